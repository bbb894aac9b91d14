"""The CPU code under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle, and the host side of the HIP library (argument validation, the tag
arithmetic, the allocation-free entry point's refusals), each rebuilt with
the sanitizers and exercised by the existing CPU tests in a child process
whose interpreter has the sanitizer runtime preloaded.  Any report aborts the
child.  No GPU code is instrumented (the library's kernels are compiled as
usual; only host code gets the sanitizer flags)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV_BASE = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
            "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run_child(preload, setup, tests, tmp_path):
    env = dict(os.environ)
    env.update(ENV_BASE)
    env["LD_PRELOAD"] = preload
    env["PYTHONPATH"] = ROOT + os.pathsep + os.path.join(ROOT, "tests")
    code = (setup + "\nimport pytest, sys\n"
            f"sys.exit(pytest.main({tests!r} + ['-q', '-m', 'not gpu', '-p', 'no:cacheprovider']))\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    rt = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("gcc's AddressSanitizer runtime not found")
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call([gcc, "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                           "-fno-builtin-popcount", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "fl_oracle.c"), "-o", lib,
                           "-lm"])
    setup = f"import oracle.search as s\ns._LIB = {lib!r}\n"
    _run_child(rt, setup, ["tests/test_oracle_search.py"], tmp_path)


@pytest.mark.slow
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2603_17201_amd import build as B
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    res = subprocess.run([hipcc, "-print-resource-dir"], capture_output=True, text=True).stdout.strip()
    rt = os.path.join(res, "lib", "linux", "libclang_rt.asan-x86_64.so")
    if not os.path.exists(rt):
        pytest.skip("clang's AddressSanitizer runtime not found")
    lib = str(tmp_path / "libfastloop_asan.so")
    flags = [f for f in B.compile_flags() if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer"]
    # the sanitizers for the host pass only
    flags += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all"]
    r = subprocess.run([hipcc] + flags + [os.path.join(ROOT, "paper_2603_17201_amd", "csrc", "fastloop.hip"),
                                          "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    setup = f"from paper_2603_17201_amd import _abi\n_abi.load({lib!r})\n"
    _run_child(rt, setup, ["tests/test_abi.py"], tmp_path)
