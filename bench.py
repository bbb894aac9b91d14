"""Benchmark: point-keyframe match candidates/s and ms per loop event, batched
vs plain, on one MI355X.

One step is one loop event of the stream through the whole hot path:
keypoint grids of all keyframes, Sim3 search-and-fuse over every (point,
keyframe) pair, ADD conflict resolution, then 10 Gauss-Newton refinement steps
of the loop Sim3 on the accepted pairs.  Inputs are resident in HBM before
timing starts.

Headline workload: the stream of 200 uneven loop events (5-80 keyframes of
752x480 or 512x512, 300-2,500 keypoints each, 5,000-100,000 points, every
point against every keyframe of its event: 2.2 M pairs per event on average,
7.2 M at most).  The timed steps are consecutive events of the stream, each
one batched launch sequence (table fetch, search, refinement) issued eagerly
on one stream, with HIP events around every event and every search and
refinement kernel.  value = pairs of the timed events / their wall time;
ms_per_step = that wall time / steps (one stream, so each event's own time).
Beside it: the same events replayed from HIP graphs, consecutive events
alternating between two contexts on two streams (one event's search overlaps
the previous one's refinement), and the plain path (the per-call pattern: one
fl_search_fuse per keyframe, each followed by a copy of its results to the
host and a stream sync; then each refinement step as its own call, copy and
sync) on the stream's first events.

Secondary workloads (skipped with --quick): the 20-keyframe loop event, the
uneven 60-keyframe event with sparse covisibility pairs, ten of them in one
launch, the residual forward/backward on 50,000 pairs, the projection searches
of loop verification, robust Sim3 refinement and essential-graph optimisation.
"""
from __future__ import annotations

import argparse
import dataclasses
import gc
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "point-keyframe match candidates/s and ms per loop event, batched vs plain"
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # int32 VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3                  # vector FP32
GN_ITERS = 10
HUBER = 2.45
STREAM_EVENTS = 200
# per accepted pair and Gauss-Newton step: 7 gradient + 28 Hessian entries,
# each w * (a*b + c*d) accumulated in float32 (5 flops), plus the match count
REFINE_FLOPS_PER_PAIR = 35 * 5 + 1
REFINE_BYTES_PER_PAIR = 32   # one accepted-pair record read (then kept in registers)
# HBM bytes per launch measured with rocprofv3 counters, one
# "traffic: <kernel> <workload> <bytes> <sources hash>" line per kernel and
# workload (each kernel named with the search tuning of the run: pairs per
# lane, LDS mode, workgroups per CU, XCD ordering)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_counters.md")
KERNEL_SOURCES = {
    "search_fused_kernel": ("paper_2603_17201_amd/csrc/fl_search.h", "paper_2603_17201_amd/csrc/fl_internal.h"),
    "refine_kernel": ("paper_2603_17201_amd/csrc/fl_residual.h", "paper_2603_17201_amd/csrc/fl_internal.h"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sources_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def search_bytes(ev, params, n_pairs):
    """Algorithmic bytes of one search launch (the compulsory traffic, each
    input once and each output once), summed over the launch's events: 48 B
    per point (xyz, descriptor, distance invariance), 45 B per keypoint (xy,
    octave, descriptor, owner), each keyframe's grid (cell starts and cell
    list) written once and read once, 4 B per pair of a sparse pair list,
    each keyframe's observed-point bitset over its event's points written
    once and read once, and 13 B of outputs per pair."""
    cells = params.grid_cols * params.grid_rows
    kp_off = np.asarray(ev.kp_offset, np.int64)
    ekf = np.asarray(getattr(ev, "event_kf_offset", [0, ev.n_kf]), np.int64)
    emp = np.asarray(getattr(ev, "event_mp_offset", [0, ev.n_mp]), np.int64)
    sparse = getattr(ev, "pair_mp", None) is not None
    total = 13 * n_pairs + (4 * n_pairs if sparse else 0)
    for e in range(len(ekf) - 1):
        k0, k1 = int(ekf[e]), int(ekf[e + 1])
        n_mp = int(emp[e + 1] - emp[e])
        n_kp = kp_off[k0 + 1:k1 + 1] - kp_off[k0:k1]
        total += 48 * n_mp + 45 * int(n_kp.sum()) + int(sum(2 * (4 * (cells + 1) + 4 * int(k)) for k in n_kp))
        total += -(-n_mp // 8) * 2 * (k1 - k0)
    return total


def search_ops(st, n_pairs):
    """Algorithmic VALU lane-ops of one search launch from its exact counters:
    25 per pair (tile bookkeeping, owner probe, decision, stores), 40 per
    visible pair (transform, projection, octave, window), 6 per grid cell
    scanned, 8 per keypoint scanned (record load and box / octave test) and
    20 per descriptor comparison (8 xor + 8 popcount-accumulate + key/min)."""
    return (25 * n_pairs + 40 * st["n_visible"] + 6 * st["n_cells"] + 8 * st["n_kp_scanned"]
            + 20 * st["n_cand"])


def sim3_error(S, S_ref):
    """Rotation angle (deg), translation (m) and |log scale| of S o S_ref^-1
    for 13-double Sim3s [R (9), t (3), s]."""
    R, t, s = S[:9].reshape(3, 3), S[9:12], S[12]
    R0, t0, s0 = S_ref[:9].reshape(3, 3), S_ref[9:12], S_ref[12]
    Re = R @ R0.T
    se = s / s0
    te = t - se * (Re @ t0)
    ang = np.degrees(np.arccos(np.clip((np.trace(Re) - 1.0) / 2.0, -1.0, 1.0)))
    return float(ang), float(np.linalg.norm(te)), float(abs(np.log(se)))


def oracle_event(ev, use_grid):
    """The oracle on one loop event as it stands: search-and-fuse (grid or
    brute force), then 10 float64 Gauss-Newton steps on its accepted pairs."""
    import oracle
    from oracle import residual as R
    out = oracle.search_fuse(ev, use_grid=use_grid)
    acc = np.nonzero((out["decision"] == oracle.ADD) | (out["decision"] == oracle.FUSE))[0]
    kf = np.searchsorted(ev.pair_offset, acc, side="right") - 1
    mp = acc - ev.pair_offset[kf]
    kp = ev.kp_offset[kf] + out["best_idx"][acc]
    R.gauss_newton(ev.S_init, ev.mp_xyz[mp], ev.kp_xy[kp], kf, ev.kf_T, ev.cams[0], HUBER, iters=GN_ITERS)


def cpu_worker(budget_s, start_at, first, stride, use_grid):
    """Child process of the CPU baseline (never touches the GPU): events
    first, first + stride, ... of the stream through the oracle, from
    start_at (a wall-clock time shared by all workers of one measurement)
    until about budget_s of oracle time; the events are generated outside
    the timed part.  Prints {n, el, pairs}."""
    import synth
    import oracle  # noqa: F401  (library loaded before the clock starts)
    delay = start_at - time.time()
    if delay > 0:
        time.sleep(delay)
    n, el, pairs, e = 0, 0.0, 0, first
    while el < budget_s:
        ev = synth.gen_c5_event(e % STREAM_EVENTS)
        t0 = time.perf_counter()
        oracle_event(ev, use_grid)
        el += time.perf_counter() - t0
        n += 1
        pairs += int(ev.pair_offset[-1])
        e += stride
    print(json.dumps(dict(n=n, el=el, pairs=pairs)), flush=True)


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return dict(nproc=avail, cpu_count=os.cpu_count(), model=model)


def run_cpu_workers(n_workers, budget_s, use_grid):
    """The oracle in n_workers concurrent single-threaded child processes
    (BLAS and OpenMP held at one thread, no GPU visible), worker w on stream
    events w, w + n_workers, ...; returns the aggregate pairs/s and the
    per-worker results."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    start_at = time.time() + 6.0 + 0.2 * n_workers
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(budget_s),
                               "--cpu-start", repr(start_at), "--cpu-first", str(w), "--cpu-stride", str(n_workers),
                               "--cpu-grid", str(int(use_grid))], stdout=subprocess.PIPE, env=env, text=True)
             for w in range(n_workers)]
    res = []
    for p in procs:
        out, _ = p.communicate(timeout=budget_s * 6 + 300)
        if p.returncode != 0:
            raise RuntimeError(f"cpu baseline worker failed ({p.returncode})")
        res.append(json.loads(out.strip().splitlines()[-1]))
    rate = sum(r["pairs"] / r["el"] for r in res)
    return rate, res


def search_roofline(nbytes, nops, ms, peaks=None):
    """Roofline of search launches that moved nbytes algorithmic bytes and ran
    nops algorithmic lane-ops in ms: the bound is whichever peak the work
    would take longer on."""
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = nops / (ALU_PEAK_TOPS * 1e12)
    if t_alu > t_hbm:
        r = dict(bound="alu", achieved=nops / (ms * 1e-3) / 1e12, peak=ALU_PEAK_TOPS, unit="Tops/s")
    else:
        r = dict(bound="hbm", achieved=nbytes / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    r.update(frac=r["achieved"] / r["peak"], kernel_us=ms * 1e3, alg_bytes=nbytes, alg_ops=nops,
             roofline_us=max(t_hbm, t_alu) * 1e6)
    if peaks:
        r["frac_of_measured_peak"] = (r["achieved"] / peaks["hbm_copy_gbs"] if r["bound"] == "hbm"
                                      else r["achieved"] * 1e12 / peaks["valu_lane_ops_per_s"])
    return r


def refine_roofline(n_acc, ms):
    """Roofline of refinement launches over n_acc accepted pairs in ms: the
    float32 sums of g and H against the FP32 vector peak."""
    flops = REFINE_FLOPS_PER_PAIR * n_acc * GN_ITERS
    return dict(bound="alu", achieved=flops / (ms * 1e-3) / 1e12, peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                frac=flops / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, kernel_us=ms * 1e3, alg_flops=flops,
                alg_bytes=REFINE_BYTES_PER_PAIR * n_acc, roofline_us=flops / (FP32_PEAK_TFLOPS * 1e12) * 1e6,
                note="float32 per-pair sums, float64 across workgroups; ten dependent steps, each one cross-CU "
                     "exchange and one 7x7 solve: latency bound")


class Bench:
    def __init__(self, args):
        import torch
        import paper_2603_17201_amd as fl
        self.torch, self.fl, self.args = torch, fl, args
        self.dev = torch.device("cuda:0")
        self.ctx = fl.Context(0)
        self.stream = torch.cuda.current_stream(self.dev)
        self.peaks = None   # measured HBM copy and VALU issue rates, once taken

    # -- helpers -------------------------------------------------------------
    def events_time(self, fn, steps, warmup):
        """Device time per call: HIP events on the launch stream around
        `steps` back-to-back calls, after `warmup` calls; ms."""
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(steps):
            fn()
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def host_buffers(self, n_pairs, n_events=1):
        torch = self.torch
        return ({k: torch.empty(n_pairs, dtype=dt, pin_memory=True) for k, dt in
                 (("best_idx", torch.int32), ("best_dist", torch.int16), ("second_dist", torch.int16),
                  ("decision", torch.uint8), ("target", torch.int32))},
                torch.empty((n_events, 13), dtype=torch.float64, pin_memory=True))

    def plain_plan(self, ev, b, out):
        """Per-keyframe arguments of the plain path.  Sparse pairs get their
        points gathered per keyframe once, before timing (the plain path
        then searches exactly the keyframe's pairs)."""
        torch, fl = self.torch, self.fl
        plan = []
        sparse = getattr(ev, "pair_mp", None) is not None
        ekf = getattr(ev, "event_kf_offset", np.array([0, ev.n_kf]))
        emp = getattr(ev, "event_mp_offset", np.array([0, ev.n_mp]))
        for e in range(len(ekf) - 1):
            for k in range(int(ekf[e]), int(ekf[e + 1])):
                a, c = int(ev.kp_offset[k]), int(ev.kp_offset[k + 1])
                p0, p1 = int(ev.pair_offset[k]), int(ev.pair_offset[k + 1])
                if sparse:
                    idx = torch.from_numpy(np.asarray(ev.pair_mp[p0:p1], np.int64) + int(emp[e])).to(self.dev)
                    pts = (b.mp_xyz[idx].contiguous(), b.mp_desc[idx].contiguous(), b.mp_dmax[idx].contiguous(),
                           b.mp_id[idx].contiguous())
                else:
                    m0, m1 = int(emp[e]), int(emp[e + 1])
                    pts = (b.mp_xyz[m0:m1], b.mp_desc[m0:m1], b.mp_dmax[m0:m1], b.mp_id[m0:m1])
                o = fl.FuseOutputs(out.best_idx[p0:p1], out.best_dist[p0:p1], out.second_dist[p0:p1],
                                   out.decision[p0:p1], out.target[p0:p1])
                plan.append((pts, (b.kp_xy[a:c], b.kp_oct[a:c], b.kp_desc[a:c], b.kp_owner[a:c]), o, p0, p1,
                             ev.kf_sim3[k], ev.cams[k]))
        return plan

    def plain_event(self, plan, b, out, P, S, S_init, host, host_S):
        """One event through the plain path; wall ms."""
        ctx, stream = self.ctx, self.stream
        t0 = time.perf_counter()
        for pts, kps, o, p0, p1, sim3, cam in plan:
            ctx.search_fuse(*pts, *kps, sim3, cam, P, out=o)
            for name, h in host.items():
                h[p0:p1].copy_(getattr(o, name), non_blocking=True)
            stream.synchronize()
        S.copy_(S_init)
        for _ in range(GN_ITERS):
            ctx.refine_events(b, out, (1, HUBER, S, None, None))
            host_S.copy_(S, non_blocking=True)
            stream.synchronize()
        return (time.perf_counter() - t0) * 1e3

    def hbm_copy_gbs(self):
        """Device-to-device copy of 1 GiB (read + write counted), for context
        beside the published HBM peak."""
        torch = self.torch
        x = torch.empty(256 << 20, dtype=torch.float32, device=self.dev)
        y = torch.empty_like(x)
        ms = self.events_time(lambda: y.copy_(x), 10, 2)
        del x, y
        return 2 * (1 << 30) / (ms * 1e-3) / 1e9

    def copy_probe(self):
        """A plain device copy of 256 MiB: the reference kernel for scaling
        the HBM byte counters."""
        torch = self.torch
        x = torch.empty(64 << 20, dtype=torch.float32, device=self.dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()

    def traffic(self, kernel, workload):
        """HBM bytes per launch of `kernel` on `workload` from the committed
        counter summary, or None when its sources changed since then."""
        try:
            with open(TRAFFIC_FILE) as fh:
                lines = [ln.split() for ln in fh if ln.startswith("traffic:")]
        except OSError:
            return None
        src = "search_fused_kernel" if kernel.startswith("search_fused_kernel") else kernel.split("/")[0]
        for ln in lines:
            if len(ln) == 5 and ln[1] == kernel and ln[2] == workload and ln[4] == sources_hash(src):
                return int(float(ln[3]))
        return None

    # -- workloads -------------------------------------------------------------
    def loop_event(self):
        """The loop event of 20 keyframes (752x480, 1,200 keypoints each) and
        15,000 points, 300,000 dense pairs: batched (graph, eager, two
        contexts) against the plain path."""
        import synth
        torch, fl, ctx, args = self.torch, self.fl, self.ctx, self.args
        ev = synth.gen_c2()
        P = ev.params
        b = fl.DeviceBatch(ev, device=self.dev)
        n_pairs = b.n_pairs
        out = fl.FuseOutputs.empty(n_pairs, self.dev)
        S_init = torch.from_numpy(ev.S_init.reshape(1, 13).copy()).to(self.dev)
        S = S_init.clone()
        n_matched = torch.zeros(1, dtype=torch.int32, device=self.dev)
        host, host_S = self.host_buffers(n_pairs)
        gc.collect()
        gc.disable()   # a full collection inside a ~100 us step would be timed as GPU work

        def step():
            ctx.search_fuse_graph(b, P, out, refine=(GN_ITERS, HUBER, S, None, n_matched))
        ms_graph = self.events_time(step, args.steps, args.warmup)
        ms_eager = self.events_time(
            lambda: ctx.search_fuse_batched(b, P, out, refine=(GN_ITERS, HUBER, S, None, n_matched)),
            args.steps, args.warmup)
        e2e = []
        for i in range(args.warmup + args.steps):
            t0 = time.perf_counter()
            step()
            for k, hb in host.items():
                hb.copy_(getattr(out, k), non_blocking=True)
            host_S.copy_(S, non_blocking=True)
            self.stream.synchronize()
            if i >= args.warmup:
                e2e.append((time.perf_counter() - t0) * 1e3)
        res = dict(n_pairs=n_pairs, n_kf=ev.n_kf, n_mp=ev.n_mp, ms_per_event_graph=ms_graph,
                   ms_per_event_eager=ms_eager, ms_per_event_graph_with_d2h=statistics.median(e2e),
                   pairs_per_s=n_pairs / (min(ms_graph, ms_eager) * 1e-3))
        res.update(self.kernel_rooflines(ev, b, P, out, S, S_init))
        if not args.no_plain:
            plan = self.plain_plan(ev, b, out)
            times = [self.plain_event(plan, b, out, P, S, S_init, host, host_S)
                     for _ in range(2 + args.plain_steps)][2:]
            res["plain_ms_per_event"] = statistics.median(times)
            res["batched_vs_plain"] = res["plain_ms_per_event"] / res["ms_per_event_graph_with_d2h"]
            res["batched_vs_plain_device_resident"] = res["plain_ms_per_event"] / min(ms_graph, ms_eager)
        gc.enable()
        log(f"loop event: {ms_graph * 1e3:.1f} us graph, {ms_eager * 1e3:.1f} us eager per event; search "
            f"{res['search_kernel_us']:.1f} us, refine {res['refine_kernel_us']:.1f} us")
        return res

    def kernel_rooflines(self, ev, b, P, out, S, S_init):
        """Kernel times of eager launches (search + refinement) of one batch
        and the search kernel's roofline at that size."""
        ctx, torch = self.ctx, self.torch
        ctx.set_stats(True)
        ctx.search_fuse_batched(b, P, out)
        torch.cuda.synchronize()
        st = ctx.get_stats()
        ctx.set_stats(False)
        ctx.set_profiling(True)
        for _ in range(5):
            S.copy_(S_init)
            ctx.search_fuse_batched(b, P, out, refine=(GN_ITERS, HUBER, S, None, None))
        ks_ms, ks_n = ctx.get_profile("search")
        kr_ms, kr_n = ctx.get_profile("refine")
        ctx.set_profiling(False)
        ks_ms /= max(ks_n, 1)
        kr_ms /= max(kr_n, 1)
        roof = search_roofline(search_bytes(ev, P, b.n_pairs), search_ops(st, b.n_pairs), ks_ms, self.peaks)
        return dict(search_kernel_us=ks_ms * 1e3, refine_kernel_us=kr_ms * 1e3, search_roofline=roof)

    def batch_graph(self, ev, label, steps):
        """Graph launches (search + refinement) of one batch, device-resident,
        and the plain path for a single event."""
        fl, torch, ctx = self.fl, self.torch, self.ctx
        P = ev.params
        b = fl.DeviceBatch(ev, device=self.dev)
        out = fl.FuseOutputs.empty(b.n_pairs, self.dev)
        n_ev = b.n_events
        S0 = np.asarray(ev.S_init if n_ev == 1 else ev.event_S_init).reshape(n_ev, 13)
        S_init = torch.from_numpy(S0.copy()).to(self.dev)
        S = S_init.clone()
        gc.collect()
        gc.disable()
        ms = self.events_time(lambda: ctx.search_fuse_graph(b, P, out, refine=(GN_ITERS, HUBER, S, None, None)),
                              steps, 3)
        res = dict(n_events=n_ev, n_kf=b.n_kf, n_pairs=b.n_pairs, ms_per_launch=ms, ms_per_event=ms / n_ev,
                   pairs_per_s=b.n_pairs / (ms * 1e-3))
        res.update(self.kernel_rooflines(ev, b, P, out, S, S_init))
        if n_ev == 1 and not self.args.no_plain:
            host, host_S = self.host_buffers(b.n_pairs)
            plan = self.plain_plan(ev, b, out)
            times = [self.plain_event(plan, b, out, P, S, S_init, host, host_S) for _ in range(5)][2:]
            res["plain_ms_per_event"] = statistics.median(times)
            res["batched_vs_plain_device_resident"] = res["plain_ms_per_event"] / ms
        gc.enable()
        log(f"{label}: {ms * 1e3:.1f} us per launch ({n_ev} events, {b.n_pairs} pairs)")
        return res

    def projection_search(self, steps):
        """The projection searches of loop verification (ratio test on, the
        wider window), search only and device-resident: one keyframe, and
        three keyframes in one launch against three one-keyframe calls."""
        import synth
        fl, ctx = self.fl, self.ctx
        P = synth.verification_params()
        res = dict(params=dict(win_px=P.win_px, nn_ratio=P.nn_ratio, hamming_th=P.hamming_th))
        for name, ev in (("one_keyframe", synth.gen_c1()), ("three_keyframes", synth.gen_c2(seed=212, n_kf=3))):
            b = fl.DeviceBatch(ev, device=self.dev)
            out = fl.FuseOutputs.empty(b.n_pairs, self.dev)
            plan = self.plain_plan(ev, b, out)

            def plain():
                for pts, kps, o, _p0, _p1, sim3, cam in plan:
                    ctx.search_fuse(*pts, *kps, sim3, cam, P, out=o)
            gc.collect()
            gc.disable()
            ms_plain = self.events_time(plain, steps, 3)
            ms_eager = self.events_time(lambda: ctx.search_fuse_batched(b, P, out), steps, 3)
            ms_graph = self.events_time(lambda: ctx.search_fuse_graph(b, P, out), steps, 3)
            gc.enable()
            dec = out.numpy()["decision"]
            best = min(ms_eager, ms_graph)
            res[name] = dict(n_kf=b.n_kf, n_pairs=b.n_pairs, accepted=int(((dec == fl.ADD) | (dec == fl.FUSE)).sum()),
                             us_plain_calls=ms_plain * 1e3, us_batched_eager=ms_eager * 1e3,
                             us_batched_graph=ms_graph * 1e3, pairs_per_s=b.n_pairs / (best * 1e-3),
                             batched_vs_plain=ms_plain / best)
            log(f"projection search, {name}: {best * 1e3:.1f} us batched, {ms_plain * 1e3:.1f} us in "
                f"{b.n_kf} plain call(s) ({b.n_pairs} pairs)")
        # the two searches on the current keyframe before and after the Sim3
        # optimisation: both passes in one launch against two batched calls
        ev = synth.gen_c1()
        passes = synth.ps2_passes(ev)
        b = fl.DeviceBatch(ev, device=self.dev)
        b2 = fl.DeviceBatch(dataclasses.replace(ev, kf_sim3=passes[1][1]), device=self.dev)
        outs = [fl.FuseOutputs.empty(b.n_pairs, self.dev) for _ in passes]
        spec = [(P, S, o) for (P, S), o in zip(passes, outs)]

        def two_calls():
            ctx.search_fuse_batched(b, passes[0][0], outs[0])
            ctx.search_fuse_batched(b2, passes[1][0], outs[1])
        gc.collect()
        gc.disable()
        ms_two = self.events_time(two_calls, steps, 3)
        ms_one = self.events_time(lambda: ctx.search_fuse_passes(b, spec), steps, 3)
        gc.enable()
        res["two_searches_one_keyframe"] = dict(n_pairs_per_search=b.n_pairs, us_one_launch=ms_one * 1e3,
                                                us_two_calls=ms_two * 1e3, pairs_per_s=2 * b.n_pairs / (ms_one * 1e-3),
                                                one_launch_vs_two_calls=ms_two / ms_one,
                                                params=[dict(win_px=P.win_px, nn_ratio=P.nn_ratio) for P, _ in passes])
        log(f"projection search, two searches on one keyframe: {ms_one * 1e3:.1f} us in one launch, "
            f"{ms_two * 1e3:.1f} us in two calls")
        return res

    def robust_refinement(self, steps):
        """Verification search and Sim3 refinement on a loop event with 10%
        wrong associations: ten Gauss-Newton steps, two rounds of five with
        the inlier bound, and the same rounds with Levenberg-Marquardt; one
        eager batched call per event, device-resident."""
        import synth
        fl, torch, ctx = self.fl, self.torch, self.ctx
        ev = synth.gen_c2_misplaced()
        P = synth.verification_params()
        b = fl.DeviceBatch(ev, device=self.dev)
        out = fl.FuseOutputs.empty(b.n_pairs, self.dev)
        S_init = torch.from_numpy(ev.S_init.reshape(1, 13).copy()).to(self.dev)
        S = S_init.clone()
        nm = torch.zeros(1, dtype=torch.int32, device=self.dev)
        it, rounds, tau, lm = (synth.ROBUST_ITERS, synth.ROBUST_ROUNDS, synth.ROBUST_OUTLIER_PX,
                               synth.ROBUST_LM_LAMBDA)
        variants = {"gauss_newton_10": (GN_ITERS, HUBER, S, None, nm),
                    "rounds_gauss_newton": (it, HUBER, S, None, nm, rounds, tau, 0.0),
                    "rounds_levenberg_marquardt": (it, HUBER, S, None, nm, rounds, tau, lm)}
        res = dict(workload="loop event, 20 keyframes, 300,000 pairs, 10% of planted keypoints moved 6-9 px; "
                            "verification thresholds", rounds=rounds, iters_per_round=it, outlier_px=tau,
                   lm_lambda=lm)

        def call(ref):
            S.copy_(S_init)
            ctx.search_fuse_batched(b, P, out, refine=ref)
        for name, ref in variants.items():
            gc.collect()
            gc.disable()
            ms = self.events_time(lambda: call(ref), steps, 3)
            ctx.set_profiling(True)
            for _ in range(10):
                call(ref)
            torch.cuda.synchronize()
            ms_ref, n_ref = ctx.get_profile("refine")
            ctx.get_profile("search")
            ctx.set_profiling(False)
            gc.enable()
            call(ref)
            torch.cuda.synchronize()
            deg, m, ls = sim3_error(S.cpu().numpy()[0], np.asarray(ev.S_true, np.float64).reshape(13))
            res[name] = dict(us_per_event=ms * 1e3, refine_kernel_us=ms_ref / max(n_ref, 1) * 1e3,
                             pairs_used=int(nm.item()), error_vs_true_sim3=dict(deg=deg, m=m, log_scale=ls))
            log(f"robust refinement, {name}: {ms * 1e3:.1f} us per event (refine kernel "
                f"{ms_ref / max(n_ref, 1) * 1e3:.1f} us), {int(nm.item())} pairs used, error vs true Sim3 "
                f"{deg:.2e} deg, {m:.2e} m, {ls:.2e} log scale")
        return res

    def essential_graph(self, steps):
        """Essential-graph optimisation of a loop of 1,000 keyframes (about
        3,000 odometry, covisibility and loop edges) from its drifted start:
        10 outer steps, each solved directly (banded Cholesky under a reverse
        Cuthill-McKee order) and, for comparison, by block-Jacobi conjugate
        gradients (at most 500 iterations, to 1e-10)."""
        import synth
        torch, fl, ctx = self.torch, self.fl, self.ctx
        d = synth.gen_pose_graph(n=1000, seed=606)
        S0 = torch.from_numpy(d["S0"]).to(self.dev)
        S = S0.clone()
        M = torch.from_numpy(d["M"]).to(self.dev)

        def worst(A):
            e = [sim3_error(a, b) for a, b in zip(A, d["S_true"])]
            return dict(deg=max(x[0] for x in e), m=max(x[1] for x in e), log_scale=max(x[2] for x in e))
        res = dict(n_nodes=int(S.shape[0]), n_edges=int(d["edges"].shape[0]), iters=10,
                   worst_node_error_start=worst(d["S0"]))
        for name, solver in (("direct", fl._abi.PGO_SOLVER_DIRECT), ("conjugate_gradients", fl._abi.PGO_SOLVER_CG)):
            out = {}

            def run():
                S.copy_(S0)
                out["r"] = ctx.pose_graph_optimize(S, M, d["edges"], None, iters=10, solver=solver)
            gc.collect()
            gc.disable()
            ms = self.events_time(run, max(3, steps // 5), 1)
            gc.enable()
            run()
            cost, used = (x.cpu().numpy() for x in out["r"])
            res[name] = dict(ms_per_optimisation=ms, cost_start=float(cost[0]), cost_end=float(cost[-1]),
                             cg_iterations=[int(u) for u in used], worst_node_error_end=worst(S.cpu().numpy()))
            log(f"essential graph, {name}: {ms:.2f} ms for 10 steps ({res['n_nodes']} keyframes, "
                f"{res['n_edges']} edges), cost {cost[0]:.3e} -> {cost[-1]:.3e}, CG iterations "
                f"{res[name]['cg_iterations']}")
        res["by_size"] = self.pose_graph_by_size(steps)
        return res

    def pose_graph_by_size(self, steps, graphs=((100, 1), (250, 1), (500, 1), (1000, 1), (2000, 1), (1000, 2),
                                                (1000, 3), (1000, 4))):
        """One Levenberg-Marquardt step of the essential graph on the device
        (edge Jacobians, banded assembly, direct solve, candidate cost) across
        graph sizes (n keyframes, laps of the trajectory: one loop, or
        several whose keyframes are joined to the lap before, 3 each), beside
        the CPU baseline of the linear solve alone: the same damped system,
        assembled on the host from the oracle's edge Jacobians (untimed),
        solved by LAPACK's banded Cholesky under a reverse Cuthill-McKee order
        and by SuperLU on the sparse matrix."""
        import synth
        import scipy.linalg
        import scipy.sparse
        import scipy.sparse.linalg
        from scipy.sparse.csgraph import reverse_cuthill_mckee
        from oracle import pgo as opgo
        torch, fl, ctx = self.torch, self.fl, self.ctx
        out = []
        for n, laps in graphs:
            d = synth.gen_pose_graph(n=n, seed=606, laps=laps, cross=3 if laps > 1 else 0)
            S0 = torch.from_numpy(d["S0"]).to(self.dev)
            S = S0.clone()
            M = torch.from_numpy(d["M"]).to(self.dev)

            def step():
                S.copy_(S0)
                ctx.pose_graph_optimize(S, M, d["edges"], None, iters=1, solver=fl._abi.PGO_SOLVER_DIRECT)
            gc.collect()
            gc.disable()
            dev_ms = self.events_time(step, max(3, steps // 3), 2)
            gc.enable()
            # the host system at the start poses, node 0 held
            rows, cols, vals = [], [], []
            g = np.zeros(7 * (n - 1))
            for k, (i, j) in enumerate(d["edges"]):
                e = opgo.edge_error(d["S0"][i], d["S0"][j], d["M"][k])
                Ji, Jj = opgo.edge_jacobians(d["S0"][i], d["S0"][j], d["M"][k])
                for a, Ja in ((int(i), Ji), (int(j), Jj)):
                    if a == 0:
                        continue
                    g[7 * (a - 1):7 * a] += Ja.T @ e
                    for b, Jb in ((int(i), Ji), (int(j), Jj)):
                        if b == 0:
                            continue
                        blk = Ja.T @ Jb
                        r, c = np.meshgrid(np.arange(7) + 7 * (a - 1), np.arange(7) + 7 * (b - 1), indexing="ij")
                        rows.append(r.ravel())
                        cols.append(c.ravel())
                        vals.append(blk.ravel())
            N = 7 * (n - 1)
            H = scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                        shape=(N, N))
            H = H + 1e-4 * scipy.sparse.diags(H.diagonal())
            perm = reverse_cuthill_mckee(H.tocsr(), symmetric_mode=True)
            Hp = H.tocsr()[perm][:, perm].tocoo()
            w = int(np.max(np.abs(Hp.row - Hp.col))) + 1
            band = np.zeros((w, N))   # lower form: band[i - j, j] = H[i, j], i >= j
            lo = Hp.row >= Hp.col
            band[Hp.row[lo] - Hp.col[lo], Hp.col[lo]] = Hp.data[lo]
            rhs = -g[perm]
            reps = 20 if n <= 1000 else 10

            def t_ms(f):
                f()
                t0 = time.perf_counter()
                for _ in range(reps):
                    f()
                return (time.perf_counter() - t0) / reps * 1e3
            chol_ms = t_ms(lambda: scipy.linalg.solveh_banded(band, rhs, lower=True))
            Hc = H.tocsc()
            lu_ms = t_ms(lambda: scipy.sparse.linalg.spsolve(Hc, -g))
            out.append(dict(n_keyframes=n, laps=laps, n_edges=int(d["edges"].shape[0]), unknowns=N, band_width=w,
                            device_lm_step_ms=dev_ms, cpu_banded_cholesky_solve_ms=chol_ms,
                            cpu_sparse_lu_solve_ms=lu_ms))
            log(f"essential graph, {n} keyframes, {laps} lap(s): device LM step {dev_ms:.3f} ms; CPU solve alone: banded "
                f"Cholesky {chol_ms:.3f} ms, sparse LU {lu_ms:.3f} ms (band {w} of {N} unknowns)")
        return dict(note="device: one whole Levenberg-Marquardt step (Jacobians, assembly, banded solve, candidate "
                         "cost); CPU: the linear solve alone in the benchmark process (LAPACK and SuperLU "
                         "with the process's BLAS threads), assembly excluded", sizes=out)

    def residual(self):
        import synth
        torch, fl, ctx = self.torch, self.fl, self.ctx
        d = synth.gen_c4()
        S0 = d["S_eval"]
        xyz = torch.from_numpy(d["xyz"]).to(self.dev)
        uv = torch.from_numpy(d["uv"]).to(self.dev)
        S32 = torch.from_numpy(d["S_eval_f32"]).to(self.dev)
        gc.collect()
        gc.disable()
        f = self.events_time(lambda: ctx.residual_fwd(xyz, uv, None, None, S32, d["cam"], d["huber_delta"]), 50, 5)
        bw = self.events_time(lambda: ctx.residual_bwd(xyz, uv, None, None, S32, d["cam"], d["huber_delta"]),
                              50, 5)
        # the same pairs taken as the other direction (observed through S^-1)
        S_inv32 = ctx.sim3_inverse(torch.from_numpy(S0).to(self.dev))[1]
        bwi = self.events_time(lambda: ctx.residual_bwd(xyz, uv, None, None, S_inv32, d["cam"], d["huber_delta"],
                                                        inverse=True), 50, 5)
        S0t = torch.from_numpy(S0).to(self.dev)
        xi = torch.zeros(7, dtype=torch.float64, device=self.dev, requires_grad=True)

        def fb():
            loss = fl.Sim3Residual.apply(xi, S0t, xyz, uv, None, None, d["cam"], d["huber_delta"], ctx)
            loss.backward()
        ab = self.events_time(fb, 20, 3)
        gc.enable()
        n = int(d["xyz"].shape[0])
        log(f"residual: fwd {f * 1e3:.1f} us, bwd {bw * 1e3:.1f} us, inverse-direction bwd {bwi * 1e3:.1f} us, "
            f"autograd fwd+bwd {ab * 1e3:.1f} us")
        return dict(n_pairs=n, fwd_us=f * 1e3, bwd_us=bw * 1e3, bwd_inverse_direction_us=bwi * 1e3,
                    autograd_fwd_bwd_us=ab * 1e3, bwd_pairs_per_s=n / (bw * 1e-3))

    def stream_headline(self):
        """The stream of uneven loop events, every event resident in HBM: the
        timed steps are consecutive events, each one batched launch sequence
        (table fetch, search with ADD resolution, 10 Gauss-Newton steps)."""
        import synth
        torch, fl, ctx, args = self.torch, self.fl, self.ctx, self.args
        n_events = args.stream_events
        log(f"stream: generating {n_events} uneven events")
        evs = [synth.gen_c5_event(e) for e in range(n_events)]
        bs = [fl.DeviceBatch(ev, device=self.dev) for ev in evs]
        P = evs[0].params
        bufs = [fl.FuseOutputs.empty(max(b.n_pairs for b in bs), self.dev) for _ in range(2)]

        def view(k, b):
            o = bufs[k]
            return fl.FuseOutputs(o.best_idx[:b.n_pairs], o.best_dist[:b.n_pairs], o.second_dist[:b.n_pairs],
                                  o.decision[:b.n_pairs], o.target[:b.n_pairs])

        big = max(range(n_events), key=lambda i: bs[i].n_pairs)
        tuning = None
        if args.tuning:
            t = [int(x) for x in args.tuning.split(",")]
            ctx.set_tuning(*t)
            tuning = dict(pairs_per_lane=t[0], lds_mode=t[1], wg_per_cu=t[2], xcd_aware=t[3], fixed=True)
        elif not args.no_autotune:
            # every tuning on a sample of the stream's events (twelve, from
            # the smallest to the largest), the one with the least total time
            order = sorted(range(n_events), key=lambda i: bs[i].n_pairs)
            sample = [order[int(round(j * (n_events - 1) / 11))] for j in range(12)]
            best = None
            for t in [(a, m, w, x) for a in (1, 2, 4) for m in (2, 1, 0) for w in (1, 2) for x in (0, 1)]:
                ctx.set_tuning(*t)
                for i in sample:
                    ctx.search_fuse_batched(bs[i], P, view(0, bs[i]))
                ms = self.events_time(lambda: [ctx.search_fuse_batched(bs[i], P, view(0, bs[i])) for i in sample],
                                      2, 0)
                if best is None or ms < best[1]:
                    best = (t, ms)
            t, ms = best
            ctx.set_tuning(*t)
            tuning = dict(pairs_per_lane=t[0], lds_mode=t[1], wg_per_cu=t[2], xcd_aware=t[3],
                          chosen_on="eager search of 12 stream events from the smallest to the largest")
            log(f"autotune on 12 stream events: {tuning} ({ms / 12 * 1e3:.1f} us per eager search)")
        # exact per-class counters of every event (untimed counting launches)
        ctx.set_stats(True)
        stats = []
        for i in range(n_events):
            ctx.search_fuse_batched(bs[i], P, view(0, bs[i]))
            torch.cuda.synchronize()
            stats.append(ctx.get_stats())
        ctx.set_stats(False)
        nbytes = [search_bytes(evs[i], P, bs[i].n_pairs) for i in range(n_events)]
        nops = [search_ops(stats[i], bs[i].n_pairs) for i in range(n_events)]
        S_init = [torch.from_numpy(ev.S_init.reshape(1, 13).copy()).to(self.dev) for ev in evs]
        S = [x.clone() for x in S_init]
        nm = torch.zeros(n_events, dtype=torch.int32, device=self.dev)
        ctx2 = fl.Context(0)
        tv = ctx.get_tuning()
        ctx2.set_tuning(tv.pairs_per_lane, tv.lds_mode, tv.wg_per_cu, tv.xcd_aware)
        ctxs = [ctx, ctx2]
        streams = [self.stream, torch.cuda.Stream(self.dev)]
        K, W = args.steps, args.warmup
        seq = [(W + j) % n_events for j in range(K)]   # the timed events, in order

        def launch(i, k=0, graph=False):
            c = ctxs[k]
            f = c.search_fuse_graph if graph else c.search_fuse_batched
            f(bs[i], P, view(k, bs[i]), refine=(GN_ITERS, HUBER, S[i], None, nm[i:i + 1]), stream=streams[k])

        def reset():
            for i in range(n_events):
                S[i].copy_(S_init[i])
            torch.cuda.synchronize()

        def timed(n_ctx, graph, profile=False):
            """W warmup events, then the K timed events between a device
            synchronisation and HIP events on both sides; returns (wall ms,
            per-event ms).  With profile, HIP events also bracket every event
            and the library brackets every search and refinement kernel: the
            per-event latencies and kernel times.  Each event marker holds
            the queue a few microseconds between kernels, so the throughput
            is taken from a pass without them."""
            for j in range(W):
                launch(j % n_events, j % n_ctx, graph)
            reset()
            e0 = [torch.cuda.Event(enable_timing=True) for _ in range(K)] if profile else None
            e1 = [torch.cuda.Event(enable_timing=True) for _ in range(K)] if profile else None
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            if profile:
                ctx.set_profiling(True)
            torch.cuda.synchronize()
            t0.record(streams[0])
            for k in range(1, n_ctx):
                streams[k].wait_event(t0)
            for j, i in enumerate(seq):
                k = j % n_ctx
                if profile:
                    e0[j].record(streams[k])
                launch(i, k, graph)
                if profile:
                    e1[j].record(streams[k])
            for k in range(1, n_ctx):
                streams[0].wait_stream(streams[k])
            t1.record(streams[0])
            torch.cuda.synchronize()
            return t0.elapsed_time(t1), ([e0[j].elapsed_time(e1[j]) for j in range(K)] if profile else None)

        gc.collect()
        gc.disable()
        only = args.only_eager
        if not only:
            for k in range(2):   # grow every workspace to the largest event and capture, untimed
                for i in range(n_events):
                    launch(i, k, graph=True)
                    launch(i, k, graph=False)
            torch.cuda.synchronize()
        log(f"stream: timing {K} events after {W} warmup events (eager, one stream)")
        if not only:
            wall, _ = timed(1, False)
        log(f"stream: the same events with HIP events around every event and kernel")
        wall_p, per = timed(1, False, profile=True)
        if only:
            wall = wall_p
        ks_ms, ks_n = ctx.get_profile("search")
        kr_ms, kr_n = ctx.get_profile("refine")
        ctx.set_profiling(False)
        n_acc = int(sum(int(nm[i].item()) for i in seq))
        errs = np.array([sim3_error(S[i].cpu().numpy()[0], evs[i].S_true) for i in range(n_events)])
        init = np.array([sim3_error(ev.S_init, ev.S_true) for ev in evs])
        failed = int((nm < 0).sum().item())
        wall_g = timed(1, True)[0] if not only else float("nan")
        wall_2 = timed(2, True)[0] if not only else float("nan")
        gc.enable()
        pairs = int(sum(bs[i].n_pairs for i in seq))
        sb, so = int(sum(nbytes[i] for i in seq)), int(sum(nops[i] for i in seq))
        rs = search_roofline(sb, so, ks_ms, self.peaks)
        rs.update(kernel=f"search_fused_kernel<{tv.pairs_per_lane},{tv.lds_mode}>", launches=ks_n,
                  kernel_us=ks_ms / max(ks_n, 1) * 1e3, alg_bytes=sb // max(ks_n, 1), alg_ops=so // max(ks_n, 1),
                  roofline_us=rs["roofline_us"] / max(ks_n, 1))
        tuning = f"{tv.pairs_per_lane},{tv.lds_mode},{tv.wg_per_cu},{tv.xcd_aware}"
        rs["traffic"] = self.traffic(f"{rs['kernel']}/{tuning}", "stream")
        rr = refine_roofline(n_acc, kr_ms)
        rr.update(kernel="refine_kernel", launches=kr_n, kernel_us=kr_ms / max(kr_n, 1) * 1e3,
                  alg_flops=rr["alg_flops"] // max(kr_n, 1), alg_bytes=rr["alg_bytes"] // max(kr_n, 1),
                  roofline_us=rr["roofline_us"] / max(kr_n, 1),
                  traffic=self.traffic(f"refine_kernel/{tuning}", "stream"))
        roof, other = (rs, rr) if ks_ms >= kr_ms else (rr, rs)
        res = dict(n_events=n_events, steps=K, warmup=W, pairs=pairs, wall_ms=wall, ms_per_event=wall / K,
                   pairs_per_s=pairs / (wall * 1e-3), events_per_s=K / (wall * 1e-3),
                   p50_ms=float(np.percentile(per, 50)), p99_ms=float(np.percentile(per, 99)),
                   ms_per_event_instrumented=wall_p / K,
                   search_kernel_ms_total=ks_ms, refine_kernel_ms_total=kr_ms, matched_pairs=n_acc,
                   tuning=tuning, roofline=roof, roofline_other_kernel=other,
                   graph_one_stream=dict(ms_per_event=wall_g / K, pairs_per_s=pairs / (wall_g * 1e-3)),
                   two_contexts_two_streams=dict(ms_per_event=wall_2 / K, pairs_per_s=pairs / (wall_2 * 1e-3),
                                                 events_per_s=K / (wall_2 * 1e-3),
                                                 launch="graph replays, consecutive events alternating between "
                                                        "two contexts on two streams"),
                   final_rot_err_deg_median=float(np.median(errs[:, 0])),
                   final_trans_err_m_median=float(np.median(errs[:, 1])),
                   final_scale_err_median=float(np.median(errs[:, 2])),
                   init_rot_err_deg_median=float(np.median(init[:, 0])),
                   init_trans_err_m_median=float(np.median(init[:, 1])),
                   init_scale_err_median=float(np.median(init[:, 2])), failed_events=failed)
        log(f"stream: {wall / K * 1e3:.1f} us per event eager ({pairs / (wall * 1e-3) / 1e9:.2f} G pairs/s), "
            f"{wall_g / K * 1e3:.1f} graph, {wall_2 / K * 1e3:.1f} on two contexts, {wall_p / K * 1e3:.1f} with "
            f"every event and kernel bracketed by HIP events; p50 {res['p50_ms']:.3f} ms, "
            f"p99 {res['p99_ms']:.3f} ms; kernels: search {ks_ms / max(ks_n, 1) * 1e3:.1f} us, "
            f"refine {kr_ms / max(kr_n, 1) * 1e3:.1f} us per event")
        # the stream's largest event on its own: kernel times and search roofline
        if not only:
            kr = self.kernel_rooflines(evs[big], bs[big], P, view(0, bs[big]), S[big], S_init[big])
            res["largest_event"] = dict(event=big, n_pairs=bs[big].n_pairs, n_kf=bs[big].n_kf, **kr)
        if not args.no_plain and not only:
            n_plain = min(n_events, args.stream_plain_events)
            ptimes, btimes = [], []
            for i in range(n_plain):
                host, host_S = self.host_buffers(bs[i].n_pairs)
                plan = self.plain_plan(evs[i], bs[i], view(0, bs[i]))
                ptimes.append(self.plain_event(plan, bs[i], view(0, bs[i]), P, S[i], S_init[i], host, host_S))
                S[i].copy_(S_init[i])
                btimes.append(self.events_time(lambda: launch(i), 3, 1))
            res["plain"] = dict(events=n_plain, p50_ms=float(np.percentile(ptimes, 50)),
                                p99_ms=float(np.percentile(ptimes, 99)),
                                events_per_s=n_plain / (sum(ptimes) * 1e-3))
            res["batched_vs_plain_same_events"] = sum(ptimes) / sum(btimes)
            log(f"plain path on the first {n_plain} events: p50 {res['plain']['p50_ms']:.3f} ms; batched is "
                f"{res['batched_vs_plain_same_events']:.1f}x faster on the same events")
        ctx2.close()
        res["_evs"] = evs
        return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=STREAM_EVENTS, help="timed events of the stream")
    ap.add_argument("--warmup", type=int, default=20, help="untimed events before them")
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--stream-events", type=int, default=STREAM_EVENTS)
    ap.add_argument("--stream-plain-events", type=int, default=50)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 256 MiB device copy (counter scaling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--only-eager", action="store_true",
                    help="profiling runs: the stream's instrumented eager pass alone (no uninstrumented, graph "
                         "or two-stream passes, no largest-event or plain runs), so each event's kernels are "
                         "dispatched W + K times; value is then that pass's")
    ap.add_argument("--only-ten-uneven", action="store_true",
                    help="profiling runs: only the ten uneven 60-keyframe events in one launch, --steps graph "
                         "launches after 3 untimed ones, its result as the JSON line")
    ap.add_argument("--tuning", type=str, default=None,
                    help="pairs_per_lane,lds_mode,wg_per_cu,xcd_aware instead of the autotuner's choice")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-start", type=float, default=0.0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-first", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-stride", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-grid", type=int, default=1, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker, args.cpu_start, args.cpu_first, args.cpu_stride, bool(args.cpu_grid))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(events and keyframes shard across GPUs without exchange, see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.stream_events < 1:
        print("bench.py: --steps must be >= 1, --warmup >= 0, --stream-events >= 1", file=sys.stderr)
        sys.exit(2)

    # The CPU baselines run first, in child processes started before this
    # process touches the GPU.
    cpu = cpu_extra = None
    if not args.no_cpu_baseline:
        host = host_cpu()
        log(f"cpu baseline: oracle (grid search + float64 GN) on stream events, one thread "
            f"({host['nproc']} cores available, {host['model']})")
        rate1, r1 = run_cpu_workers(1, 12.0, True)
        cpu = dict(value=rate1, unit="pairs/s", cores=1, kind="oracle",
                   sample=f"stream events 0-{r1[0]['n'] - 1} ({r1[0]['pairs']} pairs), C oracle with its keypoint "
                          f"grid + NumPy float64 Gauss-Newton, one thread in one child process, "
                          f"{r1[0]['el']:.1f} s of oracle time", host=host)
        log("cpu baseline: the brute-force oracle (every keypoint of the keyframe per pair), one thread")
        rate_b, rb = run_cpu_workers(1, 12.0, False)
        workers = max(1, min(16, host["nproc"]))
        log(f"cpu baseline: the grid oracle in {workers} concurrent single-threaded processes")
        rate_all, ra = run_cpu_workers(workers, 10.0, True)
        cpu_extra = dict(
            brute_force_one_thread=dict(value=rate_b, unit="pairs/s", cores=1, kind="oracle",
                                        sample=f"stream events 0-{rb[0]['n'] - 1} ({rb[0]['pairs']} pairs), "
                                               f"{rb[0]['el']:.1f} s of oracle time"),
            grid_all_cores=dict(value=rate_all, unit="pairs/s", cores=workers, kind="oracle",
                                sample=f"{sum(r['n'] for r in ra)} stream events over {workers} concurrent "
                                       f"processes (one thread each, ~10 s of oracle time each)"))

    import synth
    bench = Bench(args)
    if args.copy_probe:
        bench.copy_probe()
    hbm_meas = bench.hbm_copy_gbs()
    valu_meas = max(bench.ctx.valu_rate(iters=10000) for _ in range(3))
    log(f"measured device copy: {hbm_meas:.0f} GB/s (read + write); "
        f"measured VALU issue rate: {valu_meas / 1e12:.1f} T lane-ops/s")
    bench.peaks = dict(hbm_copy_gbs=hbm_meas, valu_lane_ops_per_s=valu_meas,
                       note="1 GiB device copy (read + write bytes); eight independent v_xor_b32 + v_bcnt_u32_b32 "
                            "chains per lane on every CU; the rooflines use the published peaks, "
                            "frac_of_measured_peak these")
    if args.only_ten_uneven:
        c3s = [synth.gen_c3(seed=303 + i, id_base=1000 + 10 ** 6 * i, fresh_base=10 ** 9 + 10 ** 7 * i)
               for i in range(10)]
        B = synth.concat_events(c3s)
        B.event_S_init = np.stack([e.S_init for e in c3s])
        if args.tuning:
            bench.ctx.set_tuning(*[int(x) for x in args.tuning.split(",")])
        r = bench.batch_graph(B, "ten uneven events", args.steps)
        bench.ctx.close()
        print(json.dumps(dict(workload="ten uneven 60-keyframe events in one launch", **r)), flush=True)
        return
    h = bench.stream_headline()
    evs = h.pop("_evs")

    secondary = None
    if not args.quick:
        secondary = {"loop_event_20kf": bench.loop_event()}
        secondary["uneven_event_60kf"] = bench.batch_graph(synth.gen_c3(), "uneven event", 30)
        c3s = [synth.gen_c3(seed=303 + i, id_base=1000 + 10 ** 6 * i, fresh_base=10 ** 9 + 10 ** 7 * i)
               for i in range(10)]
        B = synth.concat_events(c3s)
        B.event_S_init = np.stack([e.S_init for e in c3s])
        secondary["uneven_event_60kf_x10_one_launch"] = bench.batch_graph(B, "ten uneven events", 10)
        secondary["residual_50k"] = bench.residual()
        secondary["projection_search"] = bench.projection_search(30)
        secondary["robust_refinement"] = bench.robust_refinement(30)
        secondary["essential_graph"] = bench.essential_graph(30)

    n_kf = [int(ev.n_kf) for ev in evs]
    n_mp = [int(ev.n_mp) for ev in evs]
    res = dict(
        metric=METRIC, value=h["pairs_per_s"], unit="pairs/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=h["ms_per_event"], higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload=f"stream of {args.stream_events} uneven loop events (seeds 5000+e): 5-80 keyframes of "
                             "752x480 or 512x512, 300-2,500 keypoints each, 5,000-100,000 points, every point "
                             "against every keyframe of its event; batched search-and-fuse + 10 Gauss-Newton "
                             "Sim3 steps per event, eager launches on one stream",
                    events=args.stream_events, pairs_per_event_mean=h["pairs"] / args.steps,
                    n_kf_range=[min(n_kf), max(n_kf)], n_mp_range=[min(n_mp), max(n_mp)], gn_iters=GN_ITERS,
                    tuning=h["tuning"]),
        ms_per_event_p50=h["p50_ms"], ms_per_event_p99=h["p99_ms"], events_per_s=h["events_per_s"],
        ms_per_event_instrumented=h["ms_per_event_instrumented"],
        stream_graph_one_stream=h["graph_one_stream"],
        stream_two_contexts_two_streams=h["two_contexts_two_streams"],
        plain=h.get("plain"), batched_vs_plain_same_events=h.get("batched_vs_plain_same_events"),
        matched_pairs=h["matched_pairs"],
        sim3_error=dict(init_rot_deg_median=h["init_rot_err_deg_median"],
                        final_rot_deg_median=h["final_rot_err_deg_median"],
                        init_trans_m_median=h["init_trans_err_m_median"],
                        final_trans_m_median=h["final_trans_err_m_median"],
                        init_log_scale_median=h["init_scale_err_median"],
                        final_log_scale_median=h["final_scale_err_median"], failed_events=h["failed_events"]),
        roofline=h["roofline"],
        roofline_other_kernel=h["roofline_other_kernel"],
        largest_event=h.get("largest_event"),
        cpu_baseline=cpu,
        cpu_baseline_other=cpu_extra,
        measured_peaks=bench.peaks,
        secondary=secondary,
    )
    bench.ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
