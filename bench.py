"""Benchmark: point-keyframe match candidates/s and ms per loop event, batched
vs plain, on one MI355X.

One step is one loop event through the whole hot path: keypoint grids of all
keyframes, Sim3 search-and-fuse over every (point, keyframe) pair, ADD
conflict resolution, then 10 Gauss-Newton refinement steps of the loop Sim3
on the accepted pairs.  Inputs are resident in HBM before timing starts.

  batched : one upload of the event tables + one launch sequence per event,
            replayed from a HIP graph, launched eagerly, or launched eagerly
            with consecutive events alternating between two contexts on two
            streams (one event's search overlaps the previous one's
            refinement); the headline takes the highest throughput
  plain   : the per-call pattern (one fl_search_fuse per keyframe, each
            followed by a copy of its results to the host and a stream sync;
            then each refinement step as its own call, copy and sync)

Prints one JSON line.  Headline workload: a loop event of 20 keyframes
(752x480, 1,200 keypoints each) and 15,000 map points, 300,000 dense pairs.
Secondary workloads (skipped with --quick): the uneven 60-keyframe event
with sparse covisibility pairs, ten of them in one launch, the residual
forward/backward on 50,000 pairs, the projection searches of loop verification
(one keyframe; three keyframes in one launch; two searches of one keyframe in
one launch), robust Sim3 refinement, essential-graph optimisation and a stream
of uneven events.
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

HBM_PEAK_GBS = 8000.0
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # int32 VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
FP64_PEAK_TFLOPS = 78.6                   # vector FP64
GN_ITERS = 10
HUBER = 2.45
# per accepted pair and Gauss-Newton step: 7 gradient + 28 Hessian entries,
# each w * (a*b + c*d) accumulated (5 FP64 flops), plus the match count
REFINE_F64_PER_PAIR = 35 * 5 + 1
REFINE_BYTES_PER_PAIR = 32   # one accepted-pair record read (then kept in registers)
# HBM bytes per launch measured with rocprofv3 counters, one "traffic:" line
# per kernel with the hash of the sources it was measured on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "loop_event_20kf.hbm_counters.md")
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
    """Algorithmic bytes of one search-kernel launch: every point's xyz,
    descriptor, distance invariance and id once (52 B), every keypoint's
    cell-ordered record and descriptor and owner once (52 B), every grid
    and owner-table entry once, every pair's 13 bytes of outputs once (and
    its 4-byte point index when pairs are sparse)."""
    cells = params.grid_cols * params.grid_rows
    n_kp = np.diff(ev.kp_offset)
    hash_bytes = 4 * sum(max(16, 1 << int(np.ceil(np.log2(max(2 * int(k), 1))))) for k in n_kp)
    sparse = 0 if getattr(ev, "pair_mp", None) is None else 4 * n_pairs
    return (52 * ev.n_mp + 52 * int(ev.kp_offset[-1]) + 4 * (cells + 1) * ev.n_kf + hash_bytes
            + 13 * n_pairs + sparse)


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


def cpu_baseline(ev, budget_s=12.0, max_events=20):
    """The oracle as it stands: brute-force search-and-fuse of the event,
    then 10 float64 Gauss-Newton steps on its accepted pairs; repeated until
    about budget_s."""
    import oracle
    from oracle import residual as R
    n = 0
    t0 = time.perf_counter()
    while True:
        out = oracle.search_fuse(ev, use_grid=False)
        acc = np.nonzero((out["decision"] == oracle.ADD) | (out["decision"] == oracle.FUSE))[0]
        kf = np.searchsorted(ev.pair_offset, acc, side="right") - 1
        mp = acc - ev.pair_offset[kf]
        kp = ev.kp_offset[kf] + out["best_idx"][acc]
        R.gauss_newton(ev.S_init, ev.mp_xyz[mp], ev.kp_xy[kp], kf, ev.kf_T, ev.cams[0], HUBER, iters=GN_ITERS)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= max_events:
            break
    return n, el


def cpu_worker(budget_s, start_at):
    """Child process of the CPU baseline (never touches the GPU): the loop
    event's oracle run from start_at (a wall-clock time shared by all
    workers of one measurement) for about budget_s; prints {n, el}."""
    import synth
    ev = synth.gen_c2()
    import oracle  # noqa: F401  (library loaded before the clock starts)
    delay = start_at - time.time()
    if delay > 0:
        time.sleep(delay)
    n, el = cpu_baseline(ev, budget_s, max_events=10 ** 6)
    print(json.dumps(dict(n=n, el=el, n_pairs=int(ev.pair_offset[-1]))), flush=True)


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


def run_cpu_workers(n_workers, budget_s):
    """The oracle in n_workers concurrent single-threaded child processes
    (BLAS and OpenMP held at one thread, no GPU visible); returns the
    aggregate pairs/s and the per-worker results."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    start_at = time.time() + 6.0 + 0.2 * n_workers
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(budget_s),
                               "--cpu-start", repr(start_at)], stdout=subprocess.PIPE, env=env, text=True)
             for _ in range(n_workers)]
    res = []
    for p in procs:
        out, _ = p.communicate(timeout=budget_s * 4 + 300)
        if p.returncode != 0:
            raise RuntimeError(f"cpu baseline worker failed ({p.returncode})")
        res.append(json.loads(out.strip().splitlines()[-1]))
    rate = sum(r["n"] * r["n_pairs"] / r["el"] for r in res)
    return rate, res


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

    def traffic(self, kernel):
        """HBM bytes per launch of `kernel` from the committed counter
        summary, or None when its sources changed since it was measured."""
        try:
            with open(TRAFFIC_FILE) as fh:
                lines = [ln.split() for ln in fh if ln.startswith("traffic:")]
        except OSError:
            return None
        src = "search_fused_kernel" if kernel.startswith("search_fused_kernel") else kernel
        for ln in lines:
            if len(ln) == 4 and ln[1] == kernel and ln[3] == sources_hash(src):
                return int(ln[2])
        return None

    # -- workloads -------------------------------------------------------------
    def headline(self):
        import synth
        torch, fl, ctx, args = self.torch, self.fl, self.ctx, self.args
        log("generating the loop event (20 keyframes x 1,200 keypoints, 15,000 points)")
        ev = synth.gen_c2()
        P = ev.params
        b = fl.DeviceBatch(ev, device=self.dev)
        n_pairs = b.n_pairs
        out = fl.FuseOutputs.empty(n_pairs, self.dev)

        tuning = None
        if not args.no_autotune:
            t, ms = ctx.autotune(b, P, out, reps=3)
            tuning = dict(pairs_per_lane=t[0], lds_mode=t[1], wg_per_cu=t[2], xcd_aware=t[3])
            log(f"autotune: {tuning} ({ms * 1e3:.1f} us per eager batched search)")

        # exact per-class counters of this workload (one untimed counting launch)
        ctx.set_stats(True)
        ctx.search_fuse_batched(b, P, out)
        torch.cuda.synchronize()
        st = ctx.get_stats()
        ctx.set_stats(False)

        S_init = torch.from_numpy(ev.S_init.reshape(1, 13).copy()).to(self.dev)
        S = S_init.clone()
        n_matched = torch.zeros(1, dtype=torch.int32, device=self.dev)
        host, host_S = self.host_buffers(n_pairs)

        gc.collect()
        gc.disable()   # a full collection inside a ~100 us step would be timed as GPU work
        # kernel times: eager search + refinement, HIP events around each kernel
        ctx.set_profiling(True)
        for _ in range(args.steps):
            S.copy_(S_init)
            ctx.search_fuse_batched(b, P, out, refine=(GN_ITERS, HUBER, S, None, n_matched))
        ks_ms, ks_n = ctx.get_profile("search")
        kr_ms, kr_n = ctx.get_profile("refine")
        ctx.set_profiling(False)
        ks_ms /= max(ks_n, 1)
        kr_ms /= max(kr_n, 1)
        n_acc = int(n_matched.item())

        plain = None
        if not args.no_plain:
            log(f"plain: {args.plain_steps} events, per-keyframe calls with copy + sync")
            plan = self.plain_plan(ev, b, out)
            times = [self.plain_event(plan, b, out, P, S, S_init, host, host_S)
                     for _ in range(2 + args.plain_steps)][2:]
            ms_plain = statistics.median(times)
            plain = dict(ms_per_event=ms_plain, pairs_per_s=n_pairs / (ms_plain * 1e-3),
                         p99_ms=float(np.percentile(times, 99)))
            log(f"plain: {ms_plain:.3f} ms per event")

        def step():
            # the refinement continues from the previous step's Sim3: the same
            # ten Gauss-Newton steps of work on every step
            ctx.search_fuse_graph(b, P, out, refine=(GN_ITERS, HUBER, S, None, n_matched))

        log(f"batched: warmup {args.warmup}, timing {args.steps} steps")
        ms_step = self.events_time(step, args.steps, args.warmup)
        log(f"batched: {ms_step * 1e3:.1f} us per event (device-resident)")
        ms_eager = self.events_time(
            lambda: ctx.search_fuse_batched(b, P, out, refine=(GN_ITERS, HUBER, S, None, n_matched)),
            args.steps, args.warmup)
        log(f"batched, eager launches: {ms_eager * 1e3:.1f} us per event (device-resident)")

        # consecutive steps alternating between two contexts on two streams
        # (each with its own outputs and Sim3; the inputs are shared, read
        # only): one step's search runs beside the previous step's refinement
        ctx2 = fl.Context(0)
        tv = ctx.get_tuning()
        ctx2.set_tuning(tv.pairs_per_lane, tv.lds_mode, tv.wg_per_cu, tv.xcd_aware)
        ctxs = [ctx, ctx2]
        strs = [self.stream, torch.cuda.Stream(self.dev)]
        outs = [out, fl.FuseOutputs.empty(n_pairs, self.dev)]
        Ss = [S, S.clone()]
        nms = [n_matched, torch.zeros_like(n_matched)]

        def two(i):
            k = i & 1
            ctxs[k].search_fuse_batched(b, P, outs[k], refine=(GN_ITERS, HUBER, Ss[k], None, nms[k]), stream=strs[k])
        for i in range(args.warmup):
            two(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            two(i)
        torch.cuda.synchronize()
        ms_two = (time.perf_counter() - t0) * 1e3 / args.steps
        ctx2.close()
        log(f"batched, two contexts on two streams: {ms_two * 1e3:.1f} us per event (throughput)")

        e2e = []
        for i in range(args.warmup + args.steps):
            t0 = time.perf_counter()
            step()
            for k, h in host.items():
                h.copy_(getattr(out, k), non_blocking=True)
            host_S.copy_(S, non_blocking=True)
            self.stream.synchronize()
            if i >= args.warmup:
                e2e.append((time.perf_counter() - t0) * 1e3)
        ms_e2e = statistics.median(e2e)
        gc.enable()

        # rooflines of both kernels; the one with the larger time leads
        nbytes = search_bytes(ev, P, n_pairs)
        nops = search_ops(st, n_pairs)
        t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
        t_alu = nops / (ALU_PEAK_TOPS * 1e12)
        if t_alu > t_hbm:
            rs = dict(bound="alu", achieved=nops / (ks_ms * 1e-3) / 1e12, peak=ALU_PEAK_TOPS, unit="Tops/s")
        else:
            rs = dict(bound="hbm", achieved=nbytes / (ks_ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
        tv = ctx.get_tuning()
        variant = f"search_fused_kernel<{tv.pairs_per_lane},{tv.lds_mode}>"   # <pairs per lane, LDS mode>
        rs.update(frac=rs["achieved"] / rs["peak"], traffic=self.traffic(variant), kernel=variant,
                  kernel_us=ks_ms * 1e3, alg_bytes=nbytes, alg_ops=nops, roofline_us=max(t_hbm, t_alu) * 1e6)
        rflops = REFINE_F64_PER_PAIR * n_acc * GN_ITERS
        t_f = rflops / (FP64_PEAK_TFLOPS * 1e12)
        rr = dict(bound="alu", achieved=rflops / (kr_ms * 1e-3) / 1e12, peak=FP64_PEAK_TFLOPS,
                  unit="TFLOP/s", traffic=self.traffic("refine_kernel"), kernel="refine_kernel", kernel_us=kr_ms * 1e3,
                  alg_flops=rflops, alg_bytes=REFINE_BYTES_PER_PAIR * n_acc, roofline_us=t_f * 1e6,
                  note="fp64; ten dependent steps, each one cross-CU exchange and one 7x7 solve: latency bound")
        rr["frac"] = rr["achieved"] / rr["peak"]
        roof, other = (rr, rs) if kr_ms > ks_ms else (rs, rr)
        log(f"kernels: search {ks_ms * 1e3:.1f} us, refine {kr_ms * 1e3:.1f} us ({n_acc} accepted pairs)")
        return dict(ev=ev, n_pairs=n_pairs, ms_step=ms_step, ms_e2e=ms_e2e, ms_eager=ms_eager, plain=plain,
                    tuning=tuning, roof=roof, other=other, n_acc=n_acc, ms_two=ms_two)

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
        nbytes, nops = search_bytes(ev, P, b.n_pairs), search_ops(st, b.n_pairs)
        t_hbm, t_alu = nbytes / (HBM_PEAK_GBS * 1e9), nops / (ALU_PEAK_TOPS * 1e12)
        if t_alu > t_hbm:
            roof = dict(bound="alu", achieved=nops / (ks_ms * 1e-3) / 1e12, peak=ALU_PEAK_TOPS, unit="Tops/s")
        else:
            roof = dict(bound="hbm", achieved=nbytes / (ks_ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
        roof.update(frac=roof["achieved"] / roof["peak"], kernel_us=ks_ms * 1e3, alg_bytes=nbytes, alg_ops=nops)
        if self.peaks:
            roof["frac_of_measured_peak"] = (roof["achieved"] / self.peaks["hbm_copy_gbs"] if roof["bound"] == "hbm"
                                             else roof["achieved"] * 1e12 / self.peaks["valu_lane_ops_per_s"])
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
        return res

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

    def stream_events(self, n_events):
        """The stream of uneven loop events: each event resident, one graph
        launch (search + 10 GN steps) per event.  Consecutive events alternate
        between two contexts on two streams, so one event's search overlaps
        the previous one's refinement (which keeps few CUs busy); the same
        stream on one context and one stream is reported beside it."""
        import synth
        torch, fl = self.torch, self.fl
        log(f"stream: generating {n_events} uneven events")
        evs = [synth.gen_c5_event(e) for e in range(n_events)]
        bs = [fl.DeviceBatch(ev, device=self.dev) for ev in evs]
        max_pairs = max(b.n_pairs for b in bs)
        ctxs = [self.ctx, fl.Context(0)]
        tv = self.ctx.get_tuning()
        ctxs[1].set_tuning(tv.pairs_per_lane, tv.lds_mode, tv.wg_per_cu, tv.xcd_aware)
        streams = [self.stream, torch.cuda.Stream(self.dev)]
        bufs = [fl.FuseOutputs.empty(max_pairs, self.dev) for _ in range(2)]

        def view(k, b):
            o = bufs[k]
            return fl.FuseOutputs(o.best_idx[:b.n_pairs], o.best_dist[:b.n_pairs], o.second_dist[:b.n_pairs],
                                  o.decision[:b.n_pairs], o.target[:b.n_pairs])

        outs = [[view(k, b) for b in bs] for k in range(2)]
        S_init = [torch.from_numpy(ev.S_init.reshape(1, 13).copy()).to(self.dev) for ev in evs]
        S = [s.clone() for s in S_init]
        nm = torch.zeros(n_events, dtype=torch.int32, device=self.dev)
        P = evs[0].params

        def launch(i, n_ctx):
            k = i % n_ctx
            ctxs[k].search_fuse_graph(bs[i], P, outs[k][i], refine=(GN_ITERS, HUBER, S[i], None, nm[i:i + 1]),
                                      stream=streams[k])

        def timed(n_ctx):
            for i in range(n_events):
                S[i].copy_(S_init[i])
            torch.cuda.synchronize()
            e0 = [torch.cuda.Event(enable_timing=True) for _ in range(n_events)]
            e1 = [torch.cuda.Event(enable_timing=True) for _ in range(n_events)]
            t0 = time.perf_counter()
            for i in range(n_events):
                e0[i].record(streams[i % n_ctx])
                launch(i, n_ctx)
                e1[i].record(streams[i % n_ctx])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            return wall, [e0[i].elapsed_time(e1[i]) for i in range(n_events)]

        gc.collect()
        gc.disable()
        for n_ctx in (1, 2):   # first passes: grow the workspaces to the largest event, capture
            for i in range(n_events):
                launch(i, n_ctx)
            torch.cuda.synchronize()
        wall1, per1 = timed(1)
        wall, per = timed(2)
        total = int(sum(b.n_pairs for b in bs))
        res = dict(n_events=n_events, total_pairs=total, events_per_s=n_events / wall, pairs_per_s=total / wall,
                   p50_ms=float(np.percentile(per, 50)), p99_ms=float(np.percentile(per, 99)),
                   launch="graph replays alternating between two contexts on two streams",
                   one_context=dict(events_per_s=n_events / wall1, pairs_per_s=total / wall1,
                                    p50_ms=float(np.percentile(per1, 50)), p99_ms=float(np.percentile(per1, 99))))
        errs = np.array([sim3_error(S[i].cpu().numpy()[0], ev.S_true) for i, ev in enumerate(evs)])
        res["final_rot_err_deg_median"] = float(np.median(errs[:, 0]))
        res["final_trans_err_m_median"] = float(np.median(errs[:, 1]))
        res["final_scale_err_median"] = float(np.median(errs[:, 2]))
        init = np.array([sim3_error(ev.S_init, ev.S_true) for ev in evs])
        res["init_rot_err_deg_median"] = float(np.median(init[:, 0]))
        res["init_trans_err_m_median"] = float(np.median(init[:, 1]))
        res["init_scale_err_median"] = float(np.median(init[:, 2]))
        res["failed_events"] = int((nm < 0).sum().item())
        # kernel times and the search roofline of the stream's largest event
        big = max(range(n_events), key=lambda i: bs[i].n_pairs)
        kr = self.kernel_rooflines(evs[big], bs[big], P, outs[0][big], S[big], S_init[big])
        res["largest_event"] = dict(event=big, n_pairs=bs[big].n_pairs, n_kf=bs[big].n_kf, **kr)
        if not self.args.no_plain:
            n_plain = min(n_events, self.args.stream_plain_events)
            ptimes = []
            for i in range(n_plain):
                host, host_S = self.host_buffers(bs[i].n_pairs)
                plan = self.plain_plan(evs[i], bs[i], outs[0][i])
                ptimes.append(self.plain_event(plan, bs[i], outs[0][i], P, S[i], S_init[i], host, host_S))
            res["plain_events"] = n_plain
            res["plain_p50_ms"] = float(np.percentile(ptimes, 50))
            res["plain_p99_ms"] = float(np.percentile(ptimes, 99))
            res["plain_events_per_s"] = n_plain / (sum(ptimes) * 1e-3)
            res["batched_vs_plain_same_events"] = sum(ptimes) / sum(per1[:n_plain])
        gc.enable()
        log(f"stream: {res['events_per_s']:.1f} events/s on two contexts and streams "
            f"({res['one_context']['events_per_s']:.1f} on one), p50 {res['p50_ms']:.3f} ms, p99 {res['p99_ms']:.3f} ms")
        ctxs[1].close()
        return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--stream-events", type=int, default=200)
    ap.add_argument("--stream-plain-events", type=int, default=50)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 256 MiB device copy (counter scaling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-worker", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-start", type=float, default=0.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker, args.cpu_start)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(events and keyframes shard across GPUs without exchange, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    # The CPU baselines run first, in child processes started before this
    # process touches the GPU.
    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        host = host_cpu()
        log(f"cpu baseline: oracle (brute-force search + float64 GN) on the same event, one thread "
            f"({host['nproc']} cores available, {host['model']})")
        rate1, r1 = run_cpu_workers(1, 12.0)
        n, el = r1[0]["n"], r1[0]["el"]
        cpu = dict(value=rate1, unit="pairs/s", cores=1, kind="oracle",
                   sample=f"{n} full loop events of this workload ({n * r1[0]['n_pairs']} pairs), "
                          f"single-threaded C oracle + NumPy float64 Gauss-Newton in one child process, {el:.1f} s",
                   ms_per_event=el / n * 1e3, host=host)
        workers = max(1, min(16, host["nproc"]))
        log(f"cpu baseline: the same oracle in {workers} concurrent single-threaded processes")
        rate_all, rs = run_cpu_workers(workers, 10.0)
        cpu_all = dict(value=rate_all, unit="pairs/s", cores=workers, kind="oracle",
                       sample=f"{sum(r['n'] for r in rs)} full loop events over {workers} concurrent processes "
                              f"(one thread each, ~10 s each, started together)", host=host)

    import synth
    bench = Bench(args)
    if args.copy_probe:
        bench.copy_probe()
    h = bench.headline()

    secondary = None
    hbm_meas = bench.hbm_copy_gbs()
    valu_meas = max(bench.ctx.valu_rate(iters=10000) for _ in range(3))
    log(f"measured device copy: {hbm_meas:.0f} GB/s (read + write); "
        f"measured VALU issue rate: {valu_meas / 1e12:.1f} T lane-ops/s")
    peaks = dict(hbm_copy_gbs=hbm_meas, valu_lane_ops_per_s=valu_meas,
                 note="1 GiB device copy (read + write bytes); eight independent v_xor_b32 + v_bcnt_u32_b32 "
                      "chains per lane on every CU; the rooflines use the published peaks, "
                      "frac_of_measured_peak these")
    bench.peaks = peaks
    for roof in (h["roof"], h["other"]):
        if roof["bound"] == "hbm":
            roof["frac_of_measured_peak"] = roof["achieved"] / hbm_meas
        elif roof["unit"] == "Tops/s":
            roof["frac_of_measured_peak"] = roof["achieved"] * 1e12 / valu_meas
    if not args.quick:
        secondary = {"uneven_event_60kf": bench.batch_graph(synth.gen_c3(), "uneven event", args.steps)}
        evs = [synth.gen_c3(seed=303 + i, id_base=1000 + 10 ** 6 * i, fresh_base=10 ** 9 + 10 ** 7 * i)
               for i in range(10)]
        B = synth.concat_events(evs)
        B.event_S_init = np.stack([e.S_init for e in evs])
        secondary["uneven_event_60kf_x10_one_launch"] = bench.batch_graph(B, "ten uneven events", 10)
        secondary["residual_50k"] = bench.residual()
        secondary["projection_search"] = bench.projection_search(args.steps)
        secondary["robust_refinement"] = bench.robust_refinement(args.steps)
        secondary["essential_graph"] = bench.essential_graph(args.steps)
        if args.stream_events > 0:
            secondary["stream"] = bench.stream_events(args.stream_events)

    ev, plain = h["ev"], h["plain"]
    # the batched path: one table upload and one launch sequence per event,
    # replayed from a HIP graph, launched eagerly, or launched eagerly with
    # consecutive events alternating between two contexts on two streams
    # (every event still runs its whole search and refinement), whichever
    # gives the higher throughput here
    launch, ms_best = min((("graph", h["ms_step"]), ("eager", h["ms_eager"]),
                           ("eager, consecutive events on two contexts and streams", h["ms_two"])),
                          key=lambda c: c[1])
    res = dict(
        metric="point-keyframe match candidates/s (batched loop event incl. 10 GN steps)",
        value=h["n_pairs"] / (ms_best * 1e-3), unit="pairs/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_best, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32", data="synthetic",
        config=dict(workload="loop event: 20 keyframes 752x480 x 1,200 keypoints, 15,000 points, "
                             "300,000 dense pairs; search-and-fuse + 10 Gauss-Newton Sim3 steps",
                    n_pairs=h["n_pairs"], n_kf=ev.n_kf, n_mp=ev.n_mp, gn_iters=GN_ITERS, tuning=h["tuning"],
                    launch=launch),
        ms_per_event_batched_graph=h["ms_step"], ms_per_event_batched_eager=h["ms_eager"],
        ms_per_event_batched_graph_with_d2h=h["ms_e2e"],
        ms_per_event_two_contexts_two_streams=h["ms_two"],
        pairs_per_s_two_contexts_two_streams=h["n_pairs"] / (h["ms_two"] * 1e-3),
        plain=plain,
        batched_vs_plain=(plain["ms_per_event"] / h["ms_e2e"]) if plain else None,
        batched_vs_plain_device_resident=(plain["ms_per_event"] / ms_best) if plain else None,
        matched_pairs=h["n_acc"],
        roofline=h["roof"],
        roofline_other_kernel=h["other"],
        cpu_baseline=cpu,
        cpu_baseline_all_cores=cpu_all,
        measured_peaks=peaks,
        secondary=secondary,
    )
    bench.ctx.close()
    print(json.dumps(res), flush=True)

if __name__ == "__main__":
    main()
