"""Benchmark: states/s of the whole-body hot path (FK + RNEA + self-collision,
forward + backward + gradient step) on the optimizer-shaped 48-DoF humanoid
workload (512 seeds x 48 timesteps = 24576 states, cost 1e-3 ||tau||^2 +
hinge(max_pen + 0.01 m)), synthetic seeded robot and states.

One "step" is one optimizer iteration over the whole batch.  Four forms are
timed on the same inputs:
  fused_graph   K iterations of the fused kernel (wb_wholebody_step) with the
                gradient step, captured in one HIP graph with a snapshot of
                state, gradient and cost every 10th iteration; after W
                eager warm-up iterations and one untimed replay (a graph's
                first launch also uploads it), the timed region is one
                replay (exactly K steps) -- the reported value; 20 more
                replays timed one by one with HIP events give its median;
  fused_graph1  a one-iteration graph of the same kernel, replayed K times;
  plain_graph   one launch per operation, captured in a HIP graph;
  plain         one launch per operation, issued eagerly (the "plain launch").
The roofline object covers the fused kernel, timed with HIP events on its
stream over an eager timed loop, with an issue-slot model beside the FLOP
model; shard_share_B3072 times the fused graph on the 3072 states one GPU
holds when the batch is split over eight; the CPU baseline is the FP64
oracle on a bounded sample of the same workload (all threads, then one).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CU x 4 SIMD x 16 lanes x 2 FLOP (FMA) x 2.4 GHz, without packed FP32
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_FP32_PUBLISHED_TFLOPS = 157.3   # needs packed FP32, which this build disables
PEAK_HBM_GBPS = 8000.0


# HBM traffic of the fused kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE passes
# (profiles/k_fused_step_humanoid48_B24576_hbm_counters.md), scaled by a copy
# calibration (FETCH x2.000, WRITE x1.000).  Valid only for the kernel sources
# and the launch shape (states per workgroup) it was measured with; reported
# as null once either changes.
TRAFFIC_MEASURED = {"sources_sha1": "34f9acce194059b226ed12f33803f5f3be188970", "states": 24576,
                    "states_per_item": 8, "bytes_per_launch": (14296.8 + 14273.5) * 1024}
FUSED_SOURCES = ("fused.hip", "sweep.h", "lanes.h", "tree.h", "spline.h", "spatial.h", "wb_internal.h")


# HBM traffic of the kinematics-outputs kernel, measured the same way
# (profiles/k_kinematics_humanoid48_B24576.md; 4 tool frames), per launch.
KIN_TRAFFIC_MEASURED = {"sources_sha1": "b54a8297dcd08b42f655f85c518d89b665149710", "states": 24576, "tools": 4,
                        "forward_bytes": (5606.6 + 133142.4) * 1024,
                        "backward_bytes": (9674.9 + 4608.0) * 1024}
KIN_SOURCES = ("kinematics.hip", "kin.h", "lanes.h", "spatial.h", "wb_internal.h")
# ... and of the three distance-transform launches on the 256 x 256 x 128 room
# (profiles/edt_room256_kernel_trace.md), summed per transform.
EDT_TRAFFIC_MEASURED = {"sources_sha1": "6204f6dc8c5a02fafb8a44743f39c46649059278", "grid": [256, 256, 128],
                        "bytes": (8242.3 + 32928.1 + 32938.4 + 32768.0 + 32768.0 + 65536.0) * 1024}
EDT_SOURCES = ("edt.hip", "edt.h")


def fused_sources_sha1(sources=FUSED_SOURCES) -> str:
    import hashlib
    h = hashlib.sha1()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2603_05493_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def nonpair_flop_per_state(L: int, S: int, n: int) -> float:
    """Work of one iteration per state outside the pair sweep (FMA = 2 FLOP),
    the per-unit figures of the work model: FK 135/link + 18/sphere; RNEA
    290/link; VJP 500/link (forward quantities kept, nothing recomputed, as
    the fused kernel does); hinge FK adjoint 2 x 15 (its two spheres) +
    38/link; cost head and step 10/joint.  Links are the jointed ones (the
    fixed root is not counted)."""
    links = L - 1
    return 135 * links + 18 * S + 290 * links + 500 * links + 30 + 38 * links + 10 * n


def algorithmic_flop_per_state(L: int, S: int, P: int, n: int) -> float:
    """The method's own work per state: every checked pair gets one distance
    (11 FLOP: difference 3, squared norm 5, radius sum and penetration 2,
    square root 1), no pruning credited, plus nonpair_flop_per_state."""
    return 11 * P + nonpair_flop_per_state(L, S, n)


BLOCK_TEST_FLOP = 9   # one link-block test: difference 3, squared norm 5, compare 1


def executed_flop_per_state(L: int, S: int, n: int, pairs_evaluated: float, block_tests: float,
                            row_tests: float = 0.0) -> float:
    """Work the fused kernel executes per state: the pairs its exact broad
    phase sweeps (padded sphere slots included), its block tests and row
    tests, plus the same non-pair work as the model."""
    return (11 * pairs_evaluated + BLOCK_TEST_FLOP * (block_tests + row_tests)
            + nonpair_flop_per_state(L, S, n))


# One VALU issue slot = one lane of one VALU instruction; the chip issues
# 256 CU x 64 lanes x 2.4 GHz of them per second (one wave64 instruction per
# SIMD every 4 cycles, 4 SIMDs per CU).
PEAK_ISSUE_TSLOTS = 256 * 64 * 2.4e9 / 1e12


def issue_slots_per_state(L: int, S: int, P: int, n: int) -> float:
    """VALU issue-slot model of one iteration per state, fixed in advance and
    crediting every pair of the pair set (no pruning): a pair costs 16 slots
    (difference 3, squared norm 3, sqrt 4 at quarter rate, radius sum and
    penetration 2, max / argmax / count selects 4); everything else is the
    FLOP model's non-pair work with every FMA paired (FLOP / 2)."""
    return 16 * P + nonpair_flop_per_state(L, S, n) / 2


def sweep_work(centres, radius, sph_link, pair_s, pair_t, nmax: int, lanes_per_state: int):
    """Pair evaluations, link-block tests and row tests that the fused
    kernel's exact broad phase executes, per state, from the kernel's own
    rule applied on the host to sphere centres `centres` [B, S, 3] (radii
    [S], link of each sphere [S], the checked pairs (pair_s, pair_t)):
      link bound: centroid C_a of the link's centres, reach R_a = max |c - C_a| + r;
      eps = 4e-6 (1 + max_a(|C_a| + R_a));
      pass 1 takes the blocks (a, b) with |C_a - C_b| <= R_a + R_b + eps and,
      in them, tests the nmax rows (sphere slots of a) against b's bound,
      evaluating the rows with |c_s - C_b| <= r_s + R_b + eps;
      if their maximum M0 < 0, pass 2 takes every block whose bound
      R_a + R_b - |C_a - C_b| >= t1 - eps, t1 = M0 or (when pass 1 evaluated
      no row) the exact maximum of the block with the largest bound, which
      costs one more block, and evaluates its rows whose row bound reaches
      t1 - eps and that pass 1 did not evaluate.
    A row costs nmax pair evaluations; each pass tests every block of the
    table, padded to a multiple of 2 x lanes_per_state.  Returns
    (pairs_evaluated [B], block_tests [B], blocks swept [B], blocks in the
    table, row_tests [B])."""
    c = np.asarray(centres, dtype=np.float64)
    r = np.asarray(radius, dtype=np.float64)
    sl = np.asarray(sph_link)
    links = np.unique(sl)
    nst = len(c)
    Cl = np.stack([c[:, sl == a].mean(1) for a in links], 1)                       # [B, nl, 3]
    Rl = np.stack([(np.linalg.norm(c[:, sl == a] - Cl[:, i:i + 1], axis=-1) + r[sl == a]).max(1)
                   for i, a in enumerate(links)], 1)                                  # [B, nl]
    ext = (np.linalg.norm(Cl, axis=-1) + Rl).max(1)
    eps = 4e-6 * (1.0 + ext)
    li = {int(a): i for i, a in enumerate(links)}
    ps, pt = np.asarray(pair_s), np.asarray(pair_t)
    la = np.array([li[int(a)] for a in sl[ps]])
    lb = np.array([li[int(b)] for b in sl[pt]])
    key = la * len(links) + lb
    blocks, inv = np.unique(key, return_inverse=True)
    A, Bb = blocks // len(links), blocks % len(links)
    d = Cl[:, A] - Cl[:, Bb]
    d2 = (d * d).sum(-1)
    s1 = Rl[:, A] + Rl[:, Bb] + eps[:, None]
    surv1 = d2 <= s1 * np.abs(s1)                                                     # [B, nblk]
    bound = Rl[:, A] + Rl[:, Bb] - np.sqrt(d2)
    diff = c[:, ps] - c[:, pt]
    pens = r[ps] + r[pt] - np.sqrt((diff * diff).sum(-1))                               # [B, P]
    # rows: (sphere s of the first link, block); their test against the second link's bound
    rkey = ps.astype(np.int64) * len(blocks) + inv
    rows, rinv = np.unique(rkey, return_inverse=True)
    r_s, r_blk = rows // len(blocks), rows % len(blocks)
    dr = c[:, r_s] - Cl[:, Bb[r_blk]]
    dr2 = (dr * dr).sum(-1)
    sr = r[r_s] + Rl[:, Bb[r_blk]] + eps[:, None]
    rpass1 = dr2 <= sr * np.abs(sr)                                                   # [B, nrows]
    rbound = r[r_s] + Rl[:, Bb[r_blk]] - np.sqrt(dr2)
    order = np.argsort(rinv, kind="stable")
    starts = np.searchsorted(rinv[order], np.arange(len(rows)))
    rmax = np.maximum.reduceat(pens[:, order], starts, axis=1)                         # [B, nrows]
    ev1 = surv1[:, r_blk] & rpass1
    M0 = np.where(ev1, rmax, -np.inf).max(1)
    need2 = M0 < 0
    none1 = ~ev1.any(1)
    border = np.argsort(inv, kind="stable")
    bstarts = np.searchsorted(inv[border], np.arange(len(blocks)))
    bmax = np.maximum.reduceat(pens[:, border], bstarts, axis=1)                       # [B, nblk]
    seed = bmax[np.arange(nst), np.argmax(bound, 1)]
    t1 = np.where(none1, seed, M0)
    lo = (t1 - eps)[:, None]
    blk2 = need2[:, None] & (bound >= lo)
    ev2 = blk2[:, r_blk] & (rbound >= lo) & ~ev1
    rows_evaluated = ev1.sum(1) + ev2.sum(1)
    swept = surv1.sum(1) + blk2.sum(1) + (need2 & none1)
    G2 = 2 * lanes_per_state
    nb = (len(blocks) + G2 - 1) // G2 * G2
    tests = nb * (1 + need2)
    row_tests = nmax * (surv1.sum(1) + blk2.sum(1))
    pairs = nmax * rows_evaluated + nmax * nmax * (need2 & none1)
    return pairs, tests, swept, len(blocks), row_tests


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=24576)
    ap.add_argument("--replays", type=int, default=20,
                    help="further replays of the K-iteration graph timed one by one with HIP events")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="seconds of FP64 oracle work timed for the CPU baseline (at most 30)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="fused_graph,fused_graph1,plain_graph,plain")
    ap.add_argument("--no-uneven", dest="uneven", action="store_false",
                    help="skip the uneven multi-tree batch measurement")
    ap.add_argument("--no-rnea-b256", dest="rnea_b256", action="store_false",
                    help="skip RNEA forward + VJP at 256 states (7-joint chain, 12-DoF tree, humanoid)")
    ap.add_argument("--no-kinematics", dest="kinematics", action="store_false",
                    help="skip the kinematics-outputs line (tool poses, CoM, Jacobians)")
    ap.add_argument("--no-ext", dest="ext", action="store_false",
                    help="skip the line of the fused variant with mimic joints and external forces")
    ap.add_argument("--no-paper-scale", dest="paper_scale", action="store_false",
                    help="skip the 162k-pair humanoid's kinematics and self-collision line")
    ap.add_argument("--no-edt", dest="edt", action="store_false",
                    help="skip the distance-transform line")
    ap.add_argument("--no-bspline", dest="bspline", action="store_false",
                    help="skip the B-spline control-point iteration measurement")
    return ap.parse_args()


def cpu_baseline(rb, st, seconds: float, chunk: int = 2048):
    """The FP64 oracle's iteration (forward + analytic backward) timed on the
    host cores: consecutive chunks of the batch's states, cycling through the
    batch, until about `seconds` of CPU work (capped at 30 s)."""
    from oracle import oracle as O
    done, i0 = 0, 0
    t0 = time.perf_counter()
    while True:
        idx = (np.arange(chunk) + i0) % st.B
        q, qd, qdd = st.q[idx], st.qd[idx], st.qdd[idx]
        R, p, c = O.fk(rb, q)
        mp, am, nc = O.self_collision(rb, c)
        tau = O.rnea(rb, q, qd, qdd)
        gc = O.self_collision_backward(rb, c, am, mp, 0.01, np.ones(len(idx)))
        O.fk_backward(rb, q, g_spheres=gc)
        O.rnea_vjp(rb, q, qd, qdd, 2e-3 * tau)
        done += len(idx)
        i0 = (i0 + chunk) % st.B
        dt = time.perf_counter() - t0
        if dt >= min(seconds, 30.0):
            break
    cores = O.num_threads()
    # the same work on one thread, over a shorter sample
    O.set_num_threads(1)
    done1, t1 = 0, time.perf_counter()
    try:
        while True:
            idx = (np.arange(256) + done1) % st.B
            q, qd, qdd = st.q[idx], st.qd[idx], st.qdd[idx]
            R, p, c = O.fk(rb, q)
            mp, am, nc = O.self_collision(rb, c)
            tau = O.rnea(rb, q, qd, qdd)
            gc = O.self_collision_backward(rb, c, am, mp, 0.01, np.ones(len(idx)))
            O.fk_backward(rb, q, g_spheres=gc)
            O.rnea_vjp(rb, q, qd, qdd, 2e-3 * tau)
            done1 += len(idx)
            dt1 = time.perf_counter() - t1
            if dt1 >= min(seconds / 3, 5.0):
                break
    finally:
        O.set_num_threads(cores)
    return {"value": done / dt, "unit": "states/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} state evaluations ({chunk}-state chunks cycling through the {st.B}-state batch) "
                      f"in {dt:.1f} s, FP64 oracle forward + analytic backward",
            "single_thread": {"value": done1 / dt1, "unit": "states/s",
                              "sample": f"{done1} state evaluations in {dt1:.1f} s on one thread"},
            "host_cpu": host_cpu_model()}


def measure_valu_peak(reps: int = 5, blocks: int = 8192, iters: int = 4096):
    """The sustained FP32 FMA rate of the GPU's vector ALUs (libwb_peak.so:
    16 independent v_fma_f32 chains per lane, packed FP32 off as in the
    library), HIP events around each launch, best of `reps`; with the clock
    it implies (256 CUs x 4 SIMDs x 16 lanes x 2 FLOP per cycle) and what
    rocminfo reports for the agent."""
    import ctypes as C
    import torch
    path = os.path.join(ROOT, "paper_2603_05493_amd", "libwb_peak.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run paper_2603_05493_amd/build.py")
    lib = C.CDLL(path)
    lib.wb_peak_fma.argtypes = [C.c_int64, C.c_int32, C.c_float, C.c_float, C.c_void_p, C.c_void_p]
    lib.wb_peak_fma.restype = C.c_int
    lib.wb_peak_fma_flop.argtypes = [C.c_int64, C.c_int32]
    lib.wb_peak_fma_flop.restype = C.c_double
    out = torch.empty(blocks * 256, device="cuda")
    s = torch.cuda.current_stream()
    launch = lambda: lib.wb_peak_fma(blocks, iters, 0.99999994, 1e-7, out.data_ptr(), s.cuda_stream)
    if launch() != 0:
        raise RuntimeError("wb_peak_fma launch failed")
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        launch()
        e1.record(s)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    assert torch.isfinite(out).all()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    tf = lib.wb_peak_fma_flop(blocks, iters) / min(ts) / 1e12
    return {"fma_tflops": tf, "implied_clock_ghz": tf * 1e3 / (cus * 4 * 16 * 2), "cus": cus,
            "kernel": "k_fma_peak: 16 independent v_fma_f32 chains per lane, 8,192 x 256 lanes x 4,096 trips",
            "rocminfo": rocminfo_agent()}


def rocminfo_agent() -> dict:
    """Compute units and maximum engine clock of the first GPU agent, as
    rocminfo prints them (empty if rocminfo is not there)."""
    import shutil
    import subprocess
    exe = shutil.which("rocminfo") or "/opt/rocm/bin/rocminfo"
    try:
        txt = subprocess.run([exe], capture_output=True, text=True, timeout=60).stdout
    except (OSError, subprocess.SubprocessError):
        return {}
    info, in_gpu = {}, False
    for line in txt.splitlines():
        line = line.strip()
        if line.startswith("Name:") and "gfx" in line:
            in_gpu = True
            info["name"] = line.split(":", 1)[1].strip()
        elif in_gpu and line.startswith("Max Clock Freq. (MHz):"):
            info["max_clock_mhz"] = int(line.split(":", 1)[1].split()[0])
        elif in_gpu and line.startswith("Compute Unit:"):
            info["compute_units"] = int(line.split(":", 1)[1].split()[0])
        if in_gpu and "max_clock_mhz" in info and "compute_units" in info:
            break
    return info


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(states shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_05493_amd import synth, wb
    from paper_2603_05493_amd.iteration import FusedIteration, OptimizerGraph, PlainIteration

    torch.cuda.set_device(0)
    B = args.batch
    rb = synth.humanoid48(seed=0)
    st = synth.states(rb, B, seed=1, q_range=1.5)
    robot = wb.Robot(rb).to_device("cuda:0")
    from paper_2603_05493_amd import tune
    tune.apply(robot, tune.load())
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a.T.astype(np.float32))).cuda()
    q0, qd0, qdd0 = d(st.q), d(st.qd), d(st.qdd)
    lr = 1e-3
    kw = dict(torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=lr)
    forms = args.forms.split(",")
    res = {}

    def make(form):
        return FusedIteration(robot, B, outputs=False, **kw) if form.startswith("fused") else \
            PlainIteration(robot, B, **kw)

    def timed_optimizer_graph(nb=None):
        sl = slice(0, nb if nb is not None else B)
        q, qd, qdd = (x[:, sl].clone() for x in (q0, qd0, qdd0))
        og = OptimizerGraph(robot, q, qd, qdd, iters=args.steps, every=10, **kw)
        for _ in range(args.warmup):
            og.lean.run(q, qd, qdd)
        og.capture()
        # one untimed replay: a captured graph's first launch also uploads it
        og.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        og.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        assert torch.isfinite(q).all() and torch.isfinite(og.hist["cost"]).all()
        # the same graph replayed `replays` more times, each bracketed by HIP
        # events on the stream it is replayed on
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.replays)]
        for e0, e1 in ev:
            e0.record(s)
            og.replay()
            e1.record(s)
        torch.cuda.synchronize()
        per_step = np.array([e0.elapsed_time(e1) for e0, e1 in ev]) / args.steps
        assert torch.isfinite(q).all()
        return dt, per_step

    def timed_graph(form):
        q, qd, qdd = q0.clone(), qd0.clone(), qdd0.clone()
        it = make(form)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            it.run(q, qd, qdd)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            it.run(q, qd, qdd)
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        assert torch.isfinite(q).all() and torch.isfinite(it.cost).all()
        return dt

    def timed_eager(form):
        q, qd, qdd = q0.clone(), qd0.clone(), qdd0.clone()
        it = make(form)
        for _ in range(args.warmup):
            it.run(q, qd, qdd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            it.run(q, qd, qdd)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps

    def timed_kernel_graph():
        """Duration of one lean fused launch: K back-to-back launches captured
        in one graph, each of `replays` replays bracketed by HIP events on
        the stream it is replayed on, divided by K.  (HIP events around each
        of K eager launches read up to 10 % more once the host falls behind
        the launch queue: the interval then holds the launch's submission.)"""
        q, qd, qdd = q0.clone(), qd0.clone(), qdd0.clone()
        it = make("fused")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            it.run(q, qd, qdd)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(args.steps):
                it.run(q, qd, qdd)
        graph.replay()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.replays)]
        for e0, e1 in ev:
            e0.record(s)
            graph.replay()
            e1.record(s)
        torch.cuda.synchronize()
        assert torch.isfinite(q).all()
        return [e0.elapsed_time(e1) / args.steps for e0, e1 in ev]

    replay_ms = None
    fused_all = None
    for form in forms:
        if form == "fused_graph":
            res[form], replay_ms = timed_optimizer_graph()
        elif "_graph" in form:
            res[form] = timed_graph(form)
        else:
            res[form] = timed_eager(form)
        # the fused kernel's own launches, timed right after the first fused
        # form (before the plain forms' memory-bound launches)
        if fused_all is None and form.startswith("fused") and robot.fused_supported:
            fused_all = timed_kernel_graph()
    fused_ms = float(np.mean(fused_all)) if fused_all is not None else None

    head = "fused_graph" if "fused_graph" in res else forms[0]
    L, S, P, n = robot.n_links, robot.n_spheres, robot.n_pairs, robot.n_dof
    flop = algorithmic_flop_per_state(L, S, P, n) * B
    out = {
        "metric": "states/s for FK+RNEA+self-collision fwd+bwd, 48-DoF, vs plain launch at 1e-4",
        "value": B / res[head],
        "unit": "states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[head] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 48-DoF humanoid tree, 240 spheres, random states)",
        "config": {"workload": "humanoid48_optimizer_B24576", "dof": n, "links": L, "spheres": S,
                   "pairs": P, "states": B, "iteration": "fk+selfcoll+rnea+cost+adjoints+sgd",
                   "form": head},
        "forms": {f: {"states_per_s": B / t, "ms_per_step": t * 1e3} for f, t in res.items()},
    }
    if replay_ms is not None:
        out["graph_replays"] = {"replays": len(replay_ms), "steps_per_replay": args.steps,
                                "ms_per_step_median": float(np.median(replay_ms)),
                                "ms_per_step_min": float(np.min(replay_ms)),
                                "states_per_s_median": B / (float(np.median(replay_ms)) * 1e-3),
                                "timing": "HIP events around each replay of the K-iteration graph"}
    if "plain" in res:
        out["speedup_vs_plain_launch"] = res["plain"] / res[head]
    if fused_ms is not None:
        achieved = flop / (fused_ms * 1e-3) / 1e12
        traffic = None
        if (fused_sources_sha1() == TRAFFIC_MEASURED["sources_sha1"] and B == TRAFFIC_MEASURED["states"]
                and robot.get_tune()["states_per_item"] == TRAFFIC_MEASURED["states_per_item"]):
            traffic = TRAFFIC_MEASURED["bytes_per_launch"]
        alg_bytes = B * (6 * 4 * n + 16)
        out["roofline"] = {"bound": "alu", "kernel": "k_fused_step", "achieved": achieved,
                           "peak": PEAK_FP32_PUBLISHED_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
                           "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                           "nonpacked_peak": PEAK_FP32_NONPACKED_TFLOPS,
                           "work": "algorithmic: every checked pair once, no pruning credited; VJP 500 FLOP/link",
                           "kernel_ms": fused_ms, "kernel_ms_median": float(np.median(fused_all)),
                           "kernel_ms_min": float(np.min(fused_all)),
                           "kernel_timing": f"{args.steps} back-to-back launches captured in one graph, HIP events "
                                            f"on the replaying stream around each of {len(fused_all)} replays, "
                                            "per launch; taken right after the optimizer-graph form",
                           "flop_per_launch": flop, "traffic": traffic,
                           "algorithmic_bytes_per_launch": alg_bytes,
                           "hbm_gbps_algorithmic": alg_bytes / (fused_ms * 1e-3) / 1e9}
        out["roofline"]["executed"] = executed_roofline(robot, rb, q0, fused_ms)
        pk = measure_valu_peak()
        pk["frac_model"] = achieved / pk["fma_tflops"]
        pk["frac_executed"] = out["roofline"]["executed"]["achieved"] / pk["fma_tflops"]
        out["roofline"]["peak_measured"] = pk
        slots = issue_slots_per_state(L, S, P, n) * B
        ach_slots = slots / (fused_ms * 1e-3) / 1e12
        out["roofline"]["issue_slot_model"] = {
            "slots_per_state": slots / B, "achieved": ach_slots, "peak": PEAK_ISSUE_TSLOTS,
            "unit": "T lane-slots/s", "frac": ach_slots / PEAK_ISSUE_TSLOTS,
            "note": "credits every pair; above 1 where the exact broad phase skips pairs the model counts"}
        if "fused_graph" in res and B > 3072:
            t_share, _ = timed_optimizer_graph(3072)
            out["shard_share_B3072"] = {
                "states": 3072, "states_per_s": 3072 / t_share, "ms_per_step": t_share * 1e3,
                "per_state_rate_vs_full_batch": (3072 / t_share) / (B / res["fused_graph"]),
                "form": "fused_graph (one GPU's share of the batch over 8 GPUs)"}
    if args.uneven:
        out["uneven_batch"] = bench_uneven(args)
    if args.ext:
        out["ext_variant"] = bench_ext_variant(args, st)
    if args.paper_scale:
        out["paper_scale_selfcollision"] = bench_paper_scale(args)
    if args.kinematics and robot.kinematics_supported:
        out["kinematics"] = bench_kinematics(args, robot, q0)
    if args.rnea_b256:
        out["rnea_fwd_bwd_B256"] = bench_rnea_b256(args)
    if args.edt:
        out["edt"] = bench_edt(args)
    if args.bspline and B % 48 == 0:
        out["bspline_front_end"] = bench_bspline(args, robot, B // 48)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(rb, st, args.cpu_seconds)
    print(json.dumps(out))


def executed_work(robot, rb, q0, G=None, sample: int = 2048):
    """The fused iteration's executed work per state on the given states:
    sphere centres from the library's own FK (wb_fk) for the first `sample`
    states and the broad phase's rule applied to them on the host
    (sweep_work) with G lanes per state (default: the robot's tuned shape)."""
    import torch
    from paper_2603_05493_amd import wb
    ns = min(sample, q0.shape[-1])
    _, sph = wb.wb_fk(robot, q0[:, :ns].contiguous(), want_pose=False)
    torch.cuda.synchronize()
    c = np.transpose(sph.cpu().numpy(), (2, 0, 1))                   # [ns, S, 3]
    ps, pt = robot.pairs()
    G = G or robot.get_tune()["lanes_per_state"]
    ev, tests, swept, nblk, rtests = sweep_work(c, rb.sphere_r, rb.sphere_link, ps, pt,
                                                robot.max_spheres_per_link, G)
    L, S, n = robot.n_links, robot.n_spheres, robot.n_dof
    return {"pairs_evaluated_per_state": float(ev.mean()), "pairs_in_model": int(robot.n_pairs),
            "blocks_swept_per_state": float(swept.mean()), "blocks": int(nblk),
            "block_tests_per_state": float(tests.mean()), "row_tests_per_state": float(rtests.mean()),
            "flop_per_state": executed_flop_per_state(L, S, n, float(ev.mean()), float(tests.mean()),
                                                      float(rtests.mean())),
            "sampled_states": ns}


def executed_roofline(robot, rb, q0, kernel_ms: float, sample: int = 2048):
    """The fused kernel's executed work on the benchmark's states
    (executed_work) times the batch over the kernel's mean time."""
    B = q0.shape[-1]
    w = executed_work(robot, rb, q0, sample=sample)
    ach = w["flop_per_state"] * B / (kernel_ms * 1e-3) / 1e12
    ns = w.pop("sampled_states")
    return {**w, "achieved": ach, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_PUBLISHED_TFLOPS,
            "frac_of_nonpacked_peak": ach / PEAK_FP32_NONPACKED_TFLOPS,
            "sample": f"broad-phase rule applied on the host to the first {ns} benchmark states' sphere centres "
                      f"(wb_fk); an evaluated row costs {robot.max_spheres_per_link} pair evaluations"}


def bench_bspline(args, robot, T: int):
    """The same optimizer load with B-spline control points as the variables:
    T trajectories of 9 control points sampled 4 times per knot interval
    (48 states each), splines -> fused iteration -> control-point gradient
    and step, one iteration captured in a HIP graph and replayed, in three
    forms: the sampling kernel writing the states for the fused iteration
    (two_launch), the fused kernel forming the samples itself from the
    control points (fused_sampling), and one kernel that also reduces the
    control-point gradient of its trajectory and steps (one_launch).  The control-point gradient carries the
    samples' dt^-1 and dt^-2 scaling, so the step is the row-normalized one:
    each joint's row of control points moves by lr = 0.01 rad RMS per
    iteration.  The summed cost before the first and after the last timed
    iteration shows the step working."""
    import torch
    from paper_2603_05493_amd import wb
    from paper_2603_05493_amd.iteration import BsplineIteration
    d, K, n_interp = robot.n_dof, 9, 4
    lr = 1e-2
    out = {"trajectories": T, "control_points": K, "n_interp": n_interp}
    for form in ("two_launch", "fused_sampling", "one_launch"):
        g = torch.Generator(device="cpu").manual_seed(3)
        U = (torch.rand((d, T, K), generator=g) * 3.0 - 1.5).cuda()
        th0 = (torch.rand((d, T), generator=g) * 3.0 - 1.5).cuda()
        it = BsplineIteration(robot, U, th0, torch.zeros_like(th0), torch.zeros_like(th0), dt=0.05,
                              n_interp=n_interp, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=lr,
                              step_rule=wb.STEP_ROW_RMS, form=form, sample_outputs=False)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            it.run(step=False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        cost0 = float(it.fused.cost.double().sum())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            it.run(step=True)
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        it.run(step=False)
        torch.cuda.synchronize()
        cost1 = float(it.fused.cost.double().sum())
        assert torch.isfinite(U).all() and np.isfinite(cost1)
        states = T * it.H
        out["states"] = states
        out[form] = {"states_per_s": states / dt, "ms_per_step": dt * 1e3,
                     "cost_sum_first": cost0, "cost_sum_last": cost1}
    out["step"] = {"rule": "row-normalized (each joint's control points move lr / rms(g) * g)", "lr": lr,
                   "iterations": args.warmup + args.steps + 1}
    out["form"] = ("two_launch: bspline_eval + fused iteration (per-joint outputs) + control-point gradient and "
                   "step; fused_sampling: the fused kernel forms the samples + the gradient and step; one_launch: "
                   "one kernel forms the samples, runs the iteration, reduces the control-point gradient of its "
                   "trajectory and steps; each captured in a graph")
    return out


def bench_paper_scale(args, batches=(1000, 3072), reps: int = 20):
    """Kinematics and self-collision at the paper's self-collision scale: the
    48-DoF humanoid with 588 spheres (162,432 checked pairs, up to 12 per
    link) at the paper's kinematics batch of 1000 states and at one GPU's
    3072-state share.  Forward: FK sphere centres (no link poses) and the
    self-collision sweep; forward + backward: FK with poses, the sweep, the
    hinge adjoint and the FK adjoint; fused iteration: the whole optimizer
    iteration (with RNEA and its adjoint and the step) in one launch.  The sweep is also timed alone in each
    of its two forms (one state per wavefront; one state per workgroup with
    its blocks over four wavefronts and a second reduce).  HIP events on the
    launching stream."""
    import torch
    from paper_2603_05493_amd import synth, wb
    rb = synth.humanoid48_paper_scale()
    from paper_2603_05493_amd import tune
    r = wb.Robot(rb).to_device("cuda:0")
    entry = tune.load().get(r.topology_key(), {})
    tune.apply(r, {r.topology_key(): entry})   # measured dispatch thresholds, if any
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    split_below = int(entry.get("sweep_split_below", 16 * cus))
    out = {"robot": "humanoid48, 588 spheres", "pairs": int(r.n_pairs), "spheres_per_link_max": r.max_spheres_per_link}

    def timed(fn):
        for _ in range(3):
            fn()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    for B in batches:
        st = synth.states(rb, B, seed=41, q_range=1.5)
        q = torch.from_numpy(np.ascontiguousarray(st.q.T.astype(np.float32))).cuda()
        S, L = r.n_spheres, r.n_links
        sph = torch.empty((S, 3, B), device="cuda")
        pose = torch.empty((L, 12, B), device="cuda")
        mp = torch.empty(B, device="cuda")
        am = torch.empty(B, dtype=torch.int32, device="cuda")
        nc = torch.empty(B, dtype=torch.int32, device="cuda")
        g_cost = torch.ones(B, device="cuda")
        g_sph = torch.empty((S, 3, B), device="cuda")
        g_q = torch.empty((r.n_dof, B), device="cuda")
        ws = r.workspace(B)
        fwd = lambda: (wb.wb_fk(r, q, spheres=sph, want_pose=False), wb.wb_self_collision(r, sph, mp, am, nc))

        def fwd_bwd():
            wb.wb_fk(r, q, link_pose=pose, spheres=sph)
            wb.wb_self_collision(r, sph, mp, am, nc)
            wb.wb_self_collision_backward(r, sph, am, mp, 0.01, g_cost, g_sph)
            wb.wb_fk_backward(r, q, g_spheres=g_sph, link_pose=pose, g_q=g_q, workspace=ws)

        t_f, t_fb = timed(fwd), timed(fwd_bwd)
        forms = {}
        for name, below in (("wave_per_state", 0), ("workgroup_per_state", 1 << 40)):
            r.set_sweep_split(below)
            forms[name] = timed(lambda: wb.wb_self_collision(r, sph, mp, am, nc)) * 1e6
        r.set_sweep_split(split_below)
        # the whole optimizer iteration in one launch (FK, RNEA, self-collision,
        # cost head, every adjoint, the step), as for the 240-sphere humanoid
        from paper_2603_05493_amd.iteration import FusedIteration
        it = FusedIteration(r, B, outputs=False, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=1e-3)
        qs, qds, qdds = q.clone(), torch.from_numpy(np.ascontiguousarray(st.qd.T.astype(np.float32))).cuda(), \
            torch.from_numpy(np.ascontiguousarray(st.qdd.T.astype(np.float32))).cuda()
        t_it = timed(lambda: it.run(qs, qds, qdds))
        assert torch.isfinite(qs).all()
        out[f"B{B}"] = {"states": B, "forward": {"states_per_s": B / t_f, "us": t_f * 1e6,
                                                  "pairs_per_s": B * r.n_pairs / t_f},
                        "forward_backward": {"states_per_s": B / t_fb, "us": t_fb * 1e6},
                        "fused_iteration": {"states_per_s": B / t_it, "us": t_it * 1e6,
                                            "form": "wb_wholebody_step with the gradient step, 12 sphere slots "
                                                    "per link, HIP events over eager launches"},
                        "sweep_us": forms, "sweep_form_by_default": "workgroup_per_state"
                        if B < split_below else "wave_per_state"}
    return out


def bench_ext_variant(args, st, reps: int = 50):
    """The fused iteration's variant with mimic joints and external link
    forces on the optimizer batch: the humanoid with each finger's distal
    joint following its proximal one (40 actuated joints for 48 links),
    forces on every link and their gradient, the step on; timed with HIP
    events, next to the lean kernel on the plain humanoid."""
    import torch
    from paper_2603_05493_amd import synth, wb
    rb = synth.humanoid48(seed=0)
    ji, jm = rb.joint_index.copy(), rb.joint_mult.copy()
    for wrist in (synth.humanoid48_tool_links()["left_wrist"], synth.humanoid48_tool_links()["right_wrist"]):
        for f in range(4):
            prox = wrist + 1 + 2 * f
            ji[prox + 1], jm[prox + 1] = ji[prox], 0.8
    remap = {j: i for i, j in enumerate(sorted(set(int(j) for j in ji if j >= 0)))}
    rb.joint_index = np.array([remap[int(j)] if j >= 0 else -1 for j in ji], dtype=np.int32)
    rb.joint_mult = synth._f32(jm)
    r = wb.Robot(rb).to_device("cuda:0")
    from paper_2603_05493_amd import tune
    tune.apply(r, tune.load())   # the same topology as the humanoid: its tuned shape
    B, n, L = st.B, rb.n_dof, rb.n_links
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a.T.astype(np.float32))).cuda()
    q, qd, qdd = d(st.q[:, :n]), d(st.qd[:, :n]), d(st.qdd[:, :n])
    g = torch.Generator(device="cpu").manual_seed(5)
    f_ext = (torch.randn((L, 6, B), generator=g) * 2.0).cuda()
    g_fext = torch.empty((L, 6, B), device="cuda")
    out = dict(cost=torch.empty(B, device="cuda"), max_pen=torch.empty(B, device="cuda"),
               argmax=torch.empty(B, dtype=torch.int32, device="cuda"),
               n_coll=torch.empty(B, dtype=torch.int32, device="cuda"))
    run = lambda: wb.wb_wholebody_step(r, q, qd, qdd, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=1e-7,
                                       f_ext=f_ext, g_fext=g_fext, **out)
    for _ in range(5):
        run()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        run()
    e1.record(s)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    return {"robot": "humanoid48 with coupled fingers (40 joints, 48 links)", "states": B, "kernel_us": t * 1e6,
            "states_per_s": B / t, "features": "mimic joints, external link forces and their gradient, step",
            "states_per_workgroup": r.get_tune()["states_per_item"]}


def bench_rnea_b256(args, reps: int = 100, B: int = 256):
    """RNEA forward and its VJP (torques, then the gradient of w . tau with
    respect to q, qd and qdd) at 256 states for a 7-joint chain, a 12-DoF
    tree and the 48-DoF humanoid, in both per-operation forms: one state per
    lane with the forward's cache, and one group of lanes per state that
    recomputes the forward in the VJP.  `reps` forward + VJP pairs captured
    in one graph (launch-bound at this size when issued eagerly), HIP events
    around its replays on the replaying stream."""
    import torch
    from paper_2603_05493_amd import synth, wb
    out = {"states": B, "timing": f"{reps} forward + VJP pairs in one graph, HIP events around 10 replays"}
    for name, rb in (("chain7", synth.serial_chain(7)), ("tree12", synth.random_tree(12)),
                     ("humanoid48", synth.humanoid48(seed=0))):
        r = wb.Robot(rb).to_device("cuda:0")
        st = synth.states(rb, B, seed=5)
        T = lambda x: torch.from_numpy(np.ascontiguousarray(x.T.astype(np.float32))).cuda()
        q, qd, qdd = T(st.q), T(st.qd), T(st.qdd)
        gt = torch.randn(q.shape, generator=torch.Generator().manual_seed(6)).cuda()
        tau, gq, gqd, gqdd = (torch.empty_like(q) for _ in range(4))
        cache = torch.empty((r.n_links, 18, B), device="cuda")
        ws = r.workspace(B)

        def cached():
            wb.wb_rnea(r, q, qd, qdd, tau=tau, cache=cache)
            wb.wb_rnea_backward(r, q, qd, qdd, cache, gt, gq, gqd, gqdd, workspace=ws)

        def recomputed():
            wb.wb_rnea(r, q, qd, qdd, tau=tau, want_cache=False)
            wb.wb_rnea_backward(r, q, qd, qdd, None, gt, gq, gqd, gqdd)

        res = {"dof": r.n_dof}
        for form, fn in (("one_state_per_lane_cached", cached), ("lane_group_recomputed", recomputed)):
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                fn()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                for _ in range(reps):
                    fn()
            graph.replay()
            torch.cuda.synchronize()
            s = torch.cuda.current_stream()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
            for e0, e1 in ev:
                e0.record(s)
                graph.replay()
                e1.record(s)
            torch.cuda.synchronize()
            us = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev])) / reps * 1e3
            assert torch.isfinite(gq).all()
            res[form] = {"us": us, "states_per_s": B / (us * 1e-6)}
        out[name] = res
    return out


def bench_kinematics(args, robot, q, reps: int = 50):
    """The kinematics outputs a least-squares solver needs at the optimizer
    batch: four tool frames (feet and wrists), the centre of mass, the four
    tool Jacobians and the CoM Jacobian in one launch, and the gradient of a
    tool-pose and CoM loss in another; each timed with HIP events on the
    stream it is launched on."""
    import torch
    from paper_2603_05493_amd import synth, wb
    names = ("left_foot", "right_foot", "left_wrist", "right_wrist")
    tl = synth.humanoid48_tool_links()
    links = [tl[k] for k in names]
    robot.set_tool_frames(links, None, np.tile([[0.0, 0.0, -0.05]], (len(links), 1)))
    n, B, T = robot.n_dof, q.shape[-1], len(links)
    out = wb.wb_kinematics(robot, q, tool_pose=True, com=True, jacobian=True, com_jacobian=True)
    g_tool = torch.randn((T, 12, B), device="cuda")
    g_com = torch.randn((3, B), device="cuda")
    g_q = torch.empty((n, B), device="cuda")

    def timed(fn):
        for _ in range(5):
            fn()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    fwd = timed(lambda: wb.wb_kinematics(robot, q, tool_pose=out["tool_pose"], com=out["com"],
                                         jacobian=out["jacobian"], com_jacobian=out["com_jacobian"]))
    bwd = timed(lambda: wb.wb_kinematics_backward(robot, q, g_tool_pose=g_tool, g_com=g_com, g_q=g_q))
    robot.set_tool_frames([])
    fwd_bytes = B * 4 * (n + 12 * T + 3 + 6 * n * T + 3 * n)
    bwd_bytes = B * 4 * (n + 12 * T + 3 + n)
    m = KIN_TRAFFIC_MEASURED
    same = (fused_sources_sha1(KIN_SOURCES) == m["sources_sha1"] and B == m["states"] and T == m["tools"])
    line = lambda t, nb, tr: {"kernel_us": t * 1e6, "states_per_s": B / t, "algorithmic_bytes_per_launch": nb,
                              "roofline": {"bound": "hbm", "achieved": nb / t / 1e9, "peak": PEAK_HBM_GBPS,
                                           "unit": "GB/s", "frac": nb / t / 1e9 / PEAK_HBM_GBPS,
                                           "traffic": tr if same else None}}
    return {"states": B, "tools": T, "kernel": "k_kinematics",
            "forward": dict(line(fwd, fwd_bytes, m["forward_bytes"]),
                            outputs="tool poses, com, tool Jacobians, com Jacobian"),
            "backward": dict(line(bwd, bwd_bytes, m["backward_bytes"]), outputs="d(tool-pose and com loss)/dq")}


def bench_edt(args, reps: int = 20):
    """The exact distance transform of a room-scan site grid: 256 x 256 x 128
    voxels (a 5.12 m x 5.12 m x 2.56 m room at the paper's 20 mm ESDF voxel),
    nearest site and distance for every voxel, three launches timed together
    with HIP events on the launching stream."""
    import torch
    from paper_2603_05493_amd import sitegrid, wb
    nx, ny, nz = 256, 256, 128
    m = torch.from_numpy(sitegrid.room(nx, ny, nz, seed=0)).cuda()
    ws = torch.empty(wb.edt_workspace_bytes(nx, ny, nz), dtype=torch.uint8, device="cuda")
    near = torch.empty((nz, ny, nx), dtype=torch.int32, device="cuda")
    dist = torch.empty((nz, ny, nx), device="cuda")
    run = lambda: wb.wb_edt(m, 0.02, nearest=near, dist=dist, workspace=ws)
    for _ in range(3):
        run()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        run()
    e1.record(s)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    N = nx * ny * nz
    # site grid read, A written; A read, Bt written; Bt read, nearest and dist written
    nbytes = N * (1 + 4 + 4 + 4 + 4 + 4 + 4)
    return {"grid": [nx, ny, nz], "voxels": N, "sites": int(m.sum().item()), "voxel_size_m": 0.02,
            "ms": t * 1e3, "voxels_per_s": N / t, "algorithmic_bytes": nbytes,
            "roofline": {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                         "frac": nbytes / t / 1e9 / PEAK_HBM_GBPS,
                         "traffic": EDT_TRAFFIC_MEASURED["bytes"]
                         if fused_sources_sha1(EDT_SOURCES) == EDT_TRAFFIC_MEASURED["sources_sha1"] else None},
            "form": "three launches: x flood (wave per row), y and z envelope+assign passes over LDS tiles"}


def bench_uneven(args):
    """Random trees of 7/12/23/48 DoF with 8192/4096/2048/1024 states: one
    persistent plan launch (the trees' shapes measured inside the plan by
    the tuner when the table has them, else the narrowest lanes with one
    round per work item; costs from the tuned table) replayed from a HIP
    graph, against one plain launch sequence per tree; the plan kernel's
    roofline from HIP events around eager launches."""
    import torch
    from paper_2603_05493_amd import synth, tune, wb
    from paper_2603_05493_amd.iteration import PlainIteration, PlanIteration

    jobs = synth.uneven_trees(seed=0)
    table = tune.load()
    robots, states = [], []
    for i, (rb, B) in enumerate(jobs):
        r = wb.Robot(rb).to_device("cuda:0")
        tune.apply(r, table)
        robots.append(r)
        st = synth.states(rb, B, seed=10 + i)
        d = lambda a: torch.from_numpy(np.ascontiguousarray(a.T.astype(np.float32))).cuda()
        states.append((d(st.q), d(st.qd), d(st.qdd)))
    Bs = [B for _, B in jobs]
    total = sum(Bs)
    kw = dict(torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=0.0)

    shapes = tune.plan_shapes(robots, Bs, table)
    measured = tune.plan_key(robots, Bs) in table
    plan = PlanIteration(robots, Bs, tunes=shapes, outputs=False, **kw)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run(states)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(states)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    t_plan = (time.perf_counter() - t0) / args.steps
    # the plan kernel alone, HIP events around each eager launch on its stream
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in ev:
        e0.record(s)
        plan.run(states)
        e1.record(s)
    torch.cuda.synchronize()
    k_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    flop = sum(algorithmic_flop_per_state(r.n_links, r.n_spheres, r.n_pairs, r.n_dof) * B
               for r, B in zip(robots, Bs))
    ach = flop / (k_ms * 1e-3) / 1e12
    # executed work: each tree's broad-phase survivors at its plan shape
    ex_trees = [executed_work(r, rb, st[0], G=shp["lanes_per_state"])
                for r, (rb, _), st, shp in zip(robots, jobs, states, shapes)]
    ex_flop = sum(w["flop_per_state"] * B for w, B in zip(ex_trees, Bs))
    ach_ex = ex_flop / (k_ms * 1e-3) / 1e12

    plains = [PlainIteration(r, B, **kw) for r, B in zip(robots, Bs)]
    for _ in range(args.warmup):
        for it, s in zip(plains, states):
            it.run(*s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for it, s in zip(plains, states):
            it.run(*s)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / args.steps
    return {"trees": [f"{rb.name}x{B}" for rb, B in jobs], "states": total,
            "plan_graph": {"states_per_s": total / t_plan, "ms_per_step": t_plan * 1e3,
                           "items": plan.plan.n_items, "workgroups": plan.plan.n_workgroups},
            "plain_per_tree": {"states_per_s": total / t_plain, "ms_per_step": t_plain * 1e3},
            "speedup": t_plain / t_plan,
            "shapes": shapes, "shapes_from": "measured inside the plan" if measured else "fixed rule",
            "roofline": {"bound": "alu", "kernel": "k_plan_step", "achieved": ach, "peak": PEAK_FP32_PUBLISHED_TFLOPS,
                         "unit": "TFLOP/s", "frac": ach / PEAK_FP32_PUBLISHED_TFLOPS,
                         "frac_of_nonpacked_peak": ach / PEAK_FP32_NONPACKED_TFLOPS, "kernel_ms": k_ms,
                         "flop_per_launch": flop,
                         "work": "algorithmic: every checked pair once, no pruning credited; VJP 500 FLOP/link",
                         "executed": {"flop_per_launch": ex_flop, "achieved": ach_ex, "unit": "TFLOP/s",
                                      "frac": ach_ex / PEAK_FP32_PUBLISHED_TFLOPS,
                                      "frac_of_nonpacked_peak": ach_ex / PEAK_FP32_NONPACKED_TFLOPS,
                                      "per_tree": [{"tree": rb.name, "states": B, "model_flop_per_state":
                                                    algorithmic_flop_per_state(r.n_links, r.n_spheres, r.n_pairs,
                                                                               r.n_dof), **w}
                                                   for (rb, B), r, w in zip(jobs, robots, ex_trees)],
                                      "sample": "broad-phase rule applied on the host to each tree's first "
                                                "2048 states' sphere centres (wb_fk) at its plan shape"}}}


if __name__ == "__main__":
    main()
