"""Benchmark: states/s of the whole-body hot path (FK + RNEA + self-collision,
forward + backward + gradient step) on the optimizer-shaped 48-DoF humanoid
workload (512 seeds x 48 timesteps = 24576 states, cost 1e-3 ||tau||^2 +
hinge(max_pen + 0.01 m)), synthetic seeded robot and states.

One "step" is one optimizer iteration over the whole batch.  Two forms are
timed: the iteration captured in a HIP graph (the reported value) and the
same kernels issued as plain per-operation launches.  The roofline object
covers the dominant kernel (the self-collision pair sweep), timed with HIP
events on its own stream during the plain-launch timed loop; the CPU
baseline is the FP64 oracle on a bounded sample of the same workload.

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

PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6: 256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz
PEAK_FP32_PUBLISHED_TFLOPS = 157.3                              # with packed FP32 (disabled in this build)
FLOP_PER_PAIR = 11.0                                           # 3 sub, 3 mul, 2 add, sqrt, add, sub


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=24576)
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def cpu_baseline(rb, st, sample: int):
    """FP64 oracle iteration (forward + analytic backward) on a sample of states."""
    from oracle import oracle as O
    idx = np.arange(min(sample, st.B))
    q, qd, qdd = st.q[idx], st.qd[idx], st.qdd[idx]
    t0 = time.perf_counter()
    R, p, c = O.fk(rb, q)
    mp, am, nc = O.self_collision(rb, c)
    tau = O.rnea(rb, q, qd, qdd)
    gc = O.self_collision_backward(rb, c, am, mp, 0.01, np.ones(len(idx)))
    O.fk_backward(rb, q, g_spheres=gc)
    O.rnea_vjp(rb, q, qd, qdd, 2e-3 * tau)
    dt = time.perf_counter() - t0
    return {"value": len(idx) / dt, "unit": "states/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"first {len(idx)} of the {st.B} states (FP64 oracle, fwd + analytic bwd)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(states shard across GPUs with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_05493_amd import synth, wb
    from paper_2603_05493_amd.iteration import PlainIteration

    torch.cuda.set_device(0)
    B = args.batch
    rb = synth.humanoid48(seed=0)
    st = synth.states(rb, B, seed=1, q_range=1.5)
    robot = wb.Robot(rb).to_device("cuda:0")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a.T.astype(np.float32))).cuda()
    q0, qd0, qdd0 = d(st.q), d(st.qd), d(st.qdd)
    lr = 1e-3

    # ---- plain per-operation launches
    q, qd, qdd = q0.clone(), qd0.clone(), qdd0.clone()
    it = PlainIteration(robot, B, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=lr)
    for _ in range(args.warmup):
        it.run(q, qd, qdd)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        wb.wb_fk(robot, q, it.pose, it.spheres)
        ev[k][0].record(stream)
        wb.wb_self_collision(robot, it.spheres, it.max_pen, it.argmax, it.n_coll)
        ev[k][1].record(stream)
        wb.wb_rnea(robot, q, qd, qdd, it.tau, it.cache)
        wb.wb_cost_head(it.tau, None, it.tw, it.max_pen, it.margin, it.hw, it.cost, it.g_tau, it.g_mp)
        wb.wb_self_collision_backward(robot, it.spheres, it.argmax, it.max_pen, it.margin, it.g_mp, it.g_spheres)
        wb.wb_fk_backward(robot, q, g_spheres=it.g_spheres, link_pose=it.pose, g_q=it.g_q_fk,
                          workspace=it.workspace)
        wb.wb_rnea_backward(robot, q, qd, qdd, it.cache, it.g_tau, it.g_q, it.g_qd, it.g_qdd, it.workspace)
        wb.wb_sgd_step(lr, q, qd, qdd, it.g_q, it.g_qd, it.g_qdd, g_q2=it.g_q_fk)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / args.steps
    sweep_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))

    # ---- the same iteration captured in a HIP graph
    q, qd, qdd = q0.clone(), qd0.clone(), qdd0.clone()
    itg = PlainIteration(robot, B, torque_weight=1e-3, margin=0.01, hinge_weight=1.0, lr=lr)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        itg.run(q, qd, qdd)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        itg.run(q, qd, qdd)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / args.steps
    assert torch.isfinite(q).all() and torch.isfinite(itg.cost).all()

    P = robot.n_pairs
    flops = FLOP_PER_PAIR * P * B
    achieved = flops / (sweep_ms * 1e-3) / 1e12
    out = {
        "metric": "states/s for FK+RNEA+self-collision fwd+bwd, 48-DoF, vs plain launch at 1e-4",
        "value": B / graph_s,
        "unit": "states/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": graph_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded 48-DoF humanoid tree, 240 spheres, random states)",
        "config": {"workload": "humanoid48_optimizer_B24576", "dof": robot.n_dof, "links": robot.n_links,
                   "spheres": robot.n_spheres, "pairs": P, "states": B,
                   "iteration": "fk+selfcoll+rnea+cost+adjoints+sgd", "form": "hip_graph"},
        "plain_launch": {"value": B / plain_s, "ms_per_step": plain_s * 1e3},
        "graph_vs_plain": plain_s / graph_s,
        "roofline": {"bound": "alu", "kernel": "k_self_collision", "achieved": achieved,
                     "peak": PEAK_FP32_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                     "frac_of_published_packed_peak": achieved / PEAK_FP32_PUBLISHED_TFLOPS,
                     "kernel_ms": sweep_ms, "flop_per_launch": flops, "traffic": None},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(rb, st, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
