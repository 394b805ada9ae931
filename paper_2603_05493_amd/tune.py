"""Per-topology autotuner for the launch shape of the fused iteration.

The paper picks its forward-kinematics kernel by robot size with a fixed
threshold (one fused kernel up to 100 spheres, two kernels above; Sec. 6.1
"adaptive kernel dispatch").  Here the shape is measured instead: for each
robot topology, every candidate (lanes per state G in {16, 32, 64} with
G >= links, states per work item) is timed on the target GPU with the whole
fused iteration, and the fastest is kept together with its measured cost per
state, which the multi-robot plan uses to balance its work list.

Results are a JSON table keyed by ``Robot.topology_key()``:
    {key: {"lanes_per_state": G, "states_per_item": c, "ns_per_state": t,
           "B": batch, "candidates": [[G, c, ns_per_state], ...],
           "sweep_split_below": n, "sweep_us": [[B, wave form us, workgroup form us], ...],
           "fk_groups_below": m, "fk_us": [[B, lane form us, group form us], ...],
           "fk_pose_groups_below": m2, "fk_pose_us": [...]}}
plus, for the uneven batch, an entry keyed by ``plan_key`` with the trees'
shapes measured inside the plan (``tune_plan``).

Usage (on the GPU):  python -m paper_2603_05493_amd.tune --out tuned.json
"""
from __future__ import annotations

import argparse
import json
import os
from typing import Dict, Iterable, Optional

import numpy as np
import torch

from . import synth, wb
from .iteration import FusedIteration

LANES = (16, 32, 64)
# states per work item: powers of two and the sizes between them, so that a
# batch can fill whole rounds of the chip's resident workgroups (a partial
# last round leaves compute units idle)
ITEMS = (4, 6, 8, 12, 16, 24, 32, 48, 64)
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "mi355x.json")


def _states(robot: wb.Robot, desc, B: int, seed: int = 0):
    st = synth.states(desc, B, seed=seed, q_range=1.5)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a.T.astype(np.float32))).to(robot.device)
    return d(st.q), d(st.qd), d(st.qdd)


def measure(robot: wb.Robot, qs, shape: Dict, reps: int = 10, warmup: int = 3) -> float:
    """Seconds per fused iteration (no step) with the given launch shape."""
    robot.set_tune(shape["lanes_per_state"], shape["states_per_item"])
    B = qs[0].shape[1]
    it = FusedIteration(robot, B, outputs=False)
    for _ in range(warmup):
        it.run(*qs, step=False)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        it.run(*qs, step=False)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) * 1e-3 / reps


def tune_robot(robot: wb.Robot, desc, B: int, lanes: Iterable[int] = LANES, items: Iterable[int] = ITEMS,
               reps: int = 20, rounds: int = 5) -> Dict:
    """Time every candidate shape `rounds` times, the candidates interleaved
    within each round so that clock and thermal drift reach all of them
    alike, and keep the one with the lowest median."""
    qs = _states(robot, desc, B)
    # a work item smaller than one round of the workgroup's 4 wavefronts
    # (4 * 64 / G states) leaves wavefronts idle, in the fused launch and in
    # a plan's work list alike: only whole rounds are candidates
    shapes = [(g, c) for g in lanes if g >= robot.n_links for c in items if c % (4 * (64 // g)) == 0]
    times = {s: [] for s in shapes}
    for _ in range(rounds):
        for g, c in shapes:
            times[(g, c)].append(measure(robot, qs, {"lanes_per_state": g, "states_per_item": c}, reps=reps))
    cands = [[g, c, float(np.median(times[(g, c)])) / B * 1e9] for g, c in shapes]
    best = min(cands, key=lambda x: x[2])
    robot.set_tune(best[0], best[1], best[2])
    return {"lanes_per_state": best[0], "states_per_item": best[1], "ns_per_state": best[2], "B": B,
            "candidates": cands}


SWEEP_BATCHES = (256, 512, 1024, 2048, 3072, 4096, 6144, 8192, 16384)


def tune_sweep_split(robot: wb.Robot, desc, batches: Iterable[int] = SWEEP_BATCHES, reps: int = 10,
                     rounds: int = 3) -> Dict:
    """The batch size below which wb_self_collision should sweep one state
    per workgroup (its blocks over four wavefronts) instead of one state per
    wavefront: both forms are timed at each batch size (interleaved rounds,
    median), and the threshold is the smallest batch from which the
    wavefront form stays at least as fast."""
    batches = list(batches)
    qs = _states(robot, desc, max(batches), seed=1)
    _, sph = wb.wb_fk(robot, qs[0], want_pose=False)
    outs = [torch.empty(max(batches), device=robot.device),
            torch.empty(max(batches), dtype=torch.int32, device=robot.device),
            torch.empty(max(batches), dtype=torch.int32, device=robot.device)]
    times = {(B, f): [] for B in batches for f in (0, 1)}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(rounds):
        for B in batches:
            sp = sph[:, :, :B].contiguous()
            o = [t[:B] for t in outs]
            for f in (0, 1):
                robot.set_dispatch((1 << 40) if f else 0, -1, -1)
                for _ in range(2):
                    wb.wb_self_collision(robot, sp, *o)
                start.record()
                for _ in range(reps):
                    wb.wb_self_collision(robot, sp, *o)
                stop.record()
                torch.cuda.synchronize()
                times[(B, f)].append(start.elapsed_time(stop) * 1e3 / reps)
    med = {k: float(np.median(v)) for k, v in times.items()}
    below = 0
    for B in batches:
        if med[(B, 1)] < med[(B, 0)]:
            below = B + 1   # the split form still wins at B
    robot.set_dispatch(below, -1, -1)
    return {"sweep_split_below": below, "sweep_us": [[B, med[(B, 0)], med[(B, 1)]] for B in batches]}


FK_BATCHES = (256, 1024, 3072, 8192, 12288, 16384, 24576)


def tune_fk_groups(robot: wb.Robot, desc, pose: bool = False, batches: Iterable[int] = FK_BATCHES, reps: int = 10,
                   rounds: int = 3) -> Dict:
    """The batch size below which wb_fk and wb_fk_backward should take one
    group of lanes per state rather than one lane per state, timed in both
    forms at each batch size (interleaved rounds, median).  pose=False: FK
    to sphere centres plus the adjoint of a sphere gradient, no link poses
    (key fk_groups_below); pose=True: FK writing link poses and sphere
    centres plus the adjoint reading the poses, as the per-operation
    iteration calls them (key fk_pose_groups_below)."""
    key = "fk_pose" if pose else "fk"
    if robot.n_links > 64:
        return {f"{key}_groups_below": 0, f"{key}_us": []}
    batches = list(batches)
    Bm = max(batches)
    qs = _states(robot, desc, Bm, seed=2)
    times = {(B, f): [] for B in batches for f in (0, 1)}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(rounds):
        for B in batches:
            q = qs[0][:, :B].contiguous()
            s_ = torch.empty((robot.n_spheres, 3, B), device=robot.device)
            lp = torch.empty((robot.n_links, 12, B), device=robot.device) if pose else None
            gq = torch.empty((robot.n_dof, B), device=robot.device)
            ws = robot.workspace(B)
            for f in (0, 1):
                t = (1 << 40) if f else 0
                robot.set_dispatch(-1, -1 if pose else t, t if pose else -1)
                run = lambda: (wb.wb_fk(robot, q, link_pose=lp, spheres=s_, want_pose=pose),
                               wb.wb_fk_backward(robot, q, g_spheres=s_, link_pose=lp, g_q=gq, workspace=ws))
                for _ in range(2):
                    run()
                start.record()
                for _ in range(reps):
                    run()
                stop.record()
                torch.cuda.synchronize()
                times[(B, f)].append(start.elapsed_time(stop) * 1e3 / reps)
    robot.set_dispatch(-1, -1, -1)
    med = {k: float(np.median(v)) for k, v in times.items()}
    below = 0
    for B in batches:
        if med[(B, 1)] < med[(B, 0)]:
            below = B + 1
    return {f"{key}_groups_below": below, f"{key}_us": [[B, med[(B, 0)], med[(B, 1)]] for B in batches]}


def apply(robot: wb.Robot, table: Dict) -> bool:
    """Set the robot's tune record (and its sweep split threshold) from a
    table entry for its topology, if any."""
    e = table.get(robot.topology_key())
    if e is None:
        return False
    robot.set_dispatch(int(e.get("sweep_split_below", -1)), int(e.get("fk_groups_below", -1)),
                       int(e.get("fk_pose_groups_below", -1)))
    if "lanes_per_state" not in e or e["lanes_per_state"] < robot.n_links or not robot.fused_supported:
        return False
    robot.set_tune(e["lanes_per_state"], e["states_per_item"], e.get("ns_per_state", 0.0))
    return True


def plan_key(robots, Bs) -> str:
    """Table key of an uneven batch: its trees' topologies and batch sizes."""
    return "plan:" + "|".join(f"{r.topology_key()}x{int(b)}" for r, b in zip(robots, Bs))


def _plan_seconds(robots, Bs, shapes, states, reps: int = 20) -> float:
    from .iteration import PlanIteration
    it = PlanIteration(robots, Bs, tunes=shapes, outputs=False, torque_weight=1e-3, margin=0.01,
                       hinge_weight=1.0, lr=0.0)
    for _ in range(3):
        it.run(states, step=False)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        it.run(states, step=False)
    stop.record()
    torch.cuda.synchronize()
    it.plan.close()
    return start.elapsed_time(stop) * 1e-3 / reps


def tune_plan(robots, descs, Bs, table: Optional[Dict] = None, passes: int = 2, rounds: int = 3) -> Dict:
    """Launch shapes of the trees of one uneven batch measured inside the
    plan: starting from plan_tune's rule, each tree's candidates (every
    group width that holds its links, one to three rounds of the workgroup
    per work item) are timed with the others held fixed -- the whole plan
    launch, median of `rounds` interleaved timings -- and the fastest kept;
    `passes` sweeps over the trees."""
    states = [_states(r, d, B, seed=7 + i) for i, (r, d, B) in enumerate(zip(robots, descs, Bs))]
    shapes = [plan_tune(r, table) for r in robots]
    history = []
    for _ in range(passes):
        for i, r in enumerate(robots):
            cands = [(g, k * 4 * (64 // g)) for g in LANES if g >= r.n_links for k in (1, 2, 3)]
            times = {c: [] for c in cands}
            for _ in range(rounds):
                for g, c in cands:
                    trial = [dict(x) for x in shapes]
                    trial[i].update(lanes_per_state=g, states_per_item=c)
                    times[(g, c)].append(_plan_seconds(robots, Bs, trial, states))
            med = {c: float(np.median(v)) for c, v in times.items()}
            g, c = min(med, key=med.get)
            shapes[i].update(lanes_per_state=g, states_per_item=c)
            history.append([i, g, c, med[(g, c)] * 1e6])
    t = _plan_seconds(robots, Bs, shapes, states)
    return {"shapes": shapes, "us": t * 1e6, "states_per_s": sum(Bs) / t, "history": history}


def plan_shapes(robots, Bs, table: Optional[Dict] = None):
    """The plan's shapes: measured ones from the table when it has this
    uneven batch, else plan_tune's rule."""
    e = (table or {}).get(plan_key(robots, Bs))
    if e is not None:
        return [dict(x) for x in e["shapes"]]
    return [plan_tune(r, table) for r in robots]


def plan_tune(robot: wb.Robot, table: Optional[Dict] = None, rounds: int = 1) -> Dict:
    """Launch shape of one tree inside a multi-robot plan.  A plan is a
    different launch from a single robot's: its workgroups (as many as the
    compute units keep resident) take work items from a balanced list, so
    fine items balance best, and the narrowest group of lanes per state
    keeps a workgroup's wavefronts on more states at once.  Measured on the
    four-tree uneven batch (trees of 7/12/23/48 joints, 8192/4096/2048/1024
    states) at three workgroups per CU: the narrowest lanes (16/16/32/64)
    with one round of the workgroup per item (4 * 64 / G states) ran at
    369-373 M states/s, with two rounds 301-312 M, and 288-289 M with the
    single-robot tune's 32 lanes for the 13-link tree.  The per-state cost
    that balances the list comes from the single-robot table when it has
    the topology."""
    g = 16 if robot.n_links <= 16 else (32 if robot.n_links <= 32 else 64)
    e = (table or {}).get(robot.topology_key(), {})
    return {"lanes_per_state": g, "states_per_item": rounds * 4 * (64 // g),
            "ns_per_state": float(e.get("ns_per_state", 0.0))}


def load(path: Optional[str] = None) -> Dict:
    path = path or DEFAULT_TABLE
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    table = {}
    jobs = [(synth.humanoid48(seed=0), 24576), (synth.serial_chain(7, 5, seed=0), 4096)]
    jobs += [(synth.random_tree(n, 6, seed=i), b) for i, (n, b) in enumerate(synth.UNEVEN_TREES)]
    robots = []
    for desc, B in jobs:
        r = wb.Robot(desc).to_device()
        res = tune_robot(r, desc, B, reps=args.reps)
        res.update(tune_sweep_split(r, desc))
        res.update(tune_fk_groups(r, desc))
        res.update(tune_fk_groups(r, desc, pose=True))
        table[r.topology_key()] = res
        robots.append((r, desc, B))
        print(desc.name, r.topology_key(),
              {k: v for k, v in res.items() if k not in ("candidates", "sweep_us", "fk_us", "fk_pose_us")}, flush=True)
    # the paper-scale humanoid: the fused iteration's shape at one GPU's 3072-state share, and the
    # per-operation thresholds
    desc = synth.humanoid48_paper_scale()
    r = wb.Robot(desc).to_device()
    e = tune_robot(r, desc, 3072, reps=args.reps)
    e.update(tune_sweep_split(r, desc))
    e.update(tune_fk_groups(r, desc))
    e.update(tune_fk_groups(r, desc, pose=True))
    table[r.topology_key()] = e
    print(desc.name, "paper scale", e["sweep_split_below"], e["fk_groups_below"], e["fk_pose_groups_below"],
          flush=True)
    # the uneven batch's shapes, measured inside the plan
    trees = robots[2:]
    pr = [t[0] for t in trees]
    Bs = [t[2] for t in trees]
    res = tune_plan(pr, [t[1] for t in trees], Bs, table)
    table[plan_key(pr, Bs)] = res
    print("plan", [(s["lanes_per_state"], s["states_per_item"]) for s in res["shapes"]], res["states_per_s"],
          flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)


if __name__ == "__main__":
    main()
