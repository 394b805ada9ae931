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
           "B": batch, "candidates": [[G, c, ns_per_state], ...]}}

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


def apply(robot: wb.Robot, table: Dict) -> bool:
    """Set the robot's tune record from a table entry for its topology, if any."""
    e = table.get(robot.topology_key())
    if e is None or e["lanes_per_state"] < robot.n_links:
        return False
    robot.set_tune(e["lanes_per_state"], e["states_per_item"], e.get("ns_per_state", 0.0))
    return True


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
    for desc, B in jobs:
        r = wb.Robot(desc).to_device()
        res = tune_robot(r, desc, B, reps=args.reps)
        table[r.topology_key()] = res
        print(desc.name, r.topology_key(), {k: v for k, v in res.items() if k != "candidates"}, flush=True)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)


if __name__ == "__main__":
    main()
