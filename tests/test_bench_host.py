"""Host-side checks of the benchmark script: the measured-traffic records
hold every key the script reads, the frozen work models keep their values,
and a request for more than one GPU ends with a message (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_traffic_records_have_the_keys_the_bench_reads():
    assert {"sources_sha1", "states", "states_per_item", "bytes_per_launch"} <= set(bench.TRAFFIC_MEASURED)
    assert {"sources_sha1", "states", "tools", "forward_bytes", "backward_bytes"} <= set(bench.KIN_TRAFFIC_MEASURED)
    assert {"sources_sha1", "grid", "bytes"} <= set(bench.EDT_TRAFFIC_MEASURED)
    for rec in (bench.TRAFFIC_MEASURED, bench.KIN_TRAFFIC_MEASURED, bench.EDT_TRAFFIC_MEASURED):
        assert len(rec["sources_sha1"]) == 40


def test_source_hashes_cover_existing_files():
    for srcs in (bench.FUSED_SOURCES, bench.KIN_SOURCES, bench.EDT_SOURCES):
        h = bench.fused_sources_sha1(srcs)
        assert len(h) == 40 and int(h, 16) >= 0


def test_work_models_are_frozen():
    # the 48-DoF humanoid: 49 links, 240 spheres, 27,040 pairs, 48 joints;
    # per jointed link FK 135 + RNEA 290 + VJP 500 + FK adjoint 38, per sphere
    # 18, per pair 11, the hinge's two spheres 30, per joint 10
    nonpair = 48 * (135 + 290 + 500 + 38) + 240 * 18 + 30 + 48 * 10
    assert bench.nonpair_flop_per_state(49, 240, 48) == nonpair == 51054
    assert bench.algorithmic_flop_per_state(49, 240, 27040, 48) == 11 * 27040 + nonpair
    assert bench.issue_slots_per_state(49, 240, 27040, 48) == 16 * 27040 + nonpair / 2
    assert bench.executed_flop_per_state(49, 240, 48, 1000.0, 100.0) == 11 * 1000 + 9 * 100 + nonpair
    assert bench.PEAK_FP32_NONPACKED_TFLOPS == pytest.approx(78.6432)
    assert bench.PEAK_ISSUE_TSLOTS == pytest.approx(39.3216)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_tuned_shapes_are_whole_workgroup_rounds():
    """Every shape in the shipped tuning table keeps all four wavefronts of
    a workgroup busy (a multiple of 4 * 64 / G states) and is valid."""
    import json
    path = os.path.join(ROOT, "paper_2603_05493_amd", "tuned", "mi355x.json")
    with open(path) as f:
        table = json.load(f)
    assert table
    for key, e in table.items():
        if key.startswith("plan:"):   # an uneven batch's shapes, measured inside the plan
            for sh in e["shapes"]:
                g, c = sh["lanes_per_state"], sh["states_per_item"]
                assert g in (16, 32, 64) and c % (4 * (64 // g)) == 0, key
            continue
        if "sweep_split_below" in e:
            assert e["sweep_split_below"] >= 0 and len(e["sweep_us"]) > 0, key
        for k in ("fk_groups_below", "fk_pose_groups_below"):
            if k in e:
                assert e[k] >= 0, key
        if "lanes_per_state" not in e:   # a robot beyond the fused iteration: the sweep split only
            continue
        g, c = e["lanes_per_state"], e["states_per_item"]
        assert g in (16, 32, 64), key
        assert c % (4 * (64 // g)) == 0, key
        assert e["ns_per_state"] > 0, key
        best = min(e["candidates"], key=lambda x: x[2])
        assert [g, c] == best[:2], key


def _bounded_robot(oracle):
    from paper_2603_05493_amd import synth
    rb = synth.humanoid48(seed=0)
    st = synth.states(rb, 64, seed=1, q_range=1.5)
    _, _, c = oracle.fk(rb, st.q)
    s, t = oracle.pairs(rb)
    return rb, c, s, t


def test_sweep_work_rule_is_exact_and_counts_what_it_sweeps(oracle):
    """The broad-phase rule the executed-work figure applies: the block and
    the row it keeps hold the state's most penetrating pair (the rule is
    exact), and its counts are consistent (nmax evaluations per evaluated
    row, nmax row tests per swept block, block tests a padded multiple of
    the table once or twice)."""
    rb, c, s, t = _bounded_robot(oracle)
    nmax = int(np.bincount(rb.sphere_link).max())
    ev, tests, swept, nblk, rtests = bench.sweep_work(c, rb.sphere_r, rb.sphere_link, s, t, nmax, 64)
    assert np.all(ev % nmax == 0) and np.all(ev >= nmax)
    assert np.all(ev <= nmax * nmax * swept)
    assert np.all(rtests <= nmax * swept) and np.all(rtests >= nmax)
    nb = (nblk + 127) // 128 * 128
    assert set(np.unique(tests)) <= {nb, 2 * nb}
    assert np.all(swept >= 1) and np.all(swept <= nblk + 1)
    # exactness: re-derive the kept block and row of an argmax pair
    mp, am, _ = oracle.self_collision(rb, c)
    sl = rb.sphere_link
    links = np.unique(sl)
    for b in range(c.shape[0]):
        C = {a: c[b, sl == a].mean(0) for a in links}
        R = {a: (np.linalg.norm(c[b, sl == a] - C[a], axis=1) + rb.sphere_r[sl == a]).max() for a in links}
        sa, la, lb = s[am[b]], sl[s[am[b]]], sl[t[am[b]]]
        bound = R[la] + R[lb] - np.linalg.norm(C[la] - C[lb])
        assert bound >= mp[b] - 1e-12          # the argmax block's bound reaches the maximum
        row = rb.sphere_r[sa] + R[lb] - np.linalg.norm(c[b, sa] - C[lb])
        assert row >= mp[b] - 1e-12            # and so does its row's
    # a state in collision sweeps only pass 1 (one round of block tests)
    coll = mp >= 0
    assert np.all(tests[coll] == nb)
