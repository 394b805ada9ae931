"""Host-side checks of the benchmark script: the measured-traffic records
hold every key the script reads, the frozen work models keep their values,
and a request for more than one GPU ends with a message (no GPU needed)."""
import os
import subprocess
import sys

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
    # the 48-DoF humanoid: 49 links, 240 spheres, 27,040 pairs, 48 joints
    assert bench.algorithmic_flop_per_state(49, 240, 27040, 48) == 365774
    assert bench.issue_slots_per_state(49, 240, 27040, 48) == 466807.0
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
        g, c = e["lanes_per_state"], e["states_per_item"]
        assert g in (16, 32, 64), key
        assert c % (4 * (64 // g)) == 0, key
        assert e["ns_per_state"] > 0, key
        best = min(e["candidates"], key=lambda x: x[2])
        assert [g, c] == best[:2], key
