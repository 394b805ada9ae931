"""GPU: the allocation-free distance transform (wb_edt_noalloc, the library's
per-device scratch array in place of a caller workspace) gives exactly the
results of wb_edt with a workspace, on calls in a row whose grids shrink
(the largest grid it accepts first), and rejects grids beyond its limit
before touching the GPU."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2603_05493_amd import sitegrid

pytestmark = pytest.mark.gpu


def _both(m, voxel_size=0.02):
    from paper_2603_05493_amd import wb
    sites = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    shape = m.shape
    near_ws, dist_ws = wb.wb_edt(sites, voxel_size)
    near = torch.full(shape, -7, dtype=torch.int32, device="cuda")
    dist = torch.full(shape, float("nan"), device="cuda")
    wb.wb_edt_noalloc(sites, voxel_size, nearest=near, dist=dist)
    torch.cuda.synchronize()
    return near_ws, dist_ws, near, dist


@pytest.mark.parametrize("label,grid", [
    ("room_256x256x128_max", lambda: sitegrid.room(256, 256, 128, seed=0)),   # exactly the limit
    ("room_160x96x72", lambda: sitegrid.room(160, 96, 72, seed=1)),          # a smaller grid next
    ("bernoulli_37x29x13", lambda: sitegrid.random_sites(13, 29, 37, 0.01, seed=2)),
    ("empty_9x5x3", lambda: np.zeros((3, 5, 9), np.uint8)),
])
def test_noalloc_matches_workspace_entry(label, grid):
    m = grid()
    near_ws, dist_ws, near, dist = _both(m)
    print(label, "voxels", m.size, "sites", int(m.sum()), flush=True)
    assert torch.equal(near, near_ws), label
    assert torch.equal(dist.view(torch.int32), dist_ws.view(torch.int32)), label   # bit for bit


def test_noalloc_consecutive_calls_shrinking():
    """Two calls in a row on the shared scratch, the second on a smaller grid."""
    big = sitegrid.room(192, 128, 96, seed=3)
    small = sitegrid.random_sites(20, 33, 48, 0.003, seed=4)
    for m in (big, small):
        near_ws, dist_ws, near, dist = _both(m)
        assert torch.equal(near, near_ws)
        assert torch.equal(dist.view(torch.int32), dist_ws.view(torch.int32))


def test_noalloc_rejects_grids_beyond_its_limit():
    from paper_2603_05493_amd import _abi, wb
    sites = torch.zeros(16, dtype=torch.uint8, device="cuda")
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    # 1024 x 1024 x 9 voxels > 2^23: refused before any launch (the pointers are never used)
    rc = _abi.lib().wb_edt_noalloc(1024, 1024, 9, C.c_void_p(sites.data_ptr()), 0.02,
                                   C.c_void_p(out.data_ptr()), None, None)
    assert rc == _abi.WB_ERR_UNSUPPORTED
    assert b"at most" in _abi.lib().wb_last_error()
    assert wb.EDT_NOALLOC_MAX_VOXELS == 1 << 23
