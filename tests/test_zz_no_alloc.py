"""The entry point that allocates nothing (ebs_coarsened_geometry_noalloc)
against ebs_coarsened_geometry, through the C ABI: two calls in a row on one
GPU, the second on a smaller grid, must both equal the allocating entry
point's results bit for bit (same kernel, so the bar is exact); a coarse
grid beyond the fixed buffer is rejected before any work."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_11959_amd as ebs  # noqa: E402


def _geometry_both(w):
    print(f"[noalloc] {w.name} {w.grid.n}", flush=True)
    c = ebs.Context(w.grid.n, w.grid.dx, w.grid.lo)
    c.build_geometry(w.h_nodes)
    ref = c.coarsened_geometry()
    got = c.coarsened_geometry(noalloc=True)
    torch.cuda.synchronize()
    c.close()
    return ref, got


def _same(ref, got):
    assert np.array_equal(ref[0], got[0])
    for d in range(3):
        assert np.array_equal(ref[1][d], got[1][d])


def test_noalloc_matches_allocating_entry_point_two_calls():
    big = synth.make_workload(2)    # 128 x 128 x 64 -> 131072 coarse cells
    small = synth.make_workload(1)  # 32^3 -> 4096 coarse cells
    r1, g1 = _geometry_both(big)
    _same(r1, g1)
    assert np.any((g1[0] > 0.0) & (g1[0] < 1.0))  # the hill cuts coarse cells
    r2, g2 = _geometry_both(small)
    _same(r2, g2)
    # the second, smaller call left the rest of the buffer from the first
    # call untouched; its own results still come out whole
    assert g2[0].shape == (16, 16, 16)


def test_noalloc_rejects_grid_beyond_buffer():
    # 512 x 512 x 32 -> 2^20 coarse cells, twice the buffer; rejected before
    # the geometry check, so no geometry build is needed
    lib = ebs.load()
    n = (512, 512, 32)
    c = ebs.Context(n, (1.0, 1.0, 1.0))
    arrs = [np.zeros(1) for _ in range(4)]
    dp = C.POINTER(C.c_double)
    st = lib.ebs_coarsened_geometry_noalloc(c.h, *[a.ctypes.data_as(dp) for a in arrs])
    assert st == ebs.EBS_E_UNSUPPORTED
    assert b"static staging buffer" in lib.ebs_last_error(c.h)
    c.close()
