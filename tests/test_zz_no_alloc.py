"""lbm_cde_reduce_noalloc: the reduction of lbm_cde_reduce with its partial
sums in the library's static device array and the result left in a device
buffer, for callers that cannot allocate or wait.  Checked against
lbm_cde_reduce (FP64 sums to 1e-12 relative; counts exact) on two calls in a
row, the second with a smaller run, for every reduction kind."""
import numpy as np
import pytest

from paper_1404_2363_amd import workloads as W

pytestmark = pytest.mark.gpu


def _check_run(wl, precision, steps):
    import torch
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    s = Solver(wl, precision)
    s.step(steps)
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda:0")
    nx = wl.shape[0]
    for kind, x_ref in ((L.LBM_CDE_RED_MASS, 0.0), (L.LBM_CDE_RED_XMOMENTS, 0.37 * nx),
                        (L.LBM_CDE_RED_NONFINITE, 0.0)):
        out.fill_(float("nan"))
        L.lbm_cde_reduce_noalloc(s.h, 0, kind, x_ref, out.data_ptr())
        got = out.cpu().numpy()
        ref, _ = L.lbm_cde_reduce(s.h, 0, kind, x_ref)
        if kind == L.LBM_CDE_RED_NONFINITE:
            assert got[3] == ref[0] == 0.0
            continue
        assert got[3] == 0.0
        scale = abs(ref[0])
        assert abs(got[0] - ref[0]) <= 1e-12 * scale, (kind, got, ref)
        if kind == L.LBM_CDE_RED_XMOMENTS:
            # S1 and S2 carry the distances d and d^2 (|d| <= nx/2)
            assert abs(got[1] - ref[1]) <= 1e-12 * scale * nx, (got, ref)
            assert abs(got[2] - ref[2]) <= 1e-12 * scale * nx * nx, (got, ref)
        else:
            assert got[1] == 0.0 and got[2] == 0.0
    s.close()


def test_reduce_noalloc_matches_reduce_two_calls():
    # first call: 19 partials of 16384 nodes (a ragged last one); second: one partial
    big = W.cellular(nx=700, ny=437, steps=30, n_hills=6, sigma=20.0)
    small = W.cellular(nx=96, ny=72, steps=30, n_hills=3, sigma=6.0)
    print("case reduce_noalloc 700x437 fp32 then 96x72 fp64", flush=True)
    _check_run(big, "fp32", 30)
    _check_run(small, "fp64", 30)


def test_reduce_noalloc_fp16_and_d3q15():
    print("case reduce_noalloc 200x136 fp16 then 40x36x20 d3q15 fp32", flush=True)
    _check_run(W.cellular(nx=200, ny=136, steps=20, n_hills=4, sigma=12.0), "fp16", 20)
    _check_run(W.sine3d(n=40, ny=36, nz=20, steps=10, n_hills=3, sigma=5.0), "fp32", 10)


def test_reduce_noalloc_rejects_bad_arguments():
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    s = Solver(W.cellular(nx=32, ny=24, steps=1, n_hills=2, sigma=4.0), "fp64")
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_reduce_noalloc(s.h, 0, 9, 0.0, 0)
    assert e.value.code == L.LBM_CDE_EINVAL
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_reduce_noalloc(s.h, 1, L.LBM_CDE_RED_MASS, 0.0, 0)
    assert e.value.code == L.LBM_CDE_EINVAL
    s.close()
