"""16-bit population storage against the FP64 oracle.

Split storage (phi in FP32, the non-equilibrium part in FP16 with a
power-of-two scale) must stay within 1e-3 of max|phi| of the oracle; the
literal form (shifted populations in FP16) is measured and reported next to
it.  Saturation is detected (EOVERFLOW), forced from the host with an
oversized scale.  The split step has a general kernel and a 32-bit-index
kernel for periodic grids; every launch shape of both gives bitwise the same
state.
"""
import os

import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W
from state_views import populations

pytestmark = pytest.mark.gpu


def gpu_run(wl, precision, steps, **kw):
    from paper_1404_2363_amd.solver import Solver
    s = Solver(wl, precision, **kw)
    m0 = s.mass()
    s.step(steps)
    phi = s.phi().cpu().numpy()
    m1 = s.mass()
    s.close()
    return phi, m0, m1


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def cellular_ref():
    wl = W.cellular(nx=200, ny=136, steps=400, n_hills=6, sigma=12.0, U0=0.05)
    ref, _ = O.run_workload(wl)
    return wl, ref


def test_split_within_tolerance(cellular_ref):
    wl, ref = cellular_ref
    phi, m0, m1 = gpu_run(wl, "fp16", 400)
    err = rel(phi, ref)
    print(f"fp16 split 200x136 x 400: max rel err {err:.3e}, mass drift {abs(m1 - m0) / m0:.2e}", flush=True)
    assert err <= 1e-3
    assert abs(m1 - m0) <= 1e-6 * m0


def test_literal_is_measured_and_worse(cellular_ref):
    wl, ref = cellular_ref
    lit, _, _ = gpu_run(wl, "fp16_literal", 400)
    spl, _, _ = gpu_run(wl, "fp16", 400)
    e_lit, e_spl = rel(lit, ref), rel(spl, ref)
    print(f"fp16 literal {e_lit:.3e} vs split {e_spl:.3e}", flush=True)
    assert np.isfinite(e_lit) and e_spl < e_lit


def test_split_gaussian_hill():
    wl = W.gaussian_hill()
    ref, _ = O.run_workload(wl)
    phi, _, _ = gpu_run(wl, "fp16", 1000)
    assert rel(phi, ref) <= 1e-3


@pytest.mark.parametrize("walls", [("periodic", "specular"), ("bounce", "bounce"), ("specular", "bounce")])
def test_split_walls(walls):
    wl = W.taylor_aris_channel(20, 12.0, 1.1, nx=150, steps=200)
    wl.walls = walls
    ref, _ = O.run_workload(wl)
    phi, _, _ = gpu_run(wl, "fp16", 200)
    assert rel(phi, ref) <= 1e-3


@pytest.mark.parametrize("shape", [(67, 45), (1, 9), (7, 1), (68, 45), (4, 9), (260, 3), (1028, 5)])
def test_split_ragged(shape):
    nx, ny = shape
    wl = W.cellular(nx=nx, ny=ny, steps=60, n_hills=4, sigma=max(2.0, min(nx, ny) / 6), U0=0.05)
    ref, _ = O.run_workload(wl)
    phi, _, _ = gpu_run(wl, "fp16", 60)
    assert rel(phi, ref) <= 1e-3


def test_saturation_reported():
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    wl = W.cellular(nx=64, ny=48, steps=5, n_hills=3, sigma=6.0)
    s = Solver(wl, "fp16", fp16_scale=2.0 ** 40)
    s.step(5)
    with pytest.raises(L.LbmCdeError) as e:
        s.mass()
    assert e.value.code == L.LBM_CDE_EOVERFLOW
    s.close()


def test_split_checkpoint_restart():
    from paper_1404_2363_amd.solver import Solver
    wl = W.cellular(nx=96, ny=64, steps=60, n_hills=3, sigma=8.0)
    a = Solver(wl, "fp16")
    a.step(25)
    ck = a.get_state()
    a.step(35)
    b = Solver(wl, "fp16")
    b.set_state(ck, 25)
    b.step(35)
    np.testing.assert_array_equal(a.phi().cpu().numpy(), b.phi().cpu().numpy())


SPLIT_VARIANTS = ["64x4", "128x2", "256x1", "64x8", "128x4", "256x2"]


def _split_state(wl, steps, tile):
    from paper_1404_2363_amd.solver import Solver
    os.environ["LBM_CDE_TILE16"] = tile
    try:
        s = Solver(wl, "fp16")
        v = s.variant()
        s.step(steps)
        out = populations(s.get_state().cpu().numpy(), 9, wl.nodes, "fp16")
        s.close()
    finally:
        del os.environ["LBM_CDE_TILE16"]
    return out, v


@pytest.mark.parametrize("case", ["periodic", "mixed_kernels", "specular_y", "bounce_y", "narrow"])
def test_split_kernels_bitwise_equal(case):
    """Every launch shape gives the same bits.  On a periodic grid the
    32-bit-index kernel runs when the grid covers a tile and the general one
    otherwise; at nx = 100 the 64-wide shapes take the first and the wider
    ones the second, so the two kernels are compared with each other."""
    if case == "narrow":
        wl = W.cellular(nx=12, ny=7, steps=30, n_hills=2, sigma=2.0)
    elif case == "periodic":
        wl = W.cellular(nx=520, ny=37, steps=30, n_hills=5, sigma=6.0)
    elif case == "mixed_kernels":
        wl = W.cellular(nx=100, ny=30, steps=30, n_hills=4, sigma=5.0)
    else:
        wl = W.taylor_aris_channel(13, 12.0, 1.1, nx=1032, steps=30,
                                   wall="specular" if case == "specular_y" else "bounce")
    print(f"case split variants {case} {wl.shape}", flush=True)
    ref, v0 = _split_state(wl, 30, SPLIT_VARIANTS[0])
    for tile in SPLIT_VARIANTS[1:]:
        out, v = _split_state(wl, 30, tile)
        assert v["block"] == tuple(int(t) for t in tile.split("x"))
        np.testing.assert_array_equal(out[0], ref[0], err_msg=tile)
        np.testing.assert_array_equal(out[1], ref[1], err_msg=tile)
