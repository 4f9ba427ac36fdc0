"""16-bit population storage against the FP64 oracle.

Split storage (phi in FP32, the non-equilibrium part in FP16 with a
power-of-two scale) must stay within 1e-3 of max|phi| of the oracle; the
literal form (shifted populations in FP16) is measured and reported next to
it.  Saturation is detected (EOVERFLOW), forced from the host with an
oversized scale.
"""
import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W

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


@pytest.mark.parametrize("shape", [(67, 45), (1, 9), (7, 1)])
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
