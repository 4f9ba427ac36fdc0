"""Pins of the oracle's discrete adjoint.

* Dot-product test: <lam, P C v> = <C^T P^T lam, v> for random lam, v, with
  a per-node D field and every wall kind (the adjoint is the exact transpose).
* The gradient of the snapshot misfit with respect to the per-node D field
  equals central finite differences of the oracle's own forward misfit.
* Checkpointed recomputation gives the same gradient as stored states.
"""
import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W


def _small_problem(walls, nx=12, ny=10, seed=0, heat=(1.0, 1.0)):
    rng = W.rng_for(90, seed)
    dfield = W.dfield_from(*(W.fourier_field(rng, nx, ny, kmax=2) for _ in range(3)))
    u = rng.uniform(-0.05, 0.05, size=(2, ny, nx))
    return O.Problem("d2q9", (nx, ny), walls, u, dfield, heat_rule=list(heat)), dfield, u


@pytest.mark.parametrize("walls", [("periodic", "periodic"), ("periodic", "bounce"), ("specular", "bounce"),
                                   ("periodic", "specular")])
def test_dot_product(walls):
    prob, _, _ = _small_problem(walls)
    rng = np.random.default_rng(3)
    lam = rng.standard_normal((9, 10, 12))
    v = rng.standard_normal((9, 10, 12))
    lhs = float((lam * prob.stream(prob.collide(v))).sum())
    rhs = float((prob.collide_T(prob.stream_T(lam)) * v).sum())
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_dot_product_d3q15():
    wl = W.sine3d(n=6, ny=5, nz=4, steps=1, n_hills=2, sigma=2.0)
    prob = O.Problem("d3q15", wl.shape, ("periodic", "specular", "bounce"), wl.u(), wl.D)
    rng = np.random.default_rng(4)
    lam = rng.standard_normal((15,) + prob.grid)
    v = rng.standard_normal((15,) + prob.grid)
    lhs = float((lam * prob.stream(prob.collide(v))).sum())
    rhs = float((prob.collide_T(prob.stream_T(lam)) * v).sum())
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _misfit_setup(walls=("periodic", "periodic")):
    nx, ny = 14, 12
    prob_true, dtrue, u = _small_problem(walls, nx, ny, seed=1)
    rng = W.rng_for(91)
    dpert = W.dfield_from(*(W.fourier_field(rng, nx, ny, kmax=2) for _ in range(3)))
    dtrial = dtrue + 0.1 * (dpert - dtrue)
    spec = W.GaussianSum(np.array([[6.3, 5.1]]), np.ones(1), np.array([2.5]), (float(nx), float(ny)))
    phi0 = spec.window([np.arange(nx), np.arange(ny)])
    snap_every, nsnap = 6, 4
    _, obs = prob_true.run(prob_true.equilibrium(phi0), snap_every * nsnap, snap_every)
    make = lambda d: O.Problem("d2q9", (nx, ny), walls, u, d, heat_rule=[1.0, 1.0])
    return make, dtrial, phi0, obs, snap_every


@pytest.mark.parametrize("walls", [("periodic", "periodic"), ("periodic", "specular")])
def test_gradient_matches_finite_differences(walls):
    make, dtrial, phi0, obs, snap_every = _misfit_setup(walls)
    J, grad = O.misfit_gradient(make(dtrial), phi0, obs, snap_every)
    assert J > 0
    eps = 1e-6
    for (c, y, x) in [(0, 3, 4), (1, 6, 7), (2, 5, 5), (2, 9, 2), (0, 0, 13)]:
        dp, dm = dtrial.copy(), dtrial.copy()
        dp[c, y, x] += eps
        dm[c, y, x] -= eps
        fd = (O.misfit(make(dp), phi0, obs, snap_every) - O.misfit(make(dm), phi0, obs, snap_every)) / (2 * eps)
        assert abs(grad[c, y, x] - fd) <= 1e-6 * np.abs(grad).max(), (c, y, x, grad[c, y, x], fd)


def test_phi0_gradient_matches_finite_differences():
    make, dtrial, phi0, obs, snap_every = _misfit_setup(("periodic", "bounce"))
    J, _, dphi0 = O.misfit_gradient(make(dtrial), phi0, obs, snap_every, return_dphi0=True)
    eps = 1e-6
    for (y, x) in [(3, 4), (6, 7), (0, 13), (11, 0)]:
        pp, pm = phi0.copy(), phi0.copy()
        pp[y, x] += eps
        pm[y, x] -= eps
        fd = (O.misfit(make(dtrial), pp, obs, snap_every) - O.misfit(make(dtrial), pm, obs, snap_every)) / (2 * eps)
        assert abs(dphi0[y, x] - fd) <= 1e-6 * np.abs(dphi0).max(), (y, x, dphi0[y, x], fd)


def test_checkpointed_gradient_equals_stored():
    make, dtrial, phi0, obs, snap_every = _misfit_setup()
    J1, g1 = O.misfit_gradient(make(dtrial), phi0, obs, snap_every)
    J2, g2 = O.misfit_gradient(make(dtrial), phi0, obs, snap_every, ckpt_every=5)
    assert J1 == J2
    np.testing.assert_array_equal(g1, g2)


def test_gradient_requires_d_independent_heat_rates():
    prob = O.Problem("d2q9", (4, 4), ("periodic", "periodic"), np.zeros((2, 4, 4)), np.eye(2) * 0.1)
    with pytest.raises(ValueError):
        O.misfit_gradient(prob, np.ones((4, 4)), [np.ones((4, 4))], 1)
