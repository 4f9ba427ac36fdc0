"""The C reference (oracle/lbm_ref.c) against the Python oracle (CPU).

The C code applies the Python oracle's collision in matrix form
f' = Cm f + phi (b_0 + sum_c u_c b_c) and streams periodically; the two must
agree to rounding on small periodic grids with spatially varying u, D2Q9 and
D3Q15, over enough steps for every population to cross the grid.  It also
conserves sum phi, and the matrix form reproduces one oracle collision of
arbitrary populations.
"""
import numpy as np
import pytest

from oracle import lbm as O
from oracle import ref as R
from paper_1404_2363_amd import workloads as W


def _problem(wl):
    return O.problem_for(wl)


@pytest.mark.parametrize("case", ["d2q9", "d3q15"])
def test_matrix_form_is_the_oracle_collision(case):
    wl = (W.cellular(nx=12, ny=10, steps=1, n_hills=2, sigma=3.0) if case == "d2q9"
          else W.sine3d(n=6, steps=1, n_hills=1, sigma=2.0))
    prob = _problem(wl)
    rng = np.random.default_rng(7)
    f = rng.normal(size=(prob.lat.Q,) + prob.grid)
    Cm, b = R.collision_form(prob)
    Q = prob.lat.Q
    flat = f.reshape(Q, -1)
    phi = flat.sum(0)
    u = prob.u.reshape(prob.lat.dim, -1)
    mine = Cm @ flat + phi * (b[0][:, None] + sum(u[c] * b[1 + c][:, None] for c in range(prob.lat.dim)))
    ref = prob.collide(f).reshape(Q, -1)
    assert np.abs(mine - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("case,steps", [("d2q9", 120), ("d3q15", 40)])
def test_reference_run_equals_oracle_run(case, steps):
    wl = (W.cellular(nx=40, ny=24, steps=steps, n_hills=4, sigma=4.0) if case == "d2q9"
          else W.sine3d(n=10, steps=steps, n_hills=2, sigma=2.5))
    prob = _problem(wl)
    f0 = prob.equilibrium(wl.phi0())
    ref, _ = prob.run(f0, steps)
    mine = R.run(prob, f0, steps)
    err = float(np.abs(mine - ref).max() / np.abs(ref).max())
    print(f"{case} {prob.grid} x {steps}: max rel difference {err:.2e}")
    assert err <= 1e-13
    assert abs(mine.sum() - f0.sum()) <= 1e-12 * abs(f0.sum())


def test_rejects_walls():
    wl = W.taylor_aris_channel(8, 5.0, 1.0, nx=16, steps=1)
    prob = _problem(wl)
    with pytest.raises(ValueError):
        R.run(prob, prob.equilibrium(wl.phi0()), 1)
