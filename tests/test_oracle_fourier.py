"""Exact long-wave pins of the oracle's collision (von Neumann analysis).

For constant u and D the step is linear and translation invariant, so a
Fourier mode exp(i k.x) evolves by the symbol G(k) = diag(exp(-i k.e_j)) C,
where C is the per-node collision matrix.  C is extracted from the oracle by
colliding unit vectors on a one-node grid.  The slowest eigenvalue lambda(k)
of G(k) gives the macroscopic equation the scheme actually solves:

    log lambda(k) = -i k.u - k^T D_eff k + O(|k|^3),

and D_eff must equal
* D for the modified model MRT-A at any constant u (Eq. 36: no deviation term),
  for D2Q9 and for D3Q15 (Eq. A.6 with the alpha reading);
* D - 3 sym(D u u^T) for MRT-B3 (Eq. 29 with grad.[3D d_t(phi u)],
  d_t phi = -u.grad phi at leading order), the deviation term;
* D for MRT-B1/B2 at constant u (Sec. 3.1: their nonlinear equilibria remove
  the deviation term for u = const).
The phase speed must equal u.  Richardson extrapolation in |k| removes the
O(|k|^2) part of D_eff(k).
"""
import math

import numpy as np
import pytest

from oracle import lbm as O


def collision_matrix(lattice, u, D, model="A", heat_rule="lambda_min"):
    lat = O.get_lattice(lattice)
    dim = lat.dim
    prob = O.Problem(lattice, (1,) * dim, (False,) * dim, np.asarray(u, float).reshape((dim,) + (1,) * dim),
                     D, model=model, heat_rule=heat_rule)
    C = np.zeros((lat.Q, lat.Q))
    for j in range(lat.Q):
        f = np.zeros((lat.Q,) + (1,) * dim)
        f[j] = 1.0
        C[:, j] = prob.collide(f).reshape(lat.Q)
    return lat, C


def slow_eigenvalue(lat, C, k):
    phase = np.exp(-1j * (lat.e[:, :lat.dim] @ k))
    ev = np.linalg.eigvals(phase[:, None] * C)
    return ev[np.argmin(np.abs(ev - 1.0))]


def effective(lattice, u, D, model="A", heat_rule="lambda_min", kmag=2e-3):
    lat, C = collision_matrix(lattice, u, D, model, heat_rule)
    dim = lat.dim
    if dim == 2:
        dirs = [np.array(d, float) for d in ((1, 0), (0, 1), (1, 1))]
    else:
        dirs = [np.array(d, float) for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1))]
    dirs = [d / np.linalg.norm(d) for d in dirs]

    def along(d, h):
        lg = np.log(slow_eigenvalue(lat, C, h * d))
        return -lg.real / h ** 2, -lg.imag / h

    vals, speeds = [], []
    for d in dirs:
        (r1, s1), (r2, s2) = along(d, kmag), along(d, 2 * kmag)
        vals.append((4 * r1 - r2) / 3)
        speeds.append((4 * s1 - s2) / 3)
    # solve d^T D d = value for the symmetric components
    rows = []
    for d in dirs:
        if dim == 2:
            rows.append([d[0] ** 2, d[1] ** 2, 2 * d[0] * d[1]])
        else:
            rows.append([d[0] ** 2, d[1] ** 2, d[2] ** 2, 2 * d[0] * d[1], 2 * d[0] * d[2], 2 * d[1] * d[2]])
    comps = np.linalg.solve(np.array(rows), np.array(vals))
    return O.components_to_tensor(comps), np.array(speeds), dirs


D_CASES_2D = [
    np.array([[0.05, 0.02], [0.02, 0.03]]),                       # Gaussian-hill tensor
    np.array([[0.0325, -0.03897114317029974], [-0.03897114317029974, 0.0775]]),  # eigen 0.01/0.1 at 30 deg
    np.array([[1e-4, 1e-4], [1e-4, 4e-4]]) * 256,                 # Eq. (42) full anisotropic, lattice units
    np.eye(2) * 0.5,
]
U_CASES_2D = [(0.0, 0.0), (0.05, 0.05), (0.1, -0.07)]


@pytest.mark.parametrize("D", D_CASES_2D)
@pytest.mark.parametrize("u", U_CASES_2D)
@pytest.mark.parametrize("heat_rule", ["lambda_min", "paper", [0.9, 1.3]])
def test_modified_model_has_no_deviation_d2q9(D, u, heat_rule):
    Deff, speeds, dirs = effective("d2q9", u, D, "A", heat_rule)
    np.testing.assert_allclose(Deff, D, rtol=0, atol=2e-7 * np.abs(D).max())
    np.testing.assert_allclose(speeds, [d @ np.array(u) for d in dirs], atol=1e-9)


@pytest.mark.parametrize("D", D_CASES_2D[:3])
@pytest.mark.parametrize("u", U_CASES_2D[1:])
def test_unmodified_b3_deviation_term(D, u):
    u = np.array(u)
    Deff, _, _ = effective("d2q9", u, D, "B3")
    Dun = D @ np.outer(u, u)
    expected = D - 3.0 * 0.5 * (Dun + Dun.T)
    dev = np.abs(expected - D).max()
    np.testing.assert_allclose(Deff, expected, rtol=0, atol=2e-3 * dev + 1e-9)
    assert np.abs(Deff - D).max() > 0.5 * dev        # and the deviation is really there


@pytest.mark.parametrize("model", ["B1", "B2"])
@pytest.mark.parametrize("u", U_CASES_2D[1:])
def test_unmodified_b1_b2_constant_u(model, u):
    D = D_CASES_2D[0]
    Deff, _, _ = effective("d2q9", u, D, model)
    # no deviation at u = const (Sec. 3.1); residual O(u^4) terms only
    np.testing.assert_allclose(Deff, D, rtol=0, atol=5e-3 * np.abs(D).max())


def _random_spd3(rng):
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    lam = rng.uniform(0.01, 0.1, 3)
    D = Q @ np.diag(lam) @ Q.T
    return 0.5 * (D + D.T)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("umag", [0.0, 0.04])
def test_modified_model_has_no_deviation_d3q15(seed, umag):
    rng = np.random.default_rng(seed)
    D = _random_spd3(rng)
    u = umag * rng.uniform(-1, 1, 3)
    Deff, speeds, dirs = effective("d3q15", u, D, "A")
    np.testing.assert_allclose(Deff, D, rtol=0, atol=2e-7 * np.abs(D).max())
    np.testing.assert_allclose(speeds, [d @ u for d in dirs], atol=1e-9)


def spectral_radius(lattice, u, D, heat_rule, nk=48):
    lat, C = collision_matrix(lattice, u, D, "A", heat_rule)
    ks = 2 * math.pi * np.arange(nk) / nk
    rho = 0.0
    if lat.dim == 2:
        for kx in ks:
            for ky in ks:
                ev = np.linalg.eigvals(np.exp(-1j * (lat.e[:, :2] @ np.array([kx, ky])))[:, None] * C)
                rho = max(rho, np.abs(ev).max())
    else:
        for kx in ks:
            for ky in ks:
                for kz in ks:
                    ev = np.linalg.eigvals(np.exp(-1j * (lat.e @ np.array([kx, ky, kz])))[:, None] * C)
                    rho = max(rho, np.abs(ev).max())
    return rho


def test_stability_of_default_heat_rates():
    """Linear stability of the chosen s4 = s6 = lambda_min(A) on the workloads' tensors."""
    for D, u in [(D_CASES_2D[0], (0, 0)), (D_CASES_2D[1], (0.05, 0.0)), (D_CASES_2D[1], (0.0, 0.05)),
                 (D_CASES_2D[1], (0.035, 0.035))]:
        assert spectral_radius("d2q9", u, D, "lambda_min") <= 1.0 + 1e-12


def test_paper_heat_rule_unstable_for_rotated_tensor():
    """s4 = s_xx, s6 = s_yy (Sec. 3.1) amplifies the checkerboard mode for the
    tensor with eigenvalues 0.01 and 0.1 rotated by 30 degrees, even at u = 0;
    this is why the library defaults to s4 = s6 = lambda_min(A)."""
    rho = spectral_radius("d2q9", (0.0, 0.0), D_CASES_2D[1], "paper", nk=16)
    assert rho > 1.005
