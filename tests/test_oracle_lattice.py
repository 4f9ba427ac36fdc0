"""Pins of the oracle's lattice constants and equilibria.

* The rows of M (Eq. 12, Eq. A.2) are the textbook moment polynomials of the
  velocities (density, energy, energy square, fluxes, heat fluxes, stresses);
  a mistyped entry or a misordered velocity breaks one of them.
* The rows are mutually orthogonal (the Gram-Schmidt construction the paper
  cites for M).
* The velocity-space equilibrium M^-1 m^eq equals the closed form printed as
  Eq. (17) for arbitrary alpha1, alpha2 (this pins Eq. 15-16 and M^-1).
* The D3Q15 equilibrium carries mass and flux phi, phi u (Eq. A.3-A.4).
"""
import copy

import numpy as np
import pytest

from oracle import lbm as O


def test_d2q9_velocities_eq2():
    e = O.D2Q9.e
    # Eq. (2): rest, 4 axis (angles 0, 90, 180, 270 deg), 4 diagonals (45, 135, 225, 315 deg)
    assert (e[0] == 0).all()
    assert (np.abs(e[1:5, :2]).sum(1) == 1).all() and (np.abs(e[5:, :2]) == 1).all()
    ang = np.degrees(np.arctan2(e[1:, 1], e[1:, 0])) % 360
    np.testing.assert_allclose(ang, [0, 90, 180, 270, 45, 135, 225, 315])


def _polys_d2q9(e):
    ex, ey = e[:, 0].astype(float), e[:, 1].astype(float)
    e2 = ex * ex + ey * ey
    return np.array([
        np.ones_like(ex),                      # rho
        -4 + 3 * e2,                           # e
        4 - 21 / 2 * e2 + 9 / 2 * e2 * e2,     # epsilon
        ex,                                    # j_x
        (-5 + 3 * e2) * ex,                    # q_x
        ey,                                    # j_y
        (-5 + 3 * e2) * ey,                    # q_y
        ex * ex - ey * ey,                     # p_xx
        ex * ey,                               # p_xy
    ])


def _polys_d3q15(e):
    ex, ey, ez = (e[:, a].astype(float) for a in range(3))
    e2 = ex * ex + ey * ey + ez * ez
    return np.array([
        np.ones_like(ex), e2 - 2, (15 * e2 * e2 - 55 * e2 + 32) / 2,
        ex, (5 * e2 - 13) / 2 * ex, ey, (5 * e2 - 13) / 2 * ey, ez, (5 * e2 - 13) / 2 * ez,
        3 * ex * ex - e2, ey * ey - ez * ez, ex * ey, ey * ez, ex * ez, ex * ey * ez,
    ])


@pytest.mark.parametrize("lat,polys", [(O.D2Q9, _polys_d2q9), (O.D3Q15, _polys_d3q15)])
def test_M_rows_are_moment_polynomials(lat, polys):
    np.testing.assert_array_equal(lat.M, polys(lat.e))


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q15])
def test_M_orthogonal_and_inverse(lat):
    G = lat.M @ lat.M.T
    np.testing.assert_array_equal(G, np.diag(np.diag(G)))
    np.testing.assert_allclose(lat.Minv @ lat.M, np.eye(lat.Q), atol=1e-15)
    assert (lat.e[lat.opp] == -lat.e).all()


def test_d3q15_velocity_set_A1():
    e = O.D3Q15.e
    norms = (e * e).sum(1)
    assert norms[0] == 0 and (norms[1:7] == 1).all() and (norms[7:] == 3).all()
    assert len({tuple(v) for v in e}) == 15


@pytest.mark.parametrize("a1,a2", [(-8.0, 8.0), (-2.0, 1.0), (3.5, -4.25)])
def test_equilibrium_matches_eq17(a1, a2):
    lat = copy.copy(O.D2Q9)
    lat.alpha1, lat.alpha2 = a1, a2
    rng = np.random.default_rng(0)
    phi = rng.uniform(0.1, 2.0, size=(5,))
    u = rng.uniform(-0.1, 0.1, size=(2, 5))
    feq = np.tensordot(lat.Minv, O.equilibrium_moments(lat, "A", phi, u), axes=(1, 0))
    eu = lat.e[:, 0, None] * u[0][None] + lat.e[:, 1, None] * u[1][None]   # c = 1
    ref = np.empty_like(feq)
    ref[0] = (-a1 + a2 + 4) / 36 * phi
    ref[1:5] = (-a1 - 2 * a2 + 16 + 48 * eu[1:5]) / 144 * phi
    ref[5:] = (2 * a1 + a2 + 16 + 12 * eu[5:]) / 144 * phi
    np.testing.assert_allclose(feq, ref, rtol=0, atol=1e-15)


def test_mrt_b1_equilibrium_is_eq6_in_moment_space():
    # Eq. (38) is the moment-space form of the SRT equilibrium Eq. (6)-(7)
    lat = O.D2Q9
    rng = np.random.default_rng(1)
    phi = rng.uniform(0.1, 2.0, size=(7,))
    u = rng.uniform(-0.1, 0.1, size=(2, 7))
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    eu = lat.e[:, 0, None] * u[0][None] + lat.e[:, 1, None] * u[1][None]
    uu = (u * u).sum(0)[None]
    feq6 = w[:, None] * phi[None] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)
    np.testing.assert_allclose(lat.M @ feq6, O.equilibrium_moments(lat, "B1", phi, u), atol=1e-15)


def test_d3q15_equilibrium_mass_and_flux():
    lat = O.D3Q15
    rng = np.random.default_rng(2)
    phi = rng.uniform(0.1, 2.0, size=(6,))
    u = rng.uniform(-0.1, 0.1, size=(3, 6))
    feq = np.tensordot(lat.Minv, O.equilibrium_moments(lat, "A", phi, u), axes=(1, 0))
    np.testing.assert_allclose(feq.sum(0), phi, rtol=1e-15)
    for a in range(3):
        np.testing.assert_allclose((lat.e[:, a, None] * feq).sum(0), phi * u[a], rtol=1e-14, atol=1e-16)
    # the reading alpha1 = -6/5, alpha2 = 192: prefactor 1/3 and rest weights 8/15, 1/30
    assert abs(lat.kappa() - 1 / 3) < 1e-15
    feq0 = np.tensordot(lat.Minv, O.equilibrium_moments(lat, "A", np.ones(1), np.zeros((3, 1))), axes=(1, 0))[:, 0]
    np.testing.assert_allclose(feq0, [8 / 15] + [1 / 30] * 14, atol=1e-15)


def test_d2q9_kappa_eq36_eq29():
    # Sec. 3: all four models share D = (I - A/2) A^-1 / 3
    assert abs(O.D2Q9.kappa(True) - 1 / 3) < 1e-15
    assert abs(O.D2Q9.kappa(False) - 1 / 3) < 1e-15


def test_relaxation_matrix_structure_eq31():
    lat = O.D2Q9
    A = np.array([[1.3, 0.2], [0.2, 1.1]])
    rates = O.default_rates(lat)
    heat = np.array([0.9, 0.8])
    S = O.relaxation_matrix(lat, A, rates, heat, modified=True)
    S24 = O.relaxation_matrix(lat, A, rates, heat, modified=False)
    # outside rows 3 and 5 both are diagonal with the given rates
    for k in (0, 1, 2, 4, 6, 7, 8):
        row = np.zeros(9)
        row[k] = heat[0] if k == 4 else heat[1] if k == 6 else rates[k]
        np.testing.assert_array_equal(S[k], row)
        np.testing.assert_array_equal(S24[k], row)
    # Eq. (24): rows 3, 5 couple only the fluxes; Eq. (31) adds the heat-flux columns
    np.testing.assert_array_equal(S24[3], [0, 0, 0, 1.3, 0, 0.2, 0, 0, 0])
    np.testing.assert_allclose(S[3], [0, 0, 0, 1.3, (1.3 / 2 - 1) * 0.9, 0.2, 0.2 / 2 * 0.8, 0, 0])
    np.testing.assert_allclose(S[5], [0, 0, 0, 0.2, 0.2 / 2 * 0.9, 1.1, (1.1 / 2 - 1) * 0.8, 0, 0])
