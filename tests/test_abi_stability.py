"""The library's von Neumann stability check (host only, no GPU).

lbm_cde_spectral_radius bounds the spectral radius of the linearised step
G(k) = diag(exp(-i k.e_j)) C over a 48^2 (D2Q9) or 10^3 (D3Q15) grid of k.
It is compared with the exact eigenvalues of the same G(k) built from the
oracle's collision (colliding unit vectors on a one-node grid): the bound
must not be below the largest |eigenvalue| and may exceed it by at most
1e-5.  Runs whose bound is above 1 + 1e-5 are rejected with EUNSTABLE by
lbm_cde_workspace_bytes (and lbm_cde_init) unless the descriptor skips the
check: the paper's heat-flux rule s4 = s_xx, s6 = s_yy with the rotated
tensor of the 4096^2 workload (spectral radius 1.011), while the default
s4 = s6 = lambda_min(A) passes.
"""
import math

import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import _lib as L
from paper_1404_2363_amd import workloads as W
from paper_1404_2363_amd.solver import make_desc

C1 = np.array([[0.05, 0.02], [0.02, 0.03]])
C2 = W.rotated_tensor_2d((0.01, 0.1), math.radians(30.0))
TABLE2_FULL = W.paper_hill("full", u=(0.05, 0.05), n=16).D         # Eq. (42) tensor in lattice units


def exact_radius(lattice, u, D, heat, model="A", nk=None):
    lat = O.get_lattice(lattice)
    dim = lat.dim
    nk = nk or (48 if dim == 2 else 10)
    prob = O.Problem(lattice, (1,) * dim, (False,) * dim, np.asarray(u, float).reshape((dim,) + (1,) * dim), D,
                     model=model, heat_rule=heat)
    C = np.zeros((lat.Q, lat.Q))
    for j in range(lat.Q):
        f = np.zeros((lat.Q,) + (1,) * dim)
        f[j] = 1.0
        C[:, j] = prob.collide(f).reshape(lat.Q)
    ks = 2 * math.pi * np.arange(nk) / nk
    grids = np.meshgrid(*([ks] * dim), indexing="ij")
    kk = np.stack([g.ravel() for g in grids], 1)
    rho = 0.0
    for k in kk:
        ph = np.exp(-1j * (lat.e[:, :dim] @ k))
        rho = max(rho, float(np.abs(np.linalg.eigvals(ph[:, None] * C)).max()))
    return rho


def desc_for(lattice, u, D, heat, model="A", check=True):
    if lattice == "d2q9":
        wl = W.gaussian_hill(n=16, steps=1)
    else:
        wl = W.sine3d(n=6, steps=1, n_hills=1, sigma=2.0)
        wl.u_sep = None
    wl.D = np.asarray(D, float)
    wl.u_const = np.asarray(u, float)
    d, keep = make_desc(wl, "fp64", device="cpu", heat=heat, model=model, stability_check=check)
    return d, keep


CASES_2D = [
    (C1, (0.0, 0.0), "lambda_min", "A"),
    (C2, (0.0, 0.0), "lambda_min", "A"),
    (C2, (0.05, 0.0), "lambda_min", "A"),
    (C2, (0.0, 0.0), "paper", "A"),                      # unstable
    (TABLE2_FULL, (0.05, 0.05), "paper", "A"),           # the paper's Table 2 set-up: unstable
    (TABLE2_FULL, (0.05, 0.05), "paper", "B2"),          # unstable
    (TABLE2_FULL, (0.05, 0.05), "paper", "B1"),
    (np.eye(2) * 0.5, (0.1, -0.07), [0.9, 1.3], "A"),
]


@pytest.mark.parametrize("D,u,heat,model", CASES_2D)
def test_spectral_radius_bound_matches_exact_eigenvalues_d2q9(D, u, heat, model):
    d, keep = desc_for("d2q9", u, D, heat, model)
    bound = L.lbm_cde_spectral_radius(d)
    exact = exact_radius("d2q9", u, D, heat, model)
    print(f"D2Q9 {model} {heat} u={u}: bound {bound:.9f}, exact {exact:.9f}")
    assert exact - 1e-9 <= bound <= exact + 1e-5


@pytest.mark.parametrize("heat,umag", [("lambda_min", 0.0), ("lambda_min", 0.04), ("paper", 0.0)])
def test_spectral_radius_bound_matches_exact_eigenvalues_d3q15(heat, umag):
    D = W.sine3d(n=4, steps=1, n_hills=1, sigma=1.0).D
    u = umag * np.array([0.6, -0.8, 0.5])
    d, keep = desc_for("d3q15", u, D, heat)
    bound = L.lbm_cde_spectral_radius(d)
    exact = exact_radius("d3q15", u, D, heat)
    print(f"D3Q15 {heat} |u|={umag}: bound {bound:.9f}, exact {exact:.9f}")
    assert exact - 1e-9 <= bound <= exact + 1e-5


def test_paper_rule_with_rotated_tensor_is_rejected():
    d, keep = desc_for("d2q9", (0.0, 0.0), C2, "paper")
    assert L.lbm_cde_spectral_radius(d) > 1.005
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_workspace_bytes([d])
    assert e.value.code == L.LBM_CDE_EUNSTABLE
    assert "spectral radius" in L.lbm_cde_last_error(None)
    ok, keep2 = desc_for("d2q9", (0.0, 0.0), C2, "lambda_min")
    assert L.lbm_cde_spectral_radius(ok) <= 1.0 + 1e-5
    assert L.lbm_cde_workspace_bytes([ok]) > 0
    skip, keep3 = desc_for("d2q9", (0.0, 0.0), C2, "paper", check=False)
    assert L.lbm_cde_workspace_bytes([skip]) > 0


def test_paper_table2_setup_is_unstable_for_short_waves():
    """Table 2 (u = 0.05 (1, 1), s4 = s_xx, s6 = s_yy, D of Eq. (42) at
    dx = 1/256) amplifies short waves by 1.2 % per step for MRT-A; the
    table reproduction therefore skips the check."""
    d, keep = desc_for("d2q9", (0.05, 0.05), TABLE2_FULL, "paper")
    assert L.lbm_cde_spectral_radius(d) > 1.01
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_workspace_bytes([d])
    assert e.value.code == L.LBM_CDE_EUNSTABLE


def test_d3q15_paper_rule_rejected():
    D = W.sine3d(n=4, steps=1, n_hills=1, sigma=1.0).D
    d, keep = desc_for("d3q15", (0.0, 0.0, 0.0), D, "paper")
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_workspace_bytes([d])
    assert e.value.code == L.LBM_CDE_EUNSTABLE


def test_spectral_radius_needs_constant_fields():
    wl = W.cellular(nx=16, ny=16, steps=1, n_hills=1, sigma=3.0)       # separable u
    d, keep = make_desc(wl, "fp64", device="cpu")
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_spectral_radius(d)
    assert e.value.code == L.LBM_CDE_EUNSUPPORTED
