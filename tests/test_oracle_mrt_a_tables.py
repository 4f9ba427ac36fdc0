"""The printed Taylor-Aris errors of Tables 3-5 (Sec. 3.2) from the oracle's
one-step symbol, and what the printed MRT-A column says about the rates.

For a channel that is uniform along x the oracle's step splits into three
column-to-column maps (oracle.channel_transfer, built from the oracle's own
step with the plate rule of Sec. 3.2); the eigenvalue nearest 1 of their
Fourier symbol gives the asymptotic longitudinal dispersion coefficient, the
value that Eq. (49)'s convergence test approaches (oracle.channel_dispersion),
and the x-moment recursion gives the whole variance history of Eq. (46)-(47)
(oracle.channel_moment_history).  Both are pinned here against the direct
oracle run.

What the tables then show, for the rates the paper states (s1 = s2 = 1.1,
s7 = s8 = 1.2, s4 = s6 = s_xx = s_yy = 1/tau):
* all 36 printed MRT-B1/B2/B3 errors are reproduced to 0.75 %;
* MRT-A's are not: ours / printed is 1.314 (tau = 2), 2.058 (tau = 1) and
  0.955-0.961 (tau = 0.55), the same at every Pe of a table;
* the B models' errors do not depend on s2 at all (m2 does not enter the
  flux equation Eq. (27)), while MRT-A's do, strongly (m2 enters Eq. (34));
  s1, s7 and s8 move the B errors and are pinned by them near the stated
  values, s2 is the one rate the B columns cannot see;
* with s2 near 0.94 and every other rate as stated, MRT-A's twelve printed
  errors are met to within 3 % (each table alone needs s2 = 0.952, 0.939,
  0.930), and the same s2 moves MRT-A's Table 1 errors (Sec. 3.1, u = 0)
  from 0.91-0.93 to 0.98-1.00 of the printed values while the B models'
  stay put.  (Table 2 does not take part: there even the B models differ
  from the printed values by 2-25 %.)  This is recorded as an observation
  about the printed numbers; the oracle keeps the stated s2 = 1.1.
"""
import json
import os

import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
MODELS = GOLDEN["models"]
TABLES = {3: 2.0, 4: 1.0, 5: 0.55}


def rates(s1=1.1, s2=1.1, s7=1.2, s8=1.2):
    r = O.default_rates(O.D2Q9).copy()
    r[[1, 2, 7, 8]] = [s1, s2, s7, s8]
    return r


def plate_problem(model, tau, Pe, r=None, nx=3):
    wl = W.plate_channel(tau, Pe, length=1, steps=1)
    ny = wl.shape[1]
    return O.problem_for(wl, idx=[np.arange(nx), np.arange(ny)], model=model, heat_rule=[1.0 / tau] * 2,
                         rates=rates() if r is None else r), wl


def signed_error(model, tau, Pe, r=None):
    prob, wl = plate_problem(model, tau, Pe, r)
    K, _ = O.channel_dispersion(prob)
    return K / wl.meta["K"] - 1.0


def plate_weights(ny):
    w = np.ones(ny)
    w[0] = w[-1] = 0.5
    return w


def test_moment_history_equals_the_oracle_run():
    """The x-moment recursion against the oracle stepped on a finite channel
    (832 nodes, top-hat pulse, tau = 2, Pe = 2, MRT-A): the variance of the
    plate-weighted cross-section sum (about the nearest image of the moving
    centre) differs by the top-hat's own variance only, at every sample,
    while the pulse (sigma <= 21) stays far from the period."""
    tau, Pe, every, steps = 2.0, 2.0, 50, 400
    wl = W.plate_channel(tau, Pe, length=26, steps=steps)
    nx, ny = wl.shape
    prob = O.problem_for(wl, model="A", heat_rule=[1.0 / tau] * 2, rates=rates())
    wy = plate_weights(ny)
    x = np.arange(nx, dtype=np.float64)
    f = prob.equilibrium(wl.phi0())
    pb0 = (O.phi_of(f) * wy[:, None]).sum(0)
    d0 = x - wl.meta["x0"]
    var0 = (pb0 * d0 * d0).sum() / pb0.sum() - ((pb0 * d0).sum() / pb0.sum()) ** 2
    direct = []
    for k in range(1, steps // every + 1):
        f, _ = prob.run(f, every)
        pb = (O.phi_of(f) * wy[:, None]).sum(0)
        d = x - (wl.meta["x0"] + wl.meta["U_node_mean"] * k * every)
        d -= nx * np.floor(d / nx + 0.5)
        S0, S1, S2 = pb.sum(), (pb * d).sum(), (pb * d * d).sum()
        direct.append(S2 / S0 - (S1 / S0) ** 2)
    chan, _ = plate_problem("A", tau, Pe)
    t, S0, S1, S2 = O.channel_moment_history(chan, wy, steps, every, drift=wl.meta["U_node_mean"])
    hist = S2 / S0 - (S1 / S0) ** 2 + var0
    assert np.allclose(hist, direct, rtol=1e-11, atol=0.0), (hist, direct)


@pytest.mark.parametrize("model", MODELS)
def test_dispersion_of_the_symbol_equals_the_converged_history(model):
    """tau = 1, Pe = 8: the variance slope of the recursion after 25 e-folds
    of the slowest plate mode equals the eigenvalue's K."""
    tau, Pe = 1.0, 8.0
    prob, wl = plate_problem(model, tau, Pe)
    horizon = W.plate_channel(tau, Pe).steps
    t, S0, S1, S2 = O.channel_moment_history(prob, plate_weights(wl.shape[1]), horizon + 100, 100,
                                             drift=wl.meta["U_node_mean"])
    var = S2 / S0 - (S1 / S0) ** 2
    K, _ = O.channel_dispersion(prob)
    assert abs((var[-1] - var[-2]) / 200.0 / K - 1.0) <= 1e-7      # the eigenvalue route: ~2e-8


def table_rows():
    for tab, tau in TABLES.items():
        for Pe, printed in GOLDEN[f"table{tab}"]["Er_x100"].items():
            yield tab, tau, float(Pe), printed


@pytest.mark.parametrize("tab,tau,Pe,printed", list(table_rows()))
def test_tables_3_to_5_at_the_stated_rates(tab, tau, Pe, printed):
    """Every printed B-model Er (Eq. 48) within 0.75 %; MRT-A off by the
    table's own factor (recorded, not a property of the method)."""
    ratio = [abs(signed_error(m, tau, Pe)) * 100.0 / p for m, p in zip(MODELS, printed)]
    print(f"table {tab} Pe={Pe}: ours/printed " + " ".join(f"{m} {r:.4f}" for m, r in zip(MODELS, ratio)))
    for r in ratio[1:]:
        assert abs(r - 1.0) <= 7.5e-3
    expect = {3: (1.3138, 2e-3), 4: (2.058, 2e-3), 5: (0.958, 4e-3)}[tab]
    assert abs(ratio[0] / expect[0] - 1.0) <= expect[1]


@pytest.mark.parametrize("tab", [3, 4, 5])
def test_s2_moves_only_the_modified_model(tab):
    tau = TABLES[tab]
    Pe = float(next(iter(GOLDEN[f"table{tab}"]["Er_x100"])))
    for m in MODELS:
        a, b = signed_error(m, tau, Pe, rates(s2=1.1)), signed_error(m, tau, Pe, rates(s2=0.94))
        if m == "A":
            assert abs(a - b) >= 0.02 * abs(a)                # 26 % (tau = 2) .. 4 % (tau = 0.55)
        else:                       # unchanged to the eigenvalue route's precision (~2e-8 of K)
            assert abs(a - b) <= 1e-7, m


@pytest.mark.parametrize("which", ["s1", "s7", "s8"])
def test_the_other_free_rates_are_pinned_by_the_b_columns(which):
    """Moving s1, s7 or s8 by 0.1 from the stated value moves some printed
    B-model error by more than 2 % (Table 4, Pe = 8)."""
    printed = GOLDEN["table4"]["Er_x100"]["8"]
    kw = {which: {"s1": 1.0, "s7": 1.1, "s8": 1.1}[which]}
    worst = max(abs(abs(signed_error(m, 1.0, 8.0, rates(**kw))) * 100.0 / p - 1.0)
                for m, p in zip(MODELS[1:], printed[1:]))
    assert worst >= 0.02


def test_printed_mrt_a_column_is_met_near_s2_094():
    """Observation about the printed numbers (not the oracle's setting):
    s2 = 0.94 with every other rate as stated meets all twelve MRT-A values
    to within 3 %."""
    for tab, tau, Pe, printed in table_rows():
        r = abs(signed_error("A", tau, Pe, rates(s2=0.94))) * 100.0 / printed[0]
        print(f"table {tab} Pe={Pe}: MRT-A at s2 = 0.94 ours/printed {r:.4f}")
        assert abs(r - 1.0) <= 0.03


def hill_er2(kind, model, r, kcut=0.6):
    """Er_2 of Eq. (43) for the Table 1 hill (u = 0, 512^2, s4 = s_xx,
    s6 = s_yy) from the oracle's one-step symbol: phi_hat(k, t) =
    1^T (diag(exp(-i k.e)) C)^t f_eq(1) phi0_hat(k), C the oracle's collision
    of unit populations.  Modes with |k_x| or |k_y| above kcut carry less than
    1e-9 of the hill and of the exact solution and are left out."""
    from paper_1404_2363_amd.paper_tables import hill_exact
    wl = W.paper_hill(kind, (0.0, 0.0), n=512)
    n = wl.shape[0]
    prob = O.Problem("d2q9", (1, 1), ("periodic", "periodic"), np.zeros((2, 1, 1)), wl.D, model=model,
                     heat_rule="paper", rates=r)
    C = np.zeros((9, 9))
    for j in range(9):
        f = np.zeros((9, 1, 1))
        f[j] = 1.0
        C[:, j] = prob.collide(f).reshape(9)
    e0 = prob.equilibrium(np.ones((1, 1))).reshape(9)
    k = 2 * np.pi * np.fft.fftfreq(n)
    keep = np.abs(k) <= kcut
    KY, KX = np.meshgrid(k[keep], k[keep], indexing="ij")
    e = O.D2Q9.e
    G = np.exp(-1j * (KX[..., None] * e[:, 0] + KY[..., None] * e[:, 1]))[..., :, None] * C
    lam, V = np.linalg.eig(G)
    c = np.linalg.solve(V, np.broadcast_to(e0.astype(complex), lam.shape)[..., None])[..., 0]
    H = np.zeros((n, n), complex)
    H[np.ix_(keep, keep)] = np.einsum("...ij,...j->...i", V, lam ** wl.steps * c).sum(-1)
    phi = np.real(np.fft.ifft2(np.fft.fft2(wl.phi0()) * H))
    ex = hill_exact(wl, float(wl.steps))
    return float(np.sqrt(np.mean((phi - ex) ** 2)))


@pytest.mark.parametrize("kind", ["isotropic", "diagonal", "full"])
def test_table1_mrt_a_with_the_same_s2(kind):
    """Independent check of the s2 observation on Table 1 (Sec. 3.1, u = 0):
    at the stated rates MRT-A's Er_2 is 0.91-0.93 of the printed value (the
    GPU tables give the same), with s2 = 0.94 it is 0.98-1.00, while MRT-B2
    (0.94-0.95) moves by less than 1e-4."""
    pr = GOLDEN["table1"][kind]["Er2"]
    a_stated = hill_er2(kind, "A", rates()) / pr[0]
    a_094 = hill_er2(kind, "A", rates(s2=0.94)) / pr[0]
    b2 = hill_er2(kind, "B2", rates()) / pr[2]
    b2_094 = hill_er2(kind, "B2", rates(s2=0.94)) / pr[2]
    print(f"table 1 {kind}: MRT-A {a_stated:.3f} -> {a_094:.3f} at s2 = 0.94; MRT-B2 {b2:.3f} -> {b2_094:.3f}")
    assert 0.90 <= a_stated <= 0.935
    assert abs(a_094 - 1.0) <= 0.02
    assert abs(b2_094 / b2 - 1.0) <= 1e-3
