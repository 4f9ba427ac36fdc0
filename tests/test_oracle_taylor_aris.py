"""The scheme's own Taylor-Aris dispersion, from the oracle (Sec. 3.2).

oracle.channel_dispersion gives the long-time dispersion coefficient K and
drift U of the oracle's step in a channel from the eigenvalue of one step
on a Fourier mode exp(i k x) (Eq. 46-47 measure the same rate as the slope
of the variance).  It is pinned by
* pure diffusion (u = 0): K = D_m exactly and U = 0;
* the oracle run in time: the variance slope of a pulse in a small channel
  after the transverse transients have decayed equals 2 K;
* the continuum limit: K / (D_m (1 + Pe^2/210)) - 1 falls as 1/h^2 at fixed
  Pe and tau (the discrete profile and the lattice converge to the
  Taylor-Aris result, Pe with the full gap);
and then applied to every channel of the seeded 64-channel ensemble (values
stored in golden/taylor_aris_spectral.json, a sample recomputed here): the
scheme's asymptotic K is within 1 % of 1 + Pe^2/210 for each of them.
"""
import json
import os

import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W


def channel_problem(wl, tau):
    return O.problem_for(wl, idx=[np.arange(3), np.arange(wl.shape[1])], heat_rule=[1 / tau, 1 / tau])


def test_pure_diffusion_is_exact():
    tau = 0.9
    wl = W.taylor_aris_channel(12, 10.0, tau, nx=64, steps=10)
    wl.u_sep.amp[:] = 0.0                       # no flow
    K, U = O.channel_dispersion(channel_problem(wl, tau))
    # the eigenvalue is accurate to ~1e-15, log|lambda| / k^2 to ~1e-9 at k = 1e-3
    assert abs(K - wl.meta["D_m"]) <= 1e-7 * wl.meta["D_m"]
    assert abs(U) <= 1e-9


@pytest.mark.parametrize("wall", ["specular", "bounce"])
def test_variance_slope_of_the_oracle_run_equals_K(wall):
    """Oracle in time: a pulse in a 6-node channel, sigma^2 sampled every 20
    steps; its slope over [2, 6] h^2/D_m (transverse modes decayed by
    exp(-2 pi^2) and more) is 2 K of the eigenvalue analysis."""
    h, Pe, tau, nx = 6, 4.0, 1.0, 160
    wl = W.taylor_aris_channel(h, Pe, tau, nx=nx, wall=wall, steps=1300)
    m = wl.meta
    prob = O.problem_for(wl, heat_rule=[1 / tau, 1 / tau])
    f = prob.equilibrium(wl.phi0())
    T = h * h / m["D_m"]
    ts, var = [], []
    t = 0
    U = O.channel_dispersion(channel_problem(wl, tau))[1]
    while t < 6 * T:
        f, _ = prob.run(f, 20)
        t += 20
        if t >= 2 * T:
            S0, S1, S2 = O.x_moments(O.phi_of(f), (m["x0"] + U * t) % nx)
            ts.append(t)
            var.append(O.variance_from_moments(S0, S1, S2))
    slope = np.polyfit(np.array(ts, float), np.array(var), 1)[0]
    K, _ = O.channel_dispersion(channel_problem(wl, tau))
    print(f"{wall}: K from the run {slope / 2:.6f}, from the eigenvalue {K:.6f}")
    assert abs(slope / 2 / K - 1) <= 2e-3


def test_continuum_limit_second_order():
    Pe, tau = 10.0, 1.0
    dev = []
    for h in (8, 16, 32):
        wl = W.taylor_aris_channel(h, Pe, tau, nx=64, steps=10)
        m = wl.meta
        K, U = O.channel_dispersion(channel_problem(wl, tau))
        Pe_n = m["U_node_mean"] * h / m["D_m"]
        dev.append(K / (m["D_m"] * (1 + Pe_n ** 2 / 210)) - 1)
        assert abs(U - m["U_node_mean"]) <= 1e-8
    print("deviations", dev)
    assert abs(dev[2]) < abs(dev[1]) < abs(dev[0])
    for a, b in zip(dev, dev[1:]):
        assert 3.5 <= a / b <= 4.5                  # second order in 1/h


GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "taylor_aris_spectral.json")))


def test_golden_file_is_the_seeded_ensemble():
    runs = W.taylor_aris_batch()
    assert len(GOLDEN["channels"]) == len(runs) == 64
    for g, r in zip(GOLDEN["channels"], runs):
        assert (g["h"], g["tau"]) == (r.meta["h"], r.meta["tau"])
        assert abs(g["Pe"] - r.meta["U_node_mean"] * r.meta["h"] / r.meta["D_m"]) <= 1e-12 * g["Pe"]


@pytest.mark.parametrize("which", [0, 18, 30, 44, 62])
def test_golden_values_reproduce(which):
    """A sample of the stored values (the worst wrap-limited channel h = 48,
    Pe = 97.2 among them) recomputed from the oracle."""
    g = GOLDEN["channels"][which]
    m = W.taylor_aris_batch()[which].meta
    K, U = O.channel_dispersion(channel_problem(W.taylor_aris_channel(m["h"], m["Pe"], m["tau"], nx=64, steps=1),
                                                m["tau"]))
    assert abs(K / g["K_scheme"] - 1) <= 1e-9 and abs(U / g["U_scheme"] - 1) <= 1e-9


def test_every_ensemble_channel_within_one_percent():
    """The 1 % Taylor-Aris pin holds for the scheme on every channel of the
    seeded ensemble (h = 32 .. 128, Pe 5 .. 100, tau 0.6 .. 2): the
    asymptotic K of the oracle's step (stored by
    golden/make_taylor_aris_spectral.py), against D_m (1 + Pe^2/210).  The
    deviation is negative and largest for the narrow, fast channels."""
    rel = np.array([g["rel"] for g in GOLDEN["channels"]])
    print(f"largest |K / K_TA - 1| over the ensemble: {np.abs(rel).max():.4%}")
    assert np.all(np.abs(rel) <= 1e-2)
    assert np.all(rel < 0)
