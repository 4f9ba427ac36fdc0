"""Batched persistent stepping of uneven runs (the Taylor-Aris ensemble form).

Several channels of different length, gap, Peclet number, relaxation time
and step budget are advanced by one persistent launch per step (replayed
from captured graphs); each run is compared with the FP64 oracle run alone,
at its own budget.  The in-graph x-moment history is compared with the
oracle's moments at the sampled times.
"""
import json
import os

import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}

CHANNELS = [  # (h, Pe, tau, nx, max_steps); the first has more nodes than one pass of the x-moment blocks
    (12, 20.0, 0.8, 1400, -1),
    (20, 8.0, 1.4, 64, 47),
    (7, 40.0, 0.6, 130, -1),
    (16, 12.0, 1.1, 90, 70),
    (9, 5.0, 1.9, 77, 33),
]


def channels(wall="specular"):
    out = []
    for h, Pe, tau, nx, budget in CHANNELS:
        wl = W.taylor_aris_channel(h, Pe, tau, nx=nx, wall=wall, steps=100)
        out.append((wl, budget, tau))
    return out


def solver_for(chs, precision):
    from paper_1404_2363_amd.solver import Solver
    wls = [c[0] for c in chs]
    per_run = [{"max_steps": b, "heat": [1 / tau, 1 / tau], "xref0": wl.meta["x0"],
                "xref_drift": wl.meta["U_node_mean"]} for wl, b, tau in chs]
    return Solver(wls, precision, per_run=per_run)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("wall", ["specular", "bounce"])
def test_batch_matches_oracle_per_run(precision, wall):
    chs = channels(wall)
    s = solver_for(chs, precision)
    print(f"case batch of {len(chs)} channels {wall} {precision}", flush=True)
    s.step(100)          # 3 graph replays of 32 steps + 4 single launches
    for i, (wl, budget, tau) in enumerate(chs):
        steps = 100 if budget < 0 else budget
        assert s.steps_done(i) == steps
        ref, _ = O.run_workload(wl, steps=steps, heat_rule=[1 / tau, 1 / tau])
        err = float(np.abs(s.phi(i).cpu().numpy() - ref).max() / np.abs(ref).max())
        assert err <= TOL[precision], (i, err)
    s.close()


def test_batch_graph_equals_single_steps():
    chs = channels()
    a = solver_for(chs, "fp64")
    a.step(70)
    b = solver_for(chs, "fp64")
    for _ in range(70):
        b.step(1)
    for i in range(len(chs)):
        np.testing.assert_array_equal(a.phi(i).cpu().numpy(), b.phi(i).cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_sampled_history(precision):
    import torch
    chs = channels()
    s = solver_for(chs, precision)
    every, rows = 10, 6
    hist = torch.zeros((rows + 2, len(chs), 3), dtype=torch.float64, device="cuda:0")
    s.run_sampled(every * 3, every, hist)     # two calls continue one history
    s.run_sampled(every * 3, every, hist)
    assert s.samples_written() == rows
    h = hist.cpu().numpy()
    for i, (wl, budget, tau) in enumerate(chs):
        m = wl.meta
        prob = O.problem_for(wl, heat_rule=[1 / tau, 1 / tau])
        f = prob.equilibrium(wl.phi0())
        t = 0
        for k in range(rows):
            target = (k + 1) * every
            if budget >= 0:
                target = min(target, budget)
            f, _ = prob.run(f, target - t)
            t = target
            x_ref = (m["x0"] + m["U_node_mean"] * t) % wl.shape[0]
            ref = O.x_moments(O.phi_of(f), x_ref)
            scale = ref[0] * wl.shape[0] ** 2
            np.testing.assert_allclose(h[k, i], ref, rtol=0, atol=TOL[precision] * scale)
    s.close()


def test_mixed_precisions_fall_back_to_separate_launches():
    from paper_1404_2363_amd.solver import Solver
    chs = channels()[:2]
    s = Solver([c[0] for c in chs], "fp64", per_run=[{"precision": "fp64"}, {"precision": "fp32"}])
    s.step(40)
    for i, (wl, _, _) in enumerate(chs):
        ref, _ = O.run_workload(wl, steps=40)
        err = float(np.abs(s.phi(i).cpu().numpy() - ref).max() / np.abs(ref).max())
        assert err <= TOL["fp64" if i == 0 else "fp32"]


def test_taylor_aris_ensemble_dispersion():
    """The three cheapest channels of the seeded ensemble and the two with
    the largest Peclet numbers (whose horizon is set by the period, the
    widest pulse then 8 sigma), run batched to their own horizons: the
    fitted K within 1 % of D (1 + Pe^2/210) and within 0.3 % of the
    scheme's own asymptotic K from the oracle's one-step symbol (stored in
    golden/taylor_aris_spectral.json; the window of the fit and FP32
    storage account for the rest)."""
    from paper_1404_2363_amd.taylor_aris import run_ensemble
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "taylor_aris_spectral.json")))
    ens = W.taylor_aris_batch()
    cheap = sorted(range(len(ens)), key=lambda i: ens[i].nodes * ens[i].steps)[:3]
    fast = sorted(range(len(ens)), key=lambda i: -golden["channels"][i]["Pe"])[:2]
    pick = cheap + fast
    print(f"case taylor_aris channels {pick}", flush=True)
    res, info = run_ensemble([ens[i] for i in pick], "fp32", every=100)
    for i, r in zip(pick, res):
        g = golden["channels"][i]
        dev = r["K"] / g["K_scheme"] - 1
        print(f"h={r['h']} Pe={r['Pe']:.1f} tau={r['tau']:.3f} steps={r['steps']}: K/K_TA - 1 = {r['rel_err']:.4%}, "
              f"K/K_scheme - 1 = {dev:.4%}", flush=True)
        assert abs(r["rel_err"]) <= 1e-2, r
        assert abs(dev) <= 3e-3, (r, g)
    assert info["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_row_tiles_equal_single_runs(precision):
    """The batch's row tiles (wall rule once per row, 32-bit offsets) give
    bitwise the state of the same runs stepped alone by the general kernels,
    for every y boundary kind and a per-node velocity field."""
    from paper_1404_2363_amd.solver import Solver
    wls = [W.taylor_aris_channel(h, Pe, tau, nx=nx, wall=wall, steps=50)
           for (h, Pe, tau, nx), wall in zip([(12, 20.0, 0.8, 100), (9, 8.0, 1.3, 77), (16, 12.0, 1.1, 90)],
                                             ["specular", "bounce", "specular"])]
    wls.append(W.plate_channel(1.5, 8.0, W_lat=10, length=7, steps=50))
    per = [{"heat": [1.0, 1.0]}] * len(wls)
    fld = W.drifting_cellular(nx=64, ny=30, steps=50, n_hills=3, sigma=4.0, drift=0.0)
    wls.append(fld)
    per = per + [{"heat": [1.0, 1.0]}]
    s = Solver(wls, precision, per_run=per)
    s.step(50)
    batched = [s.phi(i).cpu().numpy() for i in range(len(wls))]
    s.close()
    for i, wl in enumerate(wls):
        one = Solver(wl, precision, per_run=[per[i]])
        one.step(50)
        np.testing.assert_array_equal(batched[i], one.phi().cpu().numpy(), err_msg=wl.name)
        one.close()


def test_full_size_ensemble_sampled_nodes():
    """The 64-channel Taylor-Aris ensemble (Nx = 4096, 17.9 M nodes) in the
    launch variant the tuner picks for it, stepped 40 times by the batched
    persistent kernel; sampled nodes of eight channels are compared with the
    oracle run on a window of the channel: every row of the gap and 2 x 41
    columns around the node, which after 40 steps depend on nothing else."""
    from paper_1404_2363_amd.solver import Solver
    runs = W.taylor_aris_batch()
    per_run = [{"heat": [1 / r.meta["tau"]] * 2, "xref0": r.meta["x0"], "xref_drift": r.meta["U_node_mean"]}
               for r in runs]
    s = Solver(runs, "fp32", per_run=per_run)
    s.tune(3)
    steps = 40
    print(f"case taylor_aris_batch 64 channels x {steps} fp32, tuned variant {s.variant()}", flush=True)
    s.step(steps)
    rng = np.random.default_rng(5)
    picks = sorted(set([0, 63] + list(rng.choice(64, 6, replace=False))))
    for i in picks:
        wl = runs[i]
        phi = s.phi(i).cpu().numpy()
        nx, h = wl.shape
        mass0 = O.mass(wl.phi0())
        assert abs(O.mass(phi) - mass0) <= 1e-5 * mass0
        scale = np.abs(wl.phi0()).max()
        for cx in (0, int(wl.meta["x0"]), int(rng.integers(0, nx))):
            idx = [np.mod(np.arange(cx - steps - 1, cx + steps + 2), nx), np.arange(h)]
            ref, _ = O.run_workload(wl, steps=steps, idx=idx, heat_rule=per_run[i]["heat"])
            c = steps + 1
            err = np.abs(phi[:, cx] - ref[:, c]).max()
            assert err <= TOL["fp32"] * scale, (i, cx, err)
    s.close()
