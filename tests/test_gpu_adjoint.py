"""GPU adjoint (reverse streaming, transposed relaxation) against the FP64 oracle
adjoint and against central finite differences.

* Parity: dJ/dD (per node, 3 components), dJ/dphi0 and J from the GPU
  rollout + backward equal the oracle's misfit_gradient on small grids,
  periodic and with walls, with checkpoint segments that do and do not divide
  the run length, with snapshots inside segments and at segment ends only.
  Bounds: 1e-10 (FP64) and 1e-4 (FP32) of max |grad|.
* Segments replayed from captured graphs equal step-by-step launches bitwise,
  and so do segments taking several steps per launch.
* Finite differences: on the inverse-problem workload (512^2, smooth random
  D field, 10 Gaussian initial conditions, 2000 steps, snapshots every 200,
  checkpoints every 100) the FP32 adjoint gradient agrees with central
  differences of the FP64 GPU forward at 20 random nodes to 1e-4.  These
  observations come from the FP64 GPU forward at D_true; the comparison is a
  consistency check of the adjoint, the oracle parity is the first part.
"""
import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W

pytestmark = pytest.mark.gpu


def _setup(nx, ny, steps, snap, walls=("periodic", "periodic"), seed=5):
    rng = W.rng_for(93, seed)
    d_true = W.dfield_from(*(W.fourier_field(rng, nx, ny, kmax=2) for _ in range(3)))
    d_pert = W.dfield_from(*(W.fourier_field(rng, nx, ny, kmax=2) for _ in range(3)))
    d_trial = d_true + 0.1 * (d_pert - d_true)
    spec = W.GaussianSum(np.array([[nx * 0.4, ny * 0.55]]), np.ones(1), np.array([nx / 7]), (float(nx), float(ny)))
    wl = W.Workload("adjoint_small", "d2q9", (nx, ny), walls, steps, spec, D_field=d_trial,
                    u_const=np.array([0.02, 0.01]))
    phi0 = wl.phi0()
    prob_true = O.Problem("d2q9", (nx, ny), walls, wl.u(), d_true, heat_rule=[1.0, 1.0])
    _, obs = prob_true.run(prob_true.equilibrium(phi0), steps, snap)
    return wl, d_trial, phi0, obs


PP = ("periodic", "periodic")


# snap < ckpt puts snapshots inside segments (launched step by step); snap >=
# ckpt puts them at segment ends only (the captured-graph replay of a segment)
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
@pytest.mark.parametrize("walls,snap,ckpt", [(PP, 10, 20), (PP, 10, 25), (PP, 10, 1), (PP, 10, 2),
                                             (("periodic", "specular"), 10, 20), (("bounce", "specular"), 10, 30),
                                             (PP, 20, 10), (PP, 20, 20), (("bounce", "specular"), 20, 7)])
def test_adjoint_matches_oracle(precision, tol, walls, snap, ckpt):
    import torch
    from paper_1404_2363_amd.adjoint import RolloutSpec, misfit
    nx, ny, steps = 24, 20, 60
    wl, d_trial, phi0, obs = _setup(nx, ny, steps, snap, walls)
    print(f"case adjoint {nx}x{ny} x {steps} {walls} snap {snap} ckpt {ckpt} {precision}", flush=True)
    J_ref, g_ref, dphi_ref = O.misfit_gradient(O.Problem("d2q9", (nx, ny), walls, wl.u(), d_trial,
                                                         heat_rule=[1.0, 1.0]), phi0, obs, snap, return_dphi0=True)
    dev = "cuda:0"
    D = torch.tensor(d_trial, dtype=torch.float64, device=dev, requires_grad=True)
    p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
    ob = torch.tensor(np.stack(obs), dtype=torch.float64, device=dev)
    spec = RolloutSpec(wl, steps, snap, ckpt, precision, (1.0, 1.0))
    J = misfit(D, p0, ob, spec)
    J.backward()
    assert abs(J.item() - J_ref) <= tol * abs(J_ref) * 10
    g = D.grad.cpu().numpy()
    assert np.abs(g - g_ref).max() <= tol * np.abs(g_ref).max(), np.abs(g - g_ref).max() / np.abs(g_ref).max()
    dp = p0.grad.cpu().numpy()
    assert np.abs(dp - dphi_ref).max() <= tol * np.abs(dphi_ref).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_segment_graphs_equal_direct_launches(precision, monkeypatch):
    """A segment replayed from its captured graphs launches the same kernels
    with the same arguments as the step-by-step path: the gradients are
    bitwise equal.  Checkpoints every 20, 40 and 7 steps with snapshots every
    40 cover whole-graph segments, a shorter last segment (a second pair of
    graphs) and segments with a snapshot inside (step by step)."""
    import torch
    from paper_1404_2363_amd.adjoint import RolloutSpec, misfit
    nx, ny, steps, snap = 64, 48, 120, 40
    wl, d_trial, phi0, obs = _setup(nx, ny, steps, snap, ("bounce", "specular"))
    dev = "cuda:0"
    ob = torch.tensor(np.stack(obs), dtype=torch.float64, device=dev)
    for ckpt in (20, 40, 7):
        out = []
        for graphs in ("1", "0"):
            monkeypatch.setenv("LBM_CDE_ADJ_GRAPHS", graphs)
            print(f"case segment graphs={graphs} {precision} ckpt {ckpt}", flush=True)
            D = torch.tensor(d_trial, dtype=torch.float64, device=dev, requires_grad=True)
            p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
            misfit(D, p0, ob, RolloutSpec(wl, steps, snap, ckpt, precision, (1.0, 1.0))).backward()
            out.append((D.grad.cpu().numpy(), p0.grad.cpu().numpy()))
        np.testing.assert_array_equal(out[0][0], out[1][0])
        np.testing.assert_array_equal(out[0][1], out[1][1])
        assert np.abs(out[0][0]).max() > 0


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_multi_step_segments_equal_one_step(precision, tol, monkeypatch):
    """On a periodic grid that spans the tiles, the segment's recomputation
    and reverse sweep take several steps per launch (forward chunks and
    reverse chunks of 4 steps in FP32, 3 in FP64; the first reverse step and
    the left-over steps one per launch): gradients bitwise those of one step
    per launch, with and without the captured graphs, for checkpoint
    intervals that leave remainders; the gradient against the oracle."""
    import torch
    from paper_1404_2363_amd.adjoint import RolloutSpec, misfit
    nx, ny, steps, snap = 150, 72, 120, 40
    wl, d_trial, phi0, obs = _setup(nx, ny, steps, snap)
    dev = "cuda:0"
    ob = torch.tensor(np.stack(obs), dtype=torch.float64, device=dev)
    for ckpt in (20, 23, 7):
        out = []
        for fused, graphs in (("1", "1"), ("1", "0"), ("0", "1")):
            monkeypatch.setenv("LBM_CDE_ADJ_FUSED", fused)
            monkeypatch.setenv("LBM_CDE_ADJ_GRAPHS", graphs)
            print(f"case adjoint multi-step={fused} graphs={graphs} {precision} ckpt {ckpt}", flush=True)
            D = torch.tensor(d_trial, dtype=torch.float64, device=dev, requires_grad=True)
            p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
            J = misfit(D, p0, ob, RolloutSpec(wl, steps, snap, ckpt, precision, (1.0, 1.0)))
            J.backward()
            out.append((D.grad.cpu().numpy(), p0.grad.cpu().numpy(), float(J.detach())))
        for o in out[1:]:
            np.testing.assert_array_equal(o[0], out[0][0])
            np.testing.assert_array_equal(o[1], out[0][1])
    monkeypatch.delenv("LBM_CDE_ADJ_FUSED")
    monkeypatch.delenv("LBM_CDE_ADJ_GRAPHS")
    J_ref, g_ref, dphi_ref = O.misfit_gradient(O.Problem("d2q9", (nx, ny), wl.walls, wl.u(), d_trial,
                                                         heat_rule=[1.0, 1.0]), phi0, obs, snap, return_dphi0=True)
    g = out[0][0]
    err = float(np.abs(g - g_ref).max() / np.abs(g_ref).max())
    print(f"oracle gradient error {err:.2e}", flush=True)
    assert err <= tol
    assert np.abs(out[0][1] - dphi_ref).max() <= tol * np.abs(dphi_ref).max()


def test_adjoint_rejects_adaptive_heat_rates():
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    import torch
    wl, d_trial, phi0, obs = _setup(16, 12, 10, 5)
    s = Solver(wl, "fp64", heat="lambda_min")
    nb = s.state_bytes()
    buf = torch.zeros(nb * 4, dtype=torch.uint8, device="cuda:0")
    grad = torch.zeros((3, 12, 16), dtype=torch.float64, device="cuda:0")
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_adjoint_segment(s.h, 0, buf.data_ptr(), 2, buf.data_ptr(), None, buf.data_ptr(),
                                  buf.data_ptr(), grad.data_ptr())
    assert e.value.code == L.LBM_CDE_EUNSUPPORTED
    s.close()


def test_adjoint_scratch_is_smaller_than_the_states():
    """The segment scratch holds two states and 2 values per node and step
    (plus an FP32 partial), far less than the K states it replaces."""
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    wl, d_trial, phi0, obs = _setup(64, 48, 10, 5)
    for precision, elem in (("fp32", 4), ("fp64", 8)):
        s = Solver(wl, precision, heat=[1.0, 1.0])
        nb = s.state_bytes()
        for K in (1, 7, 100):
            b = L.lbm_cde_adjoint_scratch_bytes(s.h, 0, K)
            assert 2 * nb + K * 2 * elem * wl.nodes <= b <= 2 * nb + K * (2 * elem * wl.nodes + 256) + 12 * wl.nodes + 256
        assert L.lbm_cde_adjoint_scratch_bytes(s.h, 0, 100) < 0.25 * 100 * nb
        s.close()


def test_checkpoint_restart_is_bitwise():
    from paper_1404_2363_amd.solver import Solver
    wl = W.cellular(nx=64, ny=40, steps=50, n_hills=3, sigma=5.0)
    a = Solver(wl, "fp32")
    a.step(20)
    ck = a.get_state()
    a.step(30)
    b = Solver(wl, "fp32")
    b.set_state(ck, 20)
    b.step(30)
    assert b.steps_done() == 50
    np.testing.assert_array_equal(a.phi().cpu().numpy(), b.phi().cpu().numpy())


def _dJ(phi_p, phi_m, obs):
    """J(+) - J(-) from field differences, avoiding cancellation at J level."""
    return 0.5 * float(((phi_p - phi_m) * (phi_p + phi_m - 2 * obs)).sum())


def test_inverse_problem_gradient_vs_finite_differences():
    import torch
    from paper_1404_2363_amd.adjoint import RolloutSpec, forward_snapshots, misfit
    inv = W.inverse_dfield()
    nx, ny = inv["shape"]
    steps, snap, ckpt = inv["steps"], inv["snap_every"], inv["ckpt_every"]
    dev = "cuda:0"
    print(f"case inverse problem {nx}x{ny}, {len(inv['ics'])} ICs x {steps} steps", flush=True)
    D_true = torch.tensor(inv["D_true"], dtype=torch.float64, device=dev)
    D_trial = torch.tensor(inv["D_trial"], dtype=torch.float64, device=dev)
    specs64 = [RolloutSpec(ic, steps, snap, ckpt, "fp64", (1.0, 1.0)) for ic in inv["ics"]]
    specs32 = [RolloutSpec(ic, steps, snap, ckpt, "fp32", (1.0, 1.0)) for ic in inv["ics"]]
    phi0s = [torch.tensor(ic.phi0(), dtype=torch.float64, device=dev) for ic in inv["ics"]]
    obs = [forward_snapshots(D_true, p, sp) for p, sp in zip(phi0s, specs64)]
    D = D_trial.clone().requires_grad_(True)
    J = sum(misfit(D, p, o, sp) for p, o, sp in zip(phi0s, obs, specs32))
    J.backward()
    g = D.grad.cpu().numpy()
    gmax = np.abs(g).max()
    eps = 1e-3 * float(D_trial.abs().max())
    worst = 0.0
    for j, (x, y) in enumerate(inv["fd_nodes"]):
        c = j % 3
        Dp, Dm = D_trial.clone(), D_trial.clone()
        Dp[c, y, x] += eps
        Dm[c, y, x] -= eps
        dJ = sum(_dJ(forward_snapshots(Dp, p, sp), forward_snapshots(Dm, p, sp), o)
                 for p, o, sp in zip(phi0s, obs, specs64))
        fd = dJ / (2 * eps)
        err = abs(g[c, y, x] - fd) / max(abs(fd), 1e-3 * gmax)
        worst = max(worst, err)
        print(f"node ({x},{y}) comp {c}: adjoint {g[c, y, x]:.6e} fd {fd:.6e} rel {err:.2e}", flush=True)
    assert worst <= 1e-4, worst


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_misfit_many_equals_sequential(precision):
    """The initial conditions run side by side, each on its own stream, give
    the gradient of the same total misfit as running them one after another
    (same kernels per condition; only the order of the final sum differs)."""
    import torch
    from paper_1404_2363_amd.adjoint import RolloutSpec, forward_snapshots, misfit, misfit_many
    inv = W.inverse_dfield(n=96, n_ic=3, steps=400, snap_every=100, ckpt_every=50, sigma0=8.0)
    dev = "cuda:0"
    print(f"case misfit_many 96^2, 3 ICs x 400 steps, {precision}", flush=True)
    specs = [RolloutSpec(ic, inv["steps"], inv["snap_every"], inv["ckpt_every"], precision, (1.0, 1.0))
             for ic in inv["ics"]]
    spec64 = [RolloutSpec(ic, inv["steps"], inv["snap_every"], inv["ckpt_every"], "fp64", (1.0, 1.0))
              for ic in inv["ics"]]
    phi0s = [torch.tensor(ic.phi0(), dtype=torch.float64, device=dev) for ic in inv["ics"]]
    D_true = torch.tensor(inv["D_true"], dtype=torch.float64, device=dev)
    obs = [forward_snapshots(D_true, p, sp) for p, sp in zip(phi0s, spec64)]
    D1 = torch.tensor(inv["D_trial"], dtype=torch.float64, device=dev, requires_grad=True)
    J1 = sum(misfit(D1, p, o, sp) for p, o, sp in zip(phi0s, obs, specs))
    J1.backward()
    D2 = torch.tensor(inv["D_trial"], dtype=torch.float64, device=dev, requires_grad=True)
    J2 = misfit_many(D2, phi0s, obs, specs)
    J2.backward()
    torch.cuda.synchronize()
    g1, g2 = D1.grad.cpu().numpy(), D2.grad.cpu().numpy()
    err = float(np.abs(g1 - g2).max() / np.abs(g1).max())
    j1, j2 = float(J1.detach()), float(J2.detach())
    print(f"J {j1:.12e} vs {j2:.12e}; gradient difference {err:.2e}", flush=True)
    assert abs(j1 - j2) <= 1e-12 * abs(j1)
    assert err <= 1e-12
