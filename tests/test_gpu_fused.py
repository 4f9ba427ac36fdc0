"""Several D2Q9 steps per launch (the LDS-blocked kernel) against one-step
launches and the FP64 oracle.

A multi-step launch computes the intermediate steps of a tile and its halo in
LDS with the same per-node arithmetic as the one-step kernel, so every result
must be bitwise that of the run's default (one-step) variant:

* every multi-step variant (steps per launch 2-5, each tile shape, each block
  order) over call sequences whose counts leave one-step remainders, fill
  captured graphs (32 steps) and read the state in between; the final state
  also against the oracle;
* the velocity as a constant, a separable product (whose factors the later
  steps of a launch take from LDS) and a per-node field;
* checkpoint and restart (get_state / set_state) in the middle of multi-step
  stepping, with the run's step budget ending inside a launch's span;
* a per-node D field (per-node relaxation parameters) and a per-node velocity
  field replaced between calls;
* a handle of two runs of which only one steps several steps per launch, so
  the runs' buffers drift apart and the graph path is left;
* a batch of channels in one multi-step launch over all their tiles, with
  budgets ending inside and at the end of 32-step blocks (one step per launch
  there), against one-step batched launches (states and sampled histories);
* walls in y (bounce-back, halfway mirror, the paper's on-node mirror) on a
  channel whose height is no multiple of the tile height;
* grids too small for a tile and its halo, walls in x, and a per-node
  velocity field with walls, are refused.
"""
import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W
from state_views import populations

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _phi(s, run=0):
    return s.phi(run).cpu().numpy()


def _pops(s, wl, precision):
    """Stored populations (9, nodes): the state without the padding between planes."""
    return populations(s.get_state().cpu().numpy(), 9, wl.nodes, precision)[0]


def _one_step(s, run=0):
    """The one-step variant with 256 x 1 tiles and streaming stores in hardware order."""
    return next(v for v in s.variants(run) if v["steps_per_launch"] == 1 and v["block"] == (256, 1)
                and v["rows_per_thread"] == 1 and v["nt_stores"] and v["block_order"] == 0)


def _multi(s, run=0):
    return [v for v in s.variants(run) if v["steps_per_launch"] > 1]


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("precision,velocity", [("fp64", "separable"), ("fp32", "separable"), ("fp32", "const")])
def test_every_multi_step_variant(precision, velocity):
    import dataclasses
    from paper_1404_2363_amd.solver import Solver
    seq = [1, 5, 32, 7, 64, 3]
    wl = W.cellular(nx=203, ny=150, steps=sum(seq), n_hills=4, sigma=7.0)
    if velocity == "const":
        wl = dataclasses.replace(wl, u_sep=None, u_const=np.array([0.04, -0.03]))
    ref = Solver(wl, precision)
    assert ref.variant()["steps_per_launch"] == 4          # the default for such runs
    ref.set_variant(_one_step(ref))
    phis = []
    for n in seq:
        ref.step(n)
        phis.append(_phi(ref))
    state = _pops(ref, wl, precision)
    variants = _multi(ref)
    ref.close()
    spl = {v["steps_per_launch"] for v in variants}
    print(f"case multi-step variants 203x150 {precision} {velocity} u: {len(variants)} variants, "
          f"steps per launch {sorted(spl)}", flush=True)
    assert spl >= {2, 3, 4, 5} and len(variants) >= 18     # 9 shapes x block orders 0 and 1
    for v in variants:
        s = Solver(wl, precision)
        s.set_variant(v)
        assert s.variant() == v
        for n, p in zip(seq, phis):
            s.step(n)
            np.testing.assert_array_equal(_phi(s), p, err_msg=str(v))
        np.testing.assert_array_equal(_pops(s, wl, precision), state, err_msg=str(v))
        assert s.steps_done() == sum(seq)
        s.close()
    oref, _ = O.run_workload(wl, steps=sum(seq))
    err = rel(phis[-1], oref)
    print(f"oracle error {err:.2e}", flush=True)
    assert err <= TOL[precision]


def test_checkpoint_restart_and_budget():
    from paper_1404_2363_amd.solver import Solver
    wl = W.cellular(nx=160, ny=96, steps=101, n_hills=3, sigma=6.0)
    ref = Solver(wl, "fp32", max_steps=101)
    ref.set_variant(_one_step(ref))
    ref.step(200)                       # stops at the budget
    assert ref.steps_done() == 101
    end = _phi(ref)
    ref.close()
    for T in (3, 4):
        a = Solver(wl, "fp32", max_steps=101)
        v = next(v for v in _multi(a) if v["steps_per_launch"] == T and v["block_order"] == 0)
        print(f"case checkpoint/budget 160x96 fp32 {v}", flush=True)
        a.set_variant(v)
        a.step(37)                      # 12 or 9 multi-step launches and a remainder
        ck, t0 = a.get_state(), a.steps_done()
        a.step(200)
        assert a.steps_done() == 101
        np.testing.assert_array_equal(_phi(a), end)
        b = Solver(wl, "fp32", max_steps=101)
        b.set_variant(v)
        b.set_state(ck, t0)
        b.step(64)
        b.step(64)
        assert b.steps_done() == 101
        np.testing.assert_array_equal(_phi(b), end)
        a.close()
        b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_node_diffusion_field(precision):
    from paper_1404_2363_amd.solver import Solver
    nx, ny, steps = 150, 72, 45
    rng = W.rng_for(93, 17)
    D = W.dfield_from(*(W.fourier_field(rng, nx, ny, kmax=2) for _ in range(3)))
    spec = W.GaussianSum(np.array([[nx * 0.4, ny * 0.55]]), np.ones(1), np.array([nx / 9]), (float(nx), float(ny)))
    wl = W.Workload("dfield_periodic", "d2q9", (nx, ny), ("periodic", "periodic"), steps, spec, D_field=D,
                    u_const=np.array([0.03, -0.02]))
    ref = Solver(wl, precision, heat=[1.0, 1.0])
    ref.set_variant(_one_step(ref))
    ref.step(steps)
    want = _phi(ref)
    variants = _multi(ref)
    ref.close()
    print(f"case per-node D 150x72 x {steps} {precision}: {len(variants)} multi-step variants", flush=True)
    for v in variants:
        if v["block_order"] != 0:
            continue
        s = Solver(wl, precision, heat=[1.0, 1.0])
        s.set_variant(v)
        s.step(steps)
        np.testing.assert_array_equal(_phi(s), want, err_msg=str(v))
        s.close()
    prob = O.Problem("d2q9", (nx, ny), wl.walls, wl.u(), D, heat_rule=[1.0, 1.0])
    f = prob.equilibrium(wl.phi0())
    for _ in range(steps):
        f = prob.step(f)
    assert rel(want, O.phi_of(f)) <= TOL[precision]


def test_velocity_field_replaced_between_calls():
    from paper_1404_2363_amd.solver import Solver
    import torch
    wl = W.drifting_cellular(nx=140, ny=90, steps=42, n_hills=4, sigma=5.0, U0=0.08, drift=0.7)
    fields = [torch.tensor(np.asarray(wl.u_schedule(7 * k)), dtype=torch.float64, device="cuda:0") for k in range(6)]

    def run(v):
        s = Solver(wl, "fp32")
        s.set_variant(v if v is not None else _one_step(s))
        for u in fields:
            s.set_velocity(u)
            s.step(7)
        out = _phi(s)
        s.close()
        return out

    want = run(None)
    s = Solver(wl, "fp32")
    variants = [v for v in _multi(s) if v["block_order"] == 0]
    s.close()
    print(f"case velocity field replaced every 7 steps 140x90: {len(variants)} multi-step variants", flush=True)
    for v in variants:
        np.testing.assert_array_equal(run(v), want, err_msg=str(v))


def test_two_runs_one_multi_step():
    from paper_1404_2363_amd.solver import Solver
    wa = W.cellular(nx=180, ny=100, steps=100, n_hills=3, sigma=6.0)
    wb = W.cellular(nx=96, ny=64, steps=100, n_hills=2, sigma=5.0, seed_id=3)
    seq = [5, 64, 3, 32]
    want = []
    for wl, prec in ((wa, "fp32"), (wb, "fp64")):
        s = Solver(wl, prec)
        s.set_variant(_one_step(s))
        s.step(sum(seq))
        want.append(_phi(s))
        s.close()
    s = Solver([wa, wb], per_run=[{"precision": "fp32"}, {"precision": "fp64"}])
    v = next(v for v in _multi(s, 0) if v["steps_per_launch"] == 3 and v["block_order"] == 0)
    print(f"case two runs, run 0 {v}", flush=True)
    s.set_variant(v, run=0)
    s.set_variant(_one_step(s, 1), run=1)
    for n in seq:
        s.step(n)
    assert s.steps_done(0) == s.steps_done(1) == sum(seq)
    np.testing.assert_array_equal(_phi(s, 0), want[0])
    np.testing.assert_array_equal(_phi(s, 1), want[1])
    s.close()


@pytest.mark.parametrize("wall", ["bounce", "specular", "node"])
def test_walls_in_y(wall):
    """A plane Poiseuille channel (x periodic, walls in y, separable velocity):
    every multi-step variant against one-step launches, and the oracle.  Tiles
    overhang the walls (ny = 37 is no multiple of the tile height); rows beyond
    a wall are skipped and pulls across it take the wall rule's source."""
    import dataclasses
    from paper_1404_2363_amd.solver import Solver
    wl = W.taylor_aris_channel(37, 12.0, 0.9, nx=150, steps=45, wall="specular")
    wl.walls = ("periodic", wall)
    for precision in ("fp64", "fp32"):
        ref = Solver(wl, precision)
        assert ref.variant()["steps_per_launch"] == 4
        ref.set_variant(_one_step(ref))
        seq = [3, 32, 10]
        phis = []
        for n in seq:
            ref.step(n)
            phis.append(_phi(ref))
        variants = _multi(ref)
        ref.close()
        print(f"case channel 150x37 walls {wall} {precision}: {len(variants)} multi-step variants", flush=True)
        assert len(variants) >= 18
        for v in variants:
            s = Solver(wl, precision)
            s.set_variant(v)
            for n, p in zip(seq, phis):
                s.step(n)
                np.testing.assert_array_equal(_phi(s), p, err_msg=str(v))
            s.close()
        oref, _ = O.run_workload(wl, steps=sum(seq))
        err = rel(phis[-1], oref)
        print(f"oracle error {err:.2e}", flush=True)
        assert err <= TOL[precision]


FBATCH = [  # (h, Pe, tau, nx, max_steps, wall): budgets inside and at the end of 32-step blocks
    (12, 20.0, 0.8, 300, -1, "specular"),
    (20, 8.0, 1.4, 150, 45, "bounce"),
    (7, 40.0, 0.6, 400, -1, "node"),
    (16, 12.0, 1.1, 200, 64, "specular"),
    (9, 5.0, 1.9, 160, 17, "bounce"),
]


def _fbatch(precision):
    from paper_1404_2363_amd.solver import Solver
    wls, per = [], []
    for h, Pe, tau, nx, budget, wall in FBATCH:
        wl = W.taylor_aris_channel(h, Pe, tau, nx=nx, wall="specular", steps=40)
        wl.walls = ("periodic", wall)
        wls.append(wl)
        per.append({"max_steps": budget, "heat": [1 / tau, 1 / tau], "xref0": wl.meta["x0"],
                    "xref_drift": wl.meta["U_node_mean"]})
    return wls, per, (lambda: Solver(wls, precision, per_run=per))


def _batch_one_step(s):
    return next(v for v in s.variants() if v["steps_per_launch"] == 1 and v["block"] == (256, 1)
                and v["nt_stores"] and v["grid"] == 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_multi_step(precision):
    """A batch of channels (walls in y of all three kinds, budgets ending inside
    and at the end of 32-step blocks): the multi-step batched launch, the
    default here, and every other multi-step candidate equal one-step batched
    launches bitwise after every call; each run equals the oracle at its own
    budget."""
    wls, per, make = _fbatch(precision)
    seq = [5, 64, 3, 32, 40]
    ref = make()
    default = ref.variant()
    assert default["steps_per_launch"] == 4
    multi = [v for v in ref.variants() if v["steps_per_launch"] > 1]
    ref.set_variant(_batch_one_step(ref))
    assert ref.variant()["steps_per_launch"] == 1
    want = []
    for n in seq:
        ref.step(n)
        want.append([_phi(ref, i) for i in range(len(wls))])
    done = [ref.steps_done(i) for i in range(len(wls))]
    ref.close()
    print(f"case batch multi-step {precision}: default {default}, {len(multi)} multi-step candidates", flush=True)
    assert len(multi) >= 3
    for v in multi:
        s = make()
        s.set_variant(v)
        assert s.variant()["steps_per_launch"] == v["steps_per_launch"]
        for k, n in enumerate(seq):
            s.step(n)
            for i in range(len(wls)):
                np.testing.assert_array_equal(_phi(s, i), want[k][i], err_msg=f"{v} call {k} run {i}")
        assert [s.steps_done(i) for i in range(len(wls))] == done
        s.close()
    for i, (wl, p) in enumerate(zip(wls, per)):
        steps = sum(seq) if p["max_steps"] < 0 else p["max_steps"]
        r, _ = O.run_workload(wl, steps=steps, heat_rule=p["heat"])
        assert rel(want[-1][i], r) <= TOL[precision], i


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_multi_step_sampled_history(precision):
    """In-graph x-moment sampling with multi-step launches (samples every 20
    steps: four-step pairs and one-step launches, and one step per launch in
    the spans where a budget ends; then every 40: multi-step only) equals the
    one-step batch bitwise, history and states."""
    import torch
    wls, per, make = _fbatch(precision)
    out = []
    for multi in (True, False):
        s = make()
        if not multi:
            s.set_variant(_batch_one_step(s))
        hist = torch.zeros((9, len(wls), 3), dtype=torch.float64, device="cuda:0")
        s.run_sampled(100, 20, hist)
        s.run_sampled(80, 40, hist)
        assert s.samples_written() == 7
        out.append((hist.cpu().numpy(), [_phi(s, i) for i in range(len(wls))]))
        s.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    for i in range(len(wls)):
        np.testing.assert_array_equal(out[0][1][i], out[1][1][i])


def test_refused_where_a_tile_and_its_halo_do_not_fit():
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    big = Solver(W.cellular(nx=160, ny=96, steps=1, n_hills=2, sigma=5.0), "fp32")
    v = next(v for v in _multi(big) if v["block"] == (128, 4) and v["steps_per_launch"] == 4)
    big.close()
    # 128 + 2 * 3 = 134 columns are needed
    small = Solver(W.cellular(nx=133, ny=96, steps=1, n_hills=2, sigma=5.0), "fp32")
    assert all(not (u["block"] == (128, 4) and u["steps_per_launch"] == 4) for u in small.variants())
    with pytest.raises(L.LbmCdeError) as e:
        small.set_variant(v)
    assert e.value.code == L.LBM_CDE_EINVAL
    small.close()
    # walls in x (only y may have walls), and a per-node velocity field with walls in y
    walls = W.taylor_aris_channel(32, 12.0, 1.1, nx=300, steps=1, wall="bounce")
    walls.walls = ("bounce", "periodic")
    s = Solver(walls, "fp32")
    assert not _multi(s)
    with pytest.raises(L.LbmCdeError):
        s.set_variant(v)
    s.close()
    fld = W.taylor_aris_channel(32, 12.0, 1.1, nx=300, steps=1, wall="bounce")
    fld.u_field, fld.u_sep = fld.u(), None
    s = Solver(fld, "fp32")
    assert not _multi(s)
    s.close()
