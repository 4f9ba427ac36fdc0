"""Every launch variant the autotuner can pick, against the oracle.

The library lists the compiled variants of a run (tile shape, streaming
stores, block order over the XCDs; for a batch also the row-tile width and
the block count of the persistent launch) and the tuner chooses among
exactly these.  Each test walks the whole list: the state after a few dozen
steps must be bitwise the state of the run's default variant (populations
and phi), and that state must match the FP64 oracle within the precision's
tolerance (1e-12 FP64, 1e-5 FP32 shifted, 1e-3 FP16 split).  So whatever
variant the tuner picks for the benchmark has been compared with the oracle.

Grids have a ragged x tail and tile-row counts divisible by 8, so the
row-interleaved block order is among the candidates.
"""
import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W
from state_views import populations

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 1e-3}
def _populations(s, wl, precision, run=0):
    """Stored populations (Q, nodes) and, for split storage, phi (nodes)."""
    Q = 9 if wl.lattice == "d2q9" else 15
    return populations(s.get_state(run).cpu().numpy(), Q, wl.nodes, precision)


def _walk(wl, precision, steps, heat="lambda_min", min_variants=1):
    from paper_1404_2363_amd.solver import Solver
    s = Solver(wl, precision, heat=heat)
    variants = s.variants()
    default = s.variant()
    s.step(steps)
    ref_pops, ref_phi = _populations(s, wl, precision)
    phi0 = s.phi().cpu().numpy()
    s.close()
    assert len(variants) >= min_variants, len(variants)
    seen_orders = set()
    for v in variants:
        s = Solver(wl, precision, heat=heat)
        s.set_variant(v)
        assert s.variant() == v
        s.step(steps)
        pops, phi = _populations(s, wl, precision)
        np.testing.assert_array_equal(pops, ref_pops, err_msg=str(v))
        if phi is not None:
            np.testing.assert_array_equal(phi, ref_phi, err_msg=str(v))
        np.testing.assert_array_equal(s.phi().cpu().numpy(), phi0, err_msg=str(v))
        s.close()
        seen_orders.add(v["block_order"])
    ref, _ = O.run_workload(wl, steps=steps, heat_rule=heat)
    err = float(np.abs(phi0 - ref).max() / np.abs(ref).max())
    print(f"{wl.name} {wl.shape} {precision}: {len(variants)} variants bitwise equal to {default}, "
          f"oracle error {err:.2e}", flush=True)
    assert err <= TOL[precision]
    return variants, seen_orders


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_d2q9_every_variant_periodic(precision):
    wl = W.cellular(nx=300, ny=128, steps=40, n_hills=5, sigma=9.0)
    variants, orders = _walk(wl, precision, 40, min_variants=54)
    assert orders == {0, 1, 2}
    assert any(v["block"] == (512, 1) and v["nt_stores"] for v in variants)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_d2q9_every_variant_walls(precision):
    wl = W.taylor_aris_channel(64, 12.0, 1.1, nx=300, steps=40, wall="bounce")
    wl.walls = ("specular", "bounce")
    _walk(wl, precision, 40, min_variants=54)


def test_d2q9_every_variant_ragged_y():
    # 77 rows: the row-interleaved order is not a candidate (77 tile rows)
    wl = W.cellular(nx=261, ny=77, steps=30, n_hills=4, sigma=7.0)
    variants, orders = _walk(wl, "fp32", 30)
    assert 2 not in {v["block_order"] for v in variants if v["block"][1] * v["rows_per_thread"] == 1}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_d3q15_every_variant(precision):
    wl = W.sine3d(n=150, ny=16, nz=8, steps=12, n_hills=3, sigma=4.0)
    variants, orders = _walk(wl, precision, 12, min_variants=30)
    assert orders == {0, 1, 2}


def test_d3q15_every_variant_walls():
    wl = W.sine3d(n=70, ny=16, nz=8, steps=10, n_hills=3, sigma=3.0)
    wl.walls = ("periodic", "bounce", "specular")
    _walk(wl, "fp32", 10)


def test_fp16_split_every_variant_periodic():
    wl = W.cellular(nx=520, ny=64, steps=30, n_hills=5, sigma=8.0)
    variants, orders = _walk(wl, "fp16", 30, min_variants=36)
    assert orders == {0, 1, 2} and any(v["nt_stores"] for v in variants)


def test_fp16_split_every_variant_walls():
    wl = W.taylor_aris_channel(32, 12.0, 1.1, nx=300, steps=30, wall="specular")
    _walk(wl, "fp16", 30)


def test_fp16_literal_every_variant():
    from paper_1404_2363_amd.solver import Solver
    wl = W.cellular(nx=300, ny=64, steps=20, n_hills=4, sigma=8.0)
    outs = []
    s0 = Solver(wl, "fp16_literal")
    variants = s0.variants()
    s0.close()
    for v in variants:
        s = Solver(wl, "fp16_literal")
        s.set_variant(v)
        s.step(20)
        outs.append(s.phi().cpu().numpy())
        s.close()
    assert len(outs) == 3
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_set_variant_rejects_unbuilt():
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    s = Solver(W.cellular(nx=64, ny=36, steps=1, n_hills=2, sigma=4.0), "fp32")
    v = dict(s.variant())
    for bad in ({**v, "block": (96, 1)}, {**v, "grid": 7}, {**v, "block_order": 3},
                {**v, "block": (256, 1), "rows_per_thread": 1, "block_order": 2}):   # 36 tile rows: not 8k
        with pytest.raises(L.LbmCdeError) as e:
            s.set_variant(bad)
        assert e.value.code == L.LBM_CDE_EINVAL
    with pytest.raises(L.LbmCdeError):
        L.lbm_cde_variant_at(s.h, 0, 10 ** 6)
    s.close()


# ---- batches: every row-tile width, store kind and block count -------------

BATCH = [  # (h, Pe, tau, nx, max_steps, wall)
    (12, 20.0, 0.8, 700, -1, "specular"),
    (20, 8.0, 1.4, 64, 23, "bounce"),
    (7, 40.0, 0.6, 1030, -1, "specular"),
    (16, 12.0, 1.1, 90, 31, "specular"),
    (9, 5.0, 1.9, 77, 17, "bounce"),
]


def _batch(precision):
    from paper_1404_2363_amd.solver import Solver
    wls, per = [], []
    for h, Pe, tau, nx, budget, wall in BATCH:
        wl = W.taylor_aris_channel(h, Pe, tau, nx=nx, wall=wall, steps=40)
        wls.append(wl)
        per.append({"max_steps": budget, "heat": [1 / tau, 1 / tau], "xref0": wl.meta["x0"],
                    "xref_drift": wl.meta["U_node_mean"]})
    return wls, per, (lambda: Solver(wls, precision, per_run=per))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_every_variant_and_grid(precision):
    """The listed batch variants plus small persistent grids (1, 7 and 61
    blocks), where every block walks many tiles of several runs at both
    buffer parities, all bitwise equal; the default equals the oracle per run
    at its own budget."""
    wls, per, make = _batch(precision)
    s = make()
    cands = s.variants()
    default = s.variant()
    s.step(40)
    ref = [s.phi(i).cpu().numpy() for i in range(len(wls))]
    tiles_256 = sum(-(-wl.shape[0] // 256) * wl.shape[1] for wl in wls)
    s.close()
    assert default["grid"] == tiles_256           # one block per tile by default
    extra = [{**c, "grid": g} for c in cands if c["grid"] == cands[0]["grid"] for g in (1, 7, 61)]
    assert len(cands) == 30 and len(extra) == 18
    for v in cands + extra:
        s = make()
        s.set_variant(v)
        got = s.variant()
        assert got["block"] == v["block"] and got["nt_stores"] == v["nt_stores"]
        assert got["grid"] == min(v["grid"], sum(-(-wl.shape[0] // v["block"][0]) * wl.shape[1] for wl in wls)) \
            or v["grid"] == 0
        s.step(40)
        for i in range(len(wls)):
            np.testing.assert_array_equal(s.phi(i).cpu().numpy(), ref[i], err_msg=f"{v} run {i}")
        s.close()
    for i, (wl, p) in enumerate(zip(wls, per)):
        steps = 40 if p["max_steps"] < 0 else p["max_steps"]
        r, _ = O.run_workload(wl, steps=steps, heat_rule=p["heat"])
        err = float(np.abs(ref[i] - r).max() / np.abs(r).max())
        assert err <= TOL[precision], (i, err)


def test_batch_tuner_keeps_state():
    wls, per, make = _batch("fp32")
    a = make()
    a.step(13)
    before = [a.phi(i).cpu().numpy() for i in range(len(wls))]
    a.tune(2)
    for i in range(len(wls)):
        np.testing.assert_array_equal(a.phi(i).cpu().numpy(), before[i])
    a.step(27)
    b = make()
    b.step(40)
    for i in range(len(wls)):
        np.testing.assert_array_equal(a.phi(i).cpu().numpy(), b.phi(i).cpu().numpy())
    print("batch tuner picked", a.variant(), flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_general_kernel_equals_compact_kernel(precision, monkeypatch):
    """A batch whose runs all have periodic x and constant D is stepped from
    compact per-run records; the general batched kernel (forced here) gives
    bitwise the same states, in every listed variant plus a 7-block grid."""
    wls, per, make = _batch(precision)
    s = make()
    cands = s.variants()
    s.close()
    picks = [cands[0], cands[7], cands[-1], {**cands[3], "grid": 7}]
    for v in picks:
        outs = []
        for general in (False, True):
            if general:
                monkeypatch.setenv("LBM_CDE_BATCH_GENERAL", "1")
            else:
                monkeypatch.delenv("LBM_CDE_BATCH_GENERAL", raising=False)
            s = make()
            s.set_variant(v)
            s.step(40)
            outs.append([s.phi(i).cpu().numpy() for i in range(len(wls))])
            s.close()
        for i in range(len(wls)):
            np.testing.assert_array_equal(outs[0][i], outs[1][i], err_msg=f"{v} run {i}")


def test_batch_with_walls_in_x_uses_general_kernel():
    """A run with walls across x (no row-tile path) makes the batch take the
    general kernel; each run still equals the oracle at its own budget."""
    from paper_1404_2363_amd.solver import Solver
    wls, per, _ = _batch("fp64")
    walled = W.taylor_aris_channel(10, 9.0, 1.2, nx=90, wall="specular", steps=40)
    walled.walls = ("bounce", "specular")
    wls = wls + [walled]
    per = per + [{"max_steps": 29, "heat": [1 / 1.2, 1 / 1.2]}]
    s = Solver(wls, "fp64", per_run=per)
    s.set_variant({**s.variant(), "grid": 5})
    s.step(40)
    for i, (wl, p) in enumerate(zip(wls, per)):
        steps = 40 if p["max_steps"] < 0 else p["max_steps"]
        r, _ = O.run_workload(wl, steps=steps, heat_rule=p["heat"])
        err = float(np.abs(s.phi(i).cpu().numpy() - r).max() / np.abs(r).max())
        assert err <= 1e-12, (i, err)
    s.close()
