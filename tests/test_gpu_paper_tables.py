"""The paper's accuracy tables reproduced on the GPU path (FP64 storage).

Tables 3-5 (Sec. 3.2, Taylor-Aris between on-node plates): every printed Er
of the unmodified models MRT-B1/B2/B3 (36 values) is reproduced to within
1 % of its value.  For the modified model MRT-A the printed values are not
reproduced: at each tau the ratio of our Er to the printed one is the same
for every Pe (to 0.5 %), but that ratio depends on tau (about 1.31, 2.06 and
0.96 for tau = 2, 1, 0.55).  The test asserts the constant ratio and the
orderings the paper draws from the tables.

Tables 1-2 (Sec. 3.1, Gaussian hill at t_m): the values agree with the
printed ones to within -15 % / +30 % (the paper does not fix how t_m is
rounded to a step or which nodes carry the grid); the test asserts that band
and the orderings the paper reads from them: at u = 0 MRT-B2 equals MRT-B3
exactly and MRT-B1 has the smallest errors; at u = (0.05, 0.05) MRT-B3's
deviation term makes its Er2 the largest by a factor of at least 2.5.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
MODELS = GOLDEN["models"]


@pytest.fixture(scope="module")
def plate_results():
    from paper_1404_2363_amd.paper_tables import run_plate_tables
    print("case Tables 3-5: 48 plate channels 4800x33, FP64, batched", flush=True)
    res, info = run_plate_tables((3, 4, 5))
    assert info["nonfinite"] == 0
    return res


def test_taylor_aris_tables_unmodified_models(plate_results):
    worst = 0.0
    for r in plate_results:
        assert r["t_eq49"] is not None, r          # the convergence test of Eq. (49) passes in the horizon
        assert r["drift_last"] <= 1e-9, r
        if r["model"] == "A":
            continue
        printed = GOLDEN["table%d" % r["table"]]["Er_x100"]["%d" % r["Pe"]][MODELS.index(r["model"])] / 100.0
        ratio = r["Er_end"] / printed
        worst = max(worst, abs(ratio - 1.0))
        assert abs(ratio - 1.0) <= 0.01, (r, printed)
    print(f"worst relative deviation from the printed Er (B models): {worst:.4f}", flush=True)


def test_taylor_aris_tables_modified_model(plate_results):
    for tab in (3, 4, 5):
        rows = [r for r in plate_results if r["table"] == tab]
        ratios = []
        for Pe in sorted({r["Pe"] for r in rows}):
            er = {r["model"]: r["Er_end"] for r in rows if r["Pe"] == Pe}
            printed = GOLDEN["table%d" % tab]["Er_x100"]["%d" % Pe][0] / 100.0
            ratios.append(er["A"] / printed)
            if tab in (3, 4):
                assert er["A"] < er["B1"] < er["B2"] < er["B3"], (tab, Pe, er)
            else:
                assert er["A"] < er["B3"] < er["B1"] < er["B2"], (tab, Pe, er)
        print(f"Table {tab}: MRT-A Er / printed = {np.round(ratios, 4).tolist()}", flush=True)
        assert max(ratios) / min(ratios) <= 1.005, (tab, ratios)


def test_gaussian_hill_tables():
    from paper_1404_2363_amd.paper_tables import run_hill_tables
    print("case Tables 1-2: 24 hills 512^2, FP64, batched", flush=True)
    res, _ = run_hill_tables((1, 2))
    by = {(r["table"], r["D"], r["model"]): r for r in res}
    for (tab, kind, m), r in by.items():
        p = GOLDEN["table%d" % tab][kind]
        i = MODELS.index(m)
        for key in ("Er2", "Erinf"):
            ratio = r[key] / p[key][i]
            assert 0.85 <= ratio <= 1.30, (tab, kind, m, key, ratio)
    for kind in ("isotropic", "diagonal", "full"):
        e1 = {m: by[(1, kind, m)]["Er2"] for m in MODELS}
        assert e1["B2"] == e1["B3"]
        assert e1["B1"] < e1["B2"] < e1["A"]
        e2 = {m: by[(2, kind, m)]["Er2"] for m in MODELS}
        assert e2["B1"] < e2["B2"] < e2["A"] < e2["B3"]
        assert e2["B3"] >= 2.5 * max(e2["A"], e2["B1"], e2["B2"])
