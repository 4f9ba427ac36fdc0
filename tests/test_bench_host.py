"""Host logic of bench.py (no GPU): the roofline's two bounds and the keys
under which committed counter profiles are looked up."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

LAUNCH = {"block": (64, 12), "rows_per_thread": 2, "nt_stores": True, "block_order": 1, "grid": 0,
          "steps_per_launch": 4}


def _variant(ms_per_launch, T=4, nodes=4096 * 4096):
    bytes_per_launch = 72 * nodes
    gbs = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    return {"nodes": nodes, "steps_per_launch": T, "ms_per_launch": ms_per_launch, "launch": dict(LAUNCH),
            "bytes_per_launch": bytes_per_launch, "achieved_gbs": gbs, "hbm_frac": gbs / bench.HBM_PEAK_GBS,
            "traffic": None}


def test_valu_peak_is_the_issue_rate_without_packed_math():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert bench.VALU_PEAK_TINSTR == pytest.approx(39.3216)


def test_algorithmic_alu_bound(monkeypatch):
    """A multi-step launch: the algorithmic lane operations (93 per update,
    each node updated T times) over the launch time; the bound is the VALU
    one when it is nearer its peak than HBM, with HBM nested."""
    monkeypatch.setattr(bench, "profiled_valu", lambda name, launch: None)
    v = _variant(0.2823)
    r = bench.roofline(v, "d2q9_4096_fp32", "float")
    ops = 93 * 4096 * 4096 * 4
    assert r["algorithmic_lane_ops_per_launch"] == ops
    assert r["achieved"] == pytest.approx(ops / 0.2823e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.VALU_PEAK_TINSTR)
    assert r["bound"] == "alu" and r["hbm"]["bound"] == "hbm"
    assert r["hbm"]["frac"] == pytest.approx(v["hbm_frac"])
    assert "issued" not in r
    assert r["kernel"] == "k_fused_d2q9<float, 64, 12, 2, 4>"


def test_issued_rate_from_the_profile(monkeypatch):
    """With a committed instruction count the issued-instruction rate sits
    beside the algorithmic one and never replaces it."""
    monkeypatch.setattr(bench, "profiled_valu", lambda name, launch: 1.45e8)
    r = bench.roofline(_variant(0.2823), "d2q9_4096_fp32", "float")
    assert r["issued"]["achieved"] == pytest.approx(1.45e8 * 64 / 0.2823e-3 / 1e12)
    assert r["issued"]["frac"] > r["frac"]


def test_one_step_launch_is_hbm_bound(monkeypatch):
    """One step per launch at 74 % of the HBM peak: the algorithmic VALU
    fraction (93 operations per 72 bytes) is far lower, so the bound is HBM
    with the VALU one nested."""
    monkeypatch.setattr(bench, "profiled_valu", lambda name, launch: None)
    v = _variant(0.2032, T=1)
    v["launch"] = {**LAUNCH, "block": (512, 1), "rows_per_thread": 1, "steps_per_launch": 1}
    r = bench.roofline(v, "d2q9_4096_fp32", "float")
    assert r["bound"] == "hbm" and r["alu"]["bound"] == "alu"
    assert r["frac"] == pytest.approx(0.743, abs=1e-3)
    assert r["alu"]["frac"] < r["frac"]
    assert r["kernel"] == "k_step_d2q9<float>"


def test_profile_keys():
    assert bench.kernel_tag(LAUNCH) == "64x12x2x1|order1|steps4"
    one = {**LAUNCH, "block": (128, 1), "rows_per_thread": 1, "steps_per_launch": 1, "grid": 139776,
           "block_order": 0}
    assert bench.kernel_tag(one) == "128x1x1x1|order0|grid139776"


def test_stale_profile_is_not_used(tmp_path):
    """A counter record is used only while the hash of the kernel sources it
    names matches the one it was taken on."""
    import hashlib
    import json
    files = ["common.hpp", "d2q9.hpp"]
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1404_2363_amd", "csrc", f), "rb").read())
    good = {"w": {"source_files": files, "source_sha": h.hexdigest()[:16], "kernels": {}}}
    stale = {"w": {"source_files": files, "source_sha": "0" * 16, "kernels": {}}}
    (tmp_path / "good.json").write_text(json.dumps(good))
    (tmp_path / "stale.json").write_text(json.dumps(stale))
    assert bench._profile("w", str(tmp_path / "good.json")) == good["w"]
    assert bench._profile("w", str(tmp_path / "stale.json")) is None
    assert bench._profile("missing", str(tmp_path / "good.json")) is None
