"""The precision forms over the full length of the large workloads.

Against the FP64 reference: the C reference (oracle/lbm_ref.c, pinned to the
Python oracle) ran both workloads to their full length on the host and
stored phi at 4096 seeded nodes (golden/full_length.json, written by
golden/make_full_length.py).  Each precision, in the tuned launch variant,
must match those values within its tolerance (1e-12, 1e-5, 1e-3 of max |phi|)
and the reference's sum phi.

Over the whole field, the reduced-precision steps are also compared with the
FP64 GPU step:

* D2Q9 4096^2 cellular flow, 5000 steps: FP32 shifted within 1e-5 and FP16
  split within 1e-3 of max |phi| (the stated tolerances); the literal FP16
  form is measured and must be worse; sum phi conserved to 1e-13 (FP64),
  1e-6 (FP32 and FP16 split; measured 3.8e-8 and 8.2e-7).
* D3Q15 256^3 sine flow, 2000 steps: FP32 shifted within 1e-5; sum phi
  conserved.
"""
import json
import os

import numpy as np
import pytest

from paper_1404_2363_amd import workloads as W

pytestmark = pytest.mark.gpu


def run(wl, precision, steps):
    from paper_1404_2363_amd.solver import Solver
    s = Solver(wl, precision)
    m0 = s.mass()
    s.step(steps)
    phi = s.phi().cpu().numpy()
    m1 = s.mass()
    assert s.nonfinite() == 0
    s.close()
    return phi, m0, m1


def test_d2q9_4096_full_length_precision_forms():
    wl = W.cellular()
    steps = wl.steps
    print(f"case cellular 4096^2 x {steps}: fp64, fp32, fp16 split, fp16 literal", flush=True)
    ref, m0, m1 = run(wl, "fp64", steps)
    assert abs(m1 - m0) <= 1e-13 * m0
    scale = np.abs(ref).max()
    out = {}
    for prec, tol, mtol in (("fp32", 1e-5, 1e-6), ("fp16", 1e-3, 1e-6)):
        phi, a, b = run(wl, prec, steps)
        err = float(np.abs(phi - ref).max() / scale)
        out[prec] = err
        print(f"{prec}: max |dphi| / max |phi| = {err:.3e}, mass drift {abs(b - a) / a:.2e}", flush=True)
        assert err <= tol, (prec, err)
        assert abs(b - a) <= mtol * a
    lit, _, _ = run(wl, "fp16_literal", steps)
    e_lit = float(np.abs(lit - ref).max() / scale)
    print(f"fp16 literal: {e_lit:.3e}", flush=True)
    assert e_lit > out["fp16"]


def test_d3q15_256_full_length_fp32():
    wl = W.sine3d()
    steps = wl.steps
    print(f"case sine3d 256^3 x {steps}: fp64, fp32", flush=True)
    ref, m0, m1 = run(wl, "fp64", steps)
    assert abs(m1 - m0) <= 1e-13 * m0
    phi, a, b = run(wl, "fp32", steps)
    err = float(np.abs(phi - ref).max() / np.abs(ref).max())
    print(f"fp32: max |dphi| / max |phi| = {err:.3e}, mass drift {abs(b - a) / a:.2e}", flush=True)
    assert err <= 1e-5
    assert abs(b - a) <= 1e-6 * a


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "full_length.json")


@pytest.mark.parametrize("case,precision,tol", [
    ("d2q9", "fp64", 1e-12), ("d2q9", "fp32", 1e-5), ("d2q9", "fp16", 1e-3),
    ("d3q15", "fp64", 1e-12), ("d3q15", "fp32", 1e-5)])
def test_full_length_against_fp64_reference(case, precision, tol):
    from paper_1404_2363_amd.solver import Solver
    gold = json.load(open(GOLDEN))[case]
    wl = W.cellular() if case == "d2q9" else W.sine3d()
    assert list(wl.shape) == gold["shape"] and wl.steps == gold["steps"]
    s = Solver(wl, precision)
    s.tune()
    print(f"case {case} {wl.shape} x {wl.steps} {precision}, tuned variant {s.variant()}", flush=True)
    s.step(wl.steps)
    phi = s.phi().cpu().numpy().ravel()
    mass = s.mass()
    assert s.nonfinite() == 0
    s.close()
    nodes = np.asarray(gold["nodes"])
    err = float(np.abs(phi[nodes] - np.asarray(gold["phi"])).max() / gold["max_abs_phi"])
    dm = abs(mass - gold["sum_phi"]) / gold["sum_phi0"]
    print(f"max |dphi| / max |phi| at {nodes.size} nodes = {err:.3e}; sum phi vs reference {dm:.2e}", flush=True)
    assert err <= tol
    assert dm <= {"fp64": 1e-12, "fp32": 1e-6, "fp16": 1e-6}[precision]
