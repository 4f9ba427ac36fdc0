"""Velocity given per node and changing in time (u = u(x, t) in Eq. 1).

* A per-node field equal to a separable flow gives the oracle's result
  (the field path of the kernels, FP64 1e-12, FP32 1e-5).
* A flow that changes every step (cellular cells drifting along x), set
  through lbm_cde_set_velocity before each step, against the oracle run with
  the same sequence of fields, periodic and with walls, single run and batch.
  The field set before the step that reaches step n relaxes the populations
  of step n; in the oracle's push form that field is used by the collision at
  the start of step n+1, which gives the same phi.
* A field set once applies to graph-replayed steps; runs made without a
  field reject the call.
"""
import numpy as np
import pytest

from oracle import lbm as O
from paper_1404_2363_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def oracle_unsteady(wl, steps, walls=None):
    prob = O.problem_for(wl)
    f = prob.equilibrium(wl.phi0())
    for n in range(steps):
        prob.u = np.asarray(wl.u_schedule(n), np.float64)
        f = prob.step(f)
    return O.phi_of(f)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_field_equals_separable_flow(precision):
    from paper_1404_2363_amd.solver import Solver
    sep = W.cellular(nx=67, ny=45, steps=80, n_hills=3, sigma=5.0, U0=0.08)
    fld = W.cellular(nx=67, ny=45, steps=80, n_hills=3, sigma=5.0, U0=0.08)
    fld.u_field, fld.u_sep = sep.u(), None
    print(f"case field vs separable 67x45 x 80 {precision}", flush=True)
    ref, _ = O.run_workload(sep, steps=80)
    s = Solver(fld, precision)
    s.step(80)
    assert rel(s.phi().cpu().numpy(), ref) <= TOL[precision]
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("walls", [("periodic", "periodic"), ("periodic", "bounce"), ("specular", "periodic")])
def test_time_dependent_velocity(precision, walls):
    from paper_1404_2363_amd.solver import Solver
    wl = W.drifting_cellular(nx=70, ny=45, steps=60, n_hills=4, sigma=5.0, U0=0.08, drift=0.7, walls=walls)
    print(f"case drifting cellular 70x45 x 60 {walls} {precision}", flush=True)
    ref = oracle_unsteady(wl, 60)
    s = Solver(wl, precision)
    for n in range(1, 61):
        s.set_velocity(wl.u_schedule(n))
        s.step(1)
    assert rel(s.phi().cpu().numpy(), ref) <= TOL[precision]
    # the flow really changed: with the step-0 field held fixed the answer differs
    frozen, _ = O.run_workload(wl, steps=60)
    assert rel(frozen, ref) > 1e3 * TOL[precision]
    s.close()


def test_time_dependent_velocity_in_a_batch():
    from paper_1404_2363_amd.solver import Solver
    a = W.drifting_cellular(nx=64, ny=40, steps=40, n_hills=3, sigma=5.0, drift=0.5)
    b = W.drifting_cellular(nx=50, ny=33, steps=40, n_hills=3, sigma=4.0, drift=-0.3, seed_id=7)
    s = Solver([a, b], "fp64")
    for n in range(1, 41):
        s.set_velocity(a.u_schedule(n), run=0)
        s.set_velocity(b.u_schedule(n), run=1)
        s.step(1)
    for i, wl in enumerate((a, b)):
        assert rel(s.phi(i).cpu().numpy(), oracle_unsteady(wl, 40)) <= 1e-12
    s.close()


def test_field_set_once_applies_to_graph_replay():
    from paper_1404_2363_amd.solver import Solver
    wl = W.drifting_cellular(nx=64, ny=48, steps=70, n_hills=3, sigma=5.0, drift=0.0)
    new = W.drifting_cellular_field(64, 48, 0.06, 9.0)
    s = Solver(wl, "fp64")
    s.set_velocity(new)
    s.step(70)                         # two graph replays of 32 steps + 6 single launches
    prob = O.problem_for(wl)
    f = prob.equilibrium(wl.phi0())
    f = prob.step(f)                   # step 1 relaxes f_0 with the field of step 0
    prob.u = new
    f, _ = prob.run(f, 69)
    assert rel(s.phi().cpu().numpy(), O.phi_of(f)) <= 1e-12
    s.close()


def test_set_velocity_needs_a_field_run():
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    s = Solver(W.cellular(nx=32, ny=24, steps=1, n_hills=1, sigma=3.0), "fp64")
    with pytest.raises(L.LbmCdeError) as e:
        s.set_velocity(np.zeros((2, 24, 32)))
    assert e.value.code == L.LBM_CDE_EINVAL
    s.close()


def test_field_speed_limit():
    """A field with |u| >= c_s is rejected at init; one set later marks the
    run, and the next reduction reports EUNSTABLE."""
    from paper_1404_2363_amd import _lib as L
    from paper_1404_2363_amd.solver import Solver
    wl = W.drifting_cellular(nx=40, ny=30, steps=4, n_hills=2, sigma=4.0, drift=0.0)
    fast = np.array(wl.u_field, copy=True)
    fast[0, 7, 11] = 0.6                               # above 1/sqrt(3) at one node
    bad = W.drifting_cellular(nx=40, ny=30, steps=4, n_hills=2, sigma=4.0, drift=0.0)
    bad.u_field = fast
    with pytest.raises(L.LbmCdeError) as e:
        Solver(bad, "fp64")
    assert e.value.code == L.LBM_CDE_EUNSTABLE
    for precision in ("fp64", "fp32"):
        s = Solver(wl, precision)
        s.step(2)
        assert s.nonfinite() == 0                     # the run's own field is fine
        s.set_velocity(fast)
        s.step(1)
        with pytest.raises(L.LbmCdeError) as e:
            s.mass()
        assert e.value.code == L.LBM_CDE_EUNSTABLE
        s.close()
