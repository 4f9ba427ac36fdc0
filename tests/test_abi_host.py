"""Host-side checks of the C ABI (no GPU needed).

* The shared library loads and exports every function that
  include/lbm_cde.h declares.
* Descriptor validation (pure host logic) rejects invalid runs with the
  documented status codes; workspace sizes follow the documented layout.
"""
import os
import re

import pytest

from paper_1404_2363_amd import _lib as L
from paper_1404_2363_amd import workloads as W
from paper_1404_2363_amd.solver import make_desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "lbm_cde.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(lbm_cde_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_function():
    lib = L.load()
    names = header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def _desc(**over):
    wl = W.cellular(nx=64, ny=48, steps=1, n_hills=2, sigma=4.0)
    d, keep = make_desc(wl, "fp64", device="cpu")
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


def test_workspace_bytes_layout():
    d, keep = _desc()
    nbytes = L.lbm_cde_workspace_bytes([d])
    plane = 64 * 48 * 8
    assert nbytes >= 2 * 9 * plane
    assert nbytes % 256 == 0
    d32, keep32 = make_desc(W.cellular(nx=64, ny=48, steps=1, n_hills=2, sigma=4.0), "fp32", device="cpu")
    assert L.lbm_cde_workspace_bytes([d32]) < nbytes
    assert L.lbm_cde_workspace_bytes([d, d32]) == nbytes + L.lbm_cde_workspace_bytes([d32])


@pytest.mark.parametrize("field,value", [("nx", 0), ("ny", -3), ("nz", 2), ("lattice", 7), ("precision", 9),
                                         ("u_kind", 5), ("heat_rule", 4), ("model", 4), ("model", -1)])
def test_invalid_descriptors_rejected(field, value):
    d, keep = _desc(**{field: value})
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_workspace_bytes([d])
    assert e.value.code == L.LBM_CDE_EINVAL
    assert L.lbm_cde_last_error(None)


def test_bad_boundary_and_missing_tables():
    d, keep = _desc()
    d.bc[1] = 4
    with pytest.raises(L.LbmCdeError):
        L.lbm_cde_workspace_bytes([d])
    d, keep = _desc()
    d.u_tables = None
    with pytest.raises(L.LbmCdeError):
        L.lbm_cde_workspace_bytes([d])


def test_null_arguments():
    lib = L.load()
    assert lib.lbm_cde_workspace_bytes(None, 1, None) == L.LBM_CDE_EINVAL
    assert lib.lbm_cde_step(None, 1) == L.LBM_CDE_EINVAL
    assert lib.lbm_cde_destroy(None) == L.LBM_CDE_EINVAL


def _plate_desc(**over):
    d, keep = _desc(**over)
    d.bc[0], d.bc[1] = L.LBM_CDE_PERIODIC, L.LBM_CDE_NODE_MIRROR
    return d, keep


def test_plate_rule_and_models_accepted():
    for model in (L.LBM_CDE_MRT_A, L.LBM_CDE_MRT_B1, L.LBM_CDE_MRT_B2, L.LBM_CDE_MRT_B3):
        for prec in (L.LBM_CDE_FP64, L.LBM_CDE_FP32_SHIFTED):
            d, keep = _plate_desc(model=model, precision=prec)
            assert L.lbm_cde_workspace_bytes([d]) > 0
    d, keep = _plate_desc()
    d.bc[0], d.bc[1] = L.LBM_CDE_NODE_MIRROR, L.LBM_CDE_PERIODIC
    assert L.lbm_cde_workspace_bytes([d]) > 0


@pytest.mark.parametrize("case", ["both_axes", "other_wall", "fp16", "fp16_literal", "d3q15", "thin"])
def test_plate_rule_limits(case):
    """The plate rule is built for D2Q9 in FP64/FP32 storage, on one axis with
    the other periodic and at least 2 nodes across."""
    d, keep = _plate_desc()
    code = L.LBM_CDE_EUNSUPPORTED
    if case == "both_axes":
        d.bc[0] = L.LBM_CDE_NODE_MIRROR
    elif case == "other_wall":
        d.bc[0] = L.LBM_CDE_SPECULAR
    elif case == "fp16":
        d.precision = L.LBM_CDE_FP16_SPLIT
    elif case == "fp16_literal":
        d.precision = L.LBM_CDE_FP16_SHIFTED
    elif case == "d3q15":
        d.lattice, d.nz = L.LBM_CDE_D3Q15, 4
        d.bc[2] = L.LBM_CDE_PERIODIC
    elif case == "thin":
        d.ny = 1
        code = L.LBM_CDE_EINVAL
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_workspace_bytes([d])
    assert e.value.code == code, L.lbm_cde_last_error(None)


@pytest.mark.parametrize("precision", [L.LBM_CDE_FP16_SPLIT, L.LBM_CDE_FP16_SHIFTED])
def test_unmodified_models_need_wide_storage(precision):
    d, keep = _desc(model=L.LBM_CDE_MRT_B1, precision=precision)
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_workspace_bytes([d])
    assert e.value.code == L.LBM_CDE_EUNSUPPORTED


def test_unmodified_models_are_d2q9_only():
    d, keep = _desc(model=L.LBM_CDE_MRT_B3, lattice=L.LBM_CDE_D3Q15, nz=4)
    with pytest.raises(L.LbmCdeError) as e:
        L.lbm_cde_workspace_bytes([d])
    assert e.value.code == L.LBM_CDE_EUNSUPPORTED
