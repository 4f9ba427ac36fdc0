"""ctypes binding of ``liblbm_cde.so`` (argument marshalling only).

Every function here forwards to the C entry point of the same name in
``include/lbm_cde.h``; all computation happens in the HIP library.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_cde.so")

# status codes
LBM_CDE_OK = 0
LBM_CDE_EINVAL = -1
LBM_CDE_ENOTSPD = -2
LBM_CDE_EUNSTABLE = -3
LBM_CDE_EHIP = -4
LBM_CDE_ENONFINITE = -5
LBM_CDE_ENOSPC = -6
LBM_CDE_EUNSUPPORTED = -7
LBM_CDE_EOVERFLOW = -8
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOTSPD", -3: "EUNSTABLE", -4: "EHIP", -5: "ENONFINITE",
                -6: "ENOSPC", -7: "EUNSUPPORTED", -8: "EOVERFLOW"}

LBM_CDE_D2Q9, LBM_CDE_D3Q15 = 0, 1
LBM_CDE_FP64, LBM_CDE_FP32_SHIFTED, LBM_CDE_FP16_SPLIT, LBM_CDE_FP16_SHIFTED = 0, 1, 2, 3
LBM_CDE_PERIODIC, LBM_CDE_BOUNCE_BACK, LBM_CDE_SPECULAR, LBM_CDE_NODE_MIRROR = 0, 1, 2, 3
LBM_CDE_MRT_A, LBM_CDE_MRT_B1, LBM_CDE_MRT_B2, LBM_CDE_MRT_B3 = 0, 1, 2, 3
LBM_CDE_U_CONST, LBM_CDE_U_SEPARABLE, LBM_CDE_U_FIELD = 0, 1, 2
LBM_CDE_HEAT_LAMBDA_MIN, LBM_CDE_HEAT_PAPER, LBM_CDE_HEAT_EXPLICIT = 0, 1, 2
LBM_CDE_RED_MASS, LBM_CDE_RED_XMOMENTS, LBM_CDE_RED_NONFINITE = 0, 1, 2


class lbm_cde_run_desc(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("bc", ctypes.c_int32 * 3),
        ("D", ctypes.c_double * 6),
        ("D_field", ctypes.c_void_p),
        ("u_kind", ctypes.c_int32),
        ("u_const", ctypes.c_double * 3),
        ("u_tables", ctypes.c_void_p),
        ("u_field", ctypes.c_void_p),
        ("heat_rule", ctypes.c_int32),
        ("heat_rates", ctypes.c_double * 3),
        ("rates", ctypes.c_double * 15),
        ("phi_ref", ctypes.c_double),
        ("fp16_scale", ctypes.c_double),
        ("xref0", ctypes.c_double),
        ("xref_drift", ctypes.c_double),
        ("max_steps", ctypes.c_int64),
        ("model", ctypes.c_int32),
        ("skip_stability_check", ctypes.c_int32),
    ]


class LbmCdeError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (built in-tree by build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1404_2363_amd/build.py "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "lbm_cde_workspace_bytes": [ctypes.POINTER(lbm_cde_run_desc), I32, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_cde_spectral_radius": [ctypes.POINTER(lbm_cde_run_desc), ctypes.POINTER(D)],
        "lbm_cde_init": [ctypes.POINTER(lbm_cde_run_desc), I32, ctypes.POINTER(ctypes.c_void_p), P,
                         ctypes.c_size_t, P, ctypes.POINTER(ctypes.c_void_p)],
        "lbm_cde_step": [P, I64],
        "lbm_cde_steps_done": [P, I32, ctypes.POINTER(I64)],
        "lbm_cde_moments": [P, I32, P],
        "lbm_cde_reduce": [P, I32, I32, D, ctypes.POINTER(D)],
        "lbm_cde_reduce_noalloc": [P, I32, I32, D, P],
        "lbm_cde_run_sampled": [P, I64, I64, P, I64],
        "lbm_cde_samples_written": [P, ctypes.POINTER(I64)],
        "lbm_cde_relaxation_matrix": [P, I32, ctypes.POINTER(D)],
        "lbm_cde_set_velocity": [P, I32, P],
        "lbm_cde_tune": [P, I32],
        "lbm_cde_get_variant": [P, I32, ctypes.POINTER(I32)],
        "lbm_cde_variant_count": [P, I32, ctypes.POINTER(I32)],
        "lbm_cde_variant_at": [P, I32, I32, ctypes.POINTER(I32)],
        "lbm_cde_set_variant": [P, I32, ctypes.POINTER(I32)],
        "lbm_cde_state_bytes": [P, I32, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_cde_get_state": [P, I32, P],
        "lbm_cde_set_state": [P, I32, P, I64],
        "lbm_cde_adjoint_scratch_bytes": [P, I32, I32, ctypes.POINTER(ctypes.c_size_t)],
        "lbm_cde_adjoint_segment": [P, I32, P, I32, P, ctypes.POINTER(ctypes.c_void_p), P, P, P],
        "lbm_cde_adjoint_phi0": [P, I32, P, P, P],
        "lbm_cde_destroy": [P],
        "lbm_cde_last_error": [P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "lbm_cde_last_error" else ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, where: str, handle=None) -> int:
    if rc != LBM_CDE_OK:
        msg = load().lbm_cde_last_error(handle)
        raise LbmCdeError(rc, where, msg.decode() if msg else "")
    return rc


# ---- same-name wrappers ----------------------------------------------------

def lbm_cde_workspace_bytes(descs) -> int:
    arr = (lbm_cde_run_desc * len(descs))(*descs)
    out = ctypes.c_size_t(0)
    _check(load().lbm_cde_workspace_bytes(arr, len(descs), ctypes.byref(out)), "lbm_cde_workspace_bytes")
    return int(out.value)


def lbm_cde_spectral_radius(desc) -> float:
    out = ctypes.c_double(0.0)
    _check(load().lbm_cde_spectral_radius(ctypes.byref(desc), ctypes.byref(out)), "lbm_cde_spectral_radius")
    return float(out.value)


def lbm_cde_init(descs, phi0_ptrs, workspace_ptr: int, ws_bytes: int, stream: int) -> int:
    arr = (lbm_cde_run_desc * len(descs))(*descs)
    ptrs = (ctypes.c_void_p * len(phi0_ptrs))(*phi0_ptrs)
    h = ctypes.c_void_p(None)
    _check(load().lbm_cde_init(arr, len(descs), ptrs, ctypes.c_void_p(workspace_ptr), ws_bytes,
                               ctypes.c_void_p(stream), ctypes.byref(h)), "lbm_cde_init")
    return h.value


def lbm_cde_step(h: int, n: int) -> None:
    _check(load().lbm_cde_step(h, n), "lbm_cde_step", h)


def lbm_cde_steps_done(h: int, run: int) -> int:
    out = ctypes.c_int64(0)
    _check(load().lbm_cde_steps_done(h, run, ctypes.byref(out)), "lbm_cde_steps_done", h)
    return int(out.value)


def lbm_cde_moments(h: int, run: int, phi_ptr: int) -> None:
    _check(load().lbm_cde_moments(h, run, ctypes.c_void_p(phi_ptr)), "lbm_cde_moments", h)


def lbm_cde_reduce(h: int, run: int, kind: int, x_ref: float = 0.0, allow_nonfinite: bool = False):
    out = (ctypes.c_double * 3)()
    rc = load().lbm_cde_reduce(h, run, kind, float(x_ref), out)
    if not (allow_nonfinite and rc == LBM_CDE_ENONFINITE):
        _check(rc, "lbm_cde_reduce", h)
    return [out[0], out[1], out[2]], rc


def lbm_cde_reduce_noalloc(h: int, run: int, kind: int, x_ref: float, out_ptr: int) -> None:
    _check(load().lbm_cde_reduce_noalloc(h, run, kind, float(x_ref), ctypes.c_void_p(out_ptr)),
           "lbm_cde_reduce_noalloc", h)


def lbm_cde_run_sampled(h: int, n: int, every: int, hist_ptr: int, capacity: int) -> None:
    _check(load().lbm_cde_run_sampled(h, n, every, ctypes.c_void_p(hist_ptr), capacity), "lbm_cde_run_sampled", h)


def lbm_cde_samples_written(h: int) -> int:
    out = ctypes.c_int64(0)
    _check(load().lbm_cde_samples_written(h, ctypes.byref(out)), "lbm_cde_samples_written", h)
    return int(out.value)


def lbm_cde_relaxation_matrix(h: int, run: int, Q: int):
    out = (ctypes.c_double * (Q * Q))()
    _check(load().lbm_cde_relaxation_matrix(h, run, out), "lbm_cde_relaxation_matrix", h)
    return [out[i] for i in range(Q * Q)]


def lbm_cde_set_velocity(h: int, run: int, u_ptr: int) -> None:
    _check(load().lbm_cde_set_velocity(h, run, u_ptr), "lbm_cde_set_velocity", h)


def lbm_cde_tune(h: int, trials: int) -> None:
    _check(load().lbm_cde_tune(h, trials), "lbm_cde_tune", h)


VARIANT_INTS = 7                # integers of a launch variant (see include/lbm_cde.h)


def _variant_dict(out) -> dict:
    return {"block": (out[0], out[1]), "rows_per_thread": out[2], "nt_stores": bool(out[3]),
            "block_order": int(out[4]), "grid": int(out[5]), "steps_per_launch": int(out[6])}


def variant_tuple(v: dict) -> tuple:
    """The seven integers of a variant dict (as returned by lbm_cde_get_variant)."""
    return (v["block"][0], v["block"][1], v["rows_per_thread"], int(v["nt_stores"]), v["block_order"], v["grid"],
            v.get("steps_per_launch", 1))


def lbm_cde_get_variant(h: int, run: int):
    out = (ctypes.c_int32 * VARIANT_INTS)()
    _check(load().lbm_cde_get_variant(h, run, out), "lbm_cde_get_variant", h)
    return _variant_dict(out)


def lbm_cde_variant_count(h: int, run: int) -> int:
    out = ctypes.c_int32(0)
    _check(load().lbm_cde_variant_count(h, run, ctypes.byref(out)), "lbm_cde_variant_count", h)
    return int(out.value)


def lbm_cde_variant_at(h: int, run: int, index: int):
    out = (ctypes.c_int32 * VARIANT_INTS)()
    _check(load().lbm_cde_variant_at(h, run, index, out), "lbm_cde_variant_at", h)
    return _variant_dict(out)


def lbm_cde_set_variant(h: int, run: int, v: dict) -> None:
    arr = (ctypes.c_int32 * VARIANT_INTS)(*variant_tuple(v))
    _check(load().lbm_cde_set_variant(h, run, arr), "lbm_cde_set_variant", h)


def lbm_cde_state_bytes(h: int, run: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().lbm_cde_state_bytes(h, run, ctypes.byref(out)), "lbm_cde_state_bytes", h)
    return int(out.value)


def lbm_cde_get_state(h: int, run: int, dst_ptr: int) -> None:
    _check(load().lbm_cde_get_state(h, run, ctypes.c_void_p(dst_ptr)), "lbm_cde_get_state", h)


def lbm_cde_set_state(h: int, run: int, src_ptr: int, steps: int) -> None:
    _check(load().lbm_cde_set_state(h, run, ctypes.c_void_p(src_ptr), steps), "lbm_cde_set_state", h)


def lbm_cde_adjoint_scratch_bytes(h: int, run: int, nsteps: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().lbm_cde_adjoint_scratch_bytes(h, run, nsteps, ctypes.byref(out)), "lbm_cde_adjoint_scratch_bytes", h)
    return int(out.value)


def lbm_cde_adjoint_segment(h: int, run: int, ckpt_ptr: int, nsteps: int, seg_ptr: int, inj_ptrs,
                            mu_ptr: int, mu_tmp_ptr: int, grad_ptr: int) -> None:
    inj = None
    if inj_ptrs is not None:
        inj = (ctypes.c_void_p * len(inj_ptrs))(*[p if p else None for p in inj_ptrs])
    _check(load().lbm_cde_adjoint_segment(h, run, ctypes.c_void_p(ckpt_ptr), nsteps, ctypes.c_void_p(seg_ptr), inj,
                                          ctypes.c_void_p(mu_ptr), ctypes.c_void_p(mu_tmp_ptr),
                                          ctypes.c_void_p(grad_ptr)), "lbm_cde_adjoint_segment", h)


def lbm_cde_adjoint_phi0(h: int, run: int, mu0_ptr: int, inj0_ptr, dphi0_ptr: int) -> None:
    _check(load().lbm_cde_adjoint_phi0(h, run, ctypes.c_void_p(mu0_ptr), ctypes.c_void_p(inj0_ptr),
                                       ctypes.c_void_p(dphi0_ptr)), "lbm_cde_adjoint_phi0", h)


def lbm_cde_destroy(h: int) -> None:
    _check(load().lbm_cde_destroy(h), "lbm_cde_destroy")


def lbm_cde_last_error(h=None) -> str:
    msg = load().lbm_cde_last_error(h)
    return msg.decode() if msg else ""
