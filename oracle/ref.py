"""ctypes front of the C reference (lbm_ref.c) for long periodic runs.

TEST INFRASTRUCTURE ONLY (see oracle/lbm.py).  The collision enters in its
matrix form f' = Cm f + phi (b_0 + sum_c u_c b_c), built here from the Python
oracle's own M, M^-1, S and MRT-A equilibrium (Eq. 11-14, 31, 37; A.2-A.5),
and the C code adds only the sums over nodes and the periodic push streaming
(Eq. 5).  Pinned against the Python oracle step by step in
tests/test_oracle_ref.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import lbm as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_ref.c")
LIB = os.path.join(HERE, "liblbm_ref.so")


def build(force: bool = False) -> str:
    """Compile liblbm_ref.so with gcc (OpenMP) when missing or older than its source."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC], check=True)
        os.replace(tmp, LIB)
    return LIB


def _lib():
    lib = ctypes.CDLL(build())
    lib.lbm_ref_run.restype = ctypes.c_int
    p = ctypes.c_void_p
    lib.lbm_ref_run.argtypes = [ctypes.c_int, ctypes.c_int, p, p, p, p, p, p, p, ctypes.c_int64, ctypes.c_int]
    return lib


def collision_form(prob: O.Problem):
    """(Cm, b) with f' = Cm f + phi (b[0] + sum_c u_c b[1 + c]) for a problem
    with a constant relaxation matrix and the (linear) MRT-A equilibrium."""
    if prob.model != "A" or np.asarray(prob.S).ndim != 2:
        raise ValueError("the C reference covers MRT-A with a constant relaxation matrix")
    lat = prob.lat
    dim = lat.dim
    Minv_S = lat.Minv @ prob.S
    Cm = np.eye(lat.Q) - Minv_S @ lat.M
    one = np.ones(1)
    zero_u = np.zeros((dim, 1))
    eq0 = O.equilibrium_moments(lat, "A", one, zero_u)[:, 0]
    b = [Minv_S @ eq0]
    for c in range(dim):
        uc = np.zeros((dim, 1))
        uc[c] = 1.0
        eqc = O.equilibrium_moments(lat, "A", one, uc)[:, 0] - eq0
        b.append(Minv_S @ eqc)
    return np.ascontiguousarray(Cm), np.ascontiguousarray(np.stack(b))


class Run:
    """Populations of a periodic problem held for the C reference; advance()
    steps them in place, .f holds them (Q, *grid)."""

    def __init__(self, prob: O.Problem, f: np.ndarray):
        if any(w != "periodic" for w in prob.walls):
            raise ValueError("the C reference is periodic on every axis")
        lat = prob.lat
        self.Q, self.dim = lat.Q, lat.dim
        self.Cm, self.b = collision_form(prob)
        grid = f.shape[1:]
        self.shape = np.array(list(reversed(grid)) + [1] * (3 - len(grid)), dtype=np.int64)
        self.e = np.ascontiguousarray(lat.e[:, :3].astype(np.int32))
        self.u = np.ascontiguousarray(np.broadcast_to(prob.u, (lat.dim,) + grid), dtype=np.float64)
        self.f = np.ascontiguousarray(f, dtype=np.float64).copy()
        self.g = np.zeros_like(self.f)
        self.lib = _lib()

    def advance(self, steps: int, threads: int = 0):
        """`steps` steps on `threads` OpenMP threads (0: the OpenMP default)."""
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        n = threads if threads > 0 else (os.cpu_count() or 1)
        if "OMP_NUM_THREADS" in os.environ and threads <= 0:
            n = int(os.environ["OMP_NUM_THREADS"])
        rc = self.lib.lbm_ref_run(self.Q, self.dim, ptr(self.shape), ptr(self.e), ptr(self.Cm), ptr(self.b),
                                  ptr(self.u), ptr(self.f), ptr(self.g), steps, n)
        if rc != 0:
            raise ValueError("lbm_ref_run rejected its arguments")


def run(prob: O.Problem, f: np.ndarray, steps: int, threads: int = 0) -> np.ndarray:
    """Advance populations f (shape (Q, *grid), FP64) by `steps` periodic steps."""
    r = Run(prob, f)
    r.advance(steps, threads)
    return r.f
