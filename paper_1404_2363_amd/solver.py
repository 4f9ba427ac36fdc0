"""Python front end of the HIP library: descriptors from workloads, torch-owned memory.

PyTorch provides device memory (the workspace, phi0, fields, outputs) and the
stream; every step, readout and reduction runs in ``liblbm_cde.so``.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L

PRECISIONS = {"fp64": L.LBM_CDE_FP64, "fp32": L.LBM_CDE_FP32_SHIFTED, "fp16": L.LBM_CDE_FP16_SPLIT,
              "fp16_literal": L.LBM_CDE_FP16_SHIFTED}
WALLS = {"periodic": L.LBM_CDE_PERIODIC, "bounce": L.LBM_CDE_BOUNCE_BACK, "specular": L.LBM_CDE_SPECULAR,
         "node": L.LBM_CDE_NODE_MIRROR, False: L.LBM_CDE_PERIODIC, True: L.LBM_CDE_BOUNCE_BACK}
MODELS = {"A": L.LBM_CDE_MRT_A, "B1": L.LBM_CDE_MRT_B1, "B2": L.LBM_CDE_MRT_B2, "B3": L.LBM_CDE_MRT_B3}
LATTICES = {"d2q9": L.LBM_CDE_D2Q9, "d3q15": L.LBM_CDE_D3Q15}
Q_OF = {"d2q9": 9, "d3q15": 15}


def _heat(desc, heat):
    if isinstance(heat, str):
        desc.heat_rule = {"lambda_min": L.LBM_CDE_HEAT_LAMBDA_MIN, "paper": L.LBM_CDE_HEAT_PAPER}[heat]
    else:
        desc.heat_rule = L.LBM_CDE_HEAT_EXPLICIT
        vals = list(heat) + [0.0] * (3 - len(heat))
        for i in range(3):
            desc.heat_rates[i] = float(vals[i])


def make_desc(wl, precision: str = "fp64", device="cuda:0", heat="lambda_min", rates=None,
              phi_ref: Optional[float] = None, max_steps: int = -1, xref0: float = 0.0,
              xref_drift: float = 0.0, fp16_scale: float = 0.0, model: str = "A",
              stability_check: bool = True):
    """Descriptor of one workload, plus the objects that must outlive init.

    ``model`` is "A" (the modified model) or "B1" | "B2" | "B3" (unmodified).
    ``stability_check=False`` accepts a constant-u, constant-D run whose
    linearised step is unstable (the library rejects it otherwise)."""
    keep = []
    d = L.lbm_cde_run_desc()
    d.lattice = LATTICES[wl.lattice]
    d.precision = PRECISIONS[precision]
    shape = tuple(wl.shape) + (1,) * (3 - len(wl.shape))
    d.nx, d.ny, d.nz = (int(s) for s in shape)
    for a, w in enumerate(wl.walls):
        d.bc[a] = WALLS[w]
    if wl.D_field is not None:
        if isinstance(wl.D_field, torch.Tensor):
            Df = wl.D_field.detach().to(device=device, dtype=torch.float64).contiguous()
        else:
            Df = torch.as_tensor(np.ascontiguousarray(wl.D_field), dtype=torch.float64, device=device)
        keep.append(Df)
        d.D_field = Df.data_ptr()
    else:
        Dm = np.asarray(wl.D, np.float64)
        comps = [Dm[0, 0], Dm[1, 1], 0.0, Dm[0, 1], 0.0, 0.0] if Dm.shape == (2, 2) else \
            [Dm[0, 0], Dm[1, 1], Dm[2, 2], Dm[0, 1], Dm[0, 2], Dm[1, 2]]
        for i, v in enumerate(comps):
            d.D[i] = float(v)
    if wl.u_field is not None:
        d.u_kind = L.LBM_CDE_U_FIELD
        Uf = torch.as_tensor(np.ascontiguousarray(wl.u_field), dtype=torch.float64, device=device)
        keep.append(Uf)
        d.u_field = Uf.data_ptr()
    elif wl.u_sep is not None:
        d.u_kind = L.LBM_CDE_U_SEPARABLE
        tab = wl.u_sep.as_flat_tables(wl.shape)
        keep.append(tab)
        d.u_tables = tab.ctypes.data
    else:
        d.u_kind = L.LBM_CDE_U_CONST
        u = np.zeros(3) if wl.u_const is None else np.asarray(wl.u_const, np.float64)
        for i in range(len(u)):
            d.u_const[i] = float(u[i])
    _heat(d, heat)
    if rates is not None:
        for k, v in rates.items():
            d.rates[int(k)] = float(v)
    d.phi_ref = float(wl.phi_ref() if phi_ref is None else phi_ref) if precision != "fp64" else 0.0
    d.fp16_scale = float(fp16_scale)
    d.xref0, d.xref_drift = float(xref0), float(xref_drift)
    d.max_steps = int(max_steps)
    d.model = MODELS[model]
    d.skip_stability_check = 0 if stability_check else 1
    return d, keep


class Solver:
    """One or more runs advanced together by the HIP library.

    ``runs`` is a workload or a list of workloads; keyword arguments are
    passed to :func:`make_desc` (a list per run is accepted via ``per_run``).
    """

    def __init__(self, runs, precision: str = "fp64", device="cuda:0", per_run: Optional[Sequence[dict]] = None,
                 phi0: Optional[Sequence[torch.Tensor]] = None, **kw):
        L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU (torch.cuda.is_available() is False)")
        self.runs = list(runs) if isinstance(runs, (list, tuple)) else [runs]
        self.device = torch.device(device)
        self.precision = precision
        descs, keep, phis = [], [], []
        for i, wl in enumerate(self.runs):
            opts = dict(kw)
            if per_run is not None:
                opts.update(per_run[i])
            d, k = make_desc(wl, opts.pop("precision", precision), device=self.device, **opts)
            descs.append(d)
            keep += k
            if phi0 is not None:
                p = phi0[i].detach().to(device=self.device, dtype=torch.float64).contiguous()
            else:
                p = torch.as_tensor(np.ascontiguousarray(wl.phi0()), dtype=torch.float64, device=self.device)
            phis.append(p)
        self.descs = descs
        self._u_keep = {}
        self.ws_bytes = L.lbm_cde_workspace_bytes(descs)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise RuntimeError("workspace is not 256-byte aligned")
        self.stream = torch.cuda.current_stream(self.device)
        self.h = L.lbm_cde_init(descs, [p.data_ptr() for p in phis], self.workspace.data_ptr(), self.ws_bytes,
                                self.stream.cuda_stream)
        torch.cuda.synchronize(self.device)
        del keep, phis

    # -- the C ABI, one call each ----------------------------------------------
    def step(self, n: int = 1) -> None:
        L.lbm_cde_step(self.h, int(n))

    def steps_done(self, run: int = 0) -> int:
        return L.lbm_cde_steps_done(self.h, run)

    def phi(self, run: int = 0) -> torch.Tensor:
        wl = self.runs[run]
        out = torch.empty(wl.grid, dtype=torch.float64, device=self.device)
        L.lbm_cde_moments(self.h, run, out.data_ptr())
        return out

    def mass(self, run: int = 0) -> float:
        return L.lbm_cde_reduce(self.h, run, L.LBM_CDE_RED_MASS)[0][0]

    def xmoments(self, run: int = 0, x_ref: float = 0.0):
        return L.lbm_cde_reduce(self.h, run, L.LBM_CDE_RED_XMOMENTS, x_ref)[0]

    def nonfinite(self, run: int = 0) -> int:
        return int(L.lbm_cde_reduce(self.h, run, L.LBM_CDE_RED_NONFINITE)[0][0])

    def relaxation_matrix(self, run: int = 0) -> np.ndarray:
        Q = Q_OF[self.runs[run].lattice]
        return np.array(L.lbm_cde_relaxation_matrix(self.h, run, Q)).reshape(Q, Q)

    def run_sampled(self, n: int, every: int, hist: torch.Tensor) -> None:
        L.lbm_cde_run_sampled(self.h, int(n), int(every), hist.data_ptr(), hist.shape[0])

    def samples_written(self) -> int:
        return L.lbm_cde_samples_written(self.h)

    def state_bytes(self, run: int = 0) -> int:
        return L.lbm_cde_state_bytes(self.h, run)

    def get_state(self, run: int = 0) -> torch.Tensor:
        out = torch.empty(self.state_bytes(run), dtype=torch.uint8, device=self.device)
        L.lbm_cde_get_state(self.h, run, out.data_ptr())
        return out

    def set_state(self, state: torch.Tensor, steps: int, run: int = 0) -> None:
        L.lbm_cde_set_state(self.h, run, state.data_ptr(), int(steps))

    def set_velocity(self, u, run: int = 0) -> None:
        """Replace the velocity field of a run made with a per-node field
        (array or tensor shaped (dim, *grid)); applies from the next step."""
        t = torch.as_tensor(u, dtype=torch.float64, device=self.device).contiguous()
        L.lbm_cde_set_velocity(self.h, run, t.data_ptr())
        self._u_keep[run] = t      # the conversion runs on the stream; keep the source alive until then

    def tune(self, trials: int = 20) -> None:
        L.lbm_cde_tune(self.h, int(trials))

    def variant(self, run: int = 0) -> dict:
        return L.lbm_cde_get_variant(self.h, run)

    def variants(self, run: int = 0) -> list:
        """Every compiled launch variant of a run (the tuner's candidates)."""
        return [L.lbm_cde_variant_at(self.h, run, i) for i in range(L.lbm_cde_variant_count(self.h, run))]

    def set_variant(self, v: dict, run: int = 0) -> None:
        L.lbm_cde_set_variant(self.h, run, v)

    def close(self) -> None:
        if getattr(self, "h", None):
            L.lbm_cde_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
