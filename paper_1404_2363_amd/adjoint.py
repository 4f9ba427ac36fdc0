"""Gradients of phi snapshots with respect to a per-node diffusion tensor field.

``Rollout`` is a ``torch.autograd.Function``: its forward advances the
modified-MRT D2Q9 model from phi0 with a per-node D field through the HIP
library, keeping a population checkpoint every ``ckpt_every`` steps and
returning the phi snapshots taken every ``snap_every`` steps; its backward
replays each checkpoint segment and runs the library's adjoint kernel over
it (reverse streaming, transposed relaxation), giving dL/dD at every node
and dL/dphi0.  The heat-flux rates are fixed (explicit), so that S depends on
D only through the flux block A = (3 D + I/2)^-1.
"""
from __future__ import annotations

import dataclasses
from typing import Sequence

import torch

from . import _lib as L
from .solver import Solver


@dataclasses.dataclass
class RolloutSpec:
    workload: object              # a D2Q9 Workload; its D_field and phi0 are replaced by the inputs
    steps: int
    snap_every: int
    ckpt_every: int
    precision: str = "fp32"
    heat: Sequence[float] = (1.0, 1.0)
    device: str = "cuda:0"


def _forward(D_field: torch.Tensor, phi0: torch.Tensor, spec: RolloutSpec):
    wl = dataclasses.replace(spec.workload, D_field=D_field)
    s = Solver(wl, spec.precision, device=spec.device, heat=list(spec.heat), phi0=[phi0])
    ckpts, snaps = {}, []
    t, T = 0, spec.steps
    while t < T:
        if t % spec.ckpt_every == 0:
            ckpts[t] = s.get_state()
        nxt = min((t // spec.ckpt_every + 1) * spec.ckpt_every, (t // spec.snap_every + 1) * spec.snap_every, T)
        s.step(nxt - t)
        t = nxt
        if t % spec.snap_every == 0:
            snaps.append(s.phi())
    return s, ckpts, torch.stack(snaps)


class Rollout(torch.autograd.Function):
    """snapshots = Rollout.apply(D_field, phi0, spec); shape (nsnap, ny, nx), FP64."""

    @staticmethod
    def forward(ctx, D_field, phi0, spec):
        s, ckpts, snaps = _forward(D_field, phi0, spec)
        ctx.solver, ctx.ckpts, ctx.spec = s, ckpts, spec
        ctx.D_dtype = D_field.dtype
        return snaps

    @staticmethod
    def backward(ctx, grad_snaps):
        s, spec = ctx.solver, ctx.spec
        g = grad_snaps.detach().to(torch.float64).contiguous()
        nb = s.state_bytes()
        ny, nx = s.runs[0].grid
        dev = s.device
        mu = torch.zeros(nb, dtype=torch.uint8, device=dev)
        mu_tmp = torch.empty(nb, dtype=torch.uint8, device=dev)
        seg = torch.empty(L.lbm_cde_adjoint_scratch_bytes(s.h, 0, spec.ckpt_every), dtype=torch.uint8, device=dev)
        grad = torch.zeros((3, ny, nx), dtype=torch.float64, device=dev)
        T = spec.steps
        for t0 in sorted(ctx.ckpts, reverse=True):
            K = min(spec.ckpt_every, T - t0)
            inj = []
            for k in range(K):
                t1 = t0 + k + 1
                inj.append(g[t1 // spec.snap_every - 1].data_ptr() if t1 % spec.snap_every == 0 else None)
            L.lbm_cde_adjoint_segment(s.h, 0, ctx.ckpts[t0].data_ptr(), K, seg.data_ptr(), inj, mu.data_ptr(),
                                      mu_tmp.data_ptr(), grad.data_ptr())
        dphi0 = torch.empty((ny, nx), dtype=torch.float64, device=dev)
        L.lbm_cde_adjoint_phi0(s.h, 0, mu.data_ptr(), None, dphi0.data_ptr())
        torch.cuda.current_stream(dev).synchronize()
        ctx.solver = None
        s.close()
        return grad.to(ctx.D_dtype), dphi0, None


def misfit(D_field: torch.Tensor, phi0: torch.Tensor, obs: torch.Tensor, spec: RolloutSpec) -> torch.Tensor:
    """J = 1/2 sum over snapshots and nodes of (phi - obs)^2 (differentiable)."""
    snaps = Rollout.apply(D_field, phi0, spec)
    return 0.5 * ((snaps - obs) ** 2).sum()


def forward_snapshots(D_field: torch.Tensor, phi0: torch.Tensor, spec: RolloutSpec) -> torch.Tensor:
    """The phi snapshots without recording for autograd."""
    s, _, snaps = _forward(D_field, phi0, spec)
    s.close()
    return snaps
