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


class RolloutMany(torch.autograd.Function):
    """J = sum over initial conditions k of 1/2 sum (phi_k - obs_k)^2 for one
    D field, the rollouts of all initial conditions advanced side by side: each
    has its own handle on a stream of its own (default priority), and the host
    issues their checkpoint segments in turn, so that the GPU overlaps runs
    that alone fill only part of it (a 512^2 step).  Forward and backward are
    those of ``Rollout``; the gradient is the sum of the per-condition
    gradients in the order of the conditions."""

    @staticmethod
    def forward(ctx, D_field, phi0s, obs, specs):
        dev = D_field.device
        main = torch.cuda.current_stream(dev)
        streams = [torch.cuda.Stream(device=dev) for _ in specs]
        runs = []
        for st, p0, spec in zip(streams, phi0s, specs):
            st.wait_stream(main)
            with torch.cuda.stream(st):
                wl = dataclasses.replace(spec.workload, D_field=D_field)
                s = Solver(wl, spec.precision, device=spec.device, heat=list(spec.heat), phi0=[p0])
            runs.append({"s": s, "ckpts": {}, "snaps": [], "t": 0})
        T = specs[0].steps
        if any(sp.steps != T or sp.snap_every != specs[0].snap_every or sp.ckpt_every != specs[0].ckpt_every
               for sp in specs):
            raise ValueError("misfit_many needs one schedule (steps, snapshots, checkpoints) for every condition")
        spec0 = specs[0]
        t = 0
        while t < T:
            nxt = min((t // spec0.ckpt_every + 1) * spec0.ckpt_every, (t // spec0.snap_every + 1) * spec0.snap_every, T)
            for st, r in zip(streams, runs):
                with torch.cuda.stream(st):
                    if t % spec0.ckpt_every == 0:
                        r["ckpts"][t] = r["s"].get_state()
                    r["s"].step(nxt - t)
                    if nxt % spec0.snap_every == 0:
                        r["snaps"].append(r["s"].phi())
            t = nxt
        J = torch.zeros((), dtype=torch.float64, device=dev)
        resid = []
        for st, r, o in zip(streams, runs, obs):
            with torch.cuda.stream(st):
                d = torch.stack(r["snaps"]) - o
                resid.append(d)
                Jk = 0.5 * (d * d).sum()
            main.wait_stream(st)
            J = J + Jk
        ctx.runs, ctx.resid, ctx.streams, ctx.specs = runs, resid, streams, specs
        ctx.D_dtype = D_field.dtype
        return J

    @staticmethod
    def backward(ctx, grad_J):
        runs, streams, spec0 = ctx.runs, ctx.streams, ctx.specs[0]
        dev = runs[0]["s"].device
        main = torch.cuda.current_stream(dev)
        ny, nx = runs[0]["s"].runs[0].grid
        T = spec0.steps
        bufs = []
        for st, r, d in zip(streams, runs, ctx.resid):
            st.wait_stream(main)
            with torch.cuda.stream(st):
                s = r["s"]
                nb = s.state_bytes()
                g = (grad_J.to(torch.float64) * d).contiguous()
                bufs.append({"g": g, "mu": torch.zeros(nb, dtype=torch.uint8, device=dev),
                             "mu_tmp": torch.empty(nb, dtype=torch.uint8, device=dev),
                             "seg": torch.empty(L.lbm_cde_adjoint_scratch_bytes(s.h, 0, spec0.ckpt_every),
                                                dtype=torch.uint8, device=dev),
                             "grad": torch.zeros((3, ny, nx), dtype=torch.float64, device=dev)})
        for t0 in sorted(runs[0]["ckpts"], reverse=True):
            K = min(spec0.ckpt_every, T - t0)
            for st, r, b in zip(streams, runs, bufs):
                inj = []
                for k in range(K):
                    t1 = t0 + k + 1
                    inj.append(b["g"][t1 // spec0.snap_every - 1].data_ptr() if t1 % spec0.snap_every == 0 else None)
                with torch.cuda.stream(st):
                    L.lbm_cde_adjoint_segment(r["s"].h, 0, r["ckpts"][t0].data_ptr(), K, b["seg"].data_ptr(), inj,
                                              b["mu"].data_ptr(), b["mu_tmp"].data_ptr(), b["grad"].data_ptr())
        grad = torch.zeros((3, ny, nx), dtype=torch.float64, device=dev)
        for st, b in zip(streams, bufs):
            main.wait_stream(st)
            grad += b["grad"]
        for st in streams:
            st.synchronize()
        for r in runs:
            r["s"].close()
        ctx.runs = None
        return grad.to(ctx.D_dtype), None, None, None


def misfit_many(D_field: torch.Tensor, phi0s: Sequence[torch.Tensor], obs: Sequence[torch.Tensor],
                specs: Sequence[RolloutSpec]) -> torch.Tensor:
    """Sum over initial conditions of the snapshot misfits, the rollouts run
    side by side (differentiable with respect to D_field only)."""
    return RolloutMany.apply(D_field, list(phi0s), list(obs), list(specs))


def misfit(D_field: torch.Tensor, phi0: torch.Tensor, obs: torch.Tensor, spec: RolloutSpec) -> torch.Tensor:
    """J = 1/2 sum over snapshots and nodes of (phi - obs)^2 (differentiable)."""
    snaps = Rollout.apply(D_field, phi0, spec)
    return 0.5 * ((snaps - obs) ** 2).sum()


def forward_snapshots(D_field: torch.Tensor, phi0: torch.Tensor, spec: RolloutSpec) -> torch.Tensor:
    """The phi snapshots without recording for autograd."""
    s, _, snaps = _forward(D_field, phi0, spec)
    s.close()
    return snaps
