"""Accuracy sweeps of Sec. 3 at GPU scale, with the throughput of each run.

* ``convergence``: pure diffusion of a Gaussian hill with dx = dt = 1/256
  fixed while the lattice grows (domain [-L, L]^2, L = dx N / 2,
  sigma0 = 0.05 L, D of Eq. 42, s4 = s_xx, s6 = s_yy), relative error Er of
  Eq. (45) at the time t_m where the exact peak halves, for each storage
  precision: the order of accuracy (Fig. 3) and where each precision stops
  converging.
* ``tau_sweep``: Er_2 of Eq. (43) on the 512^2 hill against tau for the three
  flux blocks of Eq. (44) (D = (A^-1 - I/2)/3 in lattice units), u = 0 and
  u = (0.05, 0.05), the four models (Fig. 2).
* ``fixed_u_taylor_aris``: the plate channel of Sec. 3.2 at a fixed maximum
  speed U = 0.1 with tau = 64 U / Pe + 1/2, the four models (Fig. 5).

All runs of a sweep that share a precision and lattice go through one
batched launch.

    python -m paper_1404_2363_amd.sweeps [convergence|tau|fig5]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import workloads as W
from .paper_tables import MODELS, hill_exact, plate_alpha_history
from .solver import Solver


def _hill(kind, n, u=(0.0, 0.0), D_lat=None):
    """Gaussian hill of Sec. 3.1 with dx = dt = 1/256 on n^2 nodes (sigma0 = 0.05 L)."""
    dx = 1.0 / 256.0
    sig = 0.05 * (dx * n / 2.0) / dx
    D = np.asarray(W.PAPER_HILL_D[kind], np.float64) * 1e-4 / dx if D_lat is None else np.asarray(D_lat)
    a, b, c = 4.0 * np.linalg.det(D), 2.0 * sig ** 2 * np.trace(D), -3.0 * sig ** 4
    t_m = (-b + math.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)
    spec = W.GaussianSum(np.array([[n / 2.0, n / 2.0]]), np.ones(1), np.array([sig]), (float(n), float(n)))
    return W.Workload(f"hill_{kind}_{n}", "d2q9", (n, n), ("periodic", "periodic"), int(round(t_m)), spec, D=D,
                      u_const=np.asarray(u, np.float64) * 1.0,
                      meta={"sigma0": sig, "t_m": t_m, "centre": (n / 2.0, n / 2.0), "phi_ref": 0.0, "kind": kind})


def _run_batch(runs, precision, per_run, device="cuda:0"):
    s = Solver(runs, precision, device=device, per_run=per_run)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(max(int(r.steps) for r in runs))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phis = [s.phi(i).cpu().numpy() for i in range(len(runs))]
    s.close()
    lu = sum(r.nodes * r.steps for r in runs)
    return phis, {"wall_s": wall, "lattice_updates": lu, "glups": lu / wall / 1e9}


def convergence(sizes=(128, 256, 512, 1024, 2048), precisions=("fp64", "fp32", "fp16"),
                kinds=("isotropic", "diagonal", "full")):
    out = []
    for prec in precisions:
        for n in sizes:
            runs = [_hill(k, n) for k in kinds]
            phis, info = _run_batch(runs, prec, [{"heat": "paper", "max_steps": int(r.steps),
                                                  "stability_check": False} for r in runs])
            for r, phi in zip(runs, phis):
                ex = hill_exact(r, float(r.steps))
                er = float(np.sqrt(((phi - ex) ** 2).sum()) / np.sqrt((ex ** 2).sum()))
                out.append({"precision": prec, "N": n, "D": r.meta["kind"], "steps": int(r.steps), "Er": er,
                            "glups_batch": info["glups"]})
    orders = {}
    for prec in precisions:
        for k in kinds:
            pts = [(r["N"], r["Er"]) for r in out if r["precision"] == prec and r["D"] == k]
            ns = np.log([p[0] for p in pts])
            es = np.log([p[1] for p in pts])
            orders[f"{prec}/{k}"] = {"fit_all": float(-np.polyfit(ns, es, 1)[0]),
                                     "pairwise": [float(-(es[i + 1] - es[i]) / (ns[i + 1] - ns[i]))
                                                  for i in range(len(pts) - 1)]}
    return out, orders


def eq44_D(kind, tau):
    """D = (A^-1 - I/2)/3 (lattice units) for the flux blocks of Eq. (44)."""
    if kind == "isotropic":
        Ainv = np.array([[tau, 0.0], [0.0, tau]])
    elif kind == "diagonal":
        Ainv = np.array([[tau, 0.0], [0.0, 4.0 * tau - 1.5]])
    else:
        Ainv = np.array([[tau, tau - 0.5], [tau - 0.5, 4.0 * tau - 1.5]])
    return (Ainv - 0.5 * np.eye(2)) / 3.0


def tau_sweep(taus=(0.6, 0.8, 1.0, 1.25, 1.5, 2.0), us=((0.0, 0.0), (0.05, 0.05)), precision="fp64", n=512):
    out = []
    for u in us:
        for kind in ("isotropic", "diagonal", "full"):
            runs, per = [], []
            for tau in taus:
                for m in MODELS:
                    r = _hill(kind, n, u=u, D_lat=eq44_D(kind, tau))
                    r.meta.update({"tau": tau, "model": m})
                    runs.append(r)
                    # the paper's rates; some (tau, u) points are unstable for
                    # short waves, which the sweep repeats as printed
                    per.append({"heat": "paper", "model": m, "max_steps": int(r.steps), "stability_check": False})
            phis, info = _run_batch(runs, precision, per)
            for r, phi in zip(runs, phis):
                ex = hill_exact(r, float(r.steps))
                out.append({"u": list(u), "D": kind, "tau": r.meta["tau"], "model": r.meta["model"],
                            "steps": int(r.steps), "Er2": float(np.sqrt(np.mean((phi - ex) ** 2)))})
    return out


def fixed_u_taylor_aris(pes=(2.0, 4.0, 8.0, 16.0, 25.6, 32.0, 49.2, 64.0, 128.0), U=0.1, precision="fp64",
                        every=100):
    runs, tags = [], []
    for Pe in pes:
        tau = 64.0 * U / Pe + 0.5
        for m in MODELS:
            runs.append(W.plate_channel(tau, Pe, name=f"fig5_Pe{Pe}_{m}"))
            tags.append((tau, Pe, m))
    per = [{"heat": [1.0 / t] * 2, "max_steps": int(r.steps), "xref0": r.meta["x0"],
            "xref_drift": r.meta["U_node_mean"], "model": m, "phi_ref": 0.0} for r, (t, _, m) in zip(runs, tags)]
    s = Solver(runs, precision, per_run=per)
    rows = max(int(r.steps) for r in runs) // every
    hist = torch.zeros((rows, len(runs), 3), dtype=torch.float64, device="cuda:0")
    done = 0
    while done < rows:
        k = min(100, rows - done)
        s.run_sampled(k * every, every, hist)
        done += k
    torch.cuda.synchronize()
    s.close()
    h = hist.cpu().numpy()
    out = []
    for i, (r, (tau, Pe, m)) in enumerate(zip(runs, tags)):
        a = plate_alpha_history(h[: int(r.steps) // every, i], every)
        K = r.meta["K"]
        out.append({"tau": tau, "Pe": Pe, "model": m, "U": r.meta["U"], "Er": float(abs(a[-1] - K) / K),
                    "signed": float((a[-1] - K) / K)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all", choices=["all", "convergence", "tau", "fig5"])
    args = ap.parse_args()
    if args.which in ("all", "convergence"):
        res, orders = convergence()
        for r in res:
            print(json.dumps({"sweep": "convergence", **r}), flush=True)
        print(json.dumps({"sweep": "convergence_orders", **orders}), flush=True)
    if args.which in ("all", "tau"):
        for r in tau_sweep():
            print(json.dumps({"sweep": "tau", **r}), flush=True)
    if args.which in ("all", "fig5"):
        for r in fixed_u_taylor_aris():
            print(json.dumps({"sweep": "fig5", **r}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
