"""Seeded synthetic inputs for the anisotropic convection-diffusion workloads.

This module only draws and tabulates *problem inputs* of Eq. (1): initial
scalar fields phi0(x), velocity fields u(x) and diffusion tensors D (constant
or per node).  It holds none of the lattice Boltzmann arithmetic (no moments,
equilibria, relaxation, parameter maps or streaming), so the CPU oracle and
the HIP path both take their inputs from here and from nowhere else.

Conventions
-----------
* Node ``x`` has integer coordinates ``0..n-1`` per axis (lattice units,
  dx = dt = 1).  Arrays are indexed ``[y, x]`` (2D) or ``[z, y, x]`` (3D),
  x fastest.
* A velocity component given in *separable* form is
  ``u_c(x, y, z) = amp_c * X_c[x] * Y_c[y] * Z_c[z]``, evaluated in exactly
  that order of products.  The analytic flows of the workloads (cellular 2D
  flow, plane Poiseuille profile, the 3D sine flow) all have this form.
* Every random draw comes from ``numpy.random.default_rng(SeedSequence(
  [14042363, workload_id, ...]))`` so that each workload is reproducible.

Workloads (shapes and distributions follow the paper's tests, Sec. 3):
  gaussian_hill       Sec. 3.1 analog: 128^2 periodic, u = 0, full tensor D.
  cellular            4096^2 periodic, divergence-free cellular u, rotated D,
                      64 random Gaussian hills (the spatially varying u the
                      paper's deviation-term argument is about, Sec. 2).
  taylor_aris_batch   Sec. 3.2 analog: 64 plane Poiseuille channels with
                      halfway mirror walls, uneven gaps h, Pe and tau.
  plate_channel       Sec. 3.2 as printed: W = 32 lattices between on-node
                      plates, L = 150 W, top-hat pulse, u_x = 4Uy(W-y)/W^2.
  paper_hill          Sec. 3.1 as printed: [-1, 1]^2 on 512^2 nodes,
                      dx = dt = 1/256, sigma0 = 0.05, D of Eq. (42).
  sine3d              Appendix A analog: 256^3 D3Q15, 3D sine flow, random D.
  inverse_dfield      512^2 periodic, constant u, smooth per-node D field,
                      10 Gaussian-hill initial conditions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

SEED_ROOT = 14042363


def rng_for(workload_id: int, *extra: int) -> np.random.Generator:
    """Seeded generator for one workload (and optional sub-stream)."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, workload_id, *extra]))


# --------------------------------------------------------------------------
# Building blocks
# --------------------------------------------------------------------------

def min_image(d: np.ndarray, period: Optional[float]) -> np.ndarray:
    """Signed distance folded into [-period/2, period/2) (None: no folding)."""
    if period is None:
        return d
    return d - period * np.floor(d / period + 0.5)


@dataclasses.dataclass
class GaussianSum:
    """phi0(x) = sum_j amp_j * prod_axis exp(-d_axis^2 / (2 sigma_j^2)).

    ``centres`` has shape (nhill, dim) in node coordinates; distances use the
    minimum image on periodic axes.
    """
    centres: np.ndarray
    amps: np.ndarray
    sigmas: np.ndarray
    periods: tuple  # per axis: float period or None

    def factors(self, axis: int, idx: np.ndarray) -> np.ndarray:
        """Per-hill 1D factors on the index vector ``idx`` of ``axis``: (nhill, len)."""
        idx = np.asarray(idx, dtype=np.float64)
        d = min_image(idx[None, :] - self.centres[:, axis:axis + 1], self.periods[axis])
        return np.exp(-(d * d) / (2.0 * self.sigmas[:, None] ** 2))

    def window(self, idx: Sequence[np.ndarray]) -> np.ndarray:
        """Evaluate on the tensor-product window ``idx`` = (ix, iy[, iz]).

        Returns an array indexed [y, x] or [z, y, x].
        """
        dim = len(idx)
        gx = self.factors(0, idx[0]) * self.amps[:, None]
        gy = self.factors(1, idx[1])
        if dim == 2:
            return gy.T @ gx                       # (ny, nx)
        gz = self.factors(2, idx[2])
        zy = (gz[:, :, None] * gy[:, None, :]).reshape(len(self.amps), -1)
        return (zy.T @ gx).reshape(len(idx[2]), len(idx[1]), len(idx[0]))


@dataclasses.dataclass
class SeparableU:
    """Velocity field u_c = amp_c * X_c[x] * Y_c[y] * Z_c[z] for each component c."""
    amp: np.ndarray            # (dim,)
    tables: list               # tables[c] = [X_c, Y_c, Z_c] (Z_c = [1.0] in 2D)

    def window(self, idx: Sequence[np.ndarray]) -> np.ndarray:
        dim = len(idx)
        out = []
        for c in range(dim):
            X, Y, Z = self.tables[c]
            x = np.asarray(X)[np.asarray(idx[0])]
            y = np.asarray(Y)[np.asarray(idx[1])]
            z = np.asarray(Z)[np.asarray(idx[2])] if dim == 3 else np.ones(1)
            comp = ((self.amp[c] * x[None, None, :]) * y[None, :, None]) * z[:, None, None]
            out.append(comp if dim == 3 else comp[0])
        return np.stack(out)

    def as_flat_tables(self, shape) -> np.ndarray:
        """Host table layout of the C-ABI: for each component c,
        amp_c, X_c[nx], Y_c[ny], Z_c[nz]."""
        nx, ny, nz = (tuple(shape) + (1,))[:3]
        parts = []
        for c in range(len(self.amp)):
            X, Y, Z = self.tables[c]
            parts += [np.array([self.amp[c]]), np.asarray(X, np.float64).reshape(nx),
                      np.asarray(Y, np.float64).reshape(ny), np.asarray(Z, np.float64).reshape(nz)]
        return np.ascontiguousarray(np.concatenate(parts))


@dataclasses.dataclass
class Workload:
    """One run: lattice, grid, boundaries and the inputs of Eq. (1)."""
    name: str
    lattice: str                       # "d2q9" | "d3q15"
    shape: tuple                       # (nx, ny) or (nx, ny, nz)
    walls: tuple                       # per axis: "periodic" | "bounce" | "specular" (both faces)
    steps: int
    phi0_spec: GaussianSum
    D: Optional[np.ndarray] = None     # (dim, dim) constant symmetric tensor
    D_field: Optional[np.ndarray] = None  # (ncomp, *grid): 2D (xx, yy, xy); 3D (xx, yy, zz, xy, xz, yz)
    u_const: Optional[np.ndarray] = None
    u_sep: Optional[SeparableU] = None
    meta: dict = dataclasses.field(default_factory=dict)
    u_field: Optional[np.ndarray] = None   # (dim, *grid) per-node velocity at step 0
    u_schedule: Optional[object] = None    # n -> (dim, *grid) velocity of step n (time-dependent u)

    @property
    def dim(self) -> int:
        return len(self.shape)

    @property
    def grid(self) -> tuple:
        """Array shape, slowest axis first: (ny, nx) or (nz, ny, nx)."""
        return tuple(reversed(self.shape))

    @property
    def nodes(self) -> int:
        return int(np.prod(self.shape))

    def full_index(self):
        return [np.arange(n) for n in self.shape]

    def phi0(self, idx=None) -> np.ndarray:
        return self.phi0_spec.window(self.full_index() if idx is None else idx)

    def u(self, idx=None) -> np.ndarray:
        """Velocity on a window (default: whole grid), shape (dim, *window)."""
        idx = self.full_index() if idx is None else idx
        wshape = tuple(len(i) for i in reversed(idx))
        if self.u_field is not None:
            return self.u_field[(slice(None),) + np.ix_(*reversed([np.asarray(i) for i in idx]))].copy()
        if self.u_sep is not None:
            return self.u_sep.window(idx)
        u0 = np.zeros(self.dim) if self.u_const is None else np.asarray(self.u_const, np.float64)
        return np.broadcast_to(u0.reshape((self.dim,) + (1,) * self.dim),
                               (self.dim,) + wshape).copy()

    def D_window(self, idx=None) -> np.ndarray:
        """Per-node D components on a window, shape (ncomp, *window)."""
        idx = self.full_index() if idx is None else idx
        if self.D_field is None:
            return constant_components(self.D, tuple(len(i) for i in reversed(idx)))
        return self.D_field[(slice(None),) + np.ix_(*reversed([np.asarray(i) for i in idx]))]

    def phi_ref(self) -> float:
        """Background level used by shifted storage: the minimum of phi0.

        Shifted storage keeps f - w phi_ref; the shift should remove the
        uniform background (where every node would otherwise store the same
        value and round the same way each step), which for hills on an empty
        field is zero."""
        if "phi_ref" in self.meta:
            return float(self.meta["phi_ref"])
        return float(self.phi0().min())


def tensor_components(D: np.ndarray) -> np.ndarray:
    """Symmetric tensor -> component vector (xx, yy, xy) or (xx, yy, zz, xy, xz, yz)."""
    D = np.asarray(D, np.float64)
    if D.shape == (2, 2):
        return np.array([D[0, 0], D[1, 1], D[0, 1]])
    return np.array([D[0, 0], D[1, 1], D[2, 2], D[0, 1], D[0, 2], D[1, 2]])


def components_tensor(c) -> np.ndarray:
    c = np.asarray(c, np.float64)
    if c.shape[0] == 3:
        return np.array([[c[0], c[2]], [c[2], c[1]]])
    return np.array([[c[0], c[3], c[4]], [c[3], c[1], c[5]], [c[4], c[5], c[2]]])


def constant_components(D, wshape) -> np.ndarray:
    comps = tensor_components(D)
    return np.broadcast_to(comps.reshape((-1,) + (1,) * len(wshape)), (len(comps),) + wshape).copy()


def rotation2(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def rotated_tensor_2d(eigs, theta) -> np.ndarray:
    R = rotation2(theta)
    return R @ np.diag(eigs) @ R.T


def haar_rotation3(rng: np.random.Generator) -> np.ndarray:
    """Haar-random proper rotation: QR of a Gaussian matrix with sign fix, det = +1."""
    Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def random_hills(rng, n_hills, shape, sigma, amp_lo=0.5, amp_hi=1.0, periodic=True) -> GaussianSum:
    dim = len(shape)
    centres = rng.uniform(0.0, 1.0, size=(n_hills, dim)) * np.asarray(shape, np.float64)[None, :]
    amps = rng.uniform(amp_lo, amp_hi, size=n_hills)
    periods = tuple(float(n) if periodic else None for n in shape)
    return GaussianSum(centres, amps, np.full(n_hills, float(sigma)), periods)


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------

GAUSSIAN_HILL_D = np.array([[0.05, 0.02], [0.02, 0.03]])


def gaussian_hill(n: int = 128, sigma0: float = 8.0, steps: int = 1000,
                  D=GAUSSIAN_HILL_D, u=(0.0, 0.0)) -> Workload:
    """A single hill of peak 1 at the grid centre (a node), periodic grid."""
    centre = np.array([[n // 2, n // 2]], np.float64)
    spec = GaussianSum(centre, np.ones(1), np.array([float(sigma0)]), (float(n), float(n)))
    return Workload("gaussian_hill", "d2q9", (n, n), ("periodic",) * 2, steps, spec,
                    D=np.asarray(D, np.float64), u_const=np.asarray(u, np.float64),
                    meta={"sigma0": sigma0, "centre": (n // 2, n // 2)})


CELLULAR_U0 = 0.05
CELLULAR_D = rotated_tensor_2d([0.01, 0.1], math.radians(30.0))


def cellular(nx: int = 4096, ny: Optional[int] = None, steps: int = 5000, n_hills: int = 64,
             sigma: float = 32.0, U0: float = CELLULAR_U0, D=CELLULAR_D, seed_id: int = 1) -> Workload:
    """Cellular flow u = U0 (sin kx cos ky, -cos kx sin ky), k = 2 pi / n, rotated D.

    Divergence-free for nx == ny (the full-size case); a ragged ny keeps the
    same formula with its own wavenumber, which is all parity needs.
    """
    ny = nx if ny is None else ny
    kx, ky = 2.0 * math.pi / nx, 2.0 * math.pi / ny
    X = np.arange(nx, dtype=np.float64)
    Y = np.arange(ny, dtype=np.float64)
    u_sep = SeparableU(np.array([U0, -U0]),
                       [[np.sin(kx * X), np.cos(ky * Y), np.ones(1)],
                        [np.cos(kx * X), np.sin(ky * Y), np.ones(1)]])
    spec = random_hills(rng_for(seed_id), n_hills, (nx, ny), sigma)
    return Workload("cellular", "d2q9", (nx, ny), ("periodic",) * 2, steps, spec,
                    D=np.asarray(D, np.float64), u_sep=u_sep,
                    meta={"U0": U0, "sigma": sigma, "n_hills": n_hills})


SINE3D_U0 = 0.04


def sine3d(n: int = 256, ny: Optional[int] = None, nz: Optional[int] = None, steps: int = 2000,
           n_hills: int = 32, sigma: float = 16.0, U0: float = SINE3D_U0, seed_id: int = 3) -> Workload:
    """D3Q15 workload: u = U0 (sin(2 pi y/ny), sin(2 pi z/nz), sin(2 pi x/nx)), random D."""
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = rng_for(seed_id)
    Q = haar_rotation3(rng)
    lam = rng.uniform(0.01, 0.1, size=3)
    D = Q @ np.diag(lam) @ Q.T
    D = 0.5 * (D + D.T)
    one = np.ones
    sx = np.sin(2.0 * math.pi * np.arange(nx) / nx)
    sy = np.sin(2.0 * math.pi * np.arange(ny) / ny)
    sz = np.sin(2.0 * math.pi * np.arange(nz) / nz)
    u_sep = SeparableU(np.array([U0, U0, U0]),
                       [[one(nx), sy, one(nz)], [one(nx), one(ny), sz], [sx, one(ny), one(nz)]])
    spec = random_hills(rng, n_hills, (nx, ny, nz), sigma)
    return Workload("sine3d", "d3q15", (nx, ny, nz), ("periodic",) * 3, steps, spec,
                    D=D, u_sep=u_sep, meta={"U0": U0, "eigs": lam, "rotation": Q})


# ---- Taylor-Aris ensemble ------------------------------------------------

TA_GAPS = (32, 48, 64, 96, 128)


def poiseuille_profile(h: int, u_mean: float) -> np.ndarray:
    """Parabolic u_x at node centres between walls at y = -1/2 and y = h - 1/2."""
    yh = (np.arange(h, dtype=np.float64) + 0.5) / h
    return 6.0 * u_mean * yh * (1.0 - yh)


def taylor_aris_channel(h: int, Pe: float, tau: float, nx: int = 4096, steps: Optional[int] = None,
                        name: str = "taylor_aris", wall: str = "specular") -> Workload:
    """One plane Poiseuille channel: periodic x, zero-flux walls in y halfway
    outside the first and last rows (gap h).

    ``wall`` is "specular" (mirror: only the normal velocity reverses, the
    halfway form of the paper's plate rule) or "bounce" (full reversal).

    The molecular diffusivity follows from the isotropic relaxation time,
    D_m = (tau - 1/2)/3, and the mean speed from the Peclet number based on
    the full gap, U = Pe * D_m / h.  The pulse is a Gaussian of width h/2
    released at x = nx/8, uniform across the gap.
    """
    D_m = (tau - 0.5) / 3.0
    U = Pe * D_m / h
    prof = poiseuille_profile(h, U)
    u_node_mean = float(prof.mean())
    u_sep = SeparableU(np.array([1.0, 0.0]),
                       [[np.ones(nx), prof, np.ones(1)], [np.ones(nx), np.zeros(h), np.ones(1)]])
    spec = GaussianSum(np.array([[nx / 8.0, 0.0]]), np.ones(1), np.array([h / 2.0]),
                       (float(nx), None))
    spec_x_only = _XOnly(spec)
    K = D_m * (1.0 + Pe * Pe / 210.0)
    t_taylor = h * h / D_m
    # end of the run: 8 h^2/D_m, or earlier when the pulse (8 sigma) fills the
    # period.  The variance of Eq. (47) over one period misses the tails beyond
    # +-nx/2: at 6 sigma it reads 2.7 % low at the end of the run and tilts the
    # fitted slope by up to 1.5 %, at 8 sigma by at most 0.1 %.
    sig0 = h / 2.0
    t_wrap = ((nx / 8.0) ** 2 - sig0 ** 2) / (2.0 * K)
    t_end = int(min(8.0 * t_taylor, t_wrap))
    wl = Workload(name, "d2q9", (nx, h), ("periodic", wall), t_end if steps is None else steps,
                  spec_x_only, D=D_m * np.eye(2), u_sep=u_sep,
                  meta={"h": h, "Pe": Pe, "tau": tau, "D_m": D_m, "U_mean": U,
                        "U_node_mean": u_node_mean, "U_max": 1.5 * U, "K": K,
                        "t_taylor": t_taylor, "t_end": t_end, "x0": nx / 8.0})
    return wl


class _XOnly(GaussianSum):
    """Gaussian in x only (uniform in y): the Taylor-Aris pulse."""

    def __init__(self, spec: GaussianSum):
        super().__init__(spec.centres, spec.amps, spec.sigmas, spec.periods)

    def window(self, idx):
        gx = self.factors(0, idx[0]) * self.amps[:, None]
        return np.repeat(gx.sum(0)[None, :], len(idx[1]), axis=0)


def taylor_aris_batch(n_runs: int = 64, nx: int = 4096, seed_id: int = 2, u_max_cap: float = 0.2,
                      gaps=TA_GAPS, wall: str = "specular") -> list:
    """64 channels with h ~ {32,48,64,96,128}, Pe ~ U(5,100), tau ~ U(0.6,2.0).

    A draw is kept only when the flow is slow enough to be stable
    (U_max = 1.5 U <= 0.2) and the pulse still fits the periodic length at
    twice the Taylor time (6 sigma <= nx); otherwise it is redrawn from the
    same seeded stream.
    """
    rng = rng_for(seed_id)
    runs = []
    while len(runs) < n_runs:
        h = int(rng.choice(np.asarray(gaps)))
        Pe = float(rng.uniform(5.0, 100.0))
        tau = float(rng.uniform(0.6, 2.0))
        D_m = (tau - 0.5) / 3.0
        U = Pe * D_m / h
        if 1.5 * U > u_max_cap:
            continue
        K = D_m * (1.0 + Pe * Pe / 210.0)
        sig2 = (h / 2.0) ** 2 + 2.0 * K * (2.0 * h * h / D_m)
        if 6.0 * math.sqrt(sig2) > nx:
            continue
        runs.append(taylor_aris_channel(h, Pe, tau, nx=nx, name=f"taylor_aris_{len(runs)}", wall=wall))
    return runs


# D x 10^4 of Eq. (42): isotropic, diagonal anisotropic, full anisotropic.
PAPER_HILL_D = {"isotropic": ((2.0, 0.0), (0.0, 2.0)), "diagonal": ((1.0, 0.0), (0.0, 4.0)),
                "full": ((1.0, 1.0), (1.0, 4.0))}


def paper_hill(kind: str = "isotropic", u=(0.0, 0.0), n: int = 512) -> Workload:
    """Gaussian hill of Sec. 3.1: the domain [-1, 1]^2 on n^2 periodic nodes
    x_i = -1 + i dx with dx = dt = 2/n (1/256 for n = 512), peak 1 at the
    origin (phi0 = 2 pi sigma0^2 in Eq. 40, sigma0 = 0.05), D of Eq. (42) and
    a constant u, all converted to lattice units (D dt/dx^2, u dt/dx).

    meta["t_m"] is the time at which the exact peak halves,
    sigma0^2 / sqrt(det(sigma0^2 I + 2 D t)) = 1/2, and meta["steps"] its
    nearest step."""
    dx = 2.0 / n
    dt = dx
    sig = 0.05 / dx
    D = np.asarray(PAPER_HILL_D[kind], np.float64) * 1e-4 * dt / dx ** 2
    u_lat = np.asarray(u, np.float64) * dt / dx
    # det(s^2 I + 2 D t) = 4 s^4  ->  4 det(D) t^2 + 2 s^2 tr(D) t - 3 s^4 = 0
    a, b, c = 4.0 * np.linalg.det(D), 2.0 * sig ** 2 * np.trace(D), -3.0 * sig ** 4
    t_m = (-b + math.sqrt(b * b - 4.0 * a * c)) / (2.0 * a) if a > 0 else -c / b
    centre = np.array([[n / 2.0, n / 2.0]])
    spec = GaussianSum(centre, np.ones(1), np.array([sig]), (float(n), float(n)))
    steps = int(round(t_m))
    return Workload(f"paper_hill_{kind}", "d2q9", (n, n), ("periodic", "periodic"), steps, spec,
                    D=D, u_const=u_lat, meta={"kind": kind, "sigma0": sig, "t_m": t_m, "centre": (n / 2.0, n / 2.0),
                                              "phi_ref": 0.0})


def drifting_cellular_field(nx: int, ny: int, U0: float, shift: float) -> np.ndarray:
    """u = U0 (sin k(x - s) cos ky, -cos k(x - s) sin ky), k = 2 pi / n, as a
    (2, ny, nx) array: the cellular flow translated by s nodes in x."""
    kx, ky = 2.0 * math.pi / nx, 2.0 * math.pi / ny
    X, Y = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64))
    return np.stack([U0 * np.sin(kx * (X - shift)) * np.cos(ky * Y), -U0 * np.cos(kx * (X - shift)) * np.sin(ky * Y)])


def drifting_cellular(nx: int = 512, ny: Optional[int] = None, steps: int = 400, n_hills: int = 16,
                      sigma: float = 12.0, U0: float = CELLULAR_U0, drift: float = 0.25, D=CELLULAR_D,
                      walls=("periodic", "periodic"), seed_id: int = 6) -> Workload:
    """A time-dependent flow: the cellular flow whose cells drift along x by
    `drift` nodes per step, u(x, t_n) = drifting_cellular_field(n drift),
    given as a per-node field updated every step (the case of a velocity
    that changes in space and time, Sec. 2).  Random Gaussian hills."""
    ny = nx if ny is None else ny
    rng = rng_for(seed_id)
    spec = random_hills(rng, n_hills, (nx, ny), sigma)
    wl = Workload("drifting_cellular", "d2q9", (nx, ny), tuple(walls), steps, spec, D=np.asarray(D, np.float64),
                  u_field=drifting_cellular_field(nx, ny, U0, 0.0), meta={"U0": U0, "drift": drift})
    wl.u_schedule = lambda n: drifting_cellular_field(nx, ny, U0, n * drift)
    return wl


class TopHatX:
    """phi0 = 1 on the nodes with lo <= x <= hi, 0 elsewhere, uniform in y."""

    def __init__(self, lo: float, hi: float):
        self.lo, self.hi = float(lo), float(hi)

    def window(self, idx):
        x = np.asarray(idx[0], dtype=np.float64)
        row = ((x >= self.lo) & (x <= self.hi)).astype(np.float64)
        return np.repeat(row[None, :], len(idx[1]), axis=0)


def plate_channel(tau: float, Pe: float, W_lat: int = 32, length: int = 150, name: str = "plate_channel",
                  steps: Optional[int] = None) -> Workload:
    """Taylor-Aris set-up of Sec. 3.2: the gap W is W_lat lattices with the
    plates on the first and last node (ny = W_lat + 1, walls "node"), the
    length L = length * W_lat nodes (periodic), u_x = 4 U y (W - y) / W^2,
    D = alpha I with alpha = (tau - 1/2)/3 (dx = dt = 1 in lattice units),
    U from Pe = 2 U W / (3 alpha), and a top-hat pulse on x in [0.197 L, 0.203 L].

    The default horizon lets the slowest transient that a y-symmetric pulse
    excites, the second plate mode with rate 4 pi^2 alpha / W^2, decay by
    e^-25 (rounded up to 100 steps)."""
    nx, ny = length * W_lat, W_lat + 1
    alpha = (tau - 0.5) / 3.0
    U = 3.0 * alpha * Pe / (2.0 * W_lat)
    y = np.arange(ny, dtype=np.float64)
    prof = 4.0 * y * (W_lat - y) / (W_lat * W_lat)
    wy = np.ones(ny)
    wy[0] = wy[-1] = 0.5
    u_node_mean = float(U * (prof * wy).sum() / wy.sum())
    u_sep = SeparableU(np.array([U, 0.0]), [[np.ones(nx), prof, np.ones(1)], [np.ones(nx), np.zeros(ny), np.ones(1)]])
    lam = 4.0 * math.pi ** 2 * alpha / W_lat ** 2
    horizon = int(math.ceil(25.0 / lam / 100.0)) * 100
    lo, hi = 0.197 * nx, 0.203 * nx
    return Workload(name, "d2q9", (nx, ny), ("periodic", "node"), horizon if steps is None else steps,
                    TopHatX(lo, hi), D=alpha * np.eye(2), u_sep=u_sep,
                    meta={"tau": tau, "Pe": Pe, "W": W_lat, "alpha": alpha, "U": U, "U_node_mean": u_node_mean,
                          "K": alpha * (1.0 + Pe * Pe / 210.0), "x0": 0.5 * (lo + hi), "phi_ref": 0.0})


# ---- inverse problem with a per-node D field ------------------------------

def fourier_field(rng, nx, ny, kmax=3) -> np.ndarray:
    """Smooth random periodic field with |k| <= kmax, min-max normalised to [0, 1]."""
    X, Y = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny)
    field = np.zeros((ny, nx))
    for kx in range(-kmax, kmax + 1):
        for ky in range(0, kmax + 1):
            if kx * kx + ky * ky == 0 or kx * kx + ky * ky > kmax * kmax:
                continue
            if ky == 0 and kx < 0:
                continue
            a, b = rng.standard_normal(2)
            ph = 2.0 * math.pi * (kx * X + ky * Y)
            field += a * np.cos(ph) + b * np.sin(ph)
    lo, hi = field.min(), field.max()
    return (field - lo) / (hi - lo)


def dfield_from(a, b, c, lo=0.01, hi=0.08) -> np.ndarray:
    """D(x) = R(theta) diag(l1, l2) R(theta)^T with l = lo + (hi-lo)*a, theta = pi*c."""
    l1 = lo + (hi - lo) * a
    l2 = lo + (hi - lo) * b
    th = math.pi * c
    cs, sn = np.cos(th), np.sin(th)
    xx = l1 * cs * cs + l2 * sn * sn
    yy = l1 * sn * sn + l2 * cs * cs
    xy = (l1 - l2) * sn * cs
    return np.stack([xx, yy, xy])


def inverse_dfield(n: int = 512, ny: Optional[int] = None, n_ic: int = 10, steps: int = 2000,
                   snap_every: int = 200, ckpt_every: int = 100, u=(0.02, 0.01), sigma0: float = 24.0,
                   seed_id: int = 4) -> dict:
    """Inverse-problem inputs: D_true field, an independent D_pert field, the
    trial point D_trial = D_true + 0.1 (D_pert - D_true) and n_ic hills."""
    nx = n
    ny = n if ny is None else ny
    rng = rng_for(seed_id)
    D_true = dfield_from(*(fourier_field(rng, nx, ny) for _ in range(3)))
    D_pert = dfield_from(*(fourier_field(rng, nx, ny) for _ in range(3)))
    D_trial = D_true + 0.1 * (D_pert - D_true)
    ics = []
    for j in range(n_ic):
        c = rng.uniform(0.0, 1.0, size=2) * np.array([nx, ny], np.float64)
        spec = GaussianSum(c[None, :], np.ones(1), np.array([sigma0]), (float(nx), float(ny)))
        ics.append(Workload(f"inverse_ic{j}", "d2q9", (nx, ny), ("periodic",) * 2, steps, spec,
                            D_field=D_trial, u_const=np.asarray(u, np.float64)))
    fd_nodes = rng.integers(0, [nx, ny], size=(20, 2))
    return {"D_true": D_true, "D_pert": D_pert, "D_trial": D_trial, "ics": ics,
            "snap_every": snap_every, "ckpt_every": ckpt_every, "steps": steps,
            "u": np.asarray(u, np.float64), "fd_nodes": fd_nodes, "shape": (nx, ny)}


def with_background(wl: Workload, level: float) -> Workload:
    """The same workload on a uniform background: phi0 + level."""
    spec = wl.phi0_spec

    class _Shifted(type(spec)):
        def window(self, idx):
            return spec.window(idx) + level

    shifted = _Shifted.__new__(_Shifted)
    shifted.__dict__.update(spec.__dict__)
    return dataclasses.replace(wl, phi0_spec=shifted, meta=dict(wl.meta, background=level))


def with_steps(wl: Workload, steps: int) -> Workload:
    return dataclasses.replace(wl, steps=int(steps))


def patch_index(wl: Workload, centre, half: int):
    """Index vectors of a (2*half+1)^dim window around ``centre`` (wrapped on
    periodic axes).  Used to check single nodes of full-size runs: after n
    steps a node depends only on initial data within distance n."""
    out = []
    for a, c in enumerate(centre):
        idx = np.arange(c - half, c + half + 1)
        out.append(np.mod(idx, wl.shape[a]))
    return out
