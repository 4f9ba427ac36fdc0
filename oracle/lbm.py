"""FP64 CPU oracle of the modified MRT lattice Boltzmann model for the CDE.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import this module.  The product (the HIP
library and its binding) never imports, calls or links it, and shares no
code with it.

What it computes (Huang & Wu, "A modified multiple-relaxation-time lattice
Boltzmann model for convection-diffusion equation"):

* Lattices: D2Q9 with velocities in the order of Eq. (2) and the transform M
  of Eq. (12); D3Q15 with the velocities of Eq. (A.1), ordered as the columns
  of M in Eq. (A.2) require.  M^-1 is the exact inverse of M, obtained with a
  library routine.
* Equilibrium moments: the general form Eq. (15)-(16) (D2Q9) and
  Eq. (A.3)-(A.4) (D3Q15); MRT-A and MRT-B3 use alpha1 = -8, alpha2 = 8
  (Eq. 37); MRT-B1 and MRT-B2 use Eq. (38) and Eq. (39).
* Relaxation matrices: the modified S of Eq. (31) / Eq. (A.5) for MRT-A, the
  standard anisotropic S of Eq. (24) for MRT-B1/B2/B3.
* Parameter map: D = kappa (I - A/2) A^-1 (Eq. 36, A.6; Eq. 29 for the
  unmodified models), inverted as A = (D/kappa + I/2)^-1.
* One time step in push form: collision in moment space Eq. (11), (13),
  (14), then streaming Eq. (5); phi = sum_i f_i (Eq. 8).  Walls sit halfway
  between nodes.  At a "bounce" wall a population that would leave the fluid
  returns to its node with the opposite velocity; at a "specular" wall only
  the normal velocity component reverses (a mirror, the halfway analog of the
  zero-flux rule of Sec. 3.2).
* The discrete adjoint of that step (exact transpose of the linear map) and
  the gradient of a snapshot misfit with respect to a per-node D field.

Readings of points the paper leaves open (each is also listed with the
design notes):
* D3Q15 alpha1, alpha2 are not given; alpha1 = -6/5 and alpha2 = 192 make
  the prefactor of Eq. (A.6) equal 1/3 (as in 2D) and give the equilibrium at
  rest the weights 8/15 (rest) and 1/30 (moving), the 3D analog of the
  paper's 2D choice whose rest weights are 5/9 and 1/18.
* The free rates default to s1 = s2 = 1.1, s7 = s8 = 1.2 (D2Q9, Sec. 3.1),
  and s1 = s2 = 1.1, s9..s14 = 1.2 (D3Q15).  s0 multiplies m0 - m0eq = 0 and
  never matters.
* The rates s4, s6 (s8) that the modified S couples into the flux rows are
  chosen by a rule: "lambda_min" (the smallest eigenvalue of A, default),
  "paper" (s4 = s_xx, s6 = s_yy, s8 = s_zz, Sec. 3.1) or explicit values.
* Initial populations are the equilibrium of phi0 and u.

All arrays are float64.  Populations have shape (Q, *grid) with grid
(ny, nx) or (nz, ny, nx), x fastest.

parity unpinned: nothing in this module is unpinned; every function is
checked by the oracle test suite against closed forms, the paper's
equations or brute force (see tests/test_oracle_*.py).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np

# --------------------------------------------------------------------------
# Lattices
# --------------------------------------------------------------------------

# Eq. (2): e_0 = 0; e_1..4 = axis directions at angles (i-1) pi/2;
# e_5..8 = diagonals at angles (2i-9) pi/4 (length sqrt 2).
def _d2q9_velocities():
    e = [(0, 0)]
    for i in range(1, 5):
        a = (i - 1) * math.pi / 2
        e.append((round(math.cos(a)), round(math.sin(a))))
    for i in range(5, 9):
        a = (2 * i - 9) * math.pi / 4
        e.append((round(math.sqrt(2) * math.cos(a)), round(math.sqrt(2) * math.sin(a))))
    return np.array([(ex, ey, 0) for ex, ey in e], dtype=np.int64)


# Eq. (12)
M_D2Q9 = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)

# Eq. (A.2)
M_D3Q15 = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-2, -1, -1, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1],
    [16, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1],
    [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1],
    [0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1],
    [0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
    [0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1],
    [0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, -1, -1, -1, -1],
    [0, 0, 0, 0, 0, -4, 4, 1, 1, 1, 1, -1, -1, -1, -1],
    [0, 2, 2, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1],
    [0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1],
    [0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1],
    [0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1],
], dtype=np.float64)


def _d3q15_velocities():
    # Eq. (A.1) gives the set; the order is the one in which rows 3, 5 and 7
    # of Eq. (A.2) (the x, y and z fluxes) read off the velocity components.
    e = np.stack([M_D3Q15[3], M_D3Q15[5], M_D3Q15[7]], axis=1).astype(np.int64)
    return e


class Lattice:
    """Velocity set, transform and equilibrium constants of one lattice."""

    def __init__(self, name: str):
        self.name = name
        if name == "d2q9":
            self.e = _d2q9_velocities()
            self.M = M_D2Q9.copy()
            self.dim = 2
            # Sec. 3 (Eq. 37): alpha1 = -8, alpha2 = 8; Eq. (16): c1 = 1, c1 + c2/2 = 0
            self.alpha1, self.alpha2 = -8.0, 8.0
            self.c1 = 1.0
            self.c2 = -2.0 * self.c1
            self.flux_rows = (3, 5)        # m3 = j_x, m5 = j_y
            self.heat_rows = (4, 6)        # m4 = q_x, m6 = q_y
        elif name == "d3q15":
            self.e = _d3q15_velocities()
            self.M = M_D3Q15.copy()
            self.dim = 3
            # alpha1, alpha2: reading (not given by the paper); Eq. (A.4): c1 + c2/4 = 0
            self.alpha1, self.alpha2 = -6.0 / 5.0, 192.0
            self.c1 = 1.0
            self.c2 = -4.0 * self.c1
            self.flux_rows = (3, 5, 7)
            self.heat_rows = (4, 6, 8)
        else:
            raise ValueError(name)
        self.Q = self.M.shape[0]
        self.Minv = np.linalg.inv(self.M)
        self.opp = np.array([int(np.where((self.e == -self.e[i]).all(1))[0][0]) for i in range(self.Q)])

    def kappa(self, modified: bool = True) -> float:
        """Prefactor of (I - A/2) A^-1 in the diffusion tensor.

        D2Q9 modified (Eq. 36): 2/3 + alpha1/8 + alpha2/12.
        D2Q9 unmodified (Eq. 29): 2/3 + alpha1/24.
        D3Q15 modified (Eq. A.6): 2/3 + 55 alpha1/54 + alpha2/216.
        """
        a1, a2 = self.alpha1, self.alpha2
        if self.name == "d2q9":
            return 2.0 / 3.0 + a1 / 8.0 + a2 / 12.0 if modified else 2.0 / 3.0 + a1 / 24.0
        if not modified:
            raise ValueError("the unmodified D3Q15 model is not defined by the paper")
        return 2.0 / 3.0 + 55.0 * a1 / 54.0 + a2 / 216.0


D2Q9 = Lattice("d2q9")
D3Q15 = Lattice("d3q15")


def get_lattice(name: str) -> Lattice:
    return {"d2q9": D2Q9, "d3q15": D3Q15}[name]


# --------------------------------------------------------------------------
# Models: equilibrium moments and relaxation matrices
# --------------------------------------------------------------------------

MODELS = ("A", "B1", "B2", "B3")


def equilibrium_moments(lat: Lattice, model: str, phi: np.ndarray, u: np.ndarray) -> np.ndarray:
    """m^eq(phi, u) with shape (Q, *grid).  ``u`` has shape (dim, *grid)."""
    phi = np.asarray(phi, np.float64)
    meq = np.zeros((lat.Q,) + phi.shape)
    if lat.name == "d2q9":
        ux, uy = u[0], u[1]
        if model in ("A", "B3"):
            # Eq. (15): (phi, a1 phi/4, a2 phi/4, c1 phi ux, c2 phi ux/2, c1 phi uy, c2 phi uy/2, 0, 0)
            meq[0] = phi
            meq[1] = lat.alpha1 * phi / 4.0
            meq[2] = lat.alpha2 * phi / 4.0
            meq[3] = lat.c1 * phi * ux
            meq[4] = lat.c2 * phi * ux / 2.0
            meq[5] = lat.c1 * phi * uy
            meq[6] = lat.c2 * phi * uy / 2.0
        elif model in ("B1", "B2"):
            uu = ux * ux + uy * uy
            meq[0] = phi
            meq[1] = phi * (-2.0 + 3.0 * uu)                       # Eq. (38), (39)
            meq[2] = phi * ((1.0 if model == "B1" else 2.0) - 3.0 * uu)
            meq[3] = phi * ux
            meq[4] = -phi * ux
            meq[5] = phi * uy
            meq[6] = -phi * uy
            meq[7] = phi * (ux * ux - uy * uy)
            meq[8] = phi * ux * uy
        else:
            raise ValueError(model)
        return meq
    if model not in ("A",):
        raise ValueError("D3Q15 is defined for the modified model only")
    # Eq. (A.3): (phi, 5 a1 phi/6, a2 phi/24, c1 phi u_a, c2 phi u_a/4 for a = x, y, z, 0 x 6)
    meq[0] = phi
    meq[1] = 5.0 * lat.alpha1 * phi / 6.0
    meq[2] = lat.alpha2 * phi / 24.0
    for a, (r_flux, r_heat) in enumerate(zip(lat.flux_rows, lat.heat_rows)):
        meq[r_flux] = lat.c1 * phi * u[a]
        meq[r_heat] = lat.c2 * phi * u[a] / 4.0
    return meq


def default_rates(lat: Lattice) -> np.ndarray:
    """Diagonal rates s_0..s_{Q-1}; entries on the flux rows are unused (A)."""
    s = np.zeros(lat.Q)
    s[0] = 1.0
    s[1] = s[2] = 1.1
    if lat.name == "d2q9":
        s[7] = s[8] = 1.2
    else:
        s[9:15] = 1.2
    return s


def flux_matrix(D: np.ndarray, kappa: float) -> np.ndarray:
    """A from D = kappa (I - A/2) A^-1, i.e. A = (D/kappa + I/2)^-1 (Eq. 36, A.6).

    ``D`` may be (dim, dim) or (*grid, dim, dim)."""
    D = np.asarray(D, np.float64)
    eye = np.eye(D.shape[-1])
    return np.linalg.inv(D / kappa + 0.5 * eye)


def coupled_rates(A: np.ndarray, rule="lambda_min") -> np.ndarray:
    """Rates s4, s6 (, s8) of the heat-flux moments, per the chosen rule.

    ``rule`` is "lambda_min", "paper", or an explicit sequence of values."""
    A = np.asarray(A, np.float64)
    dim = A.shape[-1]
    if isinstance(rule, str):
        if rule == "lambda_min":
            lam = np.linalg.eigvalsh(A)[..., 0]
            return np.repeat(lam[..., None], dim, axis=-1)
        if rule == "paper":
            return np.stack([A[..., a, a] for a in range(dim)], axis=-1)
        raise ValueError(rule)
    vals = np.asarray(rule, np.float64)
    return np.broadcast_to(vals, A.shape[:-2] + (dim,)).copy()


def relaxation_matrix(lat: Lattice, A: np.ndarray, rates: np.ndarray, heat: np.ndarray,
                      modified: bool = True) -> np.ndarray:
    """S of Eq. (31)/(A.5) (modified) or Eq. (24) (standard), shape (*grid, Q, Q).

    ``A`` is (*grid, dim, dim); ``rates`` the diagonal rates (Q,); ``heat`` the
    rates of the heat-flux moments (*grid, dim) (s4, s6[, s8])."""
    A = np.asarray(A, np.float64)
    batch = A.shape[:-2]
    S = np.zeros(batch + (lat.Q, lat.Q))
    for k in range(lat.Q):
        if k not in lat.flux_rows:
            S[..., k, k] = rates[k]
    for a, ra in enumerate(lat.heat_rows):
        S[..., ra, ra] = heat[..., a]
    for a, ra in enumerate(lat.flux_rows):
        for b, rb in enumerate(lat.flux_rows):
            S[..., ra, rb] = A[..., a, b]
            if modified:
                hb = lat.heat_rows[b]
                if a == b:
                    S[..., ra, hb] = (A[..., a, b] / 2.0 - 1.0) * heat[..., b]
                else:
                    S[..., ra, hb] = (A[..., a, b] / 2.0) * heat[..., b]
    return S


def relaxation_matrix_derivative(lat: Lattice, dA: np.ndarray, heat: np.ndarray,
                                 modified: bool = True) -> np.ndarray:
    """dS for a change dA of A at fixed heat-flux rates (Eq. 31 differentiated)."""
    dA = np.asarray(dA, np.float64)
    batch = dA.shape[:-2]
    dS = np.zeros(batch + (lat.Q, lat.Q))
    for a, ra in enumerate(lat.flux_rows):
        for b, rb in enumerate(lat.flux_rows):
            dS[..., ra, rb] = dA[..., a, b]
            if modified:
                dS[..., ra, lat.heat_rows[b]] = dA[..., a, b] / 2.0 * heat[..., b]
    return dS


def components_to_tensor(comps: np.ndarray) -> np.ndarray:
    """(ncomp, *grid) components (xx, yy, xy) | (xx, yy, zz, xy, xz, yz) -> (*grid, dim, dim)."""
    comps = np.asarray(comps, np.float64)
    if comps.shape[0] == 3:
        xx, yy, xy = comps
        return np.stack([np.stack([xx, xy], -1), np.stack([xy, yy], -1)], -2)
    xx, yy, zz, xy, xz, yz = comps
    return np.stack([np.stack([xx, xy, xz], -1), np.stack([xy, yy, yz], -1),
                     np.stack([xz, yz, zz], -1)], -2)


def component_unit(dim: int, c: int) -> np.ndarray:
    """Symmetric unit tensor of component c (xx, yy, xy) | (xx, yy, zz, xy, xz, yz)."""
    E = np.zeros((dim, dim))
    pairs = [(0, 0), (1, 1), (0, 1)] if dim == 2 else [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    i, j = pairs[c]
    E[i, j] = E[j, i] = 1.0
    return E


# --------------------------------------------------------------------------
# Problem, collision, streaming
# --------------------------------------------------------------------------

class Problem:
    """A grid with its boundaries, flow, diffusion and model choice.

    Parameters
    ----------
    lattice : "d2q9" | "d3q15"
    shape   : (nx, ny) or (nx, ny, nz)
    walls   : per axis "periodic", "bounce" (halfway bounce-back, True),
              "specular" (halfway mirror) or "node" (the plate rule of
              Sec. 3.2, with the first and last node on the plates) on both faces
    u       : (dim, *grid) velocity at the nodes (steady)
    D       : constant (dim, dim) tensor, or per-node components (ncomp, *grid)
    model   : "A" (modified, the paper's method) or "B1" | "B2" | "B3"
    heat_rule : rule for s4, s6 (, s8), see ``coupled_rates``
    rates   : diagonal rates (Q,), default ``default_rates``
    """

    def __init__(self, lattice: str, shape: Sequence[int], walls: Sequence[bool], u: np.ndarray,
                 D: np.ndarray, model: str = "A", heat_rule="lambda_min",
                 rates: Optional[np.ndarray] = None):
        self.lat = get_lattice(lattice)
        self.shape = tuple(int(n) for n in shape)
        self.grid = tuple(reversed(self.shape))
        self.walls = tuple(_wall_kind(w) for w in walls)
        self.model = model
        self.modified = model == "A"
        self.u = np.asarray(u, np.float64).reshape((self.lat.dim,) + self.grid)
        D = np.asarray(D, np.float64)
        self.per_node = D.ndim > 2
        self.D = components_to_tensor(D) if self.per_node else D
        self.kappa = self.lat.kappa(self.modified)
        self.A = flux_matrix(self.D, self.kappa)
        self.heat_rule = heat_rule
        self.heat = coupled_rates(self.A, heat_rule)
        self.rates = default_rates(self.lat) if rates is None else np.asarray(rates, np.float64)
        self.S = relaxation_matrix(self.lat, self.A, self.rates, self.heat, self.modified)
        # equilibrium moments per unit phi (m^eq is linear in phi for fixed u)
        self.E = equilibrium_moments(self.lat, model, np.ones(self.grid), self.u)
        self.node_axes = [a for a, w in enumerate(self.walls) if w == "node"]
        if self.node_axes and (self.lat.name != "d2q9" or len(self.node_axes) != 1
                               or any(w != "periodic" for a, w in enumerate(self.walls) if a not in self.node_axes)):
            raise ValueError("the plate rule is defined for D2Q9 with one plate axis and the other periodic")
        self._dest = [self._destinations(i) for i in range(self.lat.Q)]

    # -- helpers -------------------------------------------------------------
    def _destinations(self, i: int):
        """Where streaming sends population i of every node: (population, node) arrays.

        Periodic axes wrap.  If x + e_i leaves the fluid across a wall:
        "bounce" reverses the whole velocity and keeps the node (halfway
        bounce-back); "specular" reverses only the normal component and keeps
        the normal coordinate, moving on along the wall (halfway mirror);
        "node" drops the population (population -1), its replacement is set
        by ``stream`` from the plate rule."""
        dim = self.lat.dim
        coords = np.meshgrid(*[np.arange(n) for n in self.shape], indexing="ij")   # axis order x, y[, z]
        coords = [c.transpose(tuple(reversed(range(dim)))) for c in coords]        # to grid order
        e = self.lat.e[i, :dim]
        crossed = {k: np.zeros(self.grid, dtype=bool) for k in ("bounce", "specular", "node")}
        per_axis_cross = []
        for a in range(dim):
            raw = coords[a] + e[a]
            out = (raw < 0) | (raw >= self.shape[a])
            if self.walls[a] == "periodic":
                out = np.zeros_like(out)
            else:
                crossed[self.walls[a]] |= out
            per_axis_cross.append(out)
        bounce = crossed["bounce"]
        dest_c, vel = [], []
        for a in range(dim):
            moved = np.mod(coords[a] + e[a], self.shape[a])
            stay = per_axis_cross[a] | bounce
            dest_c.append(np.where(stay, coords[a], moved))
            va = np.where(bounce, -e[a], np.where(per_axis_cross[a], -e[a], e[a]))
            vel.append(va)
        node = np.zeros(self.grid, dtype=np.int64)
        stride = 1
        for a in range(dim):
            node += dest_c[a] * stride
            stride *= self.shape[a]
        vel = np.stack(vel, -1)
        # population index of each velocity vector: a table over the 3^dim
        # vectors with components in {-1, 0, 1}, indexed by sum_a (v_a + 1) 3^a
        code = lambda v: sum((np.asarray(v[..., a]) + 1) * 3 ** a for a in range(dim))
        table = np.full(3 ** dim, -1, dtype=np.int64)
        table[code(self.lat.e[:, :dim])] = np.arange(self.lat.Q)
        pop = table[code(vel)]
        pop = np.where(crossed["node"], -1, pop)
        return np.asarray(pop, dtype=np.int64).ravel(), node.ravel()

    def _roll(self, arr: np.ndarray, e: np.ndarray, sign: int) -> np.ndarray:
        shifts = tuple(int(sign * e[a]) for a in reversed(range(self.lat.dim)))
        return np.roll(arr, shifts, axis=tuple(range(self.lat.dim)))

    def _apply_S(self, n: np.ndarray, transpose: bool = False) -> np.ndarray:
        S = np.swapaxes(self.S, -1, -2) if transpose else self.S
        if S.ndim == 2:
            return np.tensordot(S, n, axes=(1, 0))
        return np.moveaxis(np.einsum("...ij,...j->...i", S, np.moveaxis(n, 0, -1)), -1, 0)

    # -- the method ----------------------------------------------------------
    def equilibrium(self, phi: np.ndarray) -> np.ndarray:
        """f^eq = M^-1 m^eq(phi, u) (the velocity-space form is Eq. 17)."""
        meq = equilibrium_moments(self.lat, self.model, phi, self.u)
        return np.tensordot(self.lat.Minv, meq, axes=(1, 0))

    def collide(self, f: np.ndarray) -> np.ndarray:
        """Eq. (11), (13), (14): m = M f; m' = m - S (m - m^eq); f' = M^-1 m'."""
        phi = f.sum(axis=0)                                        # Eq. (8)
        m = np.tensordot(self.lat.M, f, axes=(1, 0))               # Eq. (11)
        meq = equilibrium_moments(self.lat, self.model, phi, self.u)
        m_post = m - self._apply_S(m - meq)                        # Eq. (13)
        return np.tensordot(self.lat.Minv, m_post, axes=(1, 0))    # Eq. (14)

    def stream(self, fpost: np.ndarray) -> np.ndarray:
        """Eq. (5) push: f_i(x + e_i) = f'_i(x), with the wall rule where x + e_i is solid.

        On a "node" axis (Sec. 3.2) populations leaving the domain are lost,
        and at the plate nodes each population pointing into the fluid is
        then set to its mirror image (normal component reversed) at the same
        node: f2 = f4, f5 = f8, f6 = f7 on the low plate, the reverse on the
        high one."""
        out = np.zeros_like(fpost).reshape(self.lat.Q, -1)
        for i in range(self.lat.Q):
            pop, node = self._dest[i]
            keep = pop >= 0
            out[pop[keep], node[keep]] = fpost[i].ravel()[keep]
        out = out.reshape(fpost.shape)
        for a in self.node_axes:
            ax = self.lat.dim - 1 - a                      # grid axis of coordinate a
            for i in range(self.lat.Q):
                ea = self.lat.e[i, a]
                if ea == 0:
                    continue
                v = self.lat.e[i, :self.lat.dim].copy()
                v[a] = -ea
                j = int(np.where((self.lat.e[:, :self.lat.dim] == v).all(1))[0][0])
                plate = 0 if ea > 0 else self.shape[a] - 1
                sl = [slice(None)] * self.lat.dim
                sl[ax] = plate
                out[(i,) + tuple(sl)] = out[(j,) + tuple(sl)]
        return out

    def step(self, f: np.ndarray) -> np.ndarray:
        return self.stream(self.collide(f))

    def run(self, f: np.ndarray, steps: int, snap_every: int = 0):
        """Advance ``steps`` steps; returns (f, [phi snapshots every snap_every])."""
        snaps = []
        for t in range(1, steps + 1):
            f = self.step(f)
            if snap_every and t % snap_every == 0:
                snaps.append(phi_of(f))
        return f, snaps

    # -- the discrete adjoint --------------------------------------------------
    def collide_T(self, lam: np.ndarray) -> np.ndarray:
        """Transpose of the per-node collision map C = I - M^-1 S (M - E 1^T)."""
        w = np.tensordot(self.lat.Minv.T, lam, axes=(1, 0))
        z = self._apply_S(w, transpose=True)
        out = lam - np.tensordot(self.lat.M.T, z, axes=(1, 0))
        return out + (self.E * z).sum(axis=0)[None]

    def stream_T(self, lam: np.ndarray) -> np.ndarray:
        """Transpose of ``stream`` (a permutation): (P^T lam)_i(x) = lam at the destination of (i, x)."""
        if self.node_axes:
            raise ValueError("no adjoint is defined for the plate rule")
        flat = lam.reshape(self.lat.Q, -1)
        out = np.empty_like(flat)
        for i in range(self.lat.Q):
            pop, node = self._dest[i]
            out[i] = flat[pop, node]
        return out.reshape(lam.shape)

    def grad_D_step(self, lam_pre: np.ndarray, f: np.ndarray) -> np.ndarray:
        """Per-node d/dD_c of <lam_pre, C(D) f> with lam_pre = P^T lam_{t+1}.

        dC f = -M^-1 dS n with n = M f - m^eq(phi); dA = -A (dD/kappa) A."""
        dim = self.lat.dim
        phi = f.sum(axis=0)
        n = np.tensordot(self.lat.M, f, axes=(1, 0)) - equilibrium_moments(self.lat, self.model, phi, self.u)
        ell = np.tensordot(self.lat.Minv.T, lam_pre, axes=(1, 0))      # M^-T lam
        ncomp = 3 if dim == 2 else 6
        out = np.zeros((ncomp,) + self.grid)
        A = self.A if self.per_node else np.broadcast_to(self.A, self.grid + (dim, dim))
        heat = self.heat if self.heat.ndim > 1 else np.broadcast_to(self.heat, self.grid + (dim,))
        for c in range(ncomp):
            dA = -A @ (component_unit(dim, c) / self.kappa) @ A
            dS = relaxation_matrix_derivative(self.lat, dA, heat, self.modified)
            dSn = np.moveaxis(np.einsum("...ij,...j->...i", dS, np.moveaxis(n, 0, -1)), -1, 0)
            out[c] = -(ell * dSn).sum(axis=0)
        return out


def _wall_kind(w) -> str:
    """Boundary of one axis: "periodic", "bounce" (True), "specular" or "node"."""
    if w is True or w == 1:
        return "bounce"
    if w is False or w == 0 or w is None:
        return "periodic"
    if w in ("periodic", "bounce", "specular", "node"):
        return w
    raise ValueError(f"unknown wall kind {w!r}")


def phi_of(f: np.ndarray) -> np.ndarray:
    """Eq. (8)."""
    return f.sum(axis=0)


# --------------------------------------------------------------------------
# Snapshot misfit and its gradient
# --------------------------------------------------------------------------

def misfit(prob: Problem, phi0: np.ndarray, phi_obs: Sequence[np.ndarray], snap_every: int) -> float:
    """J = 1/2 sum_snap sum_x (phi_t - phi_obs)^2 with snapshots every snap_every steps."""
    f = prob.equilibrium(phi0)
    _, snaps = prob.run(f, snap_every * len(phi_obs), snap_every)
    return 0.5 * math.fsum(float(((s - o) ** 2).sum()) for s, o in zip(snaps, phi_obs))


def misfit_gradient(prob: Problem, phi0: np.ndarray, phi_obs: Sequence[np.ndarray], snap_every: int,
                    ckpt_every: int = 0, return_dphi0: bool = False):
    """(J, dJ/dD_field[, dJ/dphi0]) by the discrete adjoint of the push step.

    Forward: f_{t+1} = P C f_t.  Adjoint: lam_T = dJ/df_T,
    lam_t = C^T P^T lam_{t+1} + dJ/df_t, and
    dJ/dD = sum_t d<P^T lam_{t+1}, C(D) f_t>/dD.
    The forward states are stored (or recomputed from checkpoints every
    ``ckpt_every`` steps when that is set).  dJ/dphi0 follows from lam_0
    through f_0 = f_eq(phi0, u), which is linear in phi0."""
    if isinstance(prob.heat_rule, str):
        raise ValueError("the D-gradient holds for heat-flux rates that do not depend on D: "
                         "give explicit values")
    T = snap_every * len(phi_obs)
    every = ckpt_every if ckpt_every else T
    ckpts = {0: prob.equilibrium(phi0)}
    f = ckpts[0]
    J_terms = []
    for t in range(1, T + 1):
        f = prob.step(f)
        if t % snap_every == 0:
            J_terms.append(0.5 * float(((phi_of(f) - phi_obs[t // snap_every - 1]) ** 2).sum()))
        if t % every == 0 and t < T:
            ckpts[t] = f
    J = math.fsum(J_terms)
    ncomp = 3 if prob.lat.dim == 2 else 6
    grad = np.zeros((ncomp,) + prob.grid)
    lam = np.zeros((prob.lat.Q,) + prob.grid)
    for seg_start in sorted(ckpts, reverse=True):
        seg_end = min(seg_start + every, T)
        states = [ckpts[seg_start]]
        for _ in range(seg_start, seg_end - 1):
            states.append(prob.step(states[-1]))
        for t in range(seg_end, seg_start, -1):
            # dJ/df_t at snapshot times (every population of a node carries phi)
            if t % snap_every == 0:
                lam = lam + (phi_of(prob.step(states[t - 1 - seg_start])) - phi_obs[t // snap_every - 1])[None]
            lam_pre = prob.stream_T(lam)
            grad += prob.grad_D_step(lam_pre, states[t - 1 - seg_start])
            lam = prob.collide_T(lam_pre)
    if return_dphi0:
        return J, grad, (lam * prob.equilibrium(np.ones(prob.grid))).sum(axis=0)
    return J, grad


# --------------------------------------------------------------------------
# Reductions (Eq. 46-47) and error norms (Eq. 43, 45)
# --------------------------------------------------------------------------

def mass(phi: np.ndarray) -> float:
    return math.fsum(np.asarray(phi, np.float64).ravel().tolist())


def x_moments(phi: np.ndarray, x_ref: float):
    """(S0, S1, S2) of the cross-section sum phibar(x) = sum over the other axes,
    with x measured as the minimum image of x - x_ref on the periodic x axis."""
    phi = np.asarray(phi, np.float64)
    nx = phi.shape[-1]
    pbar = phi.reshape(-1, nx).sum(axis=0)
    d = np.arange(nx, dtype=np.float64) - x_ref
    d = d - nx * np.floor(d / nx + 0.5)
    return (math.fsum(pbar.tolist()), math.fsum((d * pbar).tolist()), math.fsum((d * d * pbar).tolist()))


def channel_transfer(prob: Problem) -> dict:
    """The oracle's step (Eq. 10-14, then Eq. 5 with the wall rule) on a
    channel that is periodic in x and uniform along it, split by x offset:
    T[dx] (shape (Q ny, Q ny), index i * ny + y) maps the populations of one
    column to their contribution dx columns further on.  ``prob`` has three
    columns (nx = 3) holding the channel's cross-section (walls, velocity
    profile, rates); unit populations are placed in the middle column and
    stepped, and since a population moves at most one column per step the
    three output columns are the three offsets."""
    if prob.shape[0] != 3 or prob.walls[0] != "periodic" or prob.lat.dim != 2:
        raise ValueError("a D2Q9 channel problem with nx = 3 and periodic x is needed")
    Q, ny = prob.lat.Q, prob.shape[1]
    n = Q * ny
    T = {dx: np.zeros((n, n)) for dx in (-1, 0, 1)}
    for j in range(Q):
        for y in range(ny):
            f = np.zeros((Q, ny, 3))
            f[j, y, 1] = 1.0
            g = prob.step(f)
            for dx in (-1, 0, 1):
                T[dx][:, j * ny + y] = g[:, :, 1 + dx].reshape(n)
    return T


def channel_step_symbol(prob: Problem, k: float) -> np.ndarray:
    """One step of the oracle on the Fourier mode exp(i k x) of a channel:
    a population field v(i, y) exp(i k x) becomes (G v)(i, y) exp(i k x)
    with G = sum over dx of T[dx] exp(-i k dx) (``channel_transfer``)."""
    T = channel_transfer(prob)
    return sum(np.exp(-1j * k * dx) * T[dx] for dx in (-1, 0, 1))


def channel_moment_history(prob: Problem, weights: np.ndarray, steps: int, every: int, drift: float = 0.0):
    """Exact x-moments of a pulse released at one cross-section of an
    unbounded channel (Sec. 3.2): the response to f(x, 0) = delta(x) e0(i, y)
    with e0 the equilibrium of phi = 1 at the local velocity (Eq. 17).

    With P_t, Q_t, R_t the population fields summed over x with weights
    1, x - c t, (x - c t)^2 (c = ``drift``), one step maps
        P -> sum T[dx] P,
        Q -> sum T[dx] (Q + (dx - c) P),
        R -> sum T[dx] (R + 2 (dx - c) Q + (dx - c)^2 P)
    (``channel_transfer``), and S_m = sum over i, y of weights[y] times the
    field.  A pulse of any x-profile that is uniform across the gap has
    these cumulants plus its own, so variance increments (Eq. 46-47) do not
    depend on it.  Returns (t, S0, S1, S2) sampled every ``every`` steps."""
    T = channel_transfer(prob)
    Q, ny = prob.lat.Q, prob.shape[1]
    phi1 = np.ones((ny, 3))
    e0 = prob.equilibrium(phi1)[:, :, 1].reshape(Q * ny)
    wv = np.tile(np.asarray(weights, np.float64), Q)
    P, Qm, R = e0.copy(), np.zeros_like(e0), np.zeros_like(e0)
    ts, out = [], []
    for t in range(1, steps + 1):
        nP, nQ, nR = np.zeros_like(P), np.zeros_like(P), np.zeros_like(P)
        for dx in (-1, 0, 1):
            a = dx - drift
            nP += T[dx] @ P
            nQ += T[dx] @ (Qm + a * P)
            nR += T[dx] @ (R + 2.0 * a * Qm + a * a * P)
        P, Qm, R = nP, nQ, nR
        if t % every == 0:
            ts.append(t)
            out.append((wv @ P, wv @ Qm, wv @ R))
    out = np.array(out)
    return np.array(ts), out[:, 0], out[:, 1], out[:, 2]


def channel_dispersion(prob: Problem, k: float = 1e-3):
    """Asymptotic longitudinal dispersion coefficient and drift of the
    scheme in a channel (Sec. 3.2, Eq. 46-47).  The cross-section sum of phi
    of a mode exp(i k x) decays and travels with the eigenvalue lambda(k) of
    ``channel_step_symbol`` nearest to 1, log lambda(k) = -i U k - K k^2 +
    O(k^3), and the variance of a pulse grows at 2 K for long times (the
    rate that Eq. 46-47 measure).  Returns (K, U), K from Richardson
    extrapolation of -Re log lambda / k^2 at k and 2k."""
    def at(kk):
        ev = np.linalg.eigvals(channel_step_symbol(prob, kk))
        lg = np.log(ev[np.argmax(ev.real)])
        return -lg.real / kk ** 2, -lg.imag / kk
    (K1, U1), (K2, U2) = at(k), at(2 * k)
    return (4.0 * K1 - K2) / 3.0, (4.0 * U1 - U2) / 3.0


def variance_from_moments(S0, S1, S2) -> float:
    """Eq. (47)."""
    return S2 / S0 - (S1 / S0) ** 2


def err2(num, ana) -> float:
    """Eq. (43) average error."""
    return float(np.sqrt(np.mean((np.asarray(num) - np.asarray(ana)) ** 2)))


def err_inf(num, ana) -> float:
    """Eq. (43) maximum error."""
    return float(np.max(np.abs(np.asarray(num) - np.asarray(ana))))


def err_rel(num, ana) -> float:
    """Eq. (45)."""
    num, ana = np.asarray(num), np.asarray(ana)
    return float(np.sqrt(((num - ana) ** 2).sum()) / np.sqrt((ana ** 2).sum()))


# --------------------------------------------------------------------------
# Convenience: problems from workloads
# --------------------------------------------------------------------------

def problem_for(wl, idx=None, model: str = "A", heat_rule="lambda_min", rates=None) -> Problem:
    """Oracle problem of a workload (optionally restricted to a periodic window)."""
    if idx is None:
        shape, walls = wl.shape, wl.walls
    else:
        shape, walls = tuple(len(i) for i in idx), wl.walls
    D = wl.D_window(idx) if wl.D_field is not None else wl.D
    return Problem(wl.lattice, shape, walls, wl.u(idx), D, model=model, heat_rule=heat_rule, rates=rates)


def run_workload(wl, steps: Optional[int] = None, idx=None, snap_every: int = 0, **kw):
    """phi after ``steps`` steps (default wl.steps), plus snapshots."""
    prob = problem_for(wl, idx, **kw)
    f = prob.equilibrium(wl.phi0(idx))
    f, snaps = prob.run(f, wl.steps if steps is None else steps, snap_every)
    return phi_of(f), snaps
