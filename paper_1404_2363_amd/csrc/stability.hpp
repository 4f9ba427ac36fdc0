// Host-side linear (von Neumann) stability scan of a run with constant D and u.
//
// The step is linear and translation invariant for constant D and u, so a
// Fourier mode exp(i k.x) of the populations is multiplied each step by
//   G(k) = diag(exp(-i k.e_j)) C,   C = I - M^-1 S (M - E 1^T),
// C the per-node collision of Eq. (10)-(14) with m_eq = phi E (Eq. 37, 38, 39
// or A.3-A.4) and S of Eq. (31) / (A.5) or Eq. (24).  A run is linearly
// stable if the spectral radius of G(k) is at most 1 for every k.  The scan
// samples k on an n^dim grid of [0, 2 pi)^dim (half of it: G(-k) is the
// complex conjugate of G(k)) and bounds each spectral radius from above by
// Gelfand's formula, rho = lim ||G^m||^(1/m), with m = 2^24 reached by
// repeated squaring of the normalised matrix (Frobenius norm).  The bound
// exceeds rho by at most log(c)/m for the constant c of ||G^m|| <= c rho^m,
// about 1e-6 for c as large as 1e7.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

#include "../../include/lbm_cde.h"

namespace lbm {
namespace stability {

using cplx = std::complex<double>;

struct LatticeTables {
  int Q = 9, dim = 2;
  int e[15][3] = {{0}};
  double M[15][15] = {{0}};
};

// Velocities in the order of the kernels and the rows of M as polynomials of
// e (Eq. 12 for D2Q9, Eq. A.2 for D3Q15).
inline LatticeTables tables(int lattice) {
  LatticeTables t;
  if (lattice == LBM_CDE_D2Q9) {
    const int e[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    t.Q = 9;
    t.dim = 2;
    for (int j = 0; j < 9; ++j) {
      const double ex = e[j][0], ey = e[j][1], e2 = ex * ex + ey * ey;
      t.e[j][0] = e[j][0];
      t.e[j][1] = e[j][1];
      const double row[9] = {1.0, -4.0 + 3.0 * e2, 4.0 - 10.5 * e2 + 4.5 * e2 * e2, ex, (-5.0 + 3.0 * e2) * ex, ey,
                             (-5.0 + 3.0 * e2) * ey, ex * ex - ey * ey, ex * ey};
      for (int k = 0; k < 9; ++k) t.M[k][j] = row[k];
    }
    return t;
  }
  const int e[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                        {0, 0, 1},  {0, 0, -1}, {1, 1, 1},  {-1, 1, 1},  {1, -1, 1},
                        {-1, -1, 1}, {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};
  t.Q = 15;
  t.dim = 3;
  for (int j = 0; j < 15; ++j) {
    const double ex = e[j][0], ey = e[j][1], ez = e[j][2], e2 = ex * ex + ey * ey + ez * ez;
    for (int a = 0; a < 3; ++a) t.e[j][a] = e[j][a];
    const double q = 0.5 * (5.0 * e2 - 13.0);
    const double row[15] = {1.0,         e2 - 2.0, 0.5 * (15.0 * e2 * e2 - 55.0 * e2 + 32.0),
                            ex,          q * ex,   ey,
                            q * ey,      ez,       q * ez,
                            3.0 * ex * ex - e2, ey * ey - ez * ez, ex * ey,
                            ey * ez,     ex * ez,  ex * ey * ez};
    for (int k = 0; k < 15; ++k) t.M[k][j] = row[k];
  }
  return t;
}

// Equilibrium moments per unit phi at velocity u for the model.
inline void equilibrium_moments(int lattice, int model, const double u[3], double* E) {
  if (lattice == LBM_CDE_D2Q9) {
    const bool nl = model == LBM_CDE_MRT_B1 || model == LBM_CDE_MRT_B2;
    const double u2 = u[0] * u[0] + u[1] * u[1];
    E[0] = 1.0;
    E[1] = nl ? -2.0 + 3.0 * u2 : -2.0;
    E[2] = (model == LBM_CDE_MRT_B1 ? 1.0 : 2.0) - (nl ? 3.0 * u2 : 0.0);
    E[3] = u[0];
    E[4] = -u[0];
    E[5] = u[1];
    E[6] = -u[1];
    E[7] = nl ? u[0] * u[0] - u[1] * u[1] : 0.0;
    E[8] = nl ? u[0] * u[1] : 0.0;
    return;
  }
  for (int k = 0; k < 15; ++k) E[k] = 0.0;
  E[0] = 1.0;
  E[1] = -1.0;
  E[2] = 8.0;
  E[3] = u[0];
  E[4] = -u[0];
  E[5] = u[1];
  E[6] = -u[1];
  E[7] = u[2];
  E[8] = -u[2];
}

// C = I - M^-1 S (M - E 1^T), M^-1 = M^T diag(1/|M_k|^2) (the rows of M are
// orthogonal).  S is row-major Q x Q.
inline void collision_matrix(const LatticeTables& t, const double* S, const double* E, double* C) {
  const int Q = t.Q;
  double n2[15];
  for (int k = 0; k < Q; ++k) {
    n2[k] = 0.0;
    for (int j = 0; j < Q; ++j) n2[k] += t.M[k][j] * t.M[k][j];
  }
  // B = S (M - E 1^T)
  std::vector<double> B(Q * Q, 0.0);
  for (int k = 0; k < Q; ++k)
    for (int j = 0; j < Q; ++j) {
      double s = 0.0;
      for (int l = 0; l < Q; ++l) s += S[k * Q + l] * (t.M[l][j] - E[l]);
      B[k * Q + j] = s;
    }
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      double s = 0.0;
      for (int k = 0; k < Q; ++k) s += t.M[k][i] / n2[k] * B[k * Q + j];
      C[i * Q + j] = (i == j ? 1.0 : 0.0) - s;
    }
}

// Upper bound of the spectral radius of the Q x Q matrix G (destroyed).
inline double gelfand_bound(std::vector<cplx>& G, int Q, int squarings = 24) {
  std::vector<cplx> T(Q * Q);
  double logn = 0.0;
  auto normalise = [&](std::vector<cplx>& A) -> double {
    double f = 0.0;
    for (const cplx& v : A) f += std::norm(v);
    f = std::sqrt(f);
    if (!(f > 0.0)) return -INFINITY;
    for (cplx& v : A) v /= f;
    return std::log(f);
  };
  logn = normalise(G);
  if (logn == -INFINITY) return 0.0;
  for (int s = 0; s < squarings; ++s) {
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        cplx acc = 0.0;
        for (int l = 0; l < Q; ++l) acc += G[i * Q + l] * G[l * Q + j];
        T[i * Q + j] = acc;
      }
    G.swap(T);
    const double l = normalise(G);
    if (l == -INFINITY) return 0.0;  // nilpotent part: the bound so far holds
    logn = 2.0 * logn + l;
  }
  return std::exp(logn / std::ldexp(1.0, squarings));
}

// Largest spectral-radius bound of G(k) over the k-grid (n points per axis).
inline double spectral_radius(int lattice, int model, const double* S, const double u[3], int n) {
  const LatticeTables t = tables(lattice);
  const int Q = t.Q;
  double E[15];
  equilibrium_moments(lattice, model, u, E);
  std::vector<double> C(Q * Q);
  collision_matrix(t, S, E, C.data());
  const double twopi = 6.283185307179586476925;
  double worst = 0.0;
  const int nz = t.dim == 3 ? n : 1;
  std::vector<cplx> G(Q * Q);
  for (int ix = 0; ix <= n / 2; ++ix)
    for (int iy = 0; iy < n; ++iy)
      for (int iz = 0; iz < nz; ++iz) {
        const double k[3] = {twopi * ix / n, twopi * iy / n, twopi * iz / n};
        for (int i = 0; i < Q; ++i) {
          const double ph = -(k[0] * t.e[i][0] + k[1] * t.e[i][1] + (t.dim == 3 ? k[2] * t.e[i][2] : 0.0));
          const cplx p(std::cos(ph), std::sin(ph));
          for (int j = 0; j < Q; ++j) G[i * Q + j] = p * C[i * Q + j];
        }
        worst = std::max(worst, gelfand_bound(G, Q));
      }
  return worst;
}

}  // namespace stability
}  // namespace lbm
