/* Plain FP64 reference for long periodic runs of the modified MRT step.
 *
 * TEST INFRASTRUCTURE ONLY.  Used by the oracle tests and by the script that
 * writes stored expected values under tests/golden/; the product (the HIP
 * library and its binding) never links or calls it, and shares no code with it.
 *
 * It exists because the numpy oracle needs about ten seconds per step on a
 * 4096^2 grid: the same step, written in C with OpenMP over rows, runs the
 * full-length workloads in tens of minutes on the host.
 *
 * One step in push form (Eq. 11, 13, 14, then Eq. 5), for a constant
 * relaxation matrix S:
 *   f'(x) = f(x) - M^-1 S (M f(x) - m_eq(phi(x), u(x)))
 *         = Cm f(x) + phi(x) (b_0 + sum_c u_c(x) b_c),      phi = sum_i f_i (Eq. 8)
 *   f_i(x + e_i, t + 1) = f'_i(x, t)                      (periodic on every axis)
 * with Cm = I - M^-1 S M and b = M^-1 S times the coefficient vectors of the
 * equilibrium, which for MRT-A (Eq. 37; Eq. A.3) is linear in phi and phi u.
 * Cm and b come from the Python oracle's own M, M^-1, S and equilibrium.
 *
 * Arrays are FP64, populations (Q, nz, ny, nx) with x fastest, the velocity
 * (dim, nz, ny, nx); e holds the lattice velocities as Q rows of (ex, ey, ez).
 */
#include <stdint.h>
#include <string.h>

static void one_step(int Q, int dim, int64_t nx, int64_t ny, int64_t nz, const int* e, const double* Cm,
                     const double* b, const double* u, const double* src, double* dst, int threads) {
  const int64_t N = nx * ny * nz;
#pragma omp parallel for schedule(static) num_threads(threads)
  for (int64_t row = 0; row < ny * nz; ++row) {
    const int64_t y = row % ny, z = row / ny;
    double fi[15], fo[15];
    for (int64_t x = 0; x < nx; ++x) {
      const int64_t n = row * nx + x;
      double phi = 0.0;
      for (int i = 0; i < Q; ++i) {
        fi[i] = src[i * N + n];
        phi += fi[i];
      }
      for (int i = 0; i < Q; ++i) {
        double acc = 0.0;
        for (int j = 0; j < Q; ++j) acc += Cm[i * Q + j] * fi[j];
        double eq = b[i];
        for (int c = 0; c < dim; ++c) eq += u[c * N + n] * b[(1 + c) * Q + i];
        fo[i] = acc + phi * eq;
      }
      for (int i = 0; i < Q; ++i) {
        int64_t xd = x + e[3 * i], yd = y + e[3 * i + 1], zd = z + e[3 * i + 2];
        xd = xd < 0 ? xd + nx : (xd >= nx ? xd - nx : xd);
        yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
        zd = zd < 0 ? zd + nz : (zd >= nz ? zd - nz : zd);
        dst[i * N + (zd * ny + yd) * nx + xd] = fo[i];
      }
    }
  }
}

/* Advance f (Q x N, updated in place) by `steps` steps on `threads` OpenMP
 * threads; g is scratch of the same size.  shape = (nx, ny, nz) (nz = 1 in
 * 2D).  Returns 0, or -1 for arguments outside what is built (Q > 15, a
 * velocity component outside {-1, 0, 1}, an axis shorter than 1, threads < 1). */
int lbm_ref_run(int Q, int dim, const int64_t* shape, const int* e, const double* Cm, const double* b,
                const double* u, double* f, double* g, int64_t steps, int threads) {
  const int64_t nx = shape[0], ny = shape[1], nz = shape[2];
  if (Q < 1 || Q > 15 || dim < 1 || dim > 3 || nx < 1 || ny < 1 || nz < 1 || steps < 0 || threads < 1) return -1;
  for (int k = 0; k < 3 * Q; ++k)
    if (e[k] < -1 || e[k] > 1) return -1;
  double* src = f;
  double* dst = g;
  for (int64_t t = 0; t < steps; ++t) {
    one_step(Q, dim, nx, ny, nz, e, Cm, b, u, src, dst, threads);
    double* tmp = src;
    src = dst;
    dst = tmp;
  }
  if (src != f) memcpy(f, src, sizeof(double) * (size_t)Q * (size_t)(nx * ny * nz));
  return 0;
}
