/*
 * Smooth-rule sums of the oracle in plain C (FP64), one OpenMP thread per block of target rows.
 *
 * TEST INFRASTRUCTURE ONLY: built by the oracle's loader (oracle/cfar.py); nothing in the
 * library links or calls it.
 *
 * remainder rows (Section 6.1.3, the plain Nystrom rule applied to eq:explicit_remainder
 * with c = 0):
 *     out[t][r] = sum_{j != i} w_j R(x_i, x_j) sigma_r[j],   i = targets[t],
 *     R = grad_G a(x) . rhat G'  -  a(x) G'' (n.r)^2 / r^2  +  a(x) G' (n.r)^2 / r^3
 *         - 2 a(x) H(x) (n . rhat) G',
 *     G(r; a') = log(r) / (2 pi a'),  G' = 1 / (2 pi a' r),  G'' = -1 / (2 pi a' r^2),
 * with r = x_i - x_j, a' = a(x_j) (coefficient at the source, eq:diff_param) and the target's
 * normal n, mean curvature H, coefficient a and surface gradient of a.
 *
 * parametrix rows (the representation eq:representation, same rule):
 *     out[t][r] = sum_{j != i} w_j log|x_i - x_j| / (2 pi a_j) sigma_r[j].
 *
 * Every row sums its sources in increasing j, term by term as written above; no blocking,
 * no reformulation of the kernel.  Arrays: x, n, gs row-major N x 3; sigma n_rhs rows of N;
 * out row-major n_targets x n_rhs.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

static const double kTwoPi = 6.283185307179586476925286766559;

void oracle_far_remainder(int64_t N, const double* x, const double* n, const double* H, const double* a,
                          const double* gs, const double* w, int n_rhs, const double* sigma, int64_t n_targets,
                          const int64_t* targets, double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < n_targets; ++t) {
    const int64_t i = targets[t];
    const double xi0 = x[3 * i], xi1 = x[3 * i + 1], xi2 = x[3 * i + 2];
    const double n0 = n[3 * i], n1 = n[3 * i + 1], n2 = n[3 * i + 2];
    const double g0 = gs[3 * i], g1 = gs[3 * i + 1], g2 = gs[3 * i + 2];
    const double at = a[i], Ht = H[i];
    double acc[1024];
    for (int r = 0; r < n_rhs; ++r) acc[r] = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      if (j == i) continue;
      const double r0 = xi0 - x[3 * j], r1 = xi1 - x[3 * j + 1], r2 = xi2 - x[3 * j + 2];
      const double rn = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
      const double G1 = 1.0 / (kTwoPi * a[j] * rn);
      const double G2 = -1.0 / (kTwoPi * a[j] * rn * rn);
      const double nr = n0 * r0 + n1 * r1 + n2 * r2;
      const double grh = (g0 * r0 + g1 * r1 + g2 * r2) / rn;
      const double R = grh * G1 - at * G2 * nr * nr / (rn * rn) + at * G1 * nr * nr / (rn * rn * rn) -
                       2.0 * at * Ht * (nr / rn) * G1;
      const double wr = w[j] * R;
      for (int r = 0; r < n_rhs; ++r) acc[r] += wr * sigma[(int64_t)r * N + j];
    }
    for (int r = 0; r < n_rhs; ++r) out[t * n_rhs + r] = acc[r];
  }
}

void oracle_far_parametrix(int64_t N, const double* x, const double* a, const double* w, int n_rhs,
                           const double* sigma, int64_t n_targets, const int64_t* targets, double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < n_targets; ++t) {
    const int64_t i = targets[t];
    const double xi0 = x[3 * i], xi1 = x[3 * i + 1], xi2 = x[3 * i + 2];
    double acc[1024];
    for (int r = 0; r < n_rhs; ++r) acc[r] = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      if (j == i) continue;
      const double r0 = xi0 - x[3 * j], r1 = xi1 - x[3 * j + 1], r2 = xi2 - x[3 * j + 2];
      const double K = log(sqrt(r0 * r0 + r1 * r1 + r2 * r2)) / (kTwoPi * a[j]);
      const double wk = w[j] * K;
      for (int r = 0; r < n_rhs; ++r) acc[r] += wk * sigma[(int64_t)r * N + j];
    }
    for (int r = 0; r < n_rhs; ++r) out[t * n_rhs + r] = acc[r];
  }
}

/* Threads the OpenMP runtime will use (for reporting). */
int oracle_far_threads(void) {
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
}
