// Direct far-field sums over all source nodes (smooth rule, Section 6.1.3).
//
//   phi_i = sum_{j != i} w_j R(x_i, x_j) sigma_j
//         = sum_j qt_j (1/r^2) [ (n'_i . r)^2 / r^2 + h_i . r ],   r = x_i - x_j,
//   qt_j = w_j sigma_j / a_j,  n' = sqrt(A) n,  h = g - B n,
// the c = 0 remainder of eq:explicit_remainder with G = log(r) / (2 pi a(x'))
// written with the target factors A = a/pi, B = a H/pi, g = grad_G a / (2 pi).
//
// Each thread owns one target and walks a contiguous chunk of sources.  Source
// coordinates and densities are the same for every lane of a wavefront, so they
// are read through the scalar data cache and live in scalar registers; the only
// per-pair memory traffic is zero.  The pair j = i is removed without a branch:
// r^2 gets a tiny epsilon, so the self pair has 1/r^2 finite while n.r = g.r = 0
// make its contribution exactly zero.  Partial sums per source chunk go to
// part[chunk][rhs][i] and are added in a fixed order afterwards (deterministic).
#include "pmx_internal.hpp"

namespace pmx {

namespace {
constexpr int kBlock = 256;

__device__ __forceinline__ double rcp64(double x) {
  // hardware reciprocal (about 24 correct bits), then one Newton step: 2e-15 relative
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
}  // namespace

// TPL targets per lane (targets i0 and i0 + kBlock of a 2*kBlock target tile): one
// scalar source load feeds TPL pair evaluations.
template <int NR, int TPL>
__global__ void __launch_bounds__(kBlock) k_direct64(int64_t N, const double* __restrict__ tf,
                                                     const double* __restrict__ X, const double* __restrict__ qt,
                                                     int64_t ldq, int64_t chunk, double* __restrict__ part,
                                                     int64_t ldp, int64_t ldc) {
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  double xi[TPL], yi[TPL], zi[TPL], px[TPL], py[TPL], pz[TPL], hx[TPL], hy[TPL], hz[TPL];
  int64_t it[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    it[t] = (int64_t)blockIdx.x * kBlock * TPL + t * kBlock + threadIdx.x;
    const int64_t i = it[t] < N ? it[t] : N - 1;
    xi[t] = tf[i]; yi[t] = tf[N + i]; zi[t] = tf[2 * N + i];
    px[t] = tf[3 * N + i]; py[t] = tf[4 * N + i]; pz[t] = tf[5 * N + i];
    hx[t] = tf[6 * N + i]; hy[t] = tf[7 * N + i]; hz[t] = tf[8 * N + i];
  }
  const double* __restrict__ Xs = X;
  const double* __restrict__ Ys = X + N;
  const double* __restrict__ Zs = X + 2 * N;
  double acc[TPL][NR];
#pragma unroll
  for (int t = 0; t < TPL; ++t)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[t][r] = 0.0;
#pragma unroll 2
  for (int64_t j = j0; j < j1; ++j) {
    const double xs = Xs[j], ys = Ys[j], zs = Zs[j];
    double q[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) q[r] = qt[r * ldq + j];
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
      const double dx = xi[t] - xs, dy = yi[t] - ys, dz = zi[t] - zs;
      const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-300)));
      const double inv = rcp64(r2);
      const double pr = fma(px[t], dx, fma(py[t], dy, pz[t] * dz));
      const double hr = fma(hx[t], dx, fma(hy[t], dy, hz[t] * dz));
      const double v = fma(pr * inv, pr, hr) * inv;
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[t][r] = fma(q[r], v, acc[t][r]);
    }
  }
#pragma unroll
  for (int t = 0; t < TPL; ++t)
    if (it[t] < N) {
#pragma unroll
      for (int r = 0; r < NR; ++r) part[(int64_t)blockIdx.y * ldc + r * ldp + it[t]] = acc[t][r];
    }
}

template <int NR>
__global__ void __launch_bounds__(kBlock) k_direct32(int64_t N, const float* __restrict__ t32,
                                                     const float* __restrict__ qt, int64_t ldq, int64_t chunk,
                                                     double* __restrict__ part, int64_t ldp, int64_t ldc) {
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < N ? i0 : N - 1;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  const float xi = t32[i], yi = t32[N + i], zi = t32[2 * N + i];
  const float px = t32[3 * N + i], py = t32[4 * N + i], pz = t32[5 * N + i];
  const float hx = t32[6 * N + i], hy = t32[7 * N + i], hz = t32[8 * N + i];
  const float* __restrict__ Xs = t32;
  const float* __restrict__ Ys = t32 + N;
  const float* __restrict__ Zs = t32 + 2 * N;
  float acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0f;
#pragma unroll 4
  for (int64_t j = j0; j < j1; ++j) {
    const float dx = xi - Xs[j], dy = yi - Ys[j], dz = zi - Zs[j];
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1e-30f)));
    const float inv = __builtin_amdgcn_rcpf(r2);
    const float pr = fmaf(px, dx, fmaf(py, dy, pz * dz));
    const float hr = fmaf(hx, dx, fmaf(hy, dy, hz * dz));
    const float v = fmaf(pr * inv, pr, hr) * inv;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = fmaf(qt[r * ldq + j], v, acc[r]);
  }
  if (i0 < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) part[(int64_t)blockIdx.y * ldc + r * ldp + i0] = (double)acc[r];
  }
}

// Representation far field: u_i = sum_{j != i} qt_j log(r_ij) / (2 pi), qt = w sigma / a.
template <int NR>
__global__ void __launch_bounds__(kBlock) k_direct_log(int64_t N, const double* __restrict__ X,
                                                       const double* __restrict__ qt, int64_t ldq, int64_t chunk,
                                                       double* __restrict__ part, int64_t ldp, int64_t ldc) {
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < N ? i0 : N - 1;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  const double xi = X[i], yi = X[N + i], zi = X[2 * N + i];
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    const double dx = xi - X[j], dy = yi - X[N + j], dz = zi - X[2 * N + j];
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double v = j == i ? 0.0 : 0.5 * log(r2) * 0.15915494309189533577;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = fma(qt[r * ldq + j], v, acc[r]);
  }
  if (i0 < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) part[(int64_t)blockIdx.y * ldc + r * ldp + i0] = acc[r];
  }
}

namespace {
// Source chunks so that the grid holds enough workgroups to fill 256 CUs.
int64_t n_chunks_for(int64_t N) {
  const int64_t tb = (N + 2 * kBlock - 1) / (2 * kBlock);
  int64_t c = (8 * 256 + tb - 1) / tb;
  if (c < 1) c = 1;
  if (c > 64) c = 64;
  const int64_t max_by_len = (N + 63) / 64;   // at least 64 sources per chunk
  if (c > max_by_len) c = max_by_len;
  if (c < 1) c = 1;
  return c;
}

// mode 0: FP64 remainder, 1: FP32 remainder, 2: FP64 log kernel.
template <int NR>
void launch_group(pmx_operator* op, int mode, int n_rhs, int r0, int64_t nc, hipStream_t st) {
  const int64_t N = op->s->g.N;
  const int64_t chunk = (N + nc - 1) / nc;
  dim3 grid((unsigned)((N + kBlock - 1) / kBlock), (unsigned)nc);
  double* part = op->part.p + (int64_t)r0 * N;
  const int64_t ldc = (int64_t)n_rhs * N;
  if (mode == 0) {
    constexpr int TPL = NR <= 2 ? 2 : 1;
    dim3 g64((unsigned)((N + TPL * kBlock - 1) / (TPL * kBlock)), (unsigned)nc);
    hipLaunchKernelGGL((k_direct64<NR, TPL>), g64, dim3(kBlock), 0, st, N, op->co.tf64.p, op->s->g.x.p,
                       op->qt64.p + (int64_t)r0 * N, N, chunk, part, N, ldc);
  }
  else if (mode == 1)
    hipLaunchKernelGGL(k_direct32<NR>, grid, dim3(kBlock), 0, st, N, op->co.tgt32.p, op->qt32.p + (int64_t)r0 * N,
                       N, chunk, part, N, ldc);
  else
    hipLaunchKernelGGL(k_direct_log<NR>, grid, dim3(kBlock), 0, st, N, op->s->g.x.p, op->qt64.p + (int64_t)r0 * N,
                       N, chunk, part, N, ldc);
  PMX_HIP(hipGetLastError());
}

void far_direct_mode(pmx_operator* op, int mode, int n_rhs, hipStream_t st) {
  const int64_t N = op->s->g.N;
  const int64_t nc = n_chunks_for(N);
  const size_t need = (size_t)nc * n_rhs * N;
  if (op->part.n < need) op->part.alloc(&op->s->ctx->c, need);
  int r0 = 0;
  while (r0 < n_rhs) {
    const int left = n_rhs - r0;
    if (left >= 8) { launch_group<8>(op, mode, n_rhs, r0, nc, st); r0 += 8; }
    else if (left >= 4) { launch_group<4>(op, mode, n_rhs, r0, nc, st); r0 += 4; }
    else if (left >= 2) { launch_group<2>(op, mode, n_rhs, r0, nc, st); r0 += 2; }
    else { launch_group<1>(op, mode, n_rhs, r0, nc, st); r0 += 1; }
  }
}
}  // namespace

int far_direct_chunks(const pmx_operator* op, bool) { return (int)n_chunks_for(op->s->g.N); }

void far_direct(pmx_operator* op, bool fp64, int n_rhs, hipStream_t st) { far_direct_mode(op, fp64 ? 0 : 1, n_rhs, st); }

void far_direct_log(pmx_operator* op, int n_rhs, hipStream_t st) { far_direct_mode(op, 2, n_rhs, st); }

}  // namespace pmx
