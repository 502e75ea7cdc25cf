// Direct far-field sums over all source nodes (smooth rule, Section 6.1.3).
//
//   phi_i = sum_{j != i} w_j R(x_i, x_j) sigma_j
//         = sum_j qt_j [ s_ij (A_i s_ij - B_i) + (g_i . r_ij) / r_ij^2 ],
//   s_ij = (n_i . r_ij) / r_ij^2,  qt_j = w_j sigma_j / a_j,  r_ij = x_i - x_j,
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
  // hardware reciprocal, then two Newton steps (each doubles the correct bits)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
}  // namespace

template <int NR>
__global__ void __launch_bounds__(kBlock) k_direct64(int64_t N, const double* __restrict__ tgt,
                                                     const double* __restrict__ tg, const double* __restrict__ X,
                                                     const double* __restrict__ qt, int64_t ldq, int64_t chunk,
                                                     double* __restrict__ part, int64_t ldp, int64_t ldc) {
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < N ? i0 : N - 1;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  const double xi = tgt[i], yi = tgt[N + i], zi = tgt[2 * N + i];
  const double nx = tgt[3 * N + i], ny = tgt[4 * N + i], nz = tgt[5 * N + i];
  const double A = tgt[6 * N + i], B = tgt[7 * N + i];
  const double gx = tg[i], gy = tg[N + i], gz = tg[2 * N + i];
  const double* __restrict__ Xs = X;
  const double* __restrict__ Ys = X + N;
  const double* __restrict__ Zs = X + 2 * N;
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
#pragma unroll 2
  for (int64_t j = j0; j < j1; ++j) {
    const double dx = xi - Xs[j], dy = yi - Ys[j], dz = zi - Zs[j];
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-300)));
    const double inv = rcp64(r2);
    const double nr = fma(nx, dx, fma(ny, dy, nz * dz));
    const double gr = fma(gx, dx, fma(gy, dy, gz * dz));
    const double s = nr * inv;
    const double v = fma(s, fma(A, s, -B), gr * inv);
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = fma(qt[r * ldq + j], v, acc[r]);
  }
  if (i0 < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) part[(int64_t)blockIdx.y * ldc + r * ldp + i0] = acc[r];
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
  const float nx = t32[3 * N + i], ny = t32[4 * N + i], nz = t32[5 * N + i];
  const float A = t32[6 * N + i], B = t32[7 * N + i];
  const float gx = t32[8 * N + i], gy = t32[9 * N + i], gz = t32[10 * N + i];
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
    const float nr = fmaf(nx, dx, fmaf(ny, dy, nz * dz));
    const float gr = fmaf(gx, dx, fmaf(gy, dy, gz * dz));
    const float s = nr * inv;
    const float v = fmaf(s, fmaf(A, s, -B), gr * inv);
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
  const int64_t tb = (N + kBlock - 1) / kBlock;
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
  if (mode == 0)
    hipLaunchKernelGGL(k_direct64<NR>, grid, dim3(kBlock), 0, st, N, op->co.tgt.p, op->co.tg.p, op->s->g.x.p,
                       op->qt64.p + (int64_t)r0 * N, N, chunk, part, N, ldc);
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
