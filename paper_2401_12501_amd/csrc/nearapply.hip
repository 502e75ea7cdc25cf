// Source preparation, near-field correction and combination (FP64).
//
//   s_r    = sum_j w_j sigma_rj                      (rank-one term, Section 3)
//   qt_rj  = w_j sigma_rj / a_j                      (far-field source strength)
//   y_ri   = sigma_ri + phi_ri + sum_{P in near(i)} C_{i,P,:} . sigma_r,P + s_r
//
// The correction blocks C (Sections 6.1.1-6.1.2) of target i are contiguous in
// memory, so one wavefront per target streams them with unit stride (the
// HBM-bound step of the apply); sigma of the near patches is gathered through the
// caches.  Every reduction runs in a fixed order, so results do not depend on
// timing.
#include "pmx_internal.hpp"

namespace pmx {

namespace {
constexpr int kBlock = 256;
constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
}  // namespace

__global__ void __launch_bounds__(kBlock) k_source_prep(int64_t N, int n_rhs, const double* __restrict__ sigma,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ woa, double* __restrict__ q64,
                                                        float* __restrict__ q32, double* __restrict__ spart) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double ws = 0.0;
  if (i < N) {
    const double s = sigma[(int64_t)r * N + i];
    const double qv = woa[i] * s;
    q64[(int64_t)r * N + i] = qv;
    if (q32) q32[(int64_t)r * N + i] = (float)qv;
    ws = w[i] * s;
  }
  __shared__ double red[kBlock];
  red[threadIdx.x] = ws;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) spart[(int64_t)r * gridDim.x + blockIdx.x] = red[0];
}

// Fixed-order sum of nb partials per rhs (one block per rhs).
__global__ void __launch_bounds__(kBlock) k_sum_partials(int64_t nb, const double* __restrict__ part,
                                                         double* __restrict__ out) {
  const int r = blockIdx.x;
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kBlock) acc += part[(int64_t)r * nb + b];
  __shared__ double red[kBlock];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = red[0];
}

// One wavefront per target.  identity != 0: add sigma_i and s_r (the operator A);
// identity == 0: representation (near blocks D plus far field only).  The target's
// near-patch ids sit in lane registers and are fetched by shuffle, so the loads of
// the streaming loop (C and the gathered sigma) do not wait on index loads.
// Block index of element e: e / q2 = (e * magic) >> 32, magic = ceil(2^32 / q2)
// (exact for e < 2^32 / q2; e is below 64 q2 here).
template <int NR>
__global__ void __launch_bounds__(kBlock) k_near_combine(int64_t N, int q2, uint32_t magic, int n_rhs, int r0,
                                                         const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ patch,
                                                         const double* __restrict__ Cb,
                                                         const double* __restrict__ sigma,
                                                         const double* __restrict__ far, int n_far,
                                                         const double* __restrict__ ssum, int identity,
                                                         double* __restrict__ y) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x / kWave);
  if (i >= N) return;
  const int64_t b0 = ptr[i];
  const int nb = (int)(ptr[i + 1] - b0);
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  for (int g = 0; g < nb; g += kWave) {          // groups of up to 64 near patches
    const int ng = nb - g < kWave ? nb - g : kWave;
    const int my_patch = lane < ng ? patch[b0 + g + lane] : 0;
    const double* Cg = Cb + (b0 + g) * q2;
    const uint32_t len = (uint32_t)(ng * q2);
    // wave-uniform trip count: every lane takes part in the shuffle, loads are predicated
#pragma unroll 4
    for (uint32_t e0 = 0; e0 < len; e0 += kWave) {
      const uint32_t e = e0 + lane;
      const bool ok = e < len;
      const uint32_t ee = ok ? e : len - 1;
      const uint32_t blk = (uint32_t)(((uint64_t)ee * magic) >> 32);
      const uint32_t loc = ee - blk * (uint32_t)q2;
      const int P = __shfl(my_patch, (int)blk, kWave);
      if (ok) {
        const double c = Cg[e];
        const int64_t col = (int64_t)P * q2 + loc;
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = fma(c, sigma[(int64_t)(r0 + r) * N + col], acc[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = wave_sum(acc[r]);
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int rr = r0 + r;
      double v = acc[r];
      double f = 0.0;
      for (int c = 0; c < n_far; ++c) f += far[((int64_t)c * n_rhs + rr) * N + i];
      v += f;
      if (identity) v += sigma[(int64_t)rr * N + i] + ssum[rr];
      y[(int64_t)rr * N + i] = v;
    }
  }
}

// u_r -= (sum_i w_i u_ri) / (sum_i w_i): partial sums then a fixed-order reduction.
__global__ void __launch_bounds__(kBlock) k_wdot_partial(int64_t N, const double* __restrict__ u,
                                                         const double* __restrict__ w, double* __restrict__ part) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  __shared__ double red[kBlock];
  red[threadIdx.x] = i < N ? w[i] * u[(int64_t)r * N + i] : 0.0;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)r * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_sub_mean(int64_t N, double* __restrict__ u, const double* __restrict__ s, double area) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < N) u[(int64_t)r * N + i] -= s[r] / area;
}

void source_prep(pmx_operator* op, const double* sigma, int n_rhs, bool need32, hipStream_t st) {
  const int64_t N = op->s->g.N;
  Ctx* ctx = &op->s->ctx->c;
  const int64_t nb = (N + kBlock - 1) / kBlock;
  if (op->qt64.n < (size_t)n_rhs * N) op->qt64.alloc(ctx, (size_t)n_rhs * N);
  if (need32 && op->qt32.n < (size_t)n_rhs * N) op->qt32.alloc(ctx, (size_t)n_rhs * N);
  if (op->ssum_part.n < (size_t)n_rhs * nb) op->ssum_part.alloc(ctx, (size_t)n_rhs * nb);
  if (op->ssum.n < (size_t)n_rhs) op->ssum.alloc(ctx, n_rhs);
  hipLaunchKernelGGL(k_source_prep, dim3(nb, n_rhs), dim3(kBlock), 0, st, N, n_rhs, sigma, op->s->g.w.p,
                     op->co.w_over_a.p, op->qt64.p, need32 ? op->qt32.p : (float*)nullptr, op->ssum_part.p);
  PMX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(n_rhs), dim3(kBlock), 0, st, nb, op->ssum_part.p, op->ssum.p);
  PMX_HIP(hipGetLastError());
}

template <int NR>
static void combine_group(pmx_operator* op, const double* sigma, double* y, int n_rhs, int r0, int n_far,
                          const double* far, bool parametrix, hipStream_t st) {
  const int64_t N = op->s->g.N;
  const int q2 = op->s->g.q * op->s->g.q;
  const int64_t nb = (N + (kBlock / kWave) - 1) / (kBlock / kWave);
  const uint32_t magic = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)q2 - 1) / (uint64_t)q2);
  hipLaunchKernelGGL(k_near_combine<NR>, dim3(nb), dim3(kBlock), 0, st, N, q2, magic, n_rhs, r0, op->nl.ptr.p,
                     op->nl.patch.p, parametrix ? op->nl.D.p : op->nl.C.p, sigma, far, n_far, op->ssum.p,
                     parametrix ? 0 : 1, y);
  PMX_HIP(hipGetLastError());
}

void near_combine(pmx_operator* op, const double* sigma, double* y, int n_rhs, int n_part, bool use_phi,
                  bool parametrix, hipStream_t st) {
  const double* far = use_phi ? op->phi.p : op->part.p;
  const int n_far = use_phi ? 1 : n_part;
  int r0 = 0;
  while (r0 < n_rhs) {
    const int left = n_rhs - r0;
    if (left >= 8) { combine_group<8>(op, sigma, y, n_rhs, r0, n_far, far, parametrix, st); r0 += 8; }
    else if (left >= 4) { combine_group<4>(op, sigma, y, n_rhs, r0, n_far, far, parametrix, st); r0 += 4; }
    else if (left >= 2) { combine_group<2>(op, sigma, y, n_rhs, r0, n_far, far, parametrix, st); r0 += 2; }
    else { combine_group<1>(op, sigma, y, n_rhs, r0, n_far, far, parametrix, st); r0 += 1; }
  }
}

void weighted_mean_remove(pmx_operator* op, double* u, int n_rhs, hipStream_t st) {
  const int64_t N = op->s->g.N;
  Ctx* ctx = &op->s->ctx->c;
  const int64_t nb = (N + kBlock - 1) / kBlock;
  if (op->ssum_part.n < (size_t)n_rhs * nb) op->ssum_part.alloc(ctx, (size_t)n_rhs * nb);
  DBuf<double> s;
  s.alloc(ctx, n_rhs);
  hipLaunchKernelGGL(k_wdot_partial, dim3(nb, n_rhs), dim3(kBlock), 0, st, N, u, op->s->g.w.p, op->ssum_part.p);
  PMX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(n_rhs), dim3(kBlock), 0, st, nb, op->ssum_part.p, s.p);
  PMX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sub_mean, dim3(nb, n_rhs), dim3(kBlock), 0, st, N, u, s.p, op->s->g.area);
  PMX_HIP(hipGetLastError());
  PMX_HIP(hipStreamSynchronize(st));   // s is released on return
}

}  // namespace pmx
