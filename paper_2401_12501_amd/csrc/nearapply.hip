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
#include <algorithm>

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

struct PrepArgs {
  int64_t N, nbx;                 // nodes, blocks per right-hand side
  const double* sigma;
  const double* w;
  const double* woa;              // w / a
  double* q64;
  float* q32;                     // may be null
  double* spart;                  // [rhs][nbx]
};

__global__ void __launch_bounds__(kBlock) k_source_prep(Group<PrepArgs> g) {
  int64_t lb;
  const PrepArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t r = lb / A.nbx, bx = lb - r * A.nbx;
  const int64_t N = A.N;
  const int64_t i = bx * kBlock + threadIdx.x;
  double ws = 0.0;
  if (i < N) {
    const double s = A.sigma[r * N + i];
    const double qv = A.woa[i] * s;
    A.q64[r * N + i] = qv;
    if (A.q32) A.q32[r * N + i] = (float)qv;
    ws = A.w[i] * s;
  }
  __shared__ double red[kBlock];
  red[threadIdx.x] = ws;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) A.spart[r * A.nbx + bx] = red[0];
}

// Fixed-order sum of nb partials per rhs (one block per rhs).
struct SumArgs {
  int64_t nb;
  const double* part;
  double* out;
};

__global__ void __launch_bounds__(kBlock) k_sum_partials(Group<SumArgs> g) {
  int64_t r;
  const SumArgs& A = seg_of(g, blockIdx.x, r);
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < A.nb; b += kBlock) acc += A.part[r * A.nb + b];
  __shared__ double red[kBlock];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) A.out[r] = red[0];
}

// kSub lanes per target (several targets per wavefront).  identity != 0: add sigma_i and s_r (the operator A);
// identity == 0: representation (near blocks D plus far field only).  The far field comes as
// n_far partial sums (direct sums) or not at all (n_far = 0: the FMM's L2P adds it later).  The target's
// near-patch ids sit in lane registers and are fetched by shuffle, so the loads of
// the streaming loop (C and the gathered sigma) do not wait on index loads.
// Block index of element e: e / q2 = (e * magic) >> 32, magic = ceil(2^32 / q2)
// (exact for e < 2^32 / q2; e is below kSub q2 here).
struct CombineArgs {
  int64_t N;
  int q2, n_rhs, r0, n_far, identity;
  int paired;   // q2 and N even, blocks and densities 16-byte aligned: two entries per lane and load
  int rank1;    // add sum_j w_j sigma_j (c = 0 only: the rank-one term)
  uint32_t magic;
  const int64_t* ptr;
  const int32_t* patch;
  const double* Cb;
  const double* sigma;
  const double* far;
  const double* ssum;
  double* y;
};

constexpr int kSub = 32;                  // lanes per target: two targets per wavefront
constexpr int kFarR = 64 / kSub;          // far-field partial registers per lane (up to 64 chunks)
constexpr int kTPB = kBlock / kSub;       // targets per workgroup

__device__ __forceinline__ double sub_sum(double v) {
#pragma unroll
  for (int o = kSub / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kSub);
  return v;
}

template <int NR>
__global__ void __launch_bounds__(kBlock) k_near_combine(Group<CombineArgs> g) {
  int64_t lb;
  const CombineArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t N = A.N;
  const int q2 = A.q2;
  const int sl = threadIdx.x & (kSub - 1);
  const int64_t i = lb * kTPB + (threadIdx.x / kSub);
  const bool live = i < N;                  // both halves of a wave stay for the shuffles
  const int64_t ii = live ? i : N - 1;
  const double* __restrict__ sigma = A.sigma;
  // the terms that do not depend on the near blocks are loaded first, so their latency
  // overlaps the block stream: register k of lane sl holds far-field partial k kSub + sl
  double far_p[NR][kFarR], sig_i[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int rr = A.r0 + r;
#pragma unroll
    for (int k = 0; k < kFarR; ++k) {
      const int c = k * kSub + sl;
      far_p[r][k] = c < A.n_far ? A.far[((int64_t)c * A.n_rhs + rr) * N + ii] : 0.0;
    }
    sig_i[r] = (A.identity && sl == 0) ? sigma[(int64_t)rr * N + ii] : 0.0;
  }
  const int64_t b0 = A.ptr[ii];
  const int nb = live ? (int)(A.ptr[ii + 1] - b0) : 0;
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  // the targets of a wave may differ in patch count: loop to the largest
  int nb_max = nb;
#pragma unroll
  for (int o = kSub; o < 64; o <<= 1) nb_max = max(nb_max, __shfl_xor(nb_max, o, 64));
  for (int gq = 0; gq < nb_max; gq += kSub) {     // groups of up to kSub near patches
    const int ng = nb - gq < kSub ? (nb - gq > 0 ? nb - gq : 0) : kSub;
    const int my_patch = sl < ng ? A.patch[b0 + gq + sl] : 0;
    const double* __restrict__ Cg = A.Cb + (b0 + gq) * q2;
    const uint32_t len = (uint32_t)(ng * q2);
    int ng_max = ng;
#pragma unroll
    for (int o = kSub; o < 64; o <<= 1) ng_max = max(ng_max, __shfl_xor(ng_max, o, 64));
    const uint32_t len_max = (uint32_t)(ng_max * q2);
    // trip count uniform over the wave: every lane takes part in the shuffles, loads are predicated
    if (A.paired) {
      // entries 2k and 2k+1 lie in one block (q2 even), at consecutive columns: 16-byte loads
#pragma unroll 8
      for (uint32_t e0 = 0; e0 < len_max; e0 += 2 * kSub) {
        const uint32_t e = e0 + 2 * sl;
        const bool ok = e < len;
        const uint32_t ee = ok ? e : 0;
        const uint32_t blk = (uint32_t)(((uint64_t)ee * A.magic) >> 32);
        const uint32_t loc = ee - blk * (uint32_t)q2;
        const int P = __shfl(my_patch, (int)blk, kSub);
        if (ok) {
          const double2 c = *reinterpret_cast<const double2*>(Cg + e);
          const int64_t col = (int64_t)P * q2 + loc;
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double2 sv = *reinterpret_cast<const double2*>(sigma + (int64_t)(A.r0 + r) * N + col);
            acc[r] = fma(c.y, sv.y, fma(c.x, sv.x, acc[r]));
          }
        }
      }
    } else {
#pragma unroll 8
      for (uint32_t e0 = 0; e0 < len_max; e0 += kSub) {
        const uint32_t e = e0 + sl;
        const bool ok = e < len;
        const uint32_t ee = ok ? e : 0;
        const uint32_t blk = (uint32_t)(((uint64_t)ee * A.magic) >> 32);
        const uint32_t loc = ee - blk * (uint32_t)q2;
        const int P = __shfl(my_patch, (int)blk, kSub);
        if (ok) {
          const double c = Cg[e];
          const int64_t col = (int64_t)P * q2 + loc;
#pragma unroll
          for (int r = 0; r < NR; ++r) acc[r] = fma(c, sigma[(int64_t)(A.r0 + r) * N + col], acc[r]);
        }
      }
    }
  }
  // near sum over the target's lanes, plus the far-field partials in chunk order
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = sub_sum(acc[r]);
  double f[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    f[r] = 0.0;
    for (int c = 0; c < A.n_far; ++c) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < kFarR; ++k)
        if (c / kSub == k) v = __shfl(far_p[r][k], c % kSub, kSub);
      f[r] += v;
    }
  }
  if (sl == 0 && live) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int rr = A.r0 + r;
      double v = acc[r] + f[r];
      if (A.identity) v += sig_i[r] + (A.rank1 ? A.ssum[rr] : 0.0);
      A.y[(int64_t)rr * N + i] = v;
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

// Near correction for a group of RB right-hand sides (8 or 16), one workgroup per slab of at
// most 64 target rows of a target patch T.  For every patch P in the union of the near lists of
// T's targets, the rows of T's targets with P form a q^2 x q^2 block C_{T,P} (rows of targets
// not near P are zero), and
//   Y_T += C_{T,P} Sigma_P,   Sigma_P = sigma of P's nodes for the RB right-hand sides,
// a dense contraction that runs on FP64 MFMA (16 x 16 x 4): the right-hand sides are the
// sixteen columns, each wave owns one 16-row tile of the slab, and the accumulators stay in
// registers across the union.  The contraction runs over P's nodes in chunks of kKC = 32: each
// chunk's slice of every block row of the slab (32 consecutive doubles of a row stored
// contiguously) and of Sigma_P goes straight from memory into LDS (global_load_lds, 16 bytes
// per lane), every load of the chunk in flight at once and one wait before the barrier.  Each
// target sums its patches in union order, so results are deterministic; the output goes through
// LDS so that y is written with unit stride per right-hand side.
struct TiledArgs {
  int64_t N, n_patches;
  int q2, r0;
  int n_slab;   // slabs of at most 64 rows per target patch
  const int32_t* tile_ptr;
  const int32_t* tile_patch;
  const int32_t* tile_pair;
  const double* Cb;
  const double* sigma;
  const double* ssum;
  double* y;
};

typedef double doublex4 __attribute__((ext_vector_type(4)));
constexpr int kXcds = 8;           // accelerator complex dies of the GPU, each with its own L2
constexpr int kKC = 32;            // source nodes per staged chunk: 256-byte LDS rows of 16 slots
constexpr int kLdY = 17;           // LDS row stride of the output tile (doubles)
constexpr int kSlab = 64;          // target rows per workgroup: four waves of one 16-row tile

// Sixteen zero bytes: the source of every staged slot that lies past a chunk's columns or in
// the row of a target not near P (a direct-to-LDS load cannot write a constant).
__device__ __align__(16) double near_zero16[2] = {0.0, 0.0};

// LDS rows hold 16 slots of two doubles; slot s of row t is stored at position s ^ (t & 15), so
// that the sixteen rows an MFMA operand read touches (same column, consecutive rows) fall in
// different banks.
__device__ __forceinline__ int near_swz(int t, int c) { return t * kKC + (((c >> 1) ^ (t & 15)) << 1) + (c & 1); }

__device__ __forceinline__ void lds_load16(const double* src, double* dst_wave_base) {
  __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                   (void __attribute__((address_space(3)))*)dst_wave_base, 16, 0, 0);
}

template <int RB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) k_near_tiled(Group<TiledArgs> g) {
  constexpr int kGroups = kSlab / 4 / 4;   // four-row staging groups per wave
  // LDS: block slices sC[64][kKC], then sigma slices sS[16][kKC] (right-hand side, node), both
  // swizzled; the output tile sY[64][kLdY] reuses sC once the contraction is done
  extern __shared__ double lds[];
  int64_t lb;
  const TiledArgs& A = seg_of(g, blockIdx.x, lb);
  // XCD-aware order over the slabs V = T n_slab + h: workgroups are dealt round-robin over the
  // eight XCDs, so block lb runs on XCD lb % 8; that XCD takes a contiguous range of slabs, so
  // neighbouring target patches, which share near patches, reuse densities from its L2
  const int64_t MS = A.n_patches * A.n_slab;
  const int64_t xq = MS / kXcds, xr = MS % kXcds, xc = lb % kXcds;
  const int64_t V = xc * xq + (xc < xr ? xc : xr) + lb / kXcds;
  const int64_t T = V / A.n_slab;
  const int t0 = (int)(V - T * A.n_slab) * kSlab;   // the slab's first target row
  const int64_t N = A.N;
  const int q2 = A.q2;
  const int qs = q2 - t0 < kSlab ? q2 - t0 : kSlab; // target rows of the slab
  const int rows = (qs + 15) & ~15;
  double* sC = lds;
  double* sS = lds + (size_t)kSlab * kKC;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4, col = lane & 15;
  const bool has_tile = wave * 16 < rows;        // wave w owns row tile w
  // staging: a wave-wide load writes four consecutive 256-byte rows; lane l writes slot l % 16
  // of slab row 4 G + l / 16 of its group G = wave, wave + 4, ... (that row's pair index below)
  const int lr = lane >> 4, ls = lane & 15;
  const int n_groups = rows / 4;
  doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
  const int u0 = A.tile_ptr[T], u1 = A.tile_ptr[T + 1];
  // pair indices of this lane's staged rows for union entry u, one entry ahead in registers
  auto load_pairs = [&](int u, int32_t* pr) {
#pragma unroll
    for (int i = 0; i < kGroups; ++i) {
      const int t = t0 + 4 * (wave + 4 * i) + lr;
      pr[i] = (u < u1 && t < q2) ? A.tile_pair[(int64_t)u * q2 + t] : -1;
    }
  };
  int32_t pr_cur[kGroups], pr_next[kGroups];
  load_pairs(u0, pr_cur);
  int32_t P_cur = u0 < u1 ? A.tile_patch[u0] : 0;
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the first entry's indices are in registers
  for (int u = u0; u < u1; ++u) {
    const int64_t P = P_cur;
    const int32_t P_next = u + 1 < u1 ? A.tile_patch[u + 1] : 0;   // one entry ahead, with its pairs
    load_pairs(u + 1, pr_next);
    for (int kc = 0; kc < q2; kc += kKC) {
      const int kw = q2 - kc < kKC ? q2 - kc : kKC;   // valid columns in this chunk (even)
      __syncthreads();   // the previous chunk's slices are no longer read
#pragma unroll
      for (int i = 0; i < kGroups; ++i) {
        const int G = wave + 4 * i;
        if (G < n_groups) {
          const int tl = 4 * G + lr;
          const int c = 2 * (ls ^ (tl & 15));         // the columns slot ls of slab row tl holds
          const double* src = (pr_cur[i] >= 0 && c < kw) ? A.Cb + (int64_t)pr_cur[i] * q2 + kc + c : near_zero16;
          lds_load16(src, sC + 4 * G * kKC);
        }
      }
      {   // sigma: right-hand side r = 4 wave + lr, nodes kc + c, c + 1 of P
        const int r = 4 * wave + lr;
        const int c = 2 * (ls ^ (r & 15));
        const double* src = (r < RB && c < kw) ? A.sigma + (int64_t)(A.r0 + r) * N + P * q2 + kc + c : near_zero16;
        lds_load16(src, sS + 4 * wave * kKC);
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's slices have landed
      __syncthreads();
      if (has_tile) {
#pragma unroll
        for (int ks = 0; ks < kKC; ks += 4) {
          const double bv = sS[near_swz(col, ks + kq)];
          const double av = sC[near_swz(wave * 16 + col, ks + kq)];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kGroups; ++i) pr_cur[i] = pr_next[i];
    P_cur = P_next;
  }
  __syncthreads();   // every wave is done with sC: it becomes the output tile
  double* sY = lds;
  if (has_tile) {
    // FP64 16x16x4 accumulators: register i of lane l holds row 4 i + l / 16, column l % 16
    // (the FP32 16x16x4 form holds row 4 (l / 16) + i instead)
#pragma unroll
    for (int i = 0; i < 4; ++i) sY[(wave * 16 + 4 * i + kq) * kLdY + col] = acc[i];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < RB * qs; e += 256) {
    const int r = e / qs, tl = e - r * qs;
    const int64_t at = (int64_t)(A.r0 + r) * N + T * q2 + t0 + tl;
    A.y[at] = sY[tl * kLdY + r] + A.sigma[at] + A.ssum[A.r0 + r];
  }
}

// LDS bytes of k_near_tiled (the same for every patch size: one slab of at most 64 rows).
size_t near_tiled_lds(int) {
  const size_t a = (size_t)kSlab * kKC + (size_t)16 * kKC, b = (size_t)kSlab * kLdY;
  return (a > b ? a : b) * sizeof(double);
}

int near_tiled_slabs(int q2) { return (q2 + kSlab - 1) / kSlab; }

// The tiled kernel takes even patch sizes (16-byte staged slots); odd ones use the per-target
// kernel.
bool near_tiled_fits(int q2) { return q2 % 2 == 0; }

namespace {
void size_prep_buffers(pmx_operator* op, int n_rhs, bool need32) {
  const int64_t N = op->s->g.N;
  Ctx* ctx = &op->s->ctx->c;
  const int64_t nb = (N + kBlock - 1) / kBlock;
  if (op->qt64.n < (size_t)n_rhs * N) op->qt64.alloc(ctx, (size_t)n_rhs * N);
  if (need32 && op->qt32.n < (size_t)n_rhs * N) op->qt32.alloc(ctx, (size_t)n_rhs * N);
  if (op->ssum_part.n < (size_t)n_rhs * nb) op->ssum_part.alloc(ctx, (size_t)n_rhs * nb);
  if (op->ssum.n < (size_t)n_rhs) op->ssum.alloc(ctx, n_rhs);
}
}  // namespace

void source_prep_batch(const std::vector<ApplyJob>& jobs, int n_rhs, bool need32, hipStream_t st) {
  std::vector<PrepArgs> pa;
  std::vector<SumArgs> sa;
  std::vector<int64_t> pb, sb;
  for (const ApplyJob& j : jobs) {
    pmx_operator* op = j.op;
    PMX_REQUIRE(!(j.sc && need32), PMX_ERR_INVALID, "caller scratch serves the FP64 direct apply only");
    if (!j.sc) size_prep_buffers(op, n_rhs, need32);
    double* q64 = j.sc ? j.sc->qt64 : op->qt64.p;
    double* spart = j.sc ? j.sc->spart : op->ssum_part.p;
    double* ssum = j.sc ? j.sc->ssum : op->ssum.p;
    const int64_t N = op->s->g.N, nb = (N + kBlock - 1) / kBlock;
    pa.push_back({N, nb, j.sigma, op->s->g.w.p, op->co.w_over_a.p, q64, need32 ? op->qt32.p : nullptr, spart});
    pb.push_back(nb * n_rhs);
    sa.push_back({nb, spart, ssum});
    sb.push_back(n_rhs);
  }
  launch_grouped(pa, pb, [&](const Group<PrepArgs>& g, int64_t nblk) {
    hipLaunchKernelGGL(k_source_prep, dim3((unsigned)nblk), dim3(kBlock), 0, st, g);
    PMX_HIP(hipGetLastError());
  });
  launch_grouped(sa, sb, [&](const Group<SumArgs>& g, int64_t nblk) {
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)nblk), dim3(kBlock), 0, st, g);
    PMX_HIP(hipGetLastError());
  });
}

void source_prep(pmx_operator* op, const double* sigma, int n_rhs, bool need32, hipStream_t st) {
  source_prep_batch({ApplyJob{op, sigma, nullptr}}, n_rhs, need32, st);
}

namespace {
template <int NR>
void combine_launch(const std::vector<CombineArgs>& recs, hipStream_t st) {
  std::vector<int64_t> nb;
  for (const CombineArgs& c : recs) nb.push_back((c.N + kTPB - 1) / kTPB);
  launch_grouped(recs, nb, [&](const Group<CombineArgs>& g, int64_t nblk) {
    hipLaunchKernelGGL(k_near_combine<NR>, dim3((unsigned)nblk), dim3(kBlock), 0, st, g);
    PMX_HIP(hipGetLastError());
  });
}

CombineArgs combine_args(pmx_operator* op, const double* sigma, double* y, int n_rhs, int r0, int n_far,
                         const double* far, bool parametrix, const double* ssum) {
  const int q2 = op->s->g.q * op->s->g.q;
  CombineArgs c;
  c.N = op->s->g.N;
  c.q2 = q2;
  c.n_rhs = n_rhs;
  c.r0 = r0;
  c.n_far = n_far;
  c.identity = parametrix ? 0 : 1;
  c.magic = (uint32_t)((((uint64_t)1 << 32) + (uint64_t)q2 - 1) / (uint64_t)q2);
  c.ptr = op->nl.ptr.p;
  c.patch = op->nl.patch.p;
  c.Cb = parametrix ? op->nl.D.p : op->nl.C.p;
  c.sigma = sigma;
  c.paired = (q2 % 2 == 0 && c.N % 2 == 0 && ((uintptr_t)sigma % 16) == 0 && ((uintptr_t)c.Cb % 16) == 0) ? 1 : 0;
  c.far = far;
  c.ssum = ssum;
  c.rank1 = op->co.has_c() ? 0 : 1;
  c.y = y;
  return c;
}

// Near correction and combination for several operators; n_far[k] partial far fields each.
void combine_all(const std::vector<ApplyJob>& jobs, const std::vector<int>& n_far, bool parametrix, int n_rhs,
                 hipStream_t st, int r_begin = 0) {
  int r0 = r_begin;
  while (r0 < n_rhs) {
    const int left = n_rhs - r0;
    const int nr = left >= 8 ? 8 : (left >= 4 ? 4 : (left >= 2 ? 2 : 1));
    std::vector<CombineArgs> recs;
    for (size_t k = 0; k < jobs.size(); ++k) {
      pmx_operator* op = jobs[k].op;
      const ApplyScratch* sc = jobs[k].sc;
      const double* far = n_far[k] > 0 ? (sc ? sc->part : op->part.p) : nullptr;
      recs.push_back(combine_args(op, jobs[k].sigma, jobs[k].y, n_rhs, r0, n_far[k], far, parametrix,
                                  sc ? sc->ssum : op->ssum.p));
    }
    if (nr == 8) combine_launch<8>(recs, st);
    else if (nr == 4) combine_launch<4>(recs, st);
    else if (nr == 2) combine_launch<2>(recs, st);
    else combine_launch<1>(recs, st);
    r0 += nr;
  }
}
}  // namespace

void near_combine(pmx_operator* op, const double* sigma, double* y, int n_rhs, int n_part, bool parametrix,
                  hipStream_t st) {
  combine_all({ApplyJob{op, sigma, y}}, {n_part}, parametrix, n_rhs, st);
}

// c > 0: the imaginary parts Ci of the blocks couple the two real columns of each complex
// density: after the combine has added the real parts, Re y -= Ci Im sigma and Im y += Ci Re sigma.
// Half a wavefront per target streams the target's blocks, one complex density per grid row.
struct CrossArgs {
  int64_t N;
  int q2;
  const int64_t* ptr;
  const int32_t* patch;
  const double* Ci;
  const double* sigma;   // 2 n_vec columns of N
  double* y;
};

__global__ void __launch_bounds__(kBlock) k_near_cross(CrossArgs A) {
  const int64_t N = A.N;
  const int q2 = A.q2;
  const int sl = threadIdx.x & (kSub - 1);
  const int64_t i = (int64_t)blockIdx.x * kTPB + (threadIdx.x / kSub);
  const bool live = i < N;                  // both halves of a wave stay for the shuffles
  const int64_t ii = live ? i : N - 1;
  const double* __restrict__ sr = A.sigma + (int64_t)(2 * blockIdx.y) * N;
  const double* __restrict__ si = sr + N;
  double ar = 0.0, ai = 0.0;
  for (int64_t e = A.ptr[ii]; e < A.ptr[ii + 1]; ++e) {
    const int64_t base = (int64_t)A.patch[e] * q2;
    const double* __restrict__ cb = A.Ci + e * q2;
    for (int t = sl; t < q2; t += kSub) {
      const double c = cb[t];
      ar = fma(-c, si[base + t], ar);
      ai = fma(c, sr[base + t], ai);
    }
  }
  ar = sub_sum(ar);
  ai = sub_sum(ai);
  if (live && sl == 0) {
    A.y[(int64_t)(2 * blockIdx.y) * N + i] += ar;
    A.y[(int64_t)(2 * blockIdx.y + 1) * N + i] += ai;
  }
}

void near_cross(pmx_operator* op, const double* sigma, double* y, int n_cols, bool parametrix, hipStream_t st) {
  const int64_t N = op->s->g.N;
  const double* Ci = parametrix ? op->nl.Di.p : op->nl.Ci.p;
  PMX_REQUIRE(Ci != nullptr, PMX_ERR_INVALID, "imaginary near blocks missing");
  const CrossArgs a{N, op->s->g.q * op->s->g.q, op->nl.ptr.p, op->nl.patch.p, Ci, sigma, y};
  hipLaunchKernelGGL(k_near_cross, dim3((unsigned)((N + kTPB - 1) / kTPB), (unsigned)(n_cols / 2)), dim3(kBlock), 0,
                     st, a);
  PMX_HIP(hipGetLastError());
}

void near_combine_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st) {
  std::vector<int> nf;
  for (const ApplyJob& j : jobs) nf.push_back(far_direct_chunks(j.op, true));
  combine_all(jobs, nf, false, n_rhs, st);
  for (const ApplyJob& j : jobs)
    if (j.op->cplx()) near_cross(j.op, j.sigma, j.y, n_rhs, false, st);
}

void near_only_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st) {
  // whole groups of 16 (then 8) right-hand sides by target patch, the rest per target
  bool tiles = n_rhs >= 8;
  for (const ApplyJob& j : jobs)
    tiles = tiles && j.op->nl.have_tiles && near_tiled_fits(j.op->s->g.q * j.op->s->g.q) &&
            (uintptr_t)j.sigma % 16 == 0 && (uintptr_t)j.op->nl.C.p % 16 == 0;   // 16-byte staged slots
  int r0 = 0;
  while (tiles && n_rhs - r0 >= 8) {
    const int rb = n_rhs - r0 >= 16 ? 16 : 8;
    std::vector<TiledArgs> ta;
    std::vector<int64_t> tb;
    for (const ApplyJob& j : jobs) {
      pmx_operator* op = j.op;
      const int q2 = op->s->g.q * op->s->g.q;
      const int ns = near_tiled_slabs(q2);
      ta.push_back({op->s->g.N, op->s->g.M, q2, r0, ns, op->nl.tile_ptr.p, op->nl.tile_patch.p,
                    op->nl.tile_pair.p, op->nl.C.p, j.sigma, op->ssum.p, j.y});
      tb.push_back(op->s->g.M * ns);
    }
    const size_t lds = near_tiled_lds(0);
    launch_grouped(ta, tb, [&](const Group<TiledArgs>& g, int64_t nb) {
      if (rb == 16) hipLaunchKernelGGL(k_near_tiled<16>, dim3((unsigned)nb), dim3(256), lds, st, g);
      else hipLaunchKernelGGL(k_near_tiled<8>, dim3((unsigned)nb), dim3(256), lds, st, g);
      PMX_HIP(hipGetLastError());
    });
    r0 += rb;
  }
  if (r0 == 0) {
    combine_all(jobs, std::vector<int>(jobs.size(), 0), false, n_rhs, st);
    return;
  }
  if (r0 < n_rhs)   // the remaining right-hand sides, per target
    combine_all(jobs, std::vector<int>(jobs.size(), 0), false, n_rhs, st, r0);
}

void build_near_tiles(Ctx* ctx, const Geometry& g, NearLists& nl, hipStream_t st) {
  if (nl.have_tiles) return;
  const int64_t N = g.N, M = g.M;
  const int q2 = g.q * g.q;
  PMX_REQUIRE(nl.nnz < ((int64_t)1 << 31), PMX_ERR_INVALID, "too many near pairs for the tiled near correction");
  std::vector<int64_t> ptr(N + 1);
  std::vector<int32_t> patch(nl.nnz);
  PMX_HIP(hipMemcpyAsync(ptr.data(), nl.ptr.p, (N + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  if (nl.nnz)
    PMX_HIP(hipMemcpyAsync(patch.data(), nl.patch.p, nl.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> tptr(M + 1, 0), tpatch, tpair, uni;
  for (int64_t T = 0; T < M; ++T) {
    uni.clear();
    for (int t = 0; t < q2; ++t) {
      const int64_t i = T * q2 + t;
      for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) uni.push_back(patch[e]);
    }
    std::sort(uni.begin(), uni.end());
    uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
    const size_t base = tpatch.size();
    tpatch.insert(tpatch.end(), uni.begin(), uni.end());
    tpair.resize(tpatch.size() * (size_t)q2, -1);
    for (int t = 0; t < q2; ++t) {
      const int64_t i = T * q2 + t;
      for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
        const size_t u = (size_t)(std::lower_bound(uni.begin(), uni.end(), patch[e]) - uni.begin());
        tpair[(base + u) * q2 + t] = (int32_t)e;
      }
    }
    tptr[T + 1] = (int32_t)tpatch.size();
  }
  auto up = [&](DBuf<int32_t>& buf, const std::vector<int32_t>& v) {
    buf.alloc(ctx, v.size());
    if (!v.empty()) PMX_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  };
  up(nl.tile_ptr, tptr);
  up(nl.tile_patch, tpatch);
  up(nl.tile_pair, tpair);
  PMX_HIP(hipStreamSynchronize(st));   // the host vectors go out of scope
  nl.have_tiles = true;
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
  Group<SumArgs> g;
  g.n = 1;
  g.off[1] = n_rhs;
  g.a[0] = SumArgs{nb, op->ssum_part.p, s.p};
  hipLaunchKernelGGL(k_sum_partials, dim3(n_rhs), dim3(kBlock), 0, st, g);
  PMX_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sub_mean, dim3(nb, n_rhs), dim3(kBlock), 0, st, N, u, s.p, op->s->g.area);
  PMX_HIP(hipGetLastError());
  PMX_HIP(hipStreamSynchronize(st));   // s is released on return
}

}  // namespace pmx
