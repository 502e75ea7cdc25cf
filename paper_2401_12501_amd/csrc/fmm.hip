// Chebyshev-interpolation FMM for the far field of the remainder operator (FP32).
//
// The far-field sum of the c = 0 remainder (eq:explicit_remainder) at target i is
//   phi_i = A_i n_i^T F2_i n_i - B_i n_i . F1_i + g_i . F1_i,
//   F1_i = sum_j qt_j r/r^2,  F2_i = sum_j qt_j r r^T / r^4,  r = x_i - x_j,
// (equivalently n'^T F2 n' + h . F1 with n' = sqrt(A) n, h = g - B n),
// so it needs the nine translation-invariant, homogeneous kernel components
// k(r) = [r/r^2 (3), r r^T/r^4 (6)] applied to the scalar strengths qt = w sigma / a.
// The paper accelerates the apply with an interpolative-decomposition FMM
// (Section 6.2); this file instead uses a tensor Chebyshev interpolation FMM on
// an octree of uniform depth:
//   P2M  leaf multipoles  W_m = sum_j S(t_m, x_j) qt_j  (p^3 Chebyshev nodes per box)
//   M2M  parent W from the children's W by interpolation
//   M2L  L_c,l += sum_m k_c(x_l - y_m) W_m for every well-separated pair (FP32 MFMA)
//   L2L  children's L from the parent's L by interpolation
//   L2P  F_c(x_i) = sum_l S(t_l, x_i) L_c,l, then the target contraction above
//   P2P  direct sum over adjacent leaves (the U-list), j = i excluded.
// S is the tensor product of 1-D Chebyshev interpolation weights
//   S1(t_k, x) = 1/p + (2/p) sum_{n=1}^{p-1} T_n(t_k) T_n(x).
// M2L uses translation invariance and homogeneity: for boxes of half-width h at
// offset o (in box widths), x_l - y_m = h (2 o + t_l - t_m), and the kernel of a
// unit box is generated on the fly in registers as the MFMA A operand, then
// scaled by h^-1 (F1) or h^-2 (F2).  One right-hand side: pairs are grouped by
// offset across levels, so one generated kernel block serves the 16 pairs of an
// MFMA column block, each writing its own output slot (summed per box afterwards).
// Blocks of 16 right-hand sides: the right-hand sides are the 16 columns and each
// box walks its own sources.  Several right-hand sides also share the P2P pair
// evaluations.  The P2P sums (and the caller's near correction) may run on a
// second stream while P2M, M2M, M2L and L2L run on the caller's stream.
#include <algorithm>
#include <functional>
#include <type_traits>
#include <cmath>
#include <unordered_map>

#include <hipcub/hipcub.hpp>

#include "pmx_internal.hpp"

namespace pmx {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Floats per box of the local expansions (nine components of p^3 values) and per M2L output
// slot: padded to a multiple of 4 so the slot sum reads and writes whole float4s.
constexpr int lstride_of(int p) { return (9 * p * p * p + 3) & ~3; }
template <int P>
constexpr int lstride() { return lstride_of(P); }

namespace {
constexpr int kRBlock = 16;     // right-hand sides per multi-charge P2P launch
constexpr int kMaxLevel = 20;
constexpr int kColTiles = 2;    // MFMA column tiles per M2L work item
constexpr int kItemCols = 16 * kColTiles;   // box pairs per M2L work item
}  // namespace

struct FMM {
  int p = 6, p3 = 216, L = 0;
  double c0[3] = {0, 0, 0}, h0 = 1.0;
  std::vector<int64_t> lev_off;      // first global box index of each level, size L + 2
  int64_t n_boxes = 0, n_leaves = 0;
  int64_t m2l_pairs = 0, p2p_pairs = 0;
  int64_t n_items = 0;
  DBuf<float> center;        // 3 * n_boxes
  DBuf<int32_t> child_begin; // n_boxes (global index of first child, levels < L)
  DBuf<int32_t> child_end;
  DBuf<int32_t> parent;      // n_boxes
  DBuf<int32_t> octant;      // n_boxes (child position bits x | y << 1 | z << 2)
  DBuf<int32_t> leaf_start;  // n_leaves + 1 (sorted point ranges)
  DBuf<int32_t> perm;        // N: sorted position -> node
  DBuf<float> pts;           // 9 N sorted: x y z n'x n'y n'z hx hy hz (n' = sqrt(A) n, h = g - B n)
  DBuf<float> qs;            // 4 N sorted source rows: x y z qt (one rhs at a time)
  DBuf<int32_t> u_ptr, u_idx;        // U-list of leaves (leaf-local indices)
  DBuf<int4> p2p_desc;       // P2P waves: first and end target, first and end source (sorted positions)
  DBuf<int32_t> p2p_slot;    // U-list slot of each P2P wave
  int64_t n_p2p_waves = 0;
  DBuf<int32_t> p2p_cptr;    // waves of each (leaf, 64-target chunk): [cptr[c], cptr[c + 1])
  DBuf<int2> chunks;         // (leaf, first target) of each 64-target chunk (L2P blocks)
  int64_t n_p2p_chunks = 0;
  // several right-hand sides: source rows (x, y, z, qt_0 .. qt_{R-1}, zero padding) of stride
  // rstride floats, and the P2P sums per (rhs, sorted target)
  DBuf<float> qsR, partR;
  int rstride = 0, r_cap = 0;
  // sixteen right-hand sides at once: the M2L sources of each box of levels >= 2 in slot order
  // (source box, offset code), and multipoles / locals with one slice per right-hand side
  DBuf<int2> tsrc;
  DBuf<int64_t> lev_off_d;   // device copy of lev_off
  DBuf<float> W16, L16;
  DBuf<int32_t> m2l_t, m2l_s;        // global box indices of the pairs, sorted by (offset, level)
  DBuf<int32_t> m2l_lv;              // level of each pair
  DBuf<int4> items;                  // (first pair, count, -, offset code)
  DBuf<float> tab;                   // t_k (p), M1[2][p][p], node table (3 p^3)
  DBuf<float> W, Lc;                 // multipoles n_boxes*p3, locals n_boxes*9*p3
  DBuf<float> slots;                 // M2L output per pair (9*p3 each)
  DBuf<int32_t> r_ptr;              // per box of levels >= 2: its run of output slots
  DBuf<int32_t> m2l_slot;           // output slot of each pair (a box's slots are contiguous)
  DBuf<float> phis;                  // 27 N: P2P partial sums per U-list slot (sorted order)
};

// ----------------------------------------------------------------------------- device helpers
template <int P>
__device__ __forceinline__ void cheb_weights(const float* __restrict__ t, float x, float* out) {
  // out[k] = S1(t_k, x) = 1/P + (2/P) sum_{n>=1} T_n(t_k) T_n(x)
  float Tx[P];
  Tx[0] = 1.0f;
  if (P > 1) Tx[1] = x;
#pragma unroll
  for (int n = 2; n < P; ++n) Tx[n] = 2.0f * x * Tx[n - 1] - Tx[n - 2];
  constexpr float ip = 1.0f / (float)P;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const float tk = t[k];
    float a0 = 1.0f, a1 = tk, s = 0.0f;
#pragma unroll
    for (int n = 1; n < P; ++n) {
      s = fmaf(a1, Tx[n], s);
      const float a2 = 2.0f * tk * a1 - a0;
      a0 = a1;
      a1 = a2;
    }
    out[k] = ip + 2.0f * ip * s;
  }
}

// Sorted source rows: qs[k] = (x_k, y_k, z_k, qt[perm[k]]), one 16-byte row per point.
struct PermArgs {
  int64_t N;
  const int32_t* perm;
  const float* pts;
  const float* q;
  float* qs;
};

__global__ void __launch_bounds__(256) k_permute(Group<PermArgs> g) {
  int64_t lb;
  const PermArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t N = A.N;
  const int64_t k = lb * 256 + threadIdx.x;
  if (k < N)
    reinterpret_cast<float4*>(A.qs)[k] = make_float4(A.pts[k], A.pts[N + k], A.pts[2 * N + k], A.q[A.perm[k]]);
}

typedef const __attribute__((address_space(4))) float* sfp;   // uniform loads through the scalar cache

// P2M: one block per leaf; thread m accumulates over the leaf's sources.
struct P2MArgs {
  int64_t leaf_off, N;
  float h;
  const float* tab;
  const float* center;
  const int32_t* leaf_start;
  const float* pts;
  const float* qs;
  float* W;
};

template <int P>
__global__ void __launch_bounds__(256) k_p2m(Group<P2MArgs> g) {
  constexpr int p = P, p3 = P * P * P;
  __shared__ float sw[256][3 * P + 1];
  int64_t lb;
  const P2MArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t leaf_off = A.leaf_off, N = A.N;
  const float h = A.h;
  const float* __restrict__ tab = A.tab;
  const float* __restrict__ center = A.center;
  const int32_t* __restrict__ leaf_start = A.leaf_start;
  const float* __restrict__ pts = A.pts;
  const float* __restrict__ qs = A.qs;
  float* __restrict__ W = A.W;
  const int leaf = (int)lb;
  const int64_t box = leaf_off + leaf;
  const int s0 = leaf_start[leaf], s1 = leaf_start[leaf + 1];
  const float cx = center[3 * box], cy = center[3 * box + 1], cz = center[3 * box + 2];
  const float ih = 1.0f / h;
  const int m = threadIdx.x;
  const int m1 = m / (p * p), m2 = (m / p) % p, m3 = m % p;
  float acc = 0.0f;
  for (int j0 = s0; j0 < s1; j0 += 256) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    if (j < s1) {
      const float4 sj = reinterpret_cast<const float4*>(qs)[j];
      cheb_weights<P>(tab, (sj.x - cx) * ih, &sw[threadIdx.x][0]);
      cheb_weights<P>(tab, (sj.y - cy) * ih, &sw[threadIdx.x][p]);
      cheb_weights<P>(tab, (sj.z - cz) * ih, &sw[threadIdx.x][2 * p]);
      sw[threadIdx.x][3 * p] = sj.w;
    }
    __syncthreads();
    const int lim = min(256, s1 - j0);
    if (m < p3)
      for (int t = 0; t < lim; ++t) acc = fmaf(sw[t][m1] * sw[t][p + m2] * sw[t][2 * p + m3], sw[t][3 * p], acc);
  }
  if (m < p3) W[box * p3 + m] = acc;
}

// P2M for a block of 16 right-hand sides: as k_p2m (one block per leaf, thread m per
// coefficient), with the sources' rows of the block (x, y, z, q_0 .. q_15): each source's
// Chebyshev basis product is formed once and applied to its 16 charges.  Every right-hand
// side's sum takes the same operations in the same order as k_p2m, so W16 holds the same bits.
struct P2M16Args {
  int64_t leaf_off;
  float h;
  int stride;             // source row length (x, y, z and the 16 charges first)
  const float* tab;
  const float* center;
  const int32_t* leaf_start;
  const float* qsR;
  float* W16;
  int64_t slice;          // floats between right-hand-side slices of W16
};

template <int P>
__global__ void __launch_bounds__(256) k_p2m16(Group<P2M16Args> g) {
  constexpr int p = P, p3 = P * P * P;
  constexpr int kW = 3 * P + kRBlock + 1;   // basis values, charges, one pad (odd row length)
  __shared__ float sw[256][kW];
  int64_t lb;
  const P2M16Args& A = seg_of(g, blockIdx.x, lb);
  const float* __restrict__ tab = A.tab;
  const int leaf = (int)lb;
  const int64_t box = A.leaf_off + leaf;
  const int s0 = A.leaf_start[leaf], s1 = A.leaf_start[leaf + 1];
  const float cx = A.center[3 * box], cy = A.center[3 * box + 1], cz = A.center[3 * box + 2];
  const float ih = 1.0f / A.h;
  const int m = threadIdx.x;
  const int m1 = m / (p * p), m2 = (m / p) % p, m3 = m % p;
  float acc[kRBlock];
#pragma unroll
  for (int r = 0; r < kRBlock; ++r) acc[r] = 0.0f;
  for (int j0 = s0; j0 < s1; j0 += 256) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    if (j < s1) {
      const float* __restrict__ row = A.qsR + (int64_t)j * A.stride;
      cheb_weights<P>(tab, (row[0] - cx) * ih, &sw[threadIdx.x][0]);
      cheb_weights<P>(tab, (row[1] - cy) * ih, &sw[threadIdx.x][p]);
      cheb_weights<P>(tab, (row[2] - cz) * ih, &sw[threadIdx.x][2 * p]);
#pragma unroll
      for (int r = 0; r < kRBlock; ++r) sw[threadIdx.x][3 * p + r] = row[3 + r];
    }
    __syncthreads();
    const int lim = min(256, s1 - j0);
    if (m < p3)
      for (int t = 0; t < lim; ++t) {
        const float b = sw[t][m1] * sw[t][p + m2] * sw[t][2 * p + m3];
#pragma unroll
        for (int r = 0; r < kRBlock; ++r) acc[r] = fmaf(b, sw[t][3 * p + r], acc[r]);
      }
  }
  if (m < p3) {
#pragma unroll
    for (int r = 0; r < kRBlock; ++r) A.W16[r * A.slice + box * p3 + m] = acc[r];
  }
}

// M2M: parent W from its children (one block per parent box of one level).
struct M2MArgs {
  int64_t lev_first;
  const float* tab;
  const int32_t* child_begin;
  const int32_t* child_end;
  const int32_t* octant;
  float* W;
  int64_t slice;          // floats between right-hand-side slices of W (grid y), 0 for one
};

// The interpolation operator is a tensor product, so each child's contribution is
// applied one axis at a time (3 p^4 multiply-adds instead of p^6), through LDS.  All the
// children go through each axis pass together (threads over child x node), and their
// contributions are summed in child order at the end.
template <int P>
__global__ void __launch_bounds__(256) k_m2m(Group<M2MArgs> g) {
  constexpr int p = P, p3 = P * P * P;
  __shared__ float sW[8 * p3], sT[8 * p3];
  __shared__ float sM[2 * p * p];
  __shared__ int sOct[8];
  int64_t lb;
  const M2MArgs& A = seg_of(g, blockIdx.x, lb);
  float* __restrict__ W = A.W + (int64_t)blockIdx.y * A.slice;
  const int64_t Pb = A.lev_first + lb;
  const int c0 = A.child_begin[Pb], nch = A.child_end[Pb] - c0;   // at most 8 children
  for (int e = threadIdx.x; e < 2 * p * p; e += blockDim.x) sM[e] = A.tab[p + e];   // M1[b][k][k']
  if (threadIdx.x < nch) sOct[threadIdx.x] = A.octant[c0 + threadIdx.x];
  for (int e = threadIdx.x; e < nch * p3; e += blockDim.x) sW[e] = W[(int64_t)c0 * p3 + e];
  __syncthreads();
  // z: T[c][a][b][m3] = sum_d Mz_c[m3][d] W[c][a][b][d]
  for (int e = threadIdx.x; e < nch * p3; e += blockDim.x) {
    const int ch = e / p3, m = e - ch * p3;
    const int i1 = m / (p * p), i2 = (m / p) % p, i3 = m % p;
    const float* Mz = sM + ((sOct[ch] >> 2) & 1) * p * p;
    float t = 0.0f;
    for (int d = 0; d < p; ++d) t = fmaf(Mz[i3 * p + d], sW[ch * p3 + (i1 * p + i2) * p + d], t);
    sT[e] = t;
  }
  __syncthreads();
  // y: W'[c][a][m2][m3] = sum_b My_c[m2][b] T[c][a][b][m3]
  for (int e = threadIdx.x; e < nch * p3; e += blockDim.x) {
    const int ch = e / p3, m = e - ch * p3;
    const int i1 = m / (p * p), i2 = (m / p) % p, i3 = m % p;
    const float* My = sM + ((sOct[ch] >> 1) & 1) * p * p;
    float t = 0.0f;
    for (int bb = 0; bb < p; ++bb) t = fmaf(My[i2 * p + bb], sT[ch * p3 + (i1 * p + bb) * p + i3], t);
    sW[e] = t;
  }
  __syncthreads();
  // x: out[m1][m2][m3] = sum_c sum_a Mx_c[m1][a] W'[c][a][m2][m3], children in order
  for (int m = threadIdx.x; m < p3; m += blockDim.x) {
    const int i1 = m / (p * p), i2 = (m / p) % p, i3 = m % p;
    float acc = 0.0f;
    for (int ch = 0; ch < nch; ++ch) {
      const float* Mx = sM + (sOct[ch] & 1) * p * p;
      float t = 0.0f;
      for (int aa = 0; aa < p; ++aa) t = fmaf(Mx[i1 * p + aa], sW[ch * p3 + (aa * p + i2) * p + i3], t);
      acc += t;
    }
    W[Pb * p3 + m] = acc;
  }
}

// L2L: child L += interpolation of the parent's L (one block per child box of one level).
struct L2LArgs {
  int64_t lev_first;
  const float* tab;
  const int32_t* parent;
  const int32_t* octant;
  float* Lc;
  int64_t slice;          // floats between right-hand-side slices of Lc (grid y), 0 for one
};

// Child L += the parent's L interpolated to the child, one axis at a time through LDS
// (3 p^4 multiply-adds per component instead of p^6).
template <int P>
__global__ void __launch_bounds__(256) k_l2l(Group<L2LArgs> g) {
  constexpr int p = P, p3 = P * P * P;
  constexpr int n = 9 * p3;
  __shared__ float sA[n], sB[n];
  __shared__ float sM[2 * p * p];
  int64_t lb;
  const L2LArgs& A = seg_of(g, blockIdx.x, lb);
  float* __restrict__ Lc = A.Lc + (int64_t)blockIdx.y * A.slice;
  const int64_t C = A.lev_first + lb;
  const int64_t Pb = A.parent[C];
  const int o = A.octant[C];
  for (int e = threadIdx.x; e < 2 * p * p; e += blockDim.x) sM[e] = A.tab[p + e];
  for (int e = threadIdx.x; e < n; e += blockDim.x) sA[e] = Lc[Pb * lstride<P>() + e];
  __syncthreads();
  const float* Mx = sM + (o & 1) * p * p;          // Mx[a * p + l1] = S1(t_a, child node l1)
  const float* My = sM + ((o >> 1) & 1) * p * p;
  const float* Mz = sM + ((o >> 2) & 1) * p * p;
  // z: B[c][a][b][l3] = sum_d Mz[d][l3] A[c][a][b][d]
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int l3 = e % p, r = e - l3;
    float t = 0.0f;
    for (int d = 0; d < p; ++d) t = fmaf(Mz[d * p + l3], sA[r + d], t);
    sB[e] = t;
  }
  __syncthreads();
  // y: A[c][a][l2][l3] = sum_b My[b][l2] B[c][a][b][l3]
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int l3 = e % p, l2 = (e / p) % p, r = e - l3 - l2 * p;
    float t = 0.0f;
    for (int bb = 0; bb < p; ++bb) t = fmaf(My[bb * p + l2], sB[r + bb * p + l3], t);
    sA[e] = t;
  }
  __syncthreads();
  // x: L[c][l1][l2][l3] += sum_a Mx[a][l1] A[c][a][l2][l3]
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int l23 = e % (p * p), l1 = (e / (p * p)) % p, cc = e / p3;
    float t = 0.0f;
    for (int aa = 0; aa < p; ++aa) t = fmaf(Mx[aa * p + l1], sA[cc * p3 + aa * p * p + l23], t);
    Lc[C * lstride<P>() + e] += t;
  }
}

// M2L on MFMA.  Work items of up to 32 box pairs (two MFMA column tiles) whose sources
// sit at the same offset (in box widths); a persistent grid of one workgroup per compute
// unit takes the items in turn.  By homogeneity the
// unit-box kernel of an offset is the same at every level, so an item may mix levels;
// each column is scaled by its level's h^-1 (F1) or h^-2 (F2) when written.  The
// item's source multipoles are staged in LDS once; each wave takes one 16-row tile,
// generates the unit-box kernel for all nine components of its (row, m) pairs in
// registers as MFMA A operands, each feeding both column tiles, and keeps eighteen
// accumulator tiles.  A compute unit issues MFMAs from four SIMDs, so when the row tiles
// are not a multiple of four (p = 6: 14 tiles) the split layout divides the last two
// tiles by column tile over four half waves, one in each group of four waves and one per
// SIMD whether the waves are dealt round-robin or in blocks: every SIMD then carries seven
// tile-units instead of eight on two SIMDs and six on the other two.  Its sixteen waves
// fill every SIMD's registers, so it is launched when the M2L has the compute units to
// itself; beside the second stream's kernels the 14-wave layout runs, whose two SIMDs with
// three waves leave register room for the P2P waves (measured faster that way, while the
// split layout is faster alone).  The items are many more than the resident workgroups,
// and the second stream's work fills the launch's tail.
// Each pair writes its own output slot; k_m2l_reduce then sums a target's slots in a
// fixed order, so no atomics are needed and the result does not depend on scheduling.
constexpr int kM2LStride = 226;   // LDS row stride (== 2 mod 32: conflict-free B reads)

struct M2LArgs {
  const float* tab;
  const int4* items;      // (first pair, count, -, offset code)
  const int32_t* ps;      // source box per pair
  const int32_t* plev;    // level per pair
  const int32_t* pslot;   // output slot per pair
  const float* W;
  float* slots;
  double h0;
};

// Workgroups of the persistent M2L launch: one per compute unit of the current device.
static int64_t m2l_persistent_blocks() {
  static thread_local int cached_dev = -1;
  static thread_local int64_t cached = 0;
  int dev = 0;
  PMX_HIP(hipGetDevice(&dev));
  if (dev != cached_dev) {
    int cus = 0;
    PMX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    cached = cus > 0 ? cus : 256;
    cached_dev = dev;
  }
  return cached;
}

template <int P>
constexpr int m2l_row_tiles() { return (P * P * P + 15) / 16; }   // 14, 8, 4
template <int P>
constexpr bool m2l_can_split() { return m2l_row_tiles<P>() % 4 == 2; }   // p = 6
template <int P, bool Split>
constexpr int m2l_waves() { return m2l_row_tiles<P>() + (Split ? 2 : 0); }   // 16 split; 14, 8, 4

template <int P, bool Split>
__global__ void __launch_bounds__((64 * m2l_waves<P, Split>())) k_m2l(Group<M2LArgs> g) {
  constexpr int p3 = P * P * P;
  static_assert(p3 <= kM2LStride, "multipole does not fit the LDS row");
  constexpr int n_rt = m2l_row_tiles<P>();
  constexpr int n_waves = m2l_waves<P, Split>();
  constexpr bool kSplit = Split;
  static_assert(!kSplit || (m2l_can_split<P>() && n_waves == 16),
                "half waves 0, 5, 10, 15: one per group of four and per SIMD");
  // persistent: each workgroup takes items blockIdx.x, + gridDim.x, ...; the next item's
  // multipoles travel into the other LDS buffer while the current item is computed, so the
  // staging latency is off the critical path
  __shared__ float sB[2][kItemCols * kM2LStride];
  __shared__ float4 sN[p3];
  __shared__ float sS[2][2][kItemCols];
  __shared__ int sP[2][kItemCols];
  const int64_t total = g.off[g.n];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int kq = lane >> 4, col = lane & 15;
  // this wave's row tile; a half wave (split layout) takes one column tile, hc, of it
  const bool half = kSplit && (wave >> 2) == (wave & 3);
  const int rt = !kSplit ? wave : half ? n_rt - 2 + (wave >> 3) : wave - (wave + 4) / 5;
  const int hc = (wave >> 2) & 1;
  for (int m = threadIdx.x; m < p3; m += blockDim.x) {
    const float* nd = g.a[0].tab + P + 2 * P * P + 3 * m;   // node table: the same for every operator
    sN[m] = make_float4(nd[0], nd[1], nd[2], 0.0f);
  }
  // Item bi's column multipoles go straight from memory into LDS buffer buf (global_load_lds:
  // no registers, no wait until the next item's barrier): column j of the item is W[source box
  // of column j][0, p^3), in segments of 64 values, one wave-wide load each, dealt round the
  // waves.  The columns' source boxes (sQ) and the item's record (sQit) come from LDS, filled
  // by 32 threads before a barrier, so the loads do not wait on one another.  Columns past the item's count are not
  // loaded: an MFMA output column depends on its own B column only, and those outputs are
  // never stored.
  constexpr int kSeg = (p3 + 63) / 64;
  __shared__ int sQ[kItemCols];   // source box of each column of the next item
  __shared__ int4 sQit[2];        // item records: item k's in sQit[k & 1]
  auto fetch_next = [&](int64_t bi, int slot) {   // threads below kItemCols: item bi's record, sources
    int64_t lbi;
    const M2LArgs& B = seg_of(g, bi, lbi);
    const int4 itn = B.items[lbi];
    const int j = threadIdx.x;
    sQ[j] = B.ps[itn.x + (j < itn.y ? j : 0)];
    if (j == 0) sQit[slot] = itn;
  };
  auto prefetch = [&](int64_t bi, int buf, int nc) {
    int64_t lbi;
    const M2LArgs& B = seg_of(g, bi, lbi);
    for (int t = wave; t < nc * kSeg; t += n_waves) {
      const int j = t / kSeg, m0 = (t - j * kSeg) * 64;
      const int32_t sb = __builtin_amdgcn_readfirstlane(sQ[j]);
      if (m0 + lane < p3)
        __builtin_amdgcn_global_load_lds(
            (const void __attribute__((address_space(1)))*)(B.W + (int64_t)sb * p3 + m0 + lane),
            (void __attribute__((address_space(3)))*)(&sB[buf][j * kM2LStride + m0]), 4, 0, 0);
    }
  };
  if (blockIdx.x < total) {
    if (threadIdx.x < kItemCols) fetch_next(blockIdx.x, 0);
    __syncthreads();
    prefetch(blockIdx.x, 0, __builtin_amdgcn_readfirstlane(sQit[0].y));
    __syncthreads();   // sQ is rewritten before the first item's barrier
  }
  int k = 0;
  for (int64_t bi = blockIdx.x; bi < total; bi += gridDim.x, ++k) {
    const int buf = k & 1;
    int64_t lb;
    const M2LArgs& A = seg_of(g, bi, lb);
    // this item's record (written before an earlier barrier; the next one goes to the other slot)
    const int4 it = make_int4(__builtin_amdgcn_readfirstlane(sQit[buf].x), __builtin_amdgcn_readfirstlane(sQit[buf].y),
                              0, __builtin_amdgcn_readfirstlane(sQit[buf].w));
    const int ncol = it.y;
    const int64_t bn = bi + gridDim.x;
    if (threadIdx.x < kItemCols) {   // this buffer's previous item finished before the last barrier
      const int j = threadIdx.x;
      const int jj = j < ncol ? j : 0;
      const int lev = A.plev[it.x + jj], slot = A.pslot[it.x + jj];
      if (bn < total) fetch_next(bn, buf ^ 1);   // the last prefetch read sQ before the last barrier
      const double h = A.h0 / (double)(1 << lev);
      sS[buf][0][j] = (float)(1.0 / h);
      sS[buf][1][j] = (float)(1.0 / (h * h));
      sP[buf][j] = slot;
    }
    // this wave's loads of the item's multipoles (issued during the previous item) have landed;
    // after the barrier every wave's have, and the scales and slots are in LDS
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    __syncthreads();
    const int code = it.w;
    const float ox = 2.0f * (float)(code / 49 - 3), oy = 2.0f * (float)((code / 7) % 7 - 3),
                oz = 2.0f * (float)(code % 7 - 3);
    // a generated kernel value (A operand) serves the wave's column tiles, so the
    // generation's VALU work is spread over 9 MFMAs per column tile.  Rows past p^3 (last
    // tile) use node 0: with the offset at least two box widths away the kernel stays finite
    // there, and those rows are never stored.
    const int row = rt * 16 + col;
    const float4 tl = sN[row < p3 ? row : 0];
    const float tlx = tl.x + ox, tly = tl.y + oy, tlz = tl.z + oz;
    floatx4 acc[kColTiles][9];
#pragma unroll
    for (int ct = 0; ct < kColTiles; ++ct)
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[ct][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const float* sBb = sB[buf];
    // NCT column tiles from column tile t0 on: a full wave takes all of them, a half wave one
    auto run = [&](auto nct_tag, int t0) {
      constexpr int NCT = decltype(nct_tag)::value;
#pragma unroll 2
      for (int k0 = 0; k0 < p3; k0 += 4) {
        const int m = k0 + kq;
        const float4 tm = sN[m < p3 ? m : 0];
        // k past p^3 (p^3 not a multiple of 4): a zero B row removes the term
        float b0[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          b0[ct] = (p3 % 4 == 0 || m < p3) ? sBb[((t0 + ct) * 16 + col) * kM2LStride + (m < p3 ? m : 0)]
                                           : 0.0f;
        const float rx = tlx - tm.x, ry = tly - tm.y, rz = tlz - tm.z;
        const float inv = __builtin_amdgcn_rcpf(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
        // r / r^2 and (r r^T) / r^4 = (r / r^2)(r / r^2)^T
        float a[9];
        a[0] = rx * inv; a[1] = ry * inv; a[2] = rz * inv;
        a[3] = a[0] * a[0]; a[4] = a[0] * a[1]; a[5] = a[0] * a[2];
        a[6] = a[1] * a[1]; a[7] = a[1] * a[2]; a[8] = a[2] * a[2];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int c = 0; c < 9; ++c)
            acc[ct][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], b0[ct], acc[ct][c], 0, 0, 0);
      }
    };
    // an item of at most 16 pairs (an offset's last item) fills only the first column tile:
    // the second tile's MFMAs are skipped (ncol is the same for the whole workgroup)
    static_assert(kColTiles == 2, "one or two column tiles per item");
    const bool one_tile = ncol <= 16;
    if (half) {
      if (!(one_tile && hc == 1)) run(std::integral_constant<int, 1>{}, hc);
    } else if (one_tile) {
      run(std::integral_constant<int, 1>{}, 0);
    } else {
      run(std::integral_constant<int, kColTiles>{}, 0);
    }
    // the next item's multipoles into the other buffer (its item finished before the last
    // barrier); issued after the MFMA loop, whose LDS reads would otherwise wait for them, so
    // their latency overlaps the slot stores and the barriers
    if (bn < total) prefetch(bn, buf ^ 1, __builtin_amdgcn_readfirstlane(sQit[buf ^ 1].y));
    const int l0 = rt * 16 + 4 * kq;
#pragma unroll
    for (int ct = 0; ct < kColTiles; ++ct) {
      if (half && ct > 0) break;
      const int pj = (half ? hc : ct) * 16 + col;
      if (pj < ncol) {
        float* out = A.slots + (int64_t)sP[buf][pj] * lstride<P>();
        const float s1 = sS[buf][0][pj], s2 = sS[buf][1][pj];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const float sc = c < 3 ? s1 : s2;
          if (l0 + 3 < p3 && (p3 % 4) == 0) {   // four consecutive rows: one 16-byte store
            *reinterpret_cast<float4*>(out + c * p3 + l0) =
                make_float4(sc * acc[ct][c][0], sc * acc[ct][c][1], sc * acc[ct][c][2], sc * acc[ct][c][3]);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (l0 + r < p3) out[c * p3 + l0 + r] = sc * acc[ct][c][r];
          }
        }
      }
    }
    __syncthreads();   // every wave is done with this item's LDS buffers
  }
}

// M2L for a block of 16 right-hand sides: one workgroup per box of levels >= 2 walks the
// box's M2L sources in slot order; the 16 right-hand sides are the MFMA's 16 columns, so each
// generated kernel block serves all of them and the locals stay in registers across the
// sources (no per-pair output slots and no slot sum).  The next source's multipoles are loaded
// into registers while the current one is computed, then stored to the other LDS buffer.
// One wave per 16-row tile (4 and 8 waves at p = 4, 5).  With 14 row tiles (p = 6) the last
// two are split by source node (first and second half of the p^3) over four half waves, one
// in each group of four and one per SIMD, whose two partial sums are added at the end: 16
// waves, and every SIMD carries 3.5 tile-units per source.
struct M2L16Args {
  const float* tab;
  const int32_t* rptr;    // box b's sources are [rptr[b - box2], rptr[b - box2 + 1])
  const int2* tsrc;       // (source box, offset code)
  int64_t box2, n_boxes;
  int L;                  // leaf level: boxes of level l are [lev_off[l], lev_off[l + 1])
  const int64_t* lev_first;   // device copy of lev_off (L + 2 entries)
  const float* W16;       // 16 slices of n_boxes * p^3
  float* L16;             // 16 slices of n_boxes * lstride
  double h0;
};

template <int P>
constexpr int m2l16_waves() { return m2l_row_tiles<P>() + (m2l_can_split<P>() ? 2 : 0); }   // 16, 8, 4

template <int P>
__global__ void __launch_bounds__(64 * m2l16_waves<P>()) __attribute__((amdgpu_waves_per_eu(4)))
k_m2l16(Group<M2L16Args> g) {
  constexpr int p3 = P * P * P;
  constexpr int n_rt = (p3 + 15) / 16;
  constexpr int n_waves = m2l16_waves<P>();
  constexpr bool kSplit = m2l_can_split<P>();
  static_assert(kSplit ? (n_rt == 14 && n_waves == 16 && (p3 / 2) % 4 == 0) : n_waves == n_rt,
                "12 full and 4 half waves, or one row tile per wave");
  constexpr int NT = 1;
  constexpr int kThr = 64 * n_waves;
  constexpr int kPer = (16 * p3 + kThr - 1) / kThr;   // staged multipole values per thread
  int64_t lb;
  const M2L16Args& A = seg_of(g, blockIdx.x, lb);
  const int64_t box = A.box2 + lb;
  const int s0 = A.rptr[lb], s1 = A.rptr[lb + 1];
  const int64_t slice = A.n_boxes * (int64_t)p3;
  __shared__ __align__(16) float sB[2][16 * kM2LStride];
  static_assert(!kSplit || 2 * 9 * 64 * 4 <= 2 * 16 * kM2LStride, "the half waves' sums fit in sB");
  __shared__ float4 sN[p3];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // this wave's row tile; a half wave (split layout) takes half kh of the source nodes of
  // row tile 12 or 13
  const bool hw = kSplit && (wave >> 2) == (wave & 3);
  const int rt = !kSplit ? wave : hw ? n_rt - 2 + (wave >> 3) : wave - (wave + 4) / 5;
  const int kh = (wave >> 2) & 1;
  for (int m = threadIdx.x; m < p3; m += blockDim.x) {
    const float* nd = A.tab + P + 2 * P * P + 3 * m;
    sN[m] = make_float4(nd[0], nd[1], nd[2], 0.0f);
  }
  float stage[kPer];
  auto load = [&](int si) {
    const int64_t sb = A.tsrc[si].x;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + q * kThr;
      const int j = e / p3, m = e - j * p3;
      stage[q] = e < 16 * p3 ? A.W16[j * slice + sb * p3 + m] : 0.0f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + q * kThr;
      const int j = e / p3, m = e - j * p3;
      if (e < 16 * p3) sB[buf][j * kM2LStride + m] = stage[q];
    }
  };
  if (s0 < s1) {
    load(s0);
    store(0);
  }
  __syncthreads();
  const int kq = lane >> 4, col = lane & 15;
  // one accumulator per source (its p^3-term sums), added to the running total afterwards:
  // the same two-level summation as per-pair slots, so rounding does not grow with the
  // number of sources
  floatx4 tot[NT][9];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < 9; ++c) tot[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int si = s0; si < s1; ++si) {
    floatx4 acc[NT][9];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int buf = (si - s0) & 1;
    if (si + 1 < s1) load(si + 1);
    const int code = A.tsrc[si].y;
    const float ox = 2.0f * (float)(code / 49 - 3), oy = 2.0f * (float)((code / 7) % 7 - 3),
                oz = 2.0f * (float)(code % 7 - 3);
    float tlx[NT], tly[NT], tlz[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int row = rt * 16 + col;
      const float4 tl = sN[row < p3 ? row : 0];
      tlx[t] = tl.x + ox;
      tly[t] = tl.y + oy;
      tlz[t] = tl.z + oz;
    }
    const float* sBc = sB[buf] + col * kM2LStride;
    // NK steps of four source nodes from node kb on (a compile-time count, so the loop unrolls)
    auto run = [&](auto nk_tag, int kb) {
      constexpr int NK = decltype(nk_tag)::value;
#pragma unroll 1
      for (int ks = 0; ks < NK; ++ks) {
        const int m = kb + 4 * ks + kq;
        // with p^3 a multiple of 4 every node index is below p^3; otherwise the last step's
        // extra nodes read node 0 against a zero B entry
        const int mc = p3 % 4 == 0 ? m : (m < p3 ? m : 0);
        const float4 tm = sN[mc];
        const float b0 = (p3 % 4 == 0 || m < p3) ? sBc[mc] : 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float rx = tlx[t] - tm.x, ry = tly[t] - tm.y, rz = tlz[t] - tm.z;
          const float inv = __builtin_amdgcn_rcpf(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
          float a[9];
          a[0] = rx * inv; a[1] = ry * inv; a[2] = rz * inv;
          a[3] = a[0] * a[0]; a[4] = a[0] * a[1]; a[5] = a[0] * a[2];
          a[6] = a[1] * a[1]; a[7] = a[1] * a[2]; a[8] = a[2] * a[2];
#pragma unroll
          for (int c = 0; c < 9; ++c) acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[c], b0, acc[t][c], 0, 0, 0);
        }
      }
    };
    if (hw)
      run(std::integral_constant<int, p3 / 8>{}, kh * (p3 / 2));
    else
      run(std::integral_constant<int, (p3 + 3) / 4>{}, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 9; ++c) tot[t][c] += acc[t][c];
    if (si + 1 < s1) store(buf ^ 1);
    __syncthreads();
  }
  if (kSplit) {   // the second-half waves hand their sums to the first-half waves through LDS
    floatx4* sC = reinterpret_cast<floatx4*>(&sB[0][0]);   // [2 row tiles][9][64 lanes]; sB is idle now
    const int slot = (rt - (n_rt - 2)) * 9;
    if (hw && kh == 1)
#pragma unroll
      for (int c = 0; c < 9; ++c) sC[(slot + c) * 64 + lane] = tot[0][c];
    __syncthreads();
    if (hw && kh == 0)
#pragma unroll
      for (int c = 0; c < 9; ++c) tot[0][c] += sC[(slot + c) * 64 + lane];
  }
  // every source of the box sits at the box's level: one scale per component group
  int lev = 2;
  while (lev < A.L && box >= A.lev_first[lev + 1]) ++lev;
  const double h = A.h0 / (double)(1 << lev);
  const float s1f = (float)(1.0 / h), s2f = (float)(1.0 / (h * h));
  float* out = A.L16 + (int64_t)col * A.n_boxes * lstride<P>() + box * lstride<P>();
  if (hw && kh == 1) return;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int l0 = rt * 16 + 4 * kq;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const float sc = c < 3 ? s1f : s2f;
      if (l0 + 3 < p3 && (p3 % 4) == 0) {
        *reinterpret_cast<float4*>(out + c * p3 + l0) =
            make_float4(sc * tot[t][c][0], sc * tot[t][c][1], sc * tot[t][c][2], sc * tot[t][c][3]);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (l0 + r < p3) out[c * p3 + l0 + r] = sc * tot[t][c][r];
      }
    }
  }
}

// L[T] = sum of T's M2L output slots, in pair order (one block per box of levels >= 2);
// a box's slots are contiguous, so the reads stream.
// Each thread owns four consecutive entries (float4); the pair loop is unrolled so the
// independent slot loads are in flight together.
struct RedArgs {
  int64_t box0;
  const int32_t* rptr;     // a box's slots are [rptr[b], rptr[b + 1])
  const float* slots;
  float* Lc;
};

template <int P>
__global__ void __launch_bounds__(512) k_m2l_reduce(Group<RedArgs> g) {
  constexpr int n4 = lstride<P>() / 4;   // padding entries are zero in every slot
  int64_t b;
  const RedArgs& A = seg_of(g, blockIdx.x, b);
  const int64_t box0 = A.box0;
  const int32_t* __restrict__ rptr = A.rptr;
  const float* __restrict__ slots = A.slots;
  float* __restrict__ Lc = A.Lc;
  const int k0 = rptr[b], k1 = rptr[b + 1];
  const float4* __restrict__ s4 = reinterpret_cast<const float4*>(slots);
  for (int e = threadIdx.x; e < n4; e += blockDim.x) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
    for (int k = k0; k < k1; ++k) {
      const float4 v = s4[(int64_t)k * n4 + e];
      acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    reinterpret_cast<float4*>(Lc)[(box0 + b) * n4 + e] = acc;
  }
}

// P2P over the U-list: one wave per (leaf, 64 targets, U-list slot).  The wave's
// target and source ranges come precomputed in one record, so its start needs a single
// dependent load; the source rows (x, y, z, qt) are wave-uniform and read through the
// scalar cache.  part[slot][k] is summed in slot order by L2P.
struct P2PArgs {
  int64_t N;
  const int4* desc;      // (first target, end target, first source, end source)
  const int32_t* wslot;
  const float* pts;
  const float* qs;
  float* part;
};

__global__ void __launch_bounds__(64) k_p2p(Group<P2PArgs> g) {
  int64_t lb;
  const P2PArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t N = A.N;
  const float* __restrict__ pts = A.pts;
  const int4 d = A.desc[lb];
  const int slot = A.wslot[lb];
  const int k = d.x + threadIdx.x;
  const int kk = k < d.y ? k : d.y - 1;
  const float xi = pts[kk], yi = pts[N + kk], zi = pts[2 * N + kk];
  const float px = pts[3 * N + kk], py = pts[4 * N + kk], pz = pts[5 * N + kk];
  const float hx = pts[6 * N + kk], hy = pts[7 * N + kk], hz = pts[8 * N + kk];
  const sfp src = (sfp)A.qs;
  float acc = 0.0f;
#pragma unroll 4
  for (int j = d.z; j < d.w; ++j) {
    const sfp sj = src + 4 * (int64_t)j;
    const float dx = xi - sj[0], dy = yi - sj[1], dz = zi - sj[2];
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1e-30f)));
    const float inv = __builtin_amdgcn_rcpf(r2);
    const float pr = fmaf(px, dx, fmaf(py, dy, pz * dz));
    const float hr = fmaf(hx, dx, fmaf(hy, dy, hz * dz));
    acc = fmaf(sj[3], fmaf(pr * inv, pr, hr) * inv, acc);
  }
  if (k < d.y) A.part[(int64_t)slot * N + k] = acc;
}

// Several right-hand sides: one source row per sorted point, (x, y, z, qt_0 .. qt_{R-1}) and
// zeros up to the row stride.
struct PermMArgs {
  int64_t N;
  int R, stride;
  const int32_t* perm;
  const float* pts;
  const float* q;     // R x N (node order)
  float* qsR;
};

__global__ void __launch_bounds__(256) k_permute_multi(Group<PermMArgs> g) {
  int64_t lb;
  const PermMArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t k = lb * 256 + threadIdx.x;
  if (k >= A.N) return;
  float* row = A.qsR + k * A.stride;
  const int32_t i = A.perm[k];
  row[0] = A.pts[k];
  row[1] = A.pts[A.N + k];
  row[2] = A.pts[2 * A.N + k];
  for (int r = 0; r < A.stride - 3; ++r) row[3 + r] = r < A.R ? A.q[(int64_t)r * A.N + i] : 0.0f;
}

// P2P for several right-hand sides: one wave per (leaf, 64-target chunk) takes every U-list
// slot of the chunk in order.  The pair kernel ((n'.r)^2 / r^2 + h.r) / r^2 does not depend
// on the density, so it is evaluated once per pair and applied to all R charges of the source
// row (wave-uniform, through the scalar cache); the sums stay in registers across the slots.
struct P2PMArgs {
  int64_t N;
  int R, stride;
  const int32_t* cptr;
  const int4* desc;
  const float* pts;
  const float* qsR;
  float* partR;       // R x N (sorted order)
};

template <int RMAX>
__global__ void __launch_bounds__(64) k_p2p_multi(Group<P2PMArgs> g) {
  int64_t lb;
  const P2PMArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t N = A.N;
  const float* __restrict__ pts = A.pts;
  const int w0 = A.cptr[lb], w1 = A.cptr[lb + 1];
  const int4 d0 = A.desc[w0];
  const int k = d0.x + threadIdx.x;
  const int kk = k < d0.y ? k : d0.y - 1;
  const float xi = pts[kk], yi = pts[N + kk], zi = pts[2 * N + kk];
  const float px = pts[3 * N + kk], py = pts[4 * N + kk], pz = pts[5 * N + kk];
  const float hx = pts[6 * N + kk], hy = pts[7 * N + kk], hz = pts[8 * N + kk];
  const sfp src = (sfp)A.qsR;
  const int stride = A.stride;
  float acc[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) acc[r] = 0.0f;
  for (int w = w0; w < w1; ++w) {
    const int4 d = A.desc[w];
#pragma unroll 2
    for (int j = d.z; j < d.w; ++j) {
      const sfp sj = src + (int64_t)stride * j;
      const float dx = xi - sj[0], dy = yi - sj[1], dz = zi - sj[2];
      const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1e-30f)));
      const float inv = __builtin_amdgcn_rcpf(r2);
      const float pr = fmaf(px, dx, fmaf(py, dy, pz * dz));
      const float hr = fmaf(hx, dx, fmaf(hy, dy, hz * dz));
      const float kv = fmaf(pr * inv, pr, hr) * inv;
#pragma unroll
      for (int r = 0; r < RMAX; ++r) acc[r] = fmaf(sj[3 + r], kv, acc[r]);
    }
  }
  if (k < d0.y)
    for (int r = 0; r < A.R; ++r) A.partR[(int64_t)r * N + k] = acc[r];
}

// L2P + contraction + P2P sum, added to y (FP64, node order).
struct L2PArgs {
  int64_t leaf_off, N;
  float h;
  const float* tab;
  const float* center;
  const int32_t* leaf_start;
  const float* pts;
  const float* Lc;
  const float* part;
  const int32_t* u_ptr;   // null: part holds one sum per target (several right-hand sides)
  const int32_t* perm;
  double* y;
  const int2* chunks;     // (leaf, first target) of each block's 64-target chunk
};

// The leaf's local expansion is the same for all its targets, so the evaluation
//   F_c(x_t) = sum_l S(t_l, x_t) L_c,l
// is a [targets x p^3] x [p^3 x 9] product: one MFMA tile covers 16 targets and the
// nine components (padded to 16 columns).  The K index runs over (a, b, d) with d
// padded to a multiple of 4, so a lane's share of the tensor weight S = s_x[a] s_y[b]
// s_z[d] only needs the two s_z values it owns (d = kq and 4 + kq).  The tile's nine
// components per target go through LDS to the lanes that form the contraction.
template <int P>
__global__ void __launch_bounds__(256) k_l2p(Group<L2PArgs> g) {
  constexpr int p = P, p3 = P * P * P;
  constexpr int n_h = (P + 3) / 4;                    // 4-wide d groups
  __shared__ float sL[9 * p3];
  __shared__ float sF[4][16][17];                     // per wave: [target][component]
  int64_t lb;
  const L2PArgs& A = seg_of(g, blockIdx.x, lb);
  const int64_t leaf_off = A.leaf_off, N = A.N;
  const float* __restrict__ tab = A.tab;
  const float* __restrict__ pts = A.pts;
  const int2 ch = A.chunks[lb];
  const int leaf = ch.x;
  const int64_t box = leaf_off + leaf;
  for (int e = threadIdx.x; e < 9 * p3; e += blockDim.x) sL[e] = A.Lc[box * lstride<P>() + e];
  __syncthreads();
  const float cx = A.center[3 * box], cy = A.center[3 * box + 1], cz = A.center[3 * box + 2];
  const float ih = 1.0f / A.h;
  // one block per 64-target chunk of a leaf (16 targets per wave): many more blocks than
  // leaves, so the launch fills the chip
  const int s0 = ch.y, s1 = min(ch.y + 64, A.leaf_start[leaf + 1]);
  const int n_slot = A.u_ptr ? A.u_ptr[leaf + 1] - A.u_ptr[leaf] : 1;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = lane & 15, kq = lane >> 4;
  const int c = row;                                   // B column (component) of this lane
  for (int t0 = s0 + wave * 16; t0 < s1; t0 += 64) {
    const int k = t0 + row;                            // A row (target) of this lane
    const bool kv = k < s1;
    const int kk = kv ? k : s1 - 1;
    float sx[P], sy[P], sz[P];
    cheb_weights<P>(tab, (pts[kk] - cx) * ih, sx);
    cheb_weights<P>(tab, (pts[N + kk] - cy) * ih, sy);
    cheb_weights<P>(tab, (pts[2 * N + kk] - cz) * ih, sz);
    float wz[n_h];
#pragma unroll
    for (int hq = 0; hq < n_h; ++hq) {
      float v = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * hq + q < P && kq == q) v = sz[4 * hq + q];
      wz[hq] = kv ? v : 0.0f;
    }
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < p; ++a)
#pragma unroll
      for (int b = 0; b < p; ++b) {
        const float xy = sx[a] * sy[b];
#pragma unroll
        for (int hq = 0; hq < n_h; ++hq) {
          const int d = 4 * hq + kq;
          const float bv = (c < 9 && d < P) ? sL[(c < 9 ? c : 0) * p3 + (a * p + b) * p + (d < P ? d : 0)] : 0.0f;
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(xy * wz[hq], bv, acc, 0, 0, 0);
        }
      }
    // lane holds F[component = row][targets 4 kq + r]
#pragma unroll
    for (int r = 0; r < 4; ++r) sF[wave][4 * kq + r][row] = acc[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 16 && kv) {
      const float* F = sF[wave][row];
      float near_sum = 0.0f;
      for (int sl = 0; sl < n_slot; ++sl) near_sum += A.part[(int64_t)sl * N + k];
      const float nx = pts[3 * N + k], ny = pts[4 * N + k], nz = pts[5 * N + k];
      const float hx = pts[6 * N + k], hy = pts[7 * N + k], hz = pts[8 * N + k];
      // F1 = F[0..2]; F2 = (xx, xy, xz, yy, yz, zz) = F[3..8]; phi = n'^T F2 n' + h . F1
      const float nF2n = nx * nx * F[3] + 2.f * nx * ny * F[4] + 2.f * nx * nz * F[5] + ny * ny * F[6] +
                         2.f * ny * nz * F[7] + nz * nz * F[8];
      const float hF1 = hx * F[0] + hy * F[1] + hz * F[2];
      A.y[A.perm[k]] += (double)(nF2n + hF1) + (double)near_sum;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__global__ void k_gather_pts(int64_t N, const int32_t* __restrict__ perm, const float* __restrict__ t32,
                             float* __restrict__ pts) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int64_t i = perm[k];
  for (int c = 0; c < 9; ++c) pts[c * N + k] = t32[c * N + i];
}

// ----------------------------------------------------------------------------- host: tree build
namespace {

constexpr int kBits = 21;   // Morton key bits per coordinate

__host__ __device__ inline uint64_t spread3(uint64_t v) {   // 21 bits -> every third bit
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}
__host__ __device__ inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) {
  return spread3(x) | spread3(y) << 1 | spread3(z) << 2;
}
inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ULL;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
  v = (v ^ (v >> 32)) & 0x1fffff;
  return v;
}

// Morton key of every node's cell at the finest of kBits levels (the host's arithmetic: the same
// IEEE operations on the same doubles), with the node index for the sort.
__global__ void k_morton(int64_t N, const double* __restrict__ X, double lo0, double lo1, double lo2, double w,
                         double cells, uint64_t* __restrict__ key, int32_t* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double lo[3] = {lo0, lo1, lo2};
  uint64_t ic[3];
  for (int c = 0; c < 3; ++c) {
    const double sc = (X[c * N + i] - lo[c]) / w * cells;
    int64_t v = (int64_t)floor(sc);
    v = v < 0 ? 0 : (v > ((int64_t)1 << kBits) - 1 ? ((int64_t)1 << kBits) - 1 : v);
    ic[c] = (uint64_t)v;
  }
  key[i] = morton(ic[0], ic[1], ic[2]);
  idx[i] = (int32_t)i;
}

double cheb_w_host(int p, double tk, double x) {
  double s = 0.0, a0 = 1.0, a1 = tk, b0 = 1.0, b1 = x;
  for (int n = 1; n < p; ++n) {
    s += a1 * b1;
    const double a2 = 2 * tk * a1 - a0, b2 = 2 * x * b1 - b0;
    a0 = a1; a1 = a2; b0 = b1; b1 = b2;
  }
  return 1.0 / p + 2.0 / p * s;
}

}  // namespace

void fmm_build(pmx_operator* op, hipStream_t st) {
  Ctx* ctx = &op->s->ctx->c;
  const int64_t N = op->s->g.N;
  auto* F = new FMM;
  try {
    F->p = op->opts.fmm_order;
    F->p3 = F->p * F->p * F->p;
    PMX_REQUIRE(F->p >= 4 && F->p <= 6, PMX_ERR_INVALID, "fmm_order must be 4, 5 or 6");
    const int p = F->p, p3 = F->p3;
    std::vector<double> X(3 * N);
    PMX_HIP(hipMemcpyAsync(X.data(), op->s->g.x.p, 3 * N * sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
      lo[c] = *std::min_element(X.begin() + c * N, X.begin() + (c + 1) * N);
      hi[c] = *std::max_element(X.begin() + c * N, X.begin() + (c + 1) * N);
      F->c0[c] = 0.5 * (lo[c] + hi[c]);
    }
    F->h0 = 0.5 * std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]}) * (1.0 + 1e-6) + 1e-12;
    const double cells = (double)(1u << kBits);
    // Morton keys and their sort on the GPU (a stable radix sort of (key, node) pairs, so equal
    // keys keep node order, as a sort of the pairs would), then the sorted pairs to the host
    std::vector<std::pair<uint64_t, int32_t>> key(N);
    {
      DBuf<uint64_t> k_in, k_out;
      DBuf<int32_t> i_in, i_out;
      k_in.alloc(ctx, N);
      k_out.alloc(ctx, N);
      i_in.alloc(ctx, N);
      i_out.alloc(ctx, N);
      hipLaunchKernelGGL(k_morton, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, N, op->s->g.x.p,
                         F->c0[0] - F->h0, F->c0[1] - F->h0, F->c0[2] - F->h0, 2.0 * F->h0, cells, k_in.p, i_in.p);
      PMX_HIP(hipGetLastError());
      size_t tmp_bytes = 0;
      PMX_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, k_in.p, k_out.p, i_in.p, i_out.p, (int)N, 0,
                                                 3 * kBits, st));
      DBuf<unsigned char> tmp;
      tmp.alloc(ctx, std::max<size_t>(tmp_bytes, 1));
      PMX_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, k_in.p, k_out.p, i_in.p, i_out.p, (int)N, 0,
                                                 3 * kBits, st));
      std::vector<uint64_t> hk(N);
      std::vector<int32_t> hi(N);
      PMX_HIP(hipMemcpyAsync(hk.data(), k_out.p, N * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
      PMX_HIP(hipMemcpyAsync(hi.data(), i_out.p, N * sizeof(int32_t), hipMemcpyDeviceToHost, st));
      PMX_HIP(hipStreamSynchronize(st));
      for (int64_t i = 0; i < N; ++i) key[i] = {hk[i], hi[i]};
    }
    // leaf level: smallest level >= 2 whose mean occupancy is at most fmm_leaf
    int L = 2;
    for (; L < kMaxLevel; ++L) {
      const int sh = 3 * (kBits - L);
      int64_t nb = 0;
      uint64_t prev = ~0ULL;
      for (auto& kv : key) {
        const uint64_t b = kv.first >> sh;
        if (b != prev) { ++nb; prev = b; }
      }
      if ((double)N / (double)nb <= (double)op->opts.fmm_leaf) break;
    }
    F->L = L;
    // boxes per level (sorted Morton prefixes)
    std::vector<std::vector<uint64_t>> bkey(L + 1);
    for (int l = 0; l <= L; ++l) {
      const int sh = 3 * (kBits - l);
      uint64_t prev = ~0ULL;
      for (auto& kv : key) {
        const uint64_t b = kv.first >> sh;
        if (b != prev) { bkey[l].push_back(b); prev = b; }
      }
    }
    F->lev_off.assign(L + 2, 0);
    for (int l = 0; l <= L; ++l) F->lev_off[l + 1] = F->lev_off[l] + (int64_t)bkey[l].size();
    F->n_boxes = F->lev_off[L + 1];
    F->n_leaves = (int64_t)bkey[L].size();
    std::vector<std::unordered_map<uint64_t, int32_t>> idx(L + 1);
    for (int l = 0; l <= L; ++l) {
      idx[l].reserve(bkey[l].size() * 2);
      for (size_t b = 0; b < bkey[l].size(); ++b) idx[l][bkey[l][b]] = (int32_t)b;
    }
    std::vector<float> center(3 * F->n_boxes);
    std::vector<int32_t> cb(F->n_boxes, 0), ce(F->n_boxes, 0), par(F->n_boxes, -1), oct(F->n_boxes, 0);
    for (int l = 0; l <= L; ++l) {
      const double h = F->h0 / (double)(1 << l);
      for (size_t b = 0; b < bkey[l].size(); ++b) {
        const uint64_t k = bkey[l][b];
        const int64_t g = F->lev_off[l] + b;
        const uint64_t ix = compact3(k), iy = compact3(k >> 1), iz = compact3(k >> 2);
        center[3 * g] = (float)(F->c0[0] - F->h0 + (2.0 * ix + 1.0) * h);
        center[3 * g + 1] = (float)(F->c0[1] - F->h0 + (2.0 * iy + 1.0) * h);
        center[3 * g + 2] = (float)(F->c0[2] - F->h0 + (2.0 * iz + 1.0) * h);
        if (l > 0) {
          par[g] = (int32_t)(F->lev_off[l - 1] + idx[l - 1][k >> 3]);
          oct[g] = (int32_t)(k & 7);
        }
      }
    }
    for (int l = 1; l <= L; ++l)
      for (size_t b = 0; b < bkey[l].size(); ++b) {
        const int64_t g = F->lev_off[l] + b;
        const int32_t P = par[g];
        if (ce[P] == 0) cb[P] = (int32_t)g;
        ce[P] = (int32_t)g + 1;
      }
    // leaf point ranges and permutation
    std::vector<int32_t> lstart(F->n_leaves + 1, 0), perm(N);
    {
      const int sh = 3 * (kBits - L);
      int64_t b = -1;
      uint64_t prev = ~0ULL;
      for (int64_t k = 0; k < N; ++k) {
        perm[k] = key[k].second;
        const uint64_t bk = key[k].first >> sh;
        if (bk != prev) { ++b; lstart[b] = (int32_t)k; prev = bk; }
      }
      lstart[F->n_leaves] = (int32_t)N;
    }
    auto coords = [](uint64_t k, int64_t c[3]) {
      c[0] = (int64_t)compact3(k); c[1] = (int64_t)compact3(k >> 1); c[2] = (int64_t)compact3(k >> 2);
    };
    auto lookup = [&](int l, int64_t x, int64_t y, int64_t z) -> int32_t {
      const int64_t n = (int64_t)1 << l;
      if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return -1;
      auto it = idx[l].find(morton((uint64_t)x, (uint64_t)y, (uint64_t)z));
      return it == idx[l].end() ? -1 : it->second;
    };
    // U-list of leaves
    std::vector<int32_t> uptr(F->n_leaves + 1, 0), uidx;
    int64_t p2p = 0;
    for (int64_t b = 0; b < F->n_leaves; ++b) {
      int64_t c[3];
      coords(bkey[L][b], c);
      const int64_t nt = lstart[b + 1] - lstart[b];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int32_t s = lookup(L, c[0] + dx, c[1] + dy, c[2] + dz);
            if (s >= 0) {
              uidx.push_back(s);
              p2p += nt * (int64_t)(lstart[s + 1] - lstart[s]);
            }
          }
      uptr[b + 1] = (int32_t)uidx.size();
    }
    F->p2p_pairs = p2p;
    // V-lists grouped by (level, offset)
    struct Pair { int32_t lev, code, t, s; };
    std::vector<Pair> pairs;
    for (int l = 2; l <= L; ++l) {
      for (size_t b = 0; b < bkey[l].size(); ++b) {
        int64_t cB[3];
        coords(bkey[l][b], cB);
        const int64_t pc[3] = {cB[0] >> 1, cB[1] >> 1, cB[2] >> 1};
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              const int32_t nb = lookup(l - 1, pc[0] + dx, pc[1] + dy, pc[2] + dz);
              if (nb < 0) continue;
              const int64_t gN = F->lev_off[l - 1] + nb;
              for (int32_t c = cb[gN]; c < ce[gN]; ++c) {
                int64_t cC[3];
                coords(bkey[l][c - F->lev_off[l]], cC);
                const int64_t ox = cC[0] - cB[0], oy = cC[1] - cB[1], oz = cC[2] - cB[2];
                if (std::max({std::llabs(ox), std::llabs(oy), std::llabs(oz)}) < 2) continue;
                // offset of the target relative to the source, in box widths
                const int32_t code = (int32_t)((-ox + 3) * 49 + (-oy + 3) * 7 + (-oz + 3));
                pairs.push_back({l, code, (int32_t)(F->lev_off[l] + b), c});
              }
            }
      }
    }
    // grouped by offset only: the unit-box kernel of an offset serves every level
    std::sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
      if (a.code != b.code) return a.code < b.code;
      if (a.lev != b.lev) return a.lev < b.lev;
      return a.t < b.t;
    });
    F->m2l_pairs = (int64_t)pairs.size();
    std::vector<int32_t> pt(pairs.size()), ps(pairs.size()), plv(pairs.size());
    std::vector<int4> items;
    for (size_t k = 0; k < pairs.size();) {
      size_t e = k;
      while (e < pairs.size() && pairs[e].code == pairs[k].code) ++e;
      for (size_t s = k; s < e; s += kItemCols)
        items.push_back(make_int4((int)s, (int)std::min<size_t>(kItemCols, e - s), 0, pairs[k].code));
      k = e;
    }
    for (size_t k = 0; k < pairs.size(); ++k) { pt[k] = pairs[k].t; ps[k] = pairs[k].s; plv[k] = pairs[k].lev; }
    // per-target lists of pair slots (boxes of levels >= 2, pairs in sorted order)
    const int64_t box2 = F->lev_off[2];
    std::vector<int32_t> rptr(F->n_boxes - box2 + 1, 0);
    for (auto& pr : pairs) rptr[pr.t - box2 + 1]++;
    for (size_t b = 1; b < rptr.size(); ++b) rptr[b] += rptr[b - 1];
    std::vector<int32_t> spos(pairs.size());
    {
      std::vector<int32_t> fill(rptr.begin(), rptr.end() - 1);
      for (size_t k = 0; k < pairs.size(); ++k) spos[k] = fill[pairs[k].t - box2]++;
    }
    F->n_items = (int64_t)items.size();
    std::vector<int2> tsrc(pairs.size());   // a box's sources in its slot order
    for (size_t k = 0; k < pairs.size(); ++k) tsrc[spos[k]] = make_int2(pairs[k].s, pairs[k].code);
    // P2P waves: (leaf, 64-target chunk, U-list slot) -> target and source ranges
    std::vector<int4> wd;
    std::vector<int32_t> ws;
    for (int64_t b = 0; b < F->n_leaves; ++b)
      for (int32_t f = lstart[b]; f < lstart[b + 1]; f += 64)
        for (int32_t sl = 0; sl < uptr[b + 1] - uptr[b]; ++sl) {
          const int32_t S = uidx[uptr[b] + sl];
          wd.push_back(make_int4(f, std::min(f + 64, lstart[b + 1]), lstart[S], lstart[S + 1]));
          ws.push_back(sl);
        }
    F->n_p2p_waves = (int64_t)wd.size();
    std::vector<int32_t> cptr(1, 0);   // waves are ordered by (leaf, chunk, slot)
    std::vector<int2> chunks;
    for (int64_t b = 0; b < F->n_leaves; ++b)
      for (int32_t f = lstart[b]; f < lstart[b + 1]; f += 64) {
        cptr.push_back(cptr.back() + (uptr[b + 1] - uptr[b]));
        chunks.push_back(make_int2((int)b, f));
      }
    for (int64_t b = 0; b < F->n_leaves; ++b)   // a leaf's U-list holds the leaf itself
      PMX_REQUIRE(uptr[b + 1] > uptr[b], PMX_ERR_DEVICE, "FMM leaf with an empty U-list");
    F->n_p2p_chunks = (int64_t)cptr.size() - 1;
    // tables: t_k, M1[2][p][p] (M1[b][k][k'] = S1(t_k, +-0.5 + t_k'/2)), node coordinates
    std::vector<float> tab(p + 2 * p * p + 3 * p3);
    std::vector<double> t(p);
    for (int k = 0; k < p; ++k) t[k] = std::cos((2.0 * k + 1.0) * M_PI / (2.0 * p));
    for (int k = 0; k < p; ++k) tab[k] = (float)t[k];
    for (int b = 0; b < 2; ++b)
      for (int k = 0; k < p; ++k)
        for (int kk = 0; kk < p; ++kk)
          tab[p + b * p * p + k * p + kk] = (float)cheb_w_host(p, t[k], (b ? 0.5 : -0.5) + 0.5 * t[kk]);
    for (int l = 0; l < p3; ++l) {
      tab[p + 2 * p * p + 3 * l] = (float)t[l / (p * p)];
      tab[p + 2 * p * p + 3 * l + 1] = (float)t[(l / p) % p];
      tab[p + 2 * p * p + 3 * l + 2] = (float)t[l % p];
    }
    // device copies
    auto up = [&](auto& buf, const auto& v) {
      using T = typename std::decay_t<decltype(v)>::value_type;
      buf.alloc(ctx, v.size());
      if (!v.empty()) PMX_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    };
    up(F->center, center);
    up(F->child_begin, cb);
    up(F->child_end, ce);
    up(F->parent, par);
    up(F->octant, oct);
    up(F->leaf_start, lstart);
    up(F->perm, perm);
    up(F->u_ptr, uptr);
    up(F->u_idx, uidx);
    up(F->m2l_t, pt);
    up(F->r_ptr, rptr);
    up(F->m2l_slot, spos);
    up(F->m2l_s, ps);
    up(F->m2l_lv, plv);
    up(F->items, items);
    up(F->p2p_desc, wd);
    up(F->p2p_slot, ws);
    up(F->p2p_cptr, cptr);
    up(F->chunks, chunks);
    up(F->tsrc, tsrc);
    up(F->lev_off_d, F->lev_off);
    up(F->tab, tab);
    F->pts.alloc(ctx, 9 * (size_t)N);
    F->qs.alloc(ctx, 4 * N);
    F->phis.alloc(ctx, 27 * (size_t)N);
    F->W.alloc(ctx, (size_t)F->n_boxes * p3);
    const size_t ls = (size_t)lstride_of(p);
    F->Lc.alloc(ctx, (size_t)F->n_boxes * ls);
    F->slots.alloc(ctx, (size_t)std::max<int64_t>(F->m2l_pairs, 1) * ls);
    if (ls != 9 * (size_t)p3)   // M2L never writes a slot's padding: it stays zero
      PMX_HIP(hipMemsetAsync(F->slots.p, 0, F->slots.bytes(), st));
    hipLaunchKernelGGL(k_gather_pts, dim3((N + 255) / 256), dim3(256), 0, st, N, F->perm.p, op->co.tgt32.p,
                       F->pts.p);
    PMX_HIP(hipGetLastError());
    PMX_HIP(hipStreamSynchronize(st));
  } catch (...) {
    delete F;
    throw;
  }
  op->fmm = F;
}

void fmm_destroy(FMM* f) { delete f; }

// One far-field pass for one right-hand side r of several operators: every stage
// is one launch over all operators (M2M and L2L: one launch per level).
template <int P>
static void fmm_far_rhs(const std::vector<ApplyJob>& jobs, int r, int n_rhs, Profiler* prof, hipStream_t st,
                        hipStream_t side, hipEvent_t ev_fork, hipEvent_t ev_join,
                        const std::function<void(hipStream_t)>& side_work) {
  // several right-hand sides: the P2P sums of a block of up to kRBlock of them (this rhs's
  // block starts at rb) come from one multi-charge launch at the block's first rhs
  const bool multi = n_rhs > 1;
  const int rb = (r / kRBlock) * kRBlock, nb_r = std::min(kRBlock, n_rhs - rb);
  const bool fork = !multi || r == rb;
  std::vector<pmx_operator*> ops;
  for (const ApplyJob& j : jobs) ops.push_back(j.op);
  constexpr int p3 = P * P * P;
  (void)p3;
  auto phase = [&](int ph) { return prof ? prof->begin(ph, st) : -1; };
  auto done = [&](int t) { if (prof) prof->end(t, st); };
  const size_t n = ops.size();
  int maxL = 0;
  for (pmx_operator* op : ops) maxL = std::max(maxL, op->fmm->L);

  int t = -1;
  {
    std::vector<PermArgs> pa;
    std::vector<P2MArgs> ma;
    std::vector<int64_t> pb, mb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      const int64_t N = op->s->g.N;
      pa.push_back({N, F->perm.p, F->pts.p, op->qt32.p + (int64_t)r * N, F->qs.p});
      pb.push_back((N + 255) / 256);
      const float hL = (float)(F->h0 / (double)(1 << F->L));
      ma.push_back({F->lev_off[F->L], N, hL, F->tab.p, F->center.p, F->leaf_start.p, F->pts.p, F->qs.p, F->W.p});
      mb.push_back(F->n_leaves);
    }
    launch_grouped(pa, pb, [&](const Group<PermArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_permute, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
    // fork: the caller's side work (once) and the P2P sums, which need only the permuted
    // sources, run on the side stream while P2M, M2M, M2L, its slot sum and L2L run here.
    // Measured on the ellipsoid: starting the side stream here hides more than starting it
    // with M2L, whose long launch then shares the CUs from its first wave on.
    if (multi && fork) {   // source rows with the block's charges, for the multi-charge P2P
      std::vector<PermMArgs> qm;
      std::vector<int64_t> qmb;
      for (pmx_operator* op : ops) {
        FMM* F = op->fmm;
        const int64_t N = op->s->g.N;
        qm.push_back({N, nb_r, F->rstride, F->perm.p, F->pts.p, op->qt32.p + (int64_t)rb * N, F->qsR.p});
        qmb.push_back((N + 255) / 256);
      }
      launch_grouped(qm, qmb, [&](const Group<PermMArgs>& g, int64_t nb) {
        hipLaunchKernelGGL(k_permute_multi, dim3((unsigned)nb), dim3(256), 0, st, g);
        PMX_HIP(hipGetLastError());
      });
    }
    if (fork) {
      if (side != st) {
        PMX_HIP(hipEventRecord(ev_fork, st));
        PMX_HIP(hipStreamWaitEvent(side, ev_fork, 0));
      }
      if (r == 0 && side_work) side_work(side);
      const int tp = prof ? prof->begin(PMX_PHASE_FMM_P2P, side) : -1;
      if (!multi) {
        std::vector<P2PArgs> qa;
        std::vector<int64_t> qb;
        for (pmx_operator* op : ops) {
          FMM* F = op->fmm;
          qa.push_back({op->s->g.N, F->p2p_desc.p, F->p2p_slot.p, F->pts.p, F->qs.p, F->phis.p});
          qb.push_back(F->n_p2p_waves);
        }
        launch_grouped(qa, qb, [&](const Group<P2PArgs>& g, int64_t nb) {
          hipLaunchKernelGGL(k_p2p, dim3((unsigned)nb), dim3(64), 0, side, g);
          PMX_HIP(hipGetLastError());
        });
      } else {
        std::vector<P2PMArgs> qa;
        std::vector<int64_t> qb;
        for (pmx_operator* op : ops) {
          FMM* F = op->fmm;
          qa.push_back({op->s->g.N, nb_r, F->rstride, F->p2p_cptr.p, F->p2p_desc.p, F->pts.p, F->qsR.p, F->partR.p});
          qb.push_back(F->n_p2p_chunks);
        }
        launch_grouped(qa, qb, [&](const Group<P2PMArgs>& g, int64_t nb) {
          if (nb_r <= 2) hipLaunchKernelGGL(k_p2p_multi<2>, dim3((unsigned)nb), dim3(64), 0, side, g);
          else if (nb_r <= 4) hipLaunchKernelGGL(k_p2p_multi<4>, dim3((unsigned)nb), dim3(64), 0, side, g);
          else if (nb_r <= 8) hipLaunchKernelGGL(k_p2p_multi<8>, dim3((unsigned)nb), dim3(64), 0, side, g);
          else hipLaunchKernelGGL(k_p2p_multi<16>, dim3((unsigned)nb), dim3(64), 0, side, g);
          PMX_HIP(hipGetLastError());
        });
      }
      if (prof) prof->end(tp, side);
      if (side != st) PMX_HIP(hipEventRecord(ev_join, side));
    }
    t = phase(PMX_PHASE_FMM_P2M);   // P2M alone (the permutation before it is not timed)
    launch_grouped(ma, mb, [&](const Group<P2MArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_p2m<P>, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  t = phase(PMX_PHASE_FMM_M2M);
  for (int l = maxL - 1; l >= 2; --l) {
    std::vector<M2MArgs> ma;
    std::vector<int64_t> mb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      if (l >= F->L) continue;
      ma.push_back({F->lev_off[l], F->tab.p, F->child_begin.p, F->child_end.p, F->octant.p, F->W.p});
      mb.push_back(F->lev_off[l + 1] - F->lev_off[l]);
    }
    launch_grouped(ma, mb, [&](const Group<M2MArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_m2m<P>, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  t = phase(PMX_PHASE_FMM_M2L);
  {
    std::vector<M2LArgs> la;
    std::vector<RedArgs> ra;
    std::vector<int64_t> lb, rb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      la.push_back({F->tab.p, F->items.p, F->m2l_s.p, F->m2l_lv.p, F->m2l_slot.p, F->W.p, F->slots.p, F->h0});
      lb.push_back(F->n_items);
      const int64_t box2 = F->lev_off[2];
      ra.push_back({box2, F->r_ptr.p, F->slots.p, F->Lc.p});
      rb.push_back(F->n_boxes - box2);
    }
    // the split layout when nothing runs beside this launch: the side stream's kernels are
    // in flight only after a fork onto a distinct stream
    constexpr bool kCanSplit = m2l_can_split<P>();
    const bool beside = fork && side != st;
    launch_grouped(la, lb, [&](const Group<M2LArgs>& g, int64_t nb) {
      // persistent workgroups (one resident per CU at this size), striding over the items
      const int64_t grid = std::min<int64_t>(nb, m2l_persistent_blocks());
      if (kCanSplit && !beside)
        hipLaunchKernelGGL((k_m2l<P, kCanSplit>), dim3((unsigned)grid), dim3(64 * m2l_waves<P, kCanSplit>()), 0,
                           st, g);
      else
        hipLaunchKernelGGL((k_m2l<P, false>), dim3((unsigned)grid), dim3(64 * m2l_waves<P, false>()), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
    done(t);
    t = phase(PMX_PHASE_FMM_M2L_SUM);
    launch_grouped(ra, rb, [&](const Group<RedArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_m2l_reduce<P>, dim3((unsigned)nb), dim3(512), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  t = phase(PMX_PHASE_FMM_L2L);
  for (int l = 3; l <= maxL; ++l) {
    std::vector<L2LArgs> la;
    std::vector<int64_t> lb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      if (l > F->L) continue;
      la.push_back({F->lev_off[l], F->tab.p, F->parent.p, F->octant.p, F->Lc.p});
      lb.push_back(F->lev_off[l + 1] - F->lev_off[l]);
    }
    launch_grouped(la, lb, [&](const Group<L2LArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_l2l<P>, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  if (side != st) PMX_HIP(hipStreamWaitEvent(st, ev_join, 0));   // P2P partials and the near part of y are ready
  t = phase(PMX_PHASE_FMM_L2P);
  {
    std::vector<L2PArgs> la;
    std::vector<int64_t> lb;
    for (const ApplyJob& j : jobs) {
      pmx_operator* op = j.op;
      FMM* F = op->fmm;
      const int64_t N = op->s->g.N;
      const float hL = (float)(F->h0 / (double)(1 << F->L));
      la.push_back({F->lev_off[F->L], N, hL, F->tab.p, F->center.p, F->leaf_start.p, F->pts.p, F->Lc.p,
                    multi ? F->partR.p + (int64_t)(r - rb) * N : F->phis.p, multi ? nullptr : F->u_ptr.p, F->perm.p,
                    j.y + (int64_t)r * N, F->chunks.p});
      lb.push_back(F->n_p2p_chunks);
    }
    launch_grouped(la, lb, [&](const Group<L2PArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_l2p<P>, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  (void)n;
}

// A block of 16 right-hand sides [rb, rb + 16): the upward passes for all 16 at once (P2M
// from the block's source rows, M2M with the slices along grid y) into the multipole slices,
// one M2L launch for all 16 (k_m2l16), L2L for all 16, then L2P per right-hand side.  The multi-charge P2P of the block runs on the side stream as in the
// per-rhs path, joined before the first L2P.
template <int P>
static void fmm_far_block16(const std::vector<ApplyJob>& jobs, int rb, Profiler* prof, hipStream_t st,
                            hipStream_t side, hipEvent_t ev_fork, hipEvent_t ev_join,
                            const std::function<void(hipStream_t)>& side_work) {
  constexpr int p3 = P * P * P;
  std::vector<pmx_operator*> ops;
  for (const ApplyJob& j : jobs) ops.push_back(j.op);
  auto phase = [&](int ph) { return prof ? prof->begin(ph, st) : -1; };
  auto done = [&](int t) { if (prof) prof->end(t, st); };
  int maxL = 0;
  for (pmx_operator* op : ops) maxL = std::max(maxL, op->fmm->L);
  // source rows with the block's charges, fork, near part (first block), multi-charge P2P
  {
    std::vector<PermMArgs> qm;
    std::vector<int64_t> qmb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      const int64_t N = op->s->g.N;
      qm.push_back({N, kRBlock, F->rstride, F->perm.p, F->pts.p, op->qt32.p + (int64_t)rb * N, F->qsR.p});
      qmb.push_back((N + 255) / 256);
    }
    launch_grouped(qm, qmb, [&](const Group<PermMArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_permute_multi, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
    if (side != st) {
      PMX_HIP(hipEventRecord(ev_fork, st));
      PMX_HIP(hipStreamWaitEvent(side, ev_fork, 0));
    }
    if (rb == 0 && side_work) side_work(side);
    std::vector<P2PMArgs> qa;
    std::vector<int64_t> qb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      qa.push_back({op->s->g.N, kRBlock, F->rstride, F->p2p_cptr.p, F->p2p_desc.p, F->pts.p, F->qsR.p, F->partR.p});
      qb.push_back(F->n_p2p_chunks);
    }
    const int tp = prof ? prof->begin(PMX_PHASE_FMM_P2P, side) : -1;
    launch_grouped(qa, qb, [&](const Group<P2PMArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_p2p_multi<16>, dim3((unsigned)nb), dim3(64), 0, side, g);
      PMX_HIP(hipGetLastError());
    });
    if (prof) prof->end(tp, side);
    if (side != st) PMX_HIP(hipEventRecord(ev_join, side));
  }
  // upward passes for the 16 right-hand sides together, into the multipole slices: P2M from
  // the block's source rows (built above), then M2M per level with the slices along grid y
  int t = phase(PMX_PHASE_FMM_P2M);
  {
    std::vector<P2M16Args> ma;
    std::vector<int64_t> mb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      const float hL = (float)(F->h0 / (double)(1 << F->L));
      ma.push_back({F->lev_off[F->L], hL, F->rstride, F->tab.p, F->center.p, F->leaf_start.p, F->qsR.p, F->W16.p,
                    F->n_boxes * (int64_t)p3});
      mb.push_back(F->n_leaves);
    }
    launch_grouped(ma, mb, [&](const Group<P2M16Args>& g, int64_t nb) {
      hipLaunchKernelGGL(k_p2m16<P>, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  t = phase(PMX_PHASE_FMM_M2M);
  for (int l = maxL - 1; l >= 2; --l) {
    std::vector<M2MArgs> ma;
    std::vector<int64_t> mb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      if (l >= F->L) continue;
      ma.push_back({F->lev_off[l], F->tab.p, F->child_begin.p, F->child_end.p, F->octant.p, F->W16.p,
                    F->n_boxes * (int64_t)p3});
      mb.push_back(F->lev_off[l + 1] - F->lev_off[l]);
    }
    launch_grouped(ma, mb, [&](const Group<M2MArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_m2m<P>, dim3((unsigned)nb, (unsigned)kRBlock), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  t = phase(PMX_PHASE_FMM_M2L);
  {
    std::vector<M2L16Args> la;
    std::vector<int64_t> lb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      const int64_t box2 = F->lev_off[2];
      la.push_back({F->tab.p, F->r_ptr.p, F->tsrc.p, box2, F->n_boxes, F->L, F->lev_off_d.p, F->W16.p, F->L16.p,
                    F->h0});
      lb.push_back(F->n_boxes - box2);   // one workgroup per box
    }
    launch_grouped(la, lb, [&](const Group<M2L16Args>& g, int64_t nb) {
      hipLaunchKernelGGL(k_m2l16<P>, dim3((unsigned)nb), dim3(64 * m2l16_waves<P>()), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  t = phase(PMX_PHASE_FMM_L2L);
  for (int l = 3; l <= maxL; ++l) {   // the 16 right-hand sides' slices along grid y
    std::vector<L2LArgs> la;
    std::vector<int64_t> lb;
    for (pmx_operator* op : ops) {
      FMM* F = op->fmm;
      if (l > F->L) continue;
      la.push_back({F->lev_off[l], F->tab.p, F->parent.p, F->octant.p, F->L16.p,
                    F->n_boxes * (int64_t)lstride<P>()});
      lb.push_back(F->lev_off[l + 1] - F->lev_off[l]);
    }
    launch_grouped(la, lb, [&](const Group<L2LArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_l2l<P>, dim3((unsigned)nb, (unsigned)kRBlock), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
  if (side != st) PMX_HIP(hipStreamWaitEvent(st, ev_join, 0));   // P2P sums and the near part of y
  t = phase(PMX_PHASE_FMM_L2P);
  for (int j = 0; j < kRBlock; ++j) {
    std::vector<L2PArgs> la;
    std::vector<int64_t> lb;
    for (const ApplyJob& jb : jobs) {
      pmx_operator* op = jb.op;
      FMM* F = op->fmm;
      const int64_t N = op->s->g.N;
      const float hL = (float)(F->h0 / (double)(1 << F->L));
      la.push_back({F->lev_off[F->L], N, hL, F->tab.p, F->center.p, F->leaf_start.p, F->pts.p,
                    F->L16.p + (int64_t)j * F->n_boxes * lstride<P>(), F->partR.p + (int64_t)j * N, nullptr,
                    F->perm.p, jb.y + (int64_t)(rb + j) * N, F->chunks.p});
      lb.push_back(F->n_p2p_chunks);
    }
    launch_grouped(la, lb, [&](const Group<L2PArgs>& g, int64_t nb) {
      hipLaunchKernelGGL(k_l2p<P>, dim3((unsigned)nb), dim3(256), 0, st, g);
      PMX_HIP(hipGetLastError());
    });
  }
  done(t);
}

void fmm_reserve(pmx_operator* op, int n_rhs) {
  FMM* F = op->fmm;
  if (!F || n_rhs <= 1 || F->r_cap >= std::min(n_rhs, kRBlock)) return;
  const int R = std::min(n_rhs, kRBlock);
  const int64_t N = op->s->g.N;
  Ctx* ctx = &op->s->ctx->c;
  F->rstride = (3 + kRBlock + 3) & ~3;   // rows hold the widest block's charges (k_p2p_multi<16> reads 16)
  if (F->qsR.n == 0) F->qsR.alloc(ctx, (size_t)N * F->rstride);
  F->partR.alloc(ctx, (size_t)R * N);
  if (R == kRBlock) {
    F->W16.alloc(ctx, (size_t)kRBlock * F->n_boxes * F->p3);
    F->L16.alloc(ctx, (size_t)kRBlock * F->n_boxes * lstride_of(F->p));
  }
  F->r_cap = R;
}

void fmm_far_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st, hipStream_t side,
                   hipEvent_t ev_fork, hipEvent_t ev_join, const std::function<void(hipStream_t)>& side_work) {
  int p = 0;
  for (const ApplyJob& j : jobs) fmm_reserve(j.op, n_rhs);
  for (const ApplyJob& j : jobs) {
    PMX_REQUIRE(j.op->fmm != nullptr, PMX_ERR_INVALID, "FMM tree not built");
    PMX_REQUIRE(j.y != nullptr, PMX_ERR_INVALID, "FMM far field needs the output array");
    PMX_REQUIRE(p == 0 || j.op->fmm->p == p, PMX_ERR_INVALID, "operators of one batch need the same FMM order");
    p = j.op->fmm->p;
  }
  Profiler* prof = jobs.size() == 1 ? &jobs[0].op->prof : nullptr;
  for (int r = 0; r < n_rhs;) {
    if (n_rhs - r >= kRBlock) {   // whole blocks of 16: M2L with the right-hand sides as columns
      switch (p) {
        case 4: fmm_far_block16<4>(jobs, r, prof, st, side, ev_fork, ev_join, side_work); break;
        case 5: fmm_far_block16<5>(jobs, r, prof, st, side, ev_fork, ev_join, side_work); break;
        case 6: fmm_far_block16<6>(jobs, r, prof, st, side, ev_fork, ev_join, side_work); break;
        default: throw Error(PMX_ERR_INVALID, "fmm_order must be 4, 5 or 6");
      }
      r += kRBlock;
      continue;
    }
    switch (p) {
      case 4: fmm_far_rhs<4>(jobs, r, n_rhs, prof, st, side, ev_fork, ev_join, side_work); break;
      case 5: fmm_far_rhs<5>(jobs, r, n_rhs, prof, st, side, ev_fork, ev_join, side_work); break;
      case 6: fmm_far_rhs<6>(jobs, r, n_rhs, prof, st, side, ev_fork, ev_join, side_work); break;
      default: throw Error(PMX_ERR_INVALID, "fmm_order must be 4, 5 or 6");
    }
    ++r;
  }
}

void fmm_stats(const FMM* f, pmx_operator_stats* s) {
  s->fmm_levels = f->L;
  s->fmm_boxes = f->n_boxes;
  s->fmm_m2l_pairs = f->m2l_pairs;
  s->fmm_p2p_pairs = f->p2p_pairs;
}

uint64_t fmm_bytes(const FMM* f) {
  return f->center.bytes() + f->child_begin.bytes() + f->child_end.bytes() + f->parent.bytes() +
         f->octant.bytes() + f->leaf_start.bytes() + f->perm.bytes() + f->pts.bytes() + f->qs.bytes() +
         f->u_ptr.bytes() + f->u_idx.bytes() + f->p2p_desc.bytes() + f->p2p_slot.bytes() + f->m2l_t.bytes() +
         f->m2l_s.bytes() + f->m2l_lv.bytes() + f->items.bytes() + f->tab.bytes() + f->W.bytes() + f->Lc.bytes() + f->phis.bytes() +
         f->slots.bytes() + f->r_ptr.bytes() + f->m2l_slot.bytes() + f->p2p_cptr.bytes() + f->chunks.bytes() + f->qsR.bytes() +
         f->partR.bytes() + f->tsrc.bytes() + f->lev_off_d.bytes() + f->W16.bytes() + f->L16.bytes();
}

}  // namespace pmx
