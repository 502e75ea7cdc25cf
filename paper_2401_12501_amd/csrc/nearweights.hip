// Correction blocks of the self and near rules (FP64).
//
// For a target node i and a patch P in near(i):
//   W_{i,P,j} = int_[-1,1]^2 F(x_i, y~(u,v)) l_j(u,v) J~(u,v) du dv,
//   C_{i,P,j} = W_{i,P,j} - [j != i] w_j F(x_i, x_j),
// where y~, x~_u, x~_v and a~ are tensor Lagrange interpolants of the patch's node
// data (the paper interpolates sigma to the quadrature grid, Section 6.1.1 Remark
// and Section 6.1.2), J~ = |x~_u x x~_v| and F is the remainder R or the
// parametrix K.  With c != 0 c~ is interpolated like a, F carries the c-dependent Green's function
// (G = -K0(kappa r) / (2 pi a) for c < 0; for c > 0 the complex G = -(i / 4a) H0(k r), whose real
// and imaginary parts are integrated by two launches, each an ordinary real kernel) and the
// c-term of eq:explicit_remainder, and the self rule integrates R on the dyadic radial panels of
// K, plain on the innermost one (R then has r^m log r parts).
//
// Self rule (i in P, Section 6.1.1, eq:radial_int): polar coordinates about the
// target pre-image t0.  The square splits into four triangles (t0, c_k, c_k+1);
// on the triangle of edge k the ray at angle phi from the edge normal leaves at
// L = d_k / cos(phi).  Angular panels are split at phi = 0 and where L doubles
// (cos phi = 2^-m), each with n_gl Gauss-Legendre points.  Radially R uses one
// n_gl-point panel on [0, L]; K uses the panels [L/2, L], [L/4, L/2], [L/8, L/4]
// and [0, L/8] with rho = t^3 L / 8 on the last one (log singularity).
//
// Near rule (i not in P, Section 6.1.2): the parameter square is subdivided while
// the target is within eta radii of a sub-square's centroid (centroid and radius
// from the sub-square's corner images), depth <= 20; each leaf carries an
// n_gl x n_gl tensor Gauss-Legendre rule.
//
// Layout: one workgroup per (target, patch) pair (one wave for a near pair), specialised
// on the patch order q.
// After the cells (self panels or near leaves) are built:
//  * near leaves: each wave takes whole leaves; a leaf's tensor rule turns the field
//    interpolation and the block update into chained small products on the FP64
//    MFMA (see below), about a sixth of the work of interpolating point by point;
//  * self panels: each wave takes its own batches of 64 quadrature points, one per
//    lane: the lane evaluates its point's Lagrange values (registers), interpolates
//    the ten patch fields with the node data read through the scalar cache (all
//    lanes use the same node values), evaluates the kernel and writes
//    (c l_a(u), l_b(v)) to its wave's LDS rows; the block update W += Lu^T diag(c) Lv
//    is then sixteen FP64 MFMA steps of 4 points each.
// Each wave's 16 x 16 accumulator stays in registers and the waves' accumulators are
// summed in a fixed order at the end.
#include <cmath>

#include "pmx_internal.hpp"

namespace pmx {

namespace {

constexpr int kMaxCells = 256;   // panels (self) or leaves (near) per pair
constexpr int kMaxDepth = 20;
constexpr int kNglMax = 16;
constexpr int kStage = 65;       // LDS row stride of the staging rows, in doubles (odd)

// Pointer whose loads go through the scalar cache when the address is uniform.
typedef const __attribute__((address_space(4))) double* sdp;

struct NWArgs {
  int64_t N;
  int q;
  int n_gl;
  double eta;
  const double* X;      // 3N SoA
  const double* XP;     // node-major fields x y z x_u x_v a (and c): 10 (11) per node
  const double* a;      // N
  const double* c;      // N, c < 0 (kernels 2 and 3) or c > 0 (kernels 4 and 5); null for c = 0
  const double* w;      // N
  const double* tgt;    // 8N: x y z nx ny nz A B
  const double* tg;     // 3N: grad_G a / (2 pi)
  const double* tn;     // q nodes
  const double* cinv;   // q: 1 / prod_{k != j} (t_j - t_k)
  const double* gl_t;   // n_gl Gauss-Legendre nodes on [-1, 1]
  const double* gl_w;   // n_gl weights
  const int64_t* ptr;   // N + 1: near-list rows
  const int32_t* pair_patch;
  const int32_t* pair_target;
  double* out;          // nnz * q*q
  int* err;
  int64_t pair0;
  int cpos;             // c > 0: kernels 4 and 5
  int imag;             // c > 0: 0 the real part of F, 1 the imaginary part
};

// Waves per workgroup.  Self rule: the target's panels are spread over several waves.
// Near rule: one wave per (target, patch) pair, so the subdivision's barriers and the final
// sum are those of a single wave, and many pairs are resident per CU to hide each other's
// latency (the leaves of a pair run one after another on its wave).
template <int Q, bool SELF>
constexpr int waves_for() { return SELF ? (Q <= 12 ? 4 : 2) : 1; }

// Lagrange values of the q nodes at s: l_j(s) = cinv_j prod_{k != j} (s - t_k),
// from prefix and suffix products (no division by s - t_j).
template <int Q>
__device__ inline void lagrange_q(sdp tn, sdp cinv, double s, double (&l)[Q]) {
  double d[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) d[j] = s - tn[j];
  double pre = 1.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    l[j] = pre;
    pre *= d[j];
  }
  double suf = 1.0;
#pragma unroll
  for (int j = Q - 1; j >= 0; --j) {
    l[j] *= suf * cinv[j];
    suf *= d[j];
  }
}

// Tensor interpolation of the first NF of the node fields (x, x_u, x_v, a and, with c, c;
// node-major, ST per node): g_f = sum_a l_a(u) sum_b l_b(v) X[(a q + b) ST + f].  The node values are
// uniform across the wave and come through the scalar cache; each node's loads are
// issued one node ahead of its FMAs and the scheduling barriers keep the compiler from
// hoisting more of them (which would exhaust the scalar registers).
template <int Q, int NF, int ST>
__device__ inline void interp_q(sdp XP, const double (&lu)[Q], const double (&lv)[Q], double (&g)[NF]) {
#pragma unroll
  for (int f = 0; f < NF; ++f) g[f] = 0.0;
  double cur[NF], nxt[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) cur[f] = XP[f];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    double t[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) t[f] = 0.0;
#pragma unroll
    for (int b = 0; b < Q; ++b) {
      const int n = a * Q + b;
      if (n + 1 < Q * Q) {
#pragma unroll
        for (int f = 0; f < NF; ++f) nxt[f] = XP[(n + 1) * ST + f];
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        t[f] = fma(lv[b], cur[f], t[f]);
        asm volatile("" : "+v"(t[f]));   // keep this node's FMAs ahead of the next node's loads
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int f = 0; f < NF; ++f) cur[f] = nxt[f];
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) g[f] = fma(lu[a], t[f], g[f]);
  }
}

struct Target {
  double x[3], n[3], A, B, g[3];
  double at2, ct2;   // a / (2 pi) and c / (2 pi) at the target (c != 0)
  int imag;          // c > 0: which part of the complex kernel
};

// Factored c = 0 remainder: R = (1/a') [ g.r/r^2 + A (n.r)^2/r^4 - B (n.r)/r^2 ].
__device__ inline double remainder_dev(const Target& T, const double* y, double inv_as) {
  const double r0 = T.x[0] - y[0], r1 = T.x[1] - y[1], r2 = T.x[2] - y[2];
  const double rr = r0 * r0 + r1 * r1 + r2 * r2;
  const double inv = 1.0 / rr;
  const double nr = T.n[0] * r0 + T.n[1] * r1 + T.n[2] * r2;
  const double gr = T.g[0] * r0 + T.g[1] * r1 + T.g[2] * r2;
  const double s = nr * inv;
  return inv_as * (s * (T.A * s - T.B) + gr * inv);
}

__device__ inline double parametrix_dev(const Target& T, const double* y, double inv_as) {
  const double r0 = T.x[0] - y[0], r1 = T.x[1] - y[1], r2 = T.x[2] - y[2];
  const double rr = r0 * r0 + r1 * r1 + r2 * r2;
  return log_pair(rr) * 0.07957747154594766788 * inv_as;   // log(r) / (2 pi a)
}

// c < 0: with kappa = sqrt(-c'/a') at the source, z = kappa r and k0, k1 = K0(z), K1(z),
// eq:explicit_remainder times a' is
//   kappa k1 [g.r/r + 2 at2 (n.r)^2/r^3 - B n.r/r] + at2 kappa^2 k0 ((n.r)^2/r^2 - 1) - ct2 k0
// (g = grad_G a / (2 pi), at2 = a / (2 pi), B = a H / pi, ct2 = c / (2 pi) at the target); it
// reduces to the c = 0 form as c -> 0.
__device__ inline double remainder_c_dev(const Target& T, const double* y, double inv_as, double c_s) {
  const double r0 = T.x[0] - y[0], r1 = T.x[1] - y[1], r2 = T.x[2] - y[2];
  const double rr = r0 * r0 + r1 * r1 + r2 * r2;
  const double ir = rsqrt(rr), rn = rr * ir;
  const double kap = sqrt(-c_s * inv_as);
  double k0, k1;
  bessel_k01(kap * rn, k0, k1);
  const double nr = T.n[0] * r0 + T.n[1] * r1 + T.n[2] * r2;
  const double gr = T.g[0] * r0 + T.g[1] * r1 + T.g[2] * r2;
  const double snr = nr * ir;   // n.r / r
  const double bra = fma(ir, fma(2.0 * T.at2 * snr, snr, gr), -T.B * snr);
  const double e = kap * k1 * bra + T.at2 * kap * kap * k0 * fma(snr, snr, -1.0) - T.ct2 * k0;
  return e * inv_as;
}

__device__ inline double parametrix_c_dev(const Target& T, const double* y, double inv_as, double c_s) {
  const double r0 = T.x[0] - y[0], r1 = T.x[1] - y[1], r2 = T.x[2] - y[2];
  const double rn = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
  double k0, k1;
  bessel_k01(sqrt(-c_s * inv_as) * rn, k0, k1);
  return -k0 * 0.15915494309189533577 * inv_as;   // -K0(kappa r) / (2 pi a)
}

// c > 0: with k = sqrt(c'/a') at the source, z = k r and J0, J1, Y0, Y1 at z, eq:explicit_remainder
// times a' for G = -(i / 4a') H0(k r) is (i pi / 2) {k H1 bra - m H0}, bra as above and
// m = at2 k^2 ((n.r)^2/r^2 - 1) + ct2, i.e.
//   real part (pi/2) (m Y0 - k Y1 bra),   imaginary part (pi/2) (k J1 bra - m J0).
__device__ inline double remainder_cpos_dev(const Target& T, const double* y, double inv_as, double c_s) {
  const double r0 = T.x[0] - y[0], r1 = T.x[1] - y[1], r2 = T.x[2] - y[2];
  const double rr = r0 * r0 + r1 * r1 + r2 * r2;
  const double ir = rsqrt(rr), rn = rr * ir;
  const double k = sqrt(c_s * inv_as);
  double j0, j1, y0, y1;
  bessel_jy01(k * rn, j0, j1, y0, y1);
  const double nr = T.n[0] * r0 + T.n[1] * r1 + T.n[2] * r2;
  const double gr = T.g[0] * r0 + T.g[1] * r1 + T.g[2] * r2;
  const double snr = nr * ir;
  const double bra = fma(ir, fma(2.0 * T.at2 * snr, snr, gr), -T.B * snr);
  const double m = fma(T.at2 * k * k, fma(snr, snr, -1.0), T.ct2);
  const double e = T.imag ? fma(k * j1, bra, -m * j0) : fma(m, y0, -k * y1 * bra);
  return 1.5707963267948966192 * e * inv_as;
}

// K = (Y0(k r) - i J0(k r)) / (4 a')
__device__ inline double parametrix_cpos_dev(const Target& T, const double* y, double inv_as, double c_s) {
  const double r0 = T.x[0] - y[0], r1 = T.x[1] - y[1], r2 = T.x[2] - y[2];
  const double rn = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
  double j0, j1, y0, y1;
  bessel_jy01(sqrt(c_s * inv_as) * rn, j0, j1, y0, y1);
  return 0.25 * (T.imag ? -j0 : y0) * inv_as;
}

// Kernel F at a point y with coefficients a' = 1 / inv_as (and c_s): KERNEL 0 R, 1 K (c = 0);
// 2 R, 3 K (c < 0); 4 R, 5 K (c > 0, the part T.imag selects).
template <int KERNEL>
__device__ inline double kernel_dev(const Target& T, const double* y, double inv_as, double c_s) {
  if constexpr (KERNEL == 0) return remainder_dev(T, y, inv_as);
  else if constexpr (KERNEL == 1) return parametrix_dev(T, y, inv_as);
  else if constexpr (KERNEL == 2) return remainder_c_dev(T, y, inv_as, c_s);
  else if constexpr (KERNEL == 3) return parametrix_c_dev(T, y, inv_as, c_s);
  else if constexpr (KERNEL == 4) return remainder_cpos_dev(T, y, inv_as, c_s);
  else return parametrix_cpos_dev(T, y, inv_as, c_s);
}

union Cell {                    // self: angular panel [p0, p1] of one edge; near: leaf (depth, iu, iv)
  struct { double p0, p1; } s;
  struct { int depth, iu, iv, pad; } n;
};

typedef double v4d __attribute__((ext_vector_type(4)));

// The same pointer, opaque to the optimiser: node loads through it are neither hoisted
// out of the enclosing loop nor shared between calls, so they stay next to their FMAs.
__device__ inline sdp opaque(sdp p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  return (sdp)v;
}

}  // namespace

// KERNEL: 0 = remainder R (correction blocks C), 1 = parametrix K (blocks D); 2 and 3 the same
// with c < 0, 4 and 5 with c > 0 (eleven node fields: c interpolated like a).
// SELF: one workgroup per target for the pair with its own patch; otherwise one per
// near-list pair, the self pairs leaving at once (the two launches get their own
// register allocation: the self rule is VALU work, the near rule MFMA work).
template <int KERNEL, int Q, bool SELF>
__global__ void __launch_bounds__((64 * waves_for<Q, SELF>())) __attribute__((amdgpu_waves_per_eu(2)))
k_near_weights(NWArgs A) {
  constexpr int kW = waves_for<Q, SELF>();
  constexpr int kT = 64 * kW;
  constexpr int q2 = Q * Q;
  constexpr bool kC = KERNEL >= 2;        // c != 0
  constexpr int NF = kC ? 11 : 10;        // node fields (and their stride in XP)
  extern __shared__ double lds[];
  // stage[w][2][Q][kStage]; the subdivision front and flags overlay it before the point loop
  double* stage = lds;
  int2* front = reinterpret_cast<int2*>(lds);                 // [2][kMaxCells]
  int* flag_split = reinterpret_cast<int*>(front + 2 * kMaxCells);
  double* corner_xyz = reinterpret_cast<double*>(flag_split + kT);   // [kT / 4 squares][4][3]
  __shared__ Cell cells[kMaxCells];
  __shared__ int cell_edge[kMaxCells];
  __shared__ int n_cells;
  __shared__ int n_front[2];
  __shared__ double W[q2];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  int64_t pair, i;
  int P;
  if constexpr (SELF) {
    i = A.pair0 + blockIdx.x;
    P = (int)(i / q2);
    pair = A.ptr[i];
    for (int64_t e = A.ptr[i]; e < A.ptr[i + 1]; ++e)   // a target is always near its own patch
      if (A.pair_patch[e] == P) pair = e;
  } else {
    pair = A.pair0 + blockIdx.x;
    P = A.pair_patch[pair];
    i = A.pair_target[pair];
    if (i / q2 == P) return;
  }
  const int64_t N = A.N;
  const int64_t base = (int64_t)P * q2;
  constexpr bool self = SELF;

  const sdp F = (sdp)(A.XP + base * NF);
  const sdp tn = (sdp)A.tn, cinv = (sdp)A.cinv, gl_t = (sdp)A.gl_t, gl_w = (sdp)A.gl_w;

  Target T;
  for (int c = 0; c < 3; ++c) {
    T.x[c] = A.tgt[c * N + i];
    T.n[c] = A.tgt[(3 + c) * N + i];
    T.g[c] = A.tg[c * N + i];
  }
  T.A = A.tgt[6 * N + i];
  T.B = A.tgt[7 * N + i];
  T.at2 = 0.5 * T.A;
  T.ct2 = kC ? A.c[i] * 0.15915494309189533577 : 0.0;
  T.imag = A.imag;
  const int ngl = A.n_gl;

  // ------------------------------------------------------------------ cells
  double u0 = 0.0, v0 = 0.0;
  if (self) {
    const int loc = (int)(i - base);
    u0 = tn[loc / Q];
    v0 = tn[loc % Q];
    if (tid == 0) {
      int nc = 0;
      const double dd[4] = {v0 + 1.0, 1.0 - u0, 1.0 - v0, u0 + 1.0};
      // tangential coordinate (along the edge, counter-clockwise) of the edge's two corners
      const double sa[4] = {-1.0 - u0, -1.0 - v0, u0 - 1.0, v0 - 1.0};
      const double sb[4] = {1.0 - u0, 1.0 - v0, u0 + 1.0, v0 + 1.0};
      for (int k = 0; k < 4; ++k) {
        const double pa = atan2(sa[k], dd[k]), pb = atan2(sb[k], dd[k]);
        // positive side [0, pb], then negative side [pa, 0]
        for (int side = 0; side < 2; ++side) {
          const double end = side == 0 ? pb : -pa;
          double prev = 0.0;
          for (int m = 1;; ++m) {
            const double b = acos(ldexp(1.0, -m));
            const bool last = !(b < end);
            const double hi = last ? end : b;
            if (nc < kMaxCells) {
              cells[nc].s.p0 = side == 0 ? prev : -hi;
              cells[nc].s.p1 = side == 0 ? hi : -prev;
              cell_edge[nc] = k;
            }
            ++nc;
            prev = hi;
            if (last) break;
          }
        }
      }
      n_cells = nc;
    }
  } else {
    // level-synchronous subdivision of [-1, 1]^2; a square at depth d is (iu, iv) * 2^(1-d) - 1
    if (tid == 0) {
      n_front[0] = 1;
      n_front[1] = 0;
      front[0] = make_int2(0, 0);
      n_cells = 0;
    }
    __syncthreads();
    int cur = 0;
    for (int depth = 0; depth <= kMaxDepth; ++depth) {
      const int nf = n_front[cur];
      if (nf == 0) break;
      // four threads per square, one corner image each; then one thread per square decides
      for (int f0 = 0; f0 < nf; f0 += kT / 4) {
        const int nsq = nf - f0 < kT / 4 ? nf - f0 : kT / 4;
        {
          const int sq = tid >> 2, k = tid & 3;
          if (sq < nsq) {
            const int iu = front[cur * kMaxCells + f0 + sq].x, iv = front[cur * kMaxCells + f0 + sq].y;
            const double h = 2.0 / (double)(1 << depth);
            const double ua = -1.0 + iu * h, va = -1.0 + iv * h;
            const double cu = (k == 1 || k == 2) ? ua + h : ua;   // corners (ua,va) (ub,va) (ub,vb) (ua,vb)
            const double cv = (k >= 2) ? va + h : va;
            double lu[Q], lv[Q], g[3];
            lagrange_q<Q>(tn, cinv, cu, lu);
            lagrange_q<Q>(tn, cinv, cv, lv);
            interp_q<Q, 3, NF>(opaque(F), lu, lv, g);
            corner_xyz[tid * 3] = g[0];
            corner_xyz[tid * 3 + 1] = g[1];
            corner_xyz[tid * 3 + 2] = g[2];
          }
        }
        __syncthreads();
        if (tid < nsq) {
          const double* cx = corner_xyz + tid * 12;
          double m[3];
          for (int c = 0; c < 3; ++c) m[c] = 0.25 * (cx[c] + cx[3 + c] + cx[6 + c] + cx[9 + c]);
          double rad = 0.0;
          for (int k = 0; k < 4; ++k) {
            const double d0 = cx[3 * k] - m[0], d1 = cx[3 * k + 1] - m[1], d2 = cx[3 * k + 2] - m[2];
            rad = fmax(rad, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
          }
          const double e0 = T.x[0] - m[0], e1 = T.x[1] - m[1], e2 = T.x[2] - m[2];
          const double dist = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
          flag_split[tid] = (dist < A.eta * rad && depth < kMaxDepth) ? 1 : 0;
        }
        __syncthreads();
        // compaction in square order by the first wave (nsq <= 64): a square that splits
        // appends its four children to the next front, one that does not becomes a leaf
        if (tid < 64) {
          const int nxt = cur ^ 1;
          const bool in = tid < nsq;
          const bool sp = in && flag_split[tid] != 0;
          const uint64_t m_split = __ballot(sp), m_leaf = __ballot(in && !sp);
          const uint64_t below = (1ull << tid) - 1ull;
          const int f_base = n_front[nxt], c_base = n_cells;
          if (in) {
            const int iu = front[cur * kMaxCells + f0 + tid].x, iv = front[cur * kMaxCells + f0 + tid].y;
            if (sp) {
              const int o = f_base + 4 * __popcll(m_split & below);
              const int cu2[4] = {2 * iu, 2 * iu + 1, 2 * iu, 2 * iu + 1};
              const int cv2[4] = {2 * iv, 2 * iv, 2 * iv + 1, 2 * iv + 1};
              for (int c = 0; c < 4; ++c)
                if (o + c < kMaxCells) front[nxt * kMaxCells + o + c] = make_int2(cu2[c], cv2[c]);
            } else {
              const int o = c_base + __popcll(m_leaf & below);
              if (o < kMaxCells) {
                cells[o].n.depth = depth;
                cells[o].n.iu = iu;
                cells[o].n.iv = iv;
              }
            }
          }
          __builtin_amdgcn_wave_barrier();
          if (tid == 0) {
            n_front[nxt] = f_base + 4 * __popcll(m_split);
            n_cells = c_base + __popcll(m_leaf);
          }
        }
        __syncthreads();
      }
      if (tid == 0) {
        n_front[cur] = 0;
        if (n_front[cur ^ 1] > kMaxCells) {
          atomicOr(A.err, 2);
          n_front[cur ^ 1] = 0;
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  __syncthreads();
  int nc = n_cells;
  if (nc > kMaxCells) {
    if (tid == 0) atomicOr(A.err, 2);
    nc = 0;
  }

  const int r16 = lane & 15, g4 = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};   // this wave's share of W: lane holds W[g4 + 4 r][r16]

  // ------------------------------------------------------------------ near rule: tensor leaves
  // A leaf carries a 16 x 16 tensor rule (points u_i, v_k; unused rows when n_gl < 16
  // get weight zero).  Everything is a small product done on the FP64 MFMA, in the
  // register layouts the instruction produces, so no data moves between the steps:
  //   T_f[a][k]   = sum_b X_f[a][b] l_b(v_k)          (X_f: one of the patch's ten node fields)
  //   G_f[i][k]   = sum_a l_a(u_i) T_f[a][k]          (the field at the leaf's points)
  //   c[i][k]     = w_i w_k h^2 F(x_target, y(i,k)) J(i,k)
  //   U[i][b]     = sum_k c[i][k] l_b(v_k)
  //   W[a][b]    += sum_i l_a(u_i) U[i][b]
  // (a 16 x 16 x 4 FP64 MFMA leaves D[g4 + 4 r][r16] in register r of lane 16 g4 + r16,
  // which is exactly where the next product's A operand for k-step r has to be).
  if (!self && nc > 0) {
    constexpr int KS = (Q + 3) / 4;   // k-steps over a patch index (a or b)
    // the patch's node fields go to LDS once per pair (sX[f][a][b]); the rule tables and
    // Lagrange denominators a lane needs are loaded into registers ahead of the leaves
    double* sX = stage;   // 10 q^2 doubles (the self rule's staging area is not used here)
    for (int e = tid; e < NF * q2; e += kT) {
      const int f = e / q2, j = e - f * q2;
      sX[e] = A.XP[(base + j) * NF + f];
    }
    __syncthreads();
    const bool rin = r16 < ngl;
    const double t_r = gl_t[rin ? r16 : 0], w_r = rin ? gl_w[r16] : 0.0;
    double w_g[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int m = 4 * ks + g4;
      w_g[ks] = m < ngl ? gl_w[m] : 0.0;
    }
    // per wave, per leaf: Lagrange tables Lu[i][a] = l_a(u_i), Lv[k][b] = l_b(v_k) in LDS,
    // one point's row per lane (lanes 0-15: u_i, lanes 16-31: v_k)
    double* sLu = stage + NF * q2 + (size_t)wave * 32 * Q;
    double* sLv = sLu + 16 * Q;
    for (int cell = wave; cell < nc; cell += kW) {
      const Cell C = cells[cell];
      const double h = 2.0 / (double)(1 << C.n.depth);
      const double ua = -1.0 + C.n.iu * h, va = -1.0 + C.n.iv * h;
      const double hh = 0.5 * h;
      if (lane < 32) {
        double l[Q];
        lagrange_q<Q>(tn, cinv, (lane < 16 ? ua : va) + hh * (t_r + 1.0), l);
#pragma unroll
        for (int j = 0; j < Q; ++j) sLu[lane * Q + j] = l[j];   // lane >= 16 writes the Lv rows
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double lvb[KS], lua[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int j = 4 * ks + g4;
        lvb[ks] = j < Q ? sLv[r16 * Q + (j < Q ? j : 0)] : 0.0;   // B[b][k] = l_b(v_k), b = j, k = r16
        lua[ks] = j < Q ? sLu[r16 * Q + (j < Q ? j : 0)] : 0.0;   // B[a][i] = l_a(u_i), a = j, i = r16
      }
      // G_f^T: lane holds G_f at (k = g4 + 4 r, i = r16)
      v4d acc2[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        v4d t1 = {0.0, 0.0, 0.0, 0.0};   // T_f[a = g4 + 4 r][k = r16]
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int b = 4 * ks + g4;
          const double xv = (r16 < Q && b < Q) ? sX[f * q2 + (r16 < Q ? r16 : 0) * Q + (b < Q ? b : 0)] : 0.0;
          t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(xv, lvb[ks], t1, 0, 0, 0);
        }
        acc2[f] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)   // A[k][a] = T_f[a = 4 ks + g4][k = r16] = t1[ks]
          acc2[f] = __builtin_amdgcn_mfma_f64_16x16x4f64(t1[ks], lua[ks], acc2[f], 0, 0, 0);
      }
      // kernel at the lane's four points (i = r16, k = g4 + 4 r)
      double cval[4];
      const double hh2 = hh * hh;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double gv[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) gv[f] = acc2[f][r];
        const double x0 = gv[4] * gv[8] - gv[5] * gv[7];
        const double x1 = gv[5] * gv[6] - gv[3] * gv[8];
        const double x2 = gv[3] * gv[7] - gv[4] * gv[6];
        const double Jt = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
        const double inv_as = 1.0 / gv[9];
        const double Fk = kernel_dev<KERNEL>(T, gv, inv_as, kC ? gv[NF - 1] : 0.0);
        cval[r] = w_r * w_g[r] * hh2 * Fk * Jt;   // zero weight outside the n_gl x n_gl rule
      }
      // U = C L_v: A[i][k] = c[i][k] with k = 4 ks + g4 (register ks of this lane)
      v4d accU = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const double lvk = r16 < Q ? sLv[(4 * ks + g4) * Q + (r16 < Q ? r16 : 0)] : 0.0;   // l_b(v_k), b = r16
        accU = __builtin_amdgcn_mfma_f64_16x16x4f64(cval[ks], w_g[ks] != 0.0 ? lvk : 0.0, accU, 0, 0, 0);
      }
      // W += L_u^T U: A[a][i] = l_a(u_i), B[i][b] = U[i][b] with i = 4 ks + g4 (register ks)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const double lai = r16 < Q ? sLu[(4 * ks + g4) * Q + (r16 < Q ? r16 : 0)] : 0.0;   // l_a(u_i), a = r16
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(w_g[ks] != 0.0 ? lai : 0.0, accU[ks], acc, 0, 0, 0);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // tables are rewritten for the next leaf
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }

  // ------------------------------------------------------------------ self rule: points
  const unsigned n_rad = (self && KERNEL != 0) ? 4 * ngl : ngl;   // log-graded panels for all but R, c = 0
  const unsigned ppc = self ? (unsigned)ngl * n_rad : (unsigned)(ngl * ngl);
  const unsigned n_pts = self ? ppc * (unsigned)nc : 0u;
  double* CL = stage + (size_t)wave * 2 * Q * kStage;   // c l_a(u) at [a][point]
  double* LV = CL + Q * kStage;                          // l_b(v) at [b][point]
  const int rq = r16 < Q ? r16 : 0;
  for (unsigned p0 = (unsigned)wave * 64; p0 < n_pts; p0 += kT) {
    const unsigned p = p0 + lane;
    const bool valid = p < n_pts;
    double u = 0.0, v = 0.0, wq = 0.0;
    if (valid) {
      const unsigned cell = p / ppc;
      const unsigned r = p - cell * ppc;
      if (self) {
        const int k = cell_edge[cell];
        const double c0 = cells[cell].s.p0, c1 = cells[cell].s.p1;
        const unsigned ia = r / n_rad, ir = r - ia * n_rad;
        const double dk = k == 0 ? v0 + 1.0 : (k == 1 ? 1.0 - u0 : (k == 2 ? 1.0 - v0 : u0 + 1.0));
        const double mid = 0.5 * (c0 + c1), half = 0.5 * (c1 - c0);
        const double phi = mid + half * gl_t[ia];
        double sp, cp;
        sincos(phi, &sp, &cp);
        const double L = dk / cp;
        // radial node s in (0, 1] and weight for int_0^L F rho drho = L^2 sum w F(L s)
        double s, wr;
        const unsigned pr = ir / ngl, jr = ir - pr * ngl;
        const double t = 0.5 * (gl_t[jr] + 1.0), wt = 0.5 * gl_w[jr];
        // R (c = 0): one panel [0, 1]; K: dyadic panels with rho = t^3 / 8 on the innermost;
        // R (c != 0): the dyadic panels, plain on the innermost [0, 1/8] too (the t^3 map would put
        // points within 1e-10 of the target, where r keeps too few digits of its normal component)
        if (KERNEL == 0 || pr < 3 || KERNEL == 2 || KERNEL == 4) {
          const double lo = (KERNEL == 0 || pr == 3) ? 0.0 : ldexp(1.0, -(int)(pr + 1));
          const double hi = KERNEL == 0 ? 1.0 : ldexp(1.0, -(int)pr);
          s = lo + (hi - lo) * t;
          wr = (hi - lo) * wt * s;
        } else {
          s = t * t * t * 0.125;
          wr = wt * 3.0 * t * t * t * t * t / 64.0;
        }
        wq = half * gl_w[ia] * L * L * wr;
        // direction at angle (edge normal + phi); the edge normals point along -v, +u, +v, -u
        const double ca = k == 0 ? sp : (k == 1 ? cp : (k == 2 ? -sp : -cp));
        const double sa = k == 0 ? -cp : (k == 1 ? sp : (k == 2 ? cp : -sp));
        u = u0 + L * s * ca;
        v = v0 + L * s * sa;
      } else {
        const Cell C = cells[cell];
        const unsigned ia = r / ngl, ib = r - ia * ngl;
        const double h = 2.0 / (double)(1 << C.n.depth);
        const double ua = -1.0 + C.n.iu * h, va = -1.0 + C.n.iv * h;
        const double hh = 0.5 * h;
        u = ua + hh * (gl_t[ia] + 1.0);
        v = va + hh * (gl_t[ib] + 1.0);
        wq = gl_w[ia] * gl_w[ib] * hh * hh;
      }
    }
    double lu[Q], lv[Q], g[NF];
    lagrange_q<Q>(tn, cinv, u, lu);
    lagrange_q<Q>(tn, cinv, v, lv);
    interp_q<Q, NF, NF>(opaque(F), lu, lv, g);
    const double x0 = g[4] * g[8] - g[5] * g[7];
    const double x1 = g[5] * g[6] - g[3] * g[8];
    const double x2 = g[3] * g[7] - g[4] * g[6];
    const double Jt = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
    const double inv_as = 1.0 / g[9];
    const double Fk = kernel_dev<KERNEL>(T, g, inv_as, kC ? g[NF - 1] : 0.0);
    const double c = valid ? wq * Fk * Jt : 0.0;
    // stage this wave's 64 points; LDS operations of one wave complete in order
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      CL[a * kStage + lane] = c * lu[a];
      LV[a * kStage + lane] = lv[a];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // W[a][b] += sum_t CL[a][t] LV[b][t]: A[a][k] = CL[a][4s + k], B[k][b] = LV[b][4s + k]
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const double av = CL[rq * kStage + 4 * s + g4];
      const double bv = LV[rq * kStage + 4 * s + g4];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(r16 < Q ? av : 0.0, r16 < Q ? bv : 0.0, acc, 0, 0, 0);
    }
  }

  // ------------------------------------------------------------------ sum the waves' accumulators
  __syncthreads();
  double* red = stage;   // [wave][16][16]; for the FP64 16x16x4 MFMA, lane holds D[g4 + 4 r][r16]
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wave * 256 + (g4 + 4 * r) * 16 + r16] = acc[r];
  __syncthreads();
  for (int e = tid; e < q2; e += kT) {
    const int aa = e / Q, b = e - aa * Q;
    double s = 0.0;
    for (int w = 0; w < kW; ++w) s += red[w * 256 + aa * 16 + b];
    W[e] = s;
  }
  __syncthreads();

  // ------------------------------------------------------------------ subtract the smooth rule
  for (int e = tid; e < q2; e += kT) {
    const int64_t j = base + e;
    double val = W[e];
    if (j != i) {
      const double y[3] = {A.X[j], A.X[N + j], A.X[2 * N + j]};
      const double inv_a = 1.0 / A.a[j];
      const double Fs = kernel_dev<KERNEL>(T, y, inv_a, kC ? A.c[j] : 0.0);
      val -= A.w[j] * Fs;
    }
    A.out[pair * q2 + e] = val;
  }
}

// Node-major fields for the local rules: x, x_u, x_v, a and, when c is given, c (nf = 10 or 11).
__global__ void k_interleave(int64_t N, const double* __restrict__ x, const double* __restrict__ xu,
                             const double* __restrict__ xv, const double* __restrict__ a,
                             const double* __restrict__ c, int nf, double* __restrict__ xp) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double* o = xp + j * nf;
  for (int k = 0; k < 3; ++k) {
    o[k] = x[k * N + j];
    o[3 + k] = xu[k * N + j];
    o[6 + k] = xv[k * N + j];
  }
  o[9] = a[j];
  if (nf == 11) o[10] = c[j];
}

namespace {

template <int Q, bool SELF>
size_t lds_bytes() {
  constexpr int kW = waves_for<Q, SELF>();
  // self: the waves' staging rows; near: the patch's node fields (up to 11) and each wave's
  // Lagrange tables
  const size_t stage = SELF ? (size_t)kW * 2 * Q * kStage * sizeof(double)
                            : (size_t)(11 * Q * Q + kW * 32 * Q) * sizeof(double);
  const size_t front = 2 * kMaxCells * sizeof(int2) + 64 * kW * sizeof(int) + 16 * kW * 12 * sizeof(double);
  const size_t red = (size_t)kW * 256 * sizeof(double);
  size_t m = stage > front ? stage : front;
  return m > red ? m : red;
}

template <int KERNEL, int Q>
void launch_kq(const NWArgs& A, int64_t n, bool self, hipStream_t st, size_t lds) {
  const dim3 block(64 * (self ? waves_for<Q, true>() : waves_for<Q, false>()));
  if (self) hipLaunchKernelGGL((k_near_weights<KERNEL, Q, true>), dim3(n), block, lds, st, A);
  else hipLaunchKernelGGL((k_near_weights<KERNEL, Q, false>), dim3(n), block, lds, st, A);
}

template <int Q>
void launch_q(const NWArgs& A, int64_t n, bool parametrix, bool self, hipStream_t st, size_t lds_limit) {
  const size_t lds = self ? lds_bytes<Q, true>() : lds_bytes<Q, false>();
  PMX_REQUIRE(lds + 12 * 1024 <= lds_limit, PMX_ERR_INVALID,
              "q too large for the local-rule kernel's LDS on this device");
  const bool c = A.c != nullptr;
  if (!c) {
    if (parametrix) launch_kq<1, Q>(A, n, self, st, lds);
    else launch_kq<0, Q>(A, n, self, st, lds);
  } else if (!A.cpos) {
    if (parametrix) launch_kq<3, Q>(A, n, self, st, lds);
    else launch_kq<2, Q>(A, n, self, st, lds);
  } else {
    if (parametrix) launch_kq<5, Q>(A, n, self, st, lds);
    else launch_kq<4, Q>(A, n, self, st, lds);
  }
  PMX_HIP(hipGetLastError());
}

void launch_dispatch(int q, const NWArgs& A, int64_t n, bool parametrix, bool self, hipStream_t st,
                     size_t lds_limit) {
  switch (q) {
    case 2: launch_q<2>(A, n, parametrix, self, st, lds_limit); break;
    case 3: launch_q<3>(A, n, parametrix, self, st, lds_limit); break;
    case 4: launch_q<4>(A, n, parametrix, self, st, lds_limit); break;
    case 5: launch_q<5>(A, n, parametrix, self, st, lds_limit); break;
    case 6: launch_q<6>(A, n, parametrix, self, st, lds_limit); break;
    case 7: launch_q<7>(A, n, parametrix, self, st, lds_limit); break;
    case 8: launch_q<8>(A, n, parametrix, self, st, lds_limit); break;
    case 9: launch_q<9>(A, n, parametrix, self, st, lds_limit); break;
    case 10: launch_q<10>(A, n, parametrix, self, st, lds_limit); break;
    case 11: launch_q<11>(A, n, parametrix, self, st, lds_limit); break;
    case 12: launch_q<12>(A, n, parametrix, self, st, lds_limit); break;
    case 13: launch_q<13>(A, n, parametrix, self, st, lds_limit); break;
    case 14: launch_q<14>(A, n, parametrix, self, st, lds_limit); break;
    case 15: launch_q<15>(A, n, parametrix, self, st, lds_limit); break;
    case 16: launch_q<16>(A, n, parametrix, self, st, lds_limit); break;
    default: PMX_REQUIRE(false, PMX_ERR_INVALID, "q must be in [2, 16]");
  }
}

}  // namespace

void build_near_weights(Ctx* ctx, const Geometry& g, const Coeff& co, NearLists& nl, const pmx_options& o,
                        bool parametrix, hipStream_t st) {
  const int q = g.q, q2 = q * q;
  PMX_REQUIRE(o.n_gl >= 2 && o.n_gl <= kNglMax, PMX_ERR_INVALID, "n_gl must be in [2, 16]");
  DBuf<double>& out = parametrix ? nl.D : nl.C;
  out.alloc(ctx, (size_t)nl.nnz * q2);
  DBuf<double>& out_im = parametrix ? nl.Di : nl.Ci;   // c > 0: the imaginary parts
  if (co.complex_) out_im.alloc(ctx, (size_t)nl.nnz * q2);
  // host tables: Gauss-Legendre rule of the local rules, Lagrange denominators
  std::vector<double> tn(q), tw(q), cinv(q), gt(o.n_gl), gw(o.n_gl);
  gauss_legendre_host(q, tn.data(), tw.data());
  gauss_legendre_host(o.n_gl, gt.data(), gw.data());
  for (int j = 0; j < q; ++j) {
    double d = 1.0;
    for (int k = 0; k < q; ++k)
      if (k != j) d *= (tn[j] - tn[k]);
    cinv[j] = 1.0 / d;
  }
  DBuf<double> tab;
  tab.alloc(ctx, 2 * q + 2 * o.n_gl);
  std::vector<double> h(2 * q + 2 * o.n_gl);
  for (int j = 0; j < q; ++j) { h[j] = tn[j]; h[q + j] = cinv[j]; }
  for (int j = 0; j < o.n_gl; ++j) { h[2 * q + j] = gt[j]; h[2 * q + o.n_gl + j] = gw[j]; }
  PMX_HIP(hipMemcpyAsync(tab.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
  DBuf<int> err;
  err.alloc(ctx, 1);
  PMX_HIP(hipMemsetAsync(err.p, 0, sizeof(int), st));
  NWArgs A;
  A.N = g.N; A.q = q; A.n_gl = o.n_gl; A.eta = o.eta_near;
  const int nf = co.has_c() ? 11 : 10;
  DBuf<double> xp;
  xp.alloc(ctx, (size_t)g.N * nf);
  hipLaunchKernelGGL(k_interleave, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0, st, (int64_t)g.N, g.x.p,
                     g.xu_p.p, g.xv_p.p, co.a.p, co.c.p, nf, xp.p);
  PMX_HIP(hipGetLastError());
  A.X = g.x.p; A.XP = xp.p; A.a = co.a.p; A.c = co.c.p; A.w = g.w.p;
  A.tgt = co.tgt.p; A.tg = co.tg.p;
  A.tn = tab.p; A.cinv = tab.p + q; A.gl_t = tab.p + 2 * q; A.gl_w = tab.p + 2 * q + o.n_gl;
  A.ptr = nl.ptr.p; A.pair_patch = nl.patch.p; A.pair_target = nl.target.p; A.err = err.p;
  A.cpos = co.complex_ ? 1 : 0;
  int dev = 0;
  PMX_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  PMX_HIP(hipGetDeviceProperties(&prop, dev));
  const int64_t chunk = 1 << 20;
  for (int part = 0; part < (co.complex_ ? 2 : 1); ++part) {   // c > 0: real parts, then imaginary
    A.imag = part;
    A.out = part ? out_im.p : out.p;
    for (int64_t p0 = 0; p0 < g.N; p0 += chunk) {   // self pairs, one per target
      A.pair0 = p0;
      const int64_t n = g.N - p0 < chunk ? g.N - p0 : chunk;
      launch_dispatch(q, A, n, parametrix, true, st, prop.sharedMemPerBlock);
    }
    for (int64_t p0 = 0; p0 < nl.nnz; p0 += chunk) {   // the other near pairs
      A.pair0 = p0;
      const int64_t n = nl.nnz - p0 < chunk ? nl.nnz - p0 : chunk;
      launch_dispatch(q, A, n, parametrix, false, st, prop.sharedMemPerBlock);
    }
  }
  int herr = 0;
  PMX_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  PMX_REQUIRE(herr == 0, PMX_ERR_INVALID, "local quadrature needs more cells than supported (surface too distorted)");
  if (parametrix) nl.have_D = true;
}

}  // namespace pmx
