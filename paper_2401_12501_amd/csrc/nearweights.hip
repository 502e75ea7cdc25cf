// Correction blocks of the self and near rules (FP64).
//
// For a target node i and a patch P in near(i):
//   W_{i,P,j} = int_[-1,1]^2 F(x_i, y~(u,v)) l_j(u,v) J~(u,v) du dv,
//   C_{i,P,j} = W_{i,P,j} - [j != i] w_j F(x_i, x_j),
// where y~, x~_u, x~_v and a~ are tensor Lagrange interpolants of the patch's node
// data (the paper interpolates sigma to the quadrature grid, Section 6.1.1 Remark
// and Section 6.1.2), J~ = |x~_u x x~_v| and F is the remainder R or the
// parametrix K.
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
// Layout: one workgroup per (target, patch) pair.  Quadrature points are taken in
// batches of one point per thread; each thread evaluates its point's Lagrange
// values, interpolated geometry and kernel, writes (l_a(u), l_b(v), c) to LDS, and
// the q*q block entries are then accumulated in a fixed order.
#include <cmath>

#include "pmx_internal.hpp"

namespace pmx {

namespace {

constexpr int kThreads = 256;
constexpr int kLS = kThreads + 1;   // LDS row stride (odd: rows fall in different banks)
constexpr int kMaxCells = 256;   // panels (self) or leaves (near) per pair
constexpr int kMaxDepth = 20;
constexpr int kNglMax = 16;

struct NWArgs {
  int64_t N;
  int q;
  int n_gl;
  double eta;
  const double* X;      // 3N SoA
  const double* XU;     // 3N
  const double* XV;     // 3N
  const double* a;      // N
  const double* w;      // N
  const double* tgt;    // 8N: x y z nx ny nz A B
  const double* tg;     // 3N: grad_G a / (2 pi)
  const double* tn;     // q nodes
  const double* cinv;   // q: 1 / prod_{k != j} (t_j - t_k)
  const double* gl_t;   // n_gl Gauss-Legendre nodes on [-1, 1]
  const double* gl_w;   // n_gl weights
  const int32_t* pair_patch;
  const int32_t* pair_target;
  double* out;          // nnz * q*q
  int* err;
  int64_t pair0;
};

// Lagrange values of the q nodes at s: l_j(s) = cinv_j prod_{k != j} (s - t_k),
// from prefix and suffix products (no division by s - t_j).
__device__ inline void lagrange_dev(int q, const double* tn, const double* cinv, double s, double* out,
                                    int stride) {
  double pre = 1.0;
  for (int j = 0; j < q; ++j) {
    out[j * stride] = pre;
    pre *= (s - tn[j]);
  }
  double suf = 1.0;
  for (int j = q - 1; j >= 0; --j) {
    out[j * stride] *= suf * cinv[j];
    suf *= (s - tn[j]);
  }
}

// Tensor interpolation of the patch fields at one point, with l_a(u) in Lu and
// l_b(v) in Lv (LDS rows of this thread, stride kThreads).
struct PointGeo {
  double y[3], yu[3], yv[3], as;
};

__device__ inline void interp_point(const NWArgs& A, int64_t base, const double* Lu, const double* Lv,
                                    PointGeo& pg) {
  const int q = A.q;
  const int64_t N = A.N;
  double acc[10];
  for (int f = 0; f < 10; ++f) acc[f] = 0.0;
  for (int aa = 0; aa < q; ++aa) {
    double t[10];
    for (int f = 0; f < 10; ++f) t[f] = 0.0;
    const int64_t row = base + (int64_t)aa * q;
    for (int b = 0; b < q; ++b) {
      const double lv = Lv[b * kLS];
      const int64_t j = row + b;
      t[0] = fma(lv, A.X[j], t[0]);
      t[1] = fma(lv, A.X[N + j], t[1]);
      t[2] = fma(lv, A.X[2 * N + j], t[2]);
      t[3] = fma(lv, A.XU[j], t[3]);
      t[4] = fma(lv, A.XU[N + j], t[4]);
      t[5] = fma(lv, A.XU[2 * N + j], t[5]);
      t[6] = fma(lv, A.XV[j], t[6]);
      t[7] = fma(lv, A.XV[N + j], t[7]);
      t[8] = fma(lv, A.XV[2 * N + j], t[8]);
      t[9] = fma(lv, A.a[j], t[9]);
    }
    const double lu = Lu[aa * kLS];
    for (int f = 0; f < 10; ++f) acc[f] = fma(lu, t[f], acc[f]);
  }
  pg.y[0] = acc[0]; pg.y[1] = acc[1]; pg.y[2] = acc[2];
  pg.yu[0] = acc[3]; pg.yu[1] = acc[4]; pg.yu[2] = acc[5];
  pg.yv[0] = acc[6]; pg.yv[1] = acc[7]; pg.yv[2] = acc[8];
  pg.as = acc[9];
}

struct Target {
  double x[3], n[3], A, B, g[3];
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
  return 0.5 * log(rr) * 0.15915494309189533577 * inv_as;
}

struct Cell {   // self: panel on edge k [phi0, phi1]; near: leaf (depth, iu, iv)
  double p0, p1;
  int k;
  int iu, iv;
};

}  // namespace

// KERNEL: 0 = remainder R (correction blocks C), 1 = parametrix K (blocks D).
template <int KERNEL>
__global__ void __launch_bounds__(kThreads) k_near_weights(NWArgs A) {
  extern __shared__ double lds[];
  const int q = A.q, q2 = q * q;
  const int tid = threadIdx.x;
  // LDS layout: Lu[q][kLS], Lv[q][kLS], c[kThreads], W[q2]
  double* Lu = lds;
  double* Lv = Lu + q * kLS;
  double* cw = Lv + q * kLS;
  double* W = cw + kThreads;
  __shared__ Cell cells[kMaxCells];
  __shared__ int n_cells;
  __shared__ int2 front[2][kMaxCells];  // near: sub-square (iu, iv) at the current depth
  __shared__ int n_front[2];
  __shared__ int flag_split[kThreads];

  const int64_t pair = A.pair0 + blockIdx.x;
  const int P = A.pair_patch[pair];
  const int64_t i = A.pair_target[pair];
  const int64_t N = A.N;
  const int64_t base = (int64_t)P * q2;
  const bool self = (i / q2) == P;

  Target T;
  for (int c = 0; c < 3; ++c) {
    T.x[c] = A.tgt[c * N + i];
    T.n[c] = A.tgt[(3 + c) * N + i];
    T.g[c] = A.tg[c * N + i];
  }
  T.A = A.tgt[6 * N + i];
  T.B = A.tgt[7 * N + i];

  const int ngl = A.n_gl;
  // near-rule layout (tensor leaves): Xp[10][q2] T[10][q][16] Lu16[16][q] Lv16[16][q] c[256] T2[16][q] Wn[q2]
  double* Xp = lds;
  double* Tm = Xp + 10 * q2;
  double* Lu16 = Tm + 10 * q * kNglMax;
  double* Lv16 = Lu16 + kNglMax * q;
  double* cw2 = Lv16 + kNglMax * q;
  double* T2 = cw2 + kThreads;
  double* Wn = T2 + kNglMax * q;
  double* Wacc = self ? W : Wn;
  for (int e = tid; e < q2; e += kThreads) Wacc[e] = 0.0;

  // ------------------------------------------------------------------ cells
  double u0 = 0.0, v0 = 0.0;
  if (self) {
    const int loc = (int)(i - base);
    u0 = A.tn[loc / q];
    v0 = A.tn[loc % q];
    if (tid == 0) {
      int nc = 0;
      const double PI = 3.14159265358979323846;
      const double thn[4] = {-PI / 2, 0.0, PI / 2, PI};
      const double dd[4] = {v0 + 1.0, 1.0 - u0, 1.0 - v0, u0 + 1.0};
      const double cu[4] = {-1.0, 1.0, 1.0, -1.0};
      const double cv[4] = {-1.0, -1.0, 1.0, 1.0};
      for (int k = 0; k < 4; ++k) {
        const double tx = -sin(thn[k]), ty = cos(thn[k]);
        const int k1 = (k + 1) & 3;
        const double sa = (cu[k] - u0) * tx + (cv[k] - v0) * ty;
        const double sb = (cu[k1] - u0) * tx + (cv[k1] - v0) * ty;
        const double pa = atan2(sa, dd[k]), pb = atan2(sb, dd[k]);
        // positive side [0, pb], then negative side [pa, 0]
        for (int side = 0; side < 2; ++side) {
          const double end = side == 0 ? pb : -pa;
          double prev = 0.0;
          for (int m = 1;; ++m) {
            const double b = acos(ldexp(1.0, -m));
            const bool last = !(b < end);
            const double hi = last ? end : b;
            if (nc < kMaxCells) {
              Cell& C = cells[nc];
              C.k = k;
              C.p0 = side == 0 ? prev : -hi;
              C.p1 = side == 0 ? hi : -prev;
            }
            ++nc;
            prev = hi;
            if (last) break;
          }
        }
      }
      n_cells = nc;
    }
    __syncthreads();
  } else {
    // level-synchronous subdivision of [-1, 1]^2; a square at depth d is (iu, iv) * 2^(1-d) - 1
    if (tid == 0) {
      n_front[0] = 1;
      n_front[1] = 0;
      front[0][0] = make_int2(0, 0);
      n_cells = 0;
    }
    __syncthreads();
    int cur = 0;
    for (int depth = 0; depth <= kMaxDepth; ++depth) {
      const int nf = n_front[cur];
      if (nf == 0) break;
      for (int f0 = 0; f0 < nf; f0 += kThreads) {
        const int f = f0 + tid;
        int split = 0;
        if (f < nf) {
          const int iu = front[cur][f].x, iv = front[cur][f].y;
          const double h = 2.0 / (double)(1 << depth);
          const double ua = -1.0 + iu * h, va = -1.0 + iv * h;
          const double cuu[4] = {ua, ua + h, ua + h, ua};
          const double cvv[4] = {va, va, va + h, va + h};
          double cx[4][3];
          for (int k = 0; k < 4; ++k) {
            double lu[kNglMax], lv[kNglMax];
            lagrange_dev(q, A.tn, A.cinv, cuu[k], lu, 1);
            lagrange_dev(q, A.tn, A.cinv, cvv[k], lv, 1);
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int aa = 0; aa < q; ++aa) {
              double t0 = 0.0, t1 = 0.0, t2 = 0.0;
              for (int b = 0; b < q; ++b) {
                const int64_t j = base + aa * q + b;
                t0 = fma(lv[b], A.X[j], t0);
                t1 = fma(lv[b], A.X[N + j], t1);
                t2 = fma(lv[b], A.X[2 * N + j], t2);
              }
              s0 = fma(lu[aa], t0, s0);
              s1 = fma(lu[aa], t1, s1);
              s2 = fma(lu[aa], t2, s2);
            }
            cx[k][0] = s0; cx[k][1] = s1; cx[k][2] = s2;
          }
          double m[3];
          for (int c = 0; c < 3; ++c) m[c] = 0.25 * (cx[0][c] + cx[1][c] + cx[2][c] + cx[3][c]);
          double rad = 0.0;
          for (int k = 0; k < 4; ++k) {
            const double d0 = cx[k][0] - m[0], d1 = cx[k][1] - m[1], d2 = cx[k][2] - m[2];
            rad = fmax(rad, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
          }
          const double e0 = T.x[0] - m[0], e1 = T.x[1] - m[1], e2 = T.x[2] - m[2];
          const double dist = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
          split = (dist < A.eta * rad && depth < kMaxDepth) ? 1 : 0;
        }
        flag_split[tid] = split;
        __syncthreads();
        if (tid == 0) {
          const int nxt = cur ^ 1;
          const int lim = nf - f0 < kThreads ? nf - f0 : kThreads;
          for (int t = 0; t < lim; ++t) {
            const int iu = front[cur][f0 + t].x, iv = front[cur][f0 + t].y;
            if (flag_split[t]) {
              const int cu2[4] = {2 * iu, 2 * iu + 1, 2 * iu, 2 * iu + 1};
              const int cv2[4] = {2 * iv, 2 * iv, 2 * iv + 1, 2 * iv + 1};
              for (int c = 0; c < 4; ++c) {
                if (n_front[nxt] < kMaxCells) front[nxt][n_front[nxt]] = make_int2(cu2[c], cv2[c]);
                n_front[nxt]++;
              }
            } else {
              if (n_cells < kMaxCells) {
                Cell& C = cells[n_cells];
                C.k = depth;
                C.iu = iu;
                C.iv = iv;
              }
              n_cells++;
            }
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

  // ------------------------------------------------------------------ quadrature points
  const int n_rad = (self && KERNEL == 1) ? 4 * ngl : ngl;
  const int64_t pts_per_cell = self ? (int64_t)ngl * n_rad : (int64_t)ngl * ngl;
  const int64_t n_pts = self ? pts_per_cell * nc : 0;   // near leaves use the tensor path below
  for (int64_t p0 = 0; p0 < n_pts; p0 += kThreads) {
    const int64_t p = p0 + tid;
    double c = 0.0;
    if (p < n_pts) {
      const int cell = (int)(p / pts_per_cell);
      const int r = (int)(p - (int64_t)cell * pts_per_cell);
      const Cell C = cells[cell];
      double u, v, wq;
      if (self) {
        const int ia = r / n_rad, ir = r - ia * n_rad;
        const double PI = 3.14159265358979323846;
        const double thn = (C.k == 0) ? -PI / 2 : (C.k == 1 ? 0.0 : (C.k == 2 ? PI / 2 : PI));
        const double dk = (C.k == 0) ? v0 + 1.0 : (C.k == 1 ? 1.0 - u0 : (C.k == 2 ? 1.0 - v0 : u0 + 1.0));
        const double mid = 0.5 * (C.p0 + C.p1), half = 0.5 * (C.p1 - C.p0);
        const double phi = mid + half * A.gl_t[ia];
        const double L = dk / cos(phi);
        // radial node s in (0, 1] and weight for int_0^L F rho drho = L^2 sum w F(L s)
        double s, wr;
        const int pr = ir / ngl, jr = ir - pr * ngl;
        const double t = 0.5 * (A.gl_t[jr] + 1.0), wt = 0.5 * A.gl_w[jr];
        if (KERNEL == 0 || pr < 3) {
          const double lo = KERNEL == 0 ? 0.0 : ldexp(1.0, -(pr + 1));
          const double hi = KERNEL == 0 ? 1.0 : ldexp(1.0, -pr);
          s = lo + (hi - lo) * t;
          wr = (hi - lo) * wt * s;
        } else {
          s = t * t * t * 0.125;
          wr = wt * 3.0 * t * t * t * t * t / 64.0;
        }
        wq = half * A.gl_w[ia] * L * L * wr;
        const double ang = thn + phi;
        u = u0 + L * s * cos(ang);
        v = v0 + L * s * sin(ang);
      } else {
        const int ia = r / ngl, ib = r - ia * ngl;
        const double h = 2.0 / (double)(1 << C.k);
        const double ua = -1.0 + C.iu * h, va = -1.0 + C.iv * h;
        const double hh = 0.5 * h;
        u = ua + hh * (A.gl_t[ia] + 1.0);
        v = va + hh * (A.gl_t[ib] + 1.0);
        wq = A.gl_w[ia] * A.gl_w[ib] * hh * hh;
      }
      lagrange_dev(q, A.tn, A.cinv, u, Lu + tid, kLS);
      lagrange_dev(q, A.tn, A.cinv, v, Lv + tid, kLS);
      PointGeo pg;
      interp_point(A, base, Lu + tid, Lv + tid, pg);
      const double c0 = pg.yu[1] * pg.yv[2] - pg.yu[2] * pg.yv[1];
      const double c1 = pg.yu[2] * pg.yv[0] - pg.yu[0] * pg.yv[2];
      const double c2 = pg.yu[0] * pg.yv[1] - pg.yu[1] * pg.yv[0];
      const double Jt = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
      const double inv_as = 1.0 / pg.as;
      const double F = KERNEL == 0 ? remainder_dev(T, pg.y, inv_as) : parametrix_dev(T, pg.y, inv_as);
      c = wq * F * Jt;
    } else {
      for (int aa = 0; aa < q; ++aa) {
        Lu[aa * kLS + tid] = 0.0;
        Lv[aa * kLS + tid] = 0.0;
      }
    }
    cw[tid] = c;
    __syncthreads();
    const int lim = (n_pts - p0) < kThreads ? (int)(n_pts - p0) : kThreads;
    for (int e = tid; e < q2; e += kThreads) {
      const int aa = e / q, b = e - aa * q;
      double acc = 0.0;
      for (int t = 0; t < lim; ++t) acc = fma(cw[t] * Lu[aa * kLS + t], Lv[b * kLS + t], acc);
      W[e] += acc;
    }
    __syncthreads();
  }


  // ------------------------------------------------------------------ near rule: tensor leaves
  // For a leaf with nodes u_i, v_k (i, k < n_gl): field values are Lu (X Lv^T) and the block
  // update is W += Lu^T diag(c) Lv, both as small contractions through LDS.
  if (!self && nc > 0) {
    const int64_t N = A.N;
    for (int e = tid; e < 10 * q2; e += kThreads) {
      const int f = e / q2, j = e - f * q2;
      const int64_t g = base + j;
      const double* src = f < 3 ? A.X + f * N : (f < 6 ? A.XU + (f - 3) * N : (f < 9 ? A.XV + (f - 6) * N : A.a));
      Xp[e] = src[g];
    }
    const int npt = ngl * ngl;
    for (int cell = 0; cell < nc; ++cell) {
      const Cell C = cells[cell];
      const double h = 2.0 / (double)(1 << C.k);
      const double ua = -1.0 + C.iu * h, va = -1.0 + C.iv * h;
      const double hh = 0.5 * h;
      __syncthreads();
      if (tid < ngl) lagrange_dev(q, A.tn, A.cinv, ua + hh * (A.gl_t[tid] + 1.0), Lu16 + tid * q, 1);
      else if (tid < 2 * ngl) lagrange_dev(q, A.tn, A.cinv, va + hh * (A.gl_t[tid - ngl] + 1.0), Lv16 + (tid - ngl) * q, 1);
      __syncthreads();
      // T[f][a][k] = sum_b X[f][a][b] Lv[k][b]
      for (int e = tid; e < 10 * q * ngl; e += kThreads) {
        const int f = e / (q * ngl), r = e - f * q * ngl, aa = r / ngl, k = r - aa * ngl;
        const double* xr = Xp + f * q2 + aa * q;
        const double* lv = Lv16 + k * q;
        double acc = 0.0;
        for (int b = 0; b < q; ++b) acc = fma(xr[b], lv[b], acc);
        Tm[(f * q + aa) * kNglMax + k] = acc;
      }
      __syncthreads();
      double c = 0.0;
      if (tid < npt) {
        const int i = tid / ngl, k = tid - i * ngl;
        double g[10];
        for (int f = 0; f < 10; ++f) {
          double acc = 0.0;
          for (int aa = 0; aa < q; ++aa) acc = fma(Lu16[i * q + aa], Tm[(f * q + aa) * kNglMax + k], acc);
          g[f] = acc;
        }
        const double c0 = g[4] * g[8] - g[5] * g[7];
        const double c1 = g[5] * g[6] - g[3] * g[8];
        const double c2 = g[3] * g[7] - g[4] * g[6];
        const double Jt = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        const double inv_as = 1.0 / g[9];
        const double F = KERNEL == 0 ? remainder_dev(T, g, inv_as) : parametrix_dev(T, g, inv_as);
        c = A.gl_w[i] * A.gl_w[k] * hh * hh * F * Jt;
      }
      cw2[tid] = c;
      __syncthreads();
      // T2[i][b] = sum_k c[i][k] Lv[k][b]
      for (int e = tid; e < ngl * q; e += kThreads) {
        const int i = e / q, b = e - i * q;
        double acc = 0.0;
        for (int k = 0; k < ngl; ++k) acc = fma(cw2[i * ngl + k], Lv16[k * q + b], acc);
        T2[i * q + b] = acc;
      }
      __syncthreads();
      // W[a][b] += sum_i Lu[i][a] T2[i][b]
      for (int e = tid; e < q2; e += kThreads) {
        const int aa = e / q, b = e - aa * q;
        double acc = 0.0;
        for (int i = 0; i < ngl; ++i) acc = fma(Lu16[i * q + aa], T2[i * q + b], acc);
        Wn[e] += acc;
      }
    }
    __syncthreads();
  }

  // ------------------------------------------------------------------ subtract the smooth rule
  for (int e = tid; e < q2; e += kThreads) {
    const int64_t j = base + e;
    double val = Wacc[e];
    if (j != i) {
      const double y[3] = {A.X[j], A.X[N + j], A.X[2 * N + j]};
      const double inv_a = 1.0 / A.a[j];
      const double F = KERNEL == 0 ? remainder_dev(T, y, inv_a) : parametrix_dev(T, y, inv_a);
      val -= A.w[j] * F;
    }
    A.out[pair * q2 + e] = val;
  }
}

void build_near_weights(Ctx* ctx, const Geometry& g, const Coeff& co, NearLists& nl, const pmx_options& o,
                        bool parametrix, hipStream_t st) {
  const int q = g.q, q2 = q * q;
  PMX_REQUIRE(o.n_gl >= 2 && o.n_gl <= kNglMax, PMX_ERR_INVALID, "n_gl must be in [2, 16]");
  DBuf<double>& out = parametrix ? nl.D : nl.C;
  out.alloc(ctx, (size_t)nl.nnz * q2);
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
  A.X = g.x.p; A.XU = g.xu_p.p; A.XV = g.xv_p.p; A.a = co.a.p; A.w = g.w.p;
  A.tgt = co.tgt.p; A.tg = co.tg.p;
  A.tn = tab.p; A.cinv = tab.p + q; A.gl_t = tab.p + 2 * q; A.gl_w = tab.p + 2 * q + o.n_gl;
  A.pair_patch = nl.patch.p; A.pair_target = nl.target.p; A.out = out.p; A.err = err.p;
  const size_t lds_self = (size_t)(2 * q * kLS + kThreads + q2) * sizeof(double);
  const size_t lds_near = (size_t)(11 * q2 + 10 * q * kNglMax + 3 * kNglMax * q + kThreads) * sizeof(double);
  const size_t lds = lds_self > lds_near ? lds_self : lds_near;
  int dev = 0;
  PMX_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  PMX_HIP(hipGetDeviceProperties(&prop, dev));
  PMX_REQUIRE(lds + 12 * 1024 <= prop.sharedMemPerBlock, PMX_ERR_INVALID,
              "q too large for the local-rule kernel's LDS on this device");
  const int64_t chunk = 1 << 20;
  for (int64_t p0 = 0; p0 < nl.nnz; p0 += chunk) {
    A.pair0 = p0;
    const int64_t n = nl.nnz - p0 < chunk ? nl.nnz - p0 : chunk;
    if (parametrix)
      hipLaunchKernelGGL(k_near_weights<1>, dim3(n), dim3(kThreads), lds, st, A);
    else
      hipLaunchKernelGGL(k_near_weights<0>, dim3(n), dim3(kThreads), lds, st, A);
    PMX_HIP(hipGetLastError());
  }
  int herr = 0;
  PMX_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  PMX_REQUIRE(herr == 0, PMX_ERR_INVALID, "local quadrature needs more cells than supported (surface too distorted)");
  if (parametrix) nl.have_D = true;
}

}  // namespace pmx
