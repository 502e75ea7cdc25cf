// Direct far-field sums over all source nodes (smooth rule, Section 6.1.3).
//
//   phi_i = sum_{j != i} w_j R(x_i, x_j) sigma_j
//         = sum_j qt_j (1/r^2) [ (n'_i . r)^2 / r^2 + h_i . r ],   r = x_i - x_j,
//   qt_j = w_j sigma_j / a_j,  n' = sqrt(A) n,  h = g - B n,
// the c = 0 remainder of eq:explicit_remainder with G = log(r) / (2 pi a(x'))
// written with the target factors A = a/pi, B = a H/pi, g = grad_G a / (2 pi).
//
// Each thread owns one (or two) targets and walks a contiguous chunk of sources.
// Before the sum, the sources of a group of NR right-hand sides are packed into
// rows (x, y, z, qt_1 .. qt_NR, padding): one row is the same for every lane of a
// wavefront, so it is read with one or two wide loads through the scalar data
// cache and lives in scalar registers, and consecutive sources share cache lines.
// The pair kernel is evaluated once per pair for all NR densities.  The pair
// j = i is removed without a branch: r^2 gets a tiny epsilon, so the self pair has
// 1/r^2 finite while n.r = h.r = 0 make its contribution exactly zero.  Partial
// sums per source chunk go to part[chunk][rhs][i] and are added in a fixed order
// afterwards (deterministic).
#include "pmx_internal.hpp"

namespace pmx {

namespace {
constexpr int kBlock = 256;

// Pointers whose uniform-address loads go through the scalar cache.
typedef const __attribute__((address_space(4))) double* sdp;
typedef const __attribute__((address_space(4))) float* sfp;

__device__ __forceinline__ double rcp64(double x) {
  // hardware reciprocal (about 24 correct bits), then one Newton step: 2e-15 relative
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Row length of a packed source row: x, y, z, NR densities, padded to 16 bytes.
template <int NR, typename T>
constexpr int row_len() { return sizeof(T) == 8 ? ((3 + NR + 1) / 2) * 2 : ((3 + NR + 3) / 4) * 4; }
}  // namespace

// rows[j] = (x_j, y_j, z_j, q_{r0}[j], ..., q_{r0+NR-1}[j], 0...)
template <typename T>
struct PackArgs {
  int64_t N;
  const T* X;        // 3N SoA coordinates
  const T* q;        // densities of the group's first right-hand side
  int64_t ldq;
  T* rows;
};

template <int NR, typename T>
__global__ void __launch_bounds__(kBlock) k_pack_sources(Group<PackArgs<T>> g) {
  constexpr int RL = row_len<NR, T>();
  int64_t lb;
  const PackArgs<T>& A = seg_of(g, blockIdx.x, lb);
  const int64_t N = A.N;
  const int64_t j = lb * kBlock + threadIdx.x;
  if (j >= N) return;
  T v[RL];
  v[0] = A.X[j];
  v[1] = A.X[N + j];
  v[2] = A.X[2 * N + j];
#pragma unroll
  for (int r = 0; r < NR; ++r) v[3 + r] = A.q[r * A.ldq + j];
#pragma unroll
  for (int c = 3 + NR; c < RL; ++c) v[c] = T(0);
#pragma unroll
  for (int c = 0; c < RL; ++c) A.rows[j * RL + c] = v[c];
}

// TPL targets per lane (targets i0 and i0 + kBlock of a TPL*kBlock target tile): one
// source row feeds TPL pair evaluations.  Grid: nbx target tiles x nc source chunks.
struct Direct64Args {
  int64_t N, chunk, nbx, ldp, ldc;
  const double* tf;    // 9N target factors
  const double* rows;  // packed sources
  double* part;        // part[chunk][rhs][i]
};

template <int NR, int TPL>
__global__ void __launch_bounds__(kBlock) k_direct64(Group<Direct64Args> g) {
  constexpr int RL = row_len<NR, double>();
  int64_t lb;
  const Direct64Args& A = seg_of(g, blockIdx.x, lb);
  const int64_t N = A.N;
  const int64_t by = lb / A.nbx, bx = lb - by * A.nbx;
  const int64_t j0 = by * A.chunk;
  const int64_t j1 = j0 + A.chunk < N ? j0 + A.chunk : N;
  const double* __restrict__ tf = A.tf;
  double xi[TPL], yi[TPL], zi[TPL], px[TPL], py[TPL], pz[TPL], hx[TPL], hy[TPL], hz[TPL];
  int64_t it[TPL];
#pragma unroll
  for (int t = 0; t < TPL; ++t) {
    it[t] = bx * kBlock * TPL + t * kBlock + threadIdx.x;
    const int64_t i = it[t] < N ? it[t] : N - 1;
    xi[t] = tf[i]; yi[t] = tf[N + i]; zi[t] = tf[2 * N + i];
    px[t] = tf[3 * N + i]; py[t] = tf[4 * N + i]; pz[t] = tf[5 * N + i];
    hx[t] = tf[6 * N + i]; hy[t] = tf[7 * N + i]; hz[t] = tf[8 * N + i];
  }
  const sdp S = (sdp)A.rows;
  double acc[TPL][NR];
#pragma unroll
  for (int t = 0; t < TPL; ++t)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[t][r] = 0.0;
  // several sources per step: independent pair chains for the scheduler (measured best)
#pragma unroll(NR == 1 ? 8 : 4)
  for (int64_t j = j0; j < j1; ++j) {
    const sdp row = S + j * RL;
    const double xs = row[0], ys = row[1], zs = row[2];
#pragma unroll
    for (int t = 0; t < TPL; ++t) {
      const double dx = xi[t] - xs, dy = yi[t] - ys, dz = zi[t] - zs;
      const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-300)));
      const double inv = rcp64(r2);
      const double pr = fma(px[t], dx, fma(py[t], dy, pz[t] * dz));
      const double hr = fma(hx[t], dx, fma(hy[t], dy, hz[t] * dz));
      const double v = fma(pr * inv, pr, hr) * inv;
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[t][r] = fma(row[3 + r], v, acc[t][r]);
    }
  }
#pragma unroll
  for (int t = 0; t < TPL; ++t)
    if (it[t] < N) {
#pragma unroll
      for (int r = 0; r < NR; ++r) A.part[by * A.ldc + r * A.ldp + it[t]] = acc[t][r];
    }
}

template <int NR>
__global__ void __launch_bounds__(kBlock) k_direct32(int64_t N, const float* __restrict__ t32,
                                                     const float* __restrict__ rows, int64_t chunk,
                                                     double* __restrict__ part, int64_t ldp, int64_t ldc) {
  constexpr int RL = row_len<NR, float>();
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < N ? i0 : N - 1;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  const float xi = t32[i], yi = t32[N + i], zi = t32[2 * N + i];
  const float px = t32[3 * N + i], py = t32[4 * N + i], pz = t32[5 * N + i];
  const float hx = t32[6 * N + i], hy = t32[7 * N + i], hz = t32[8 * N + i];
  const sfp S = (sfp)rows;
  float acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0f;
#pragma unroll(NR <= 4 ? 4 : 1)
  for (int64_t j = j0; j < j1; ++j) {
    const sfp row = S + j * RL;
    const float dx = xi - row[0], dy = yi - row[1], dz = zi - row[2];
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, 1e-30f)));
    const float inv = __builtin_amdgcn_rcpf(r2);
    const float pr = fmaf(px, dx, fmaf(py, dy, pz * dz));
    const float hr = fmaf(hx, dx, fmaf(hy, dy, hz * dz));
    const float v = fmaf(pr * inv, pr, hr) * inv;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = fmaf(row[3 + r], v, acc[r]);
  }
  if (i0 < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) part[(int64_t)blockIdx.y * ldc + r * ldp + i0] = (double)acc[r];
  }
}

// Representation far field: u_i = sum_{j != i} qt_j log(r_ij) / (2 pi), qt = w sigma / a.
template <int NR>
__global__ void __launch_bounds__(kBlock) k_direct_log(int64_t N, const double* __restrict__ X,
                                                       const double* __restrict__ rows, int64_t chunk,
                                                       double* __restrict__ part, int64_t ldp, int64_t ldc) {
  constexpr int RL = row_len<NR, double>();
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < N ? i0 : N - 1;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  const double xi = X[i], yi = X[N + i], zi = X[2 * N + i];
  const sdp S = (sdp)rows;
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
#pragma unroll 4
  for (int64_t j = j0; j < j1; ++j) {
    const sdp row = S + j * RL;
    const double dx = xi - row[0], dy = yi - row[1], dz = zi - row[2];
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    // log(r) / (2 pi) = log(r^2) / (4 pi).  The self pair (r2 = 0: zero mantissa) gives a finite
    // value that a zero factor drops; computing it keeps the loop free of branches
    const double v = log_pair(r2) * (j == i ? 0.0 : 0.07957747154594766788);
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = fma(row[3 + r], v, acc[r]);
  }
  if (i0 < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) part[(int64_t)blockIdx.y * ldc + r * ldp + i0] = acc[r];
  }
}

// c < 0 (the modified Helmholtz type).  Packed source rows (x, y, z, kappa, qt_1 .. qt_NR, pad),
// kappa = sqrt(-c / a) at the source.  With z = kappa r, k0, k1 = K0(z), K1(z):
//   w_j R(x_i, x_j) sigma_j = qt_j { kappa k1 [g.r/r + 2 at2 (n.r)^2/r^3 - B n.r/r]
//                                    + at2 kappa^2 k0 ((n.r)^2/r^2 - 1) - ct2 k0 },
// the eq:explicit_remainder terms with G = -K0(kappa r) / (2 pi a') (target factors g = grad_G
// a / (2 pi), at2 = a / (2 pi), B = a H / pi, ct2 = c / (2 pi)).  The self pair is removed by a
// zero factor (its argument is kept away from zero so that every value stays finite).
template <int NR>
constexpr int row_len_c() { return ((4 + NR + 1) / 2) * 2; }

struct PackCArgs {
  int64_t N;
  const double* X;       // 3N SoA
  const double* a;       // N
  const double* c;       // N
  const double* q;       // densities of the group's first right-hand side (qt = w sigma / a)
  int64_t ldq;
  double* rows;
};

template <int NR>
__global__ void __launch_bounds__(kBlock) k_pack_sources_c(PackCArgs A) {
  constexpr int RL = row_len_c<NR>();
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= A.N) return;
  const int64_t N = A.N;
  double v[RL];
  v[0] = A.X[j];
  v[1] = A.X[N + j];
  v[2] = A.X[2 * N + j];
  v[3] = sqrt(-A.c[j] / A.a[j]);
#pragma unroll
  for (int r = 0; r < NR; ++r) v[4 + r] = A.q[r * A.ldq + j];
#pragma unroll
  for (int k = 4 + NR; k < RL; ++k) v[k] = 0.0;
#pragma unroll
  for (int k = 0; k < RL; ++k) A.rows[j * RL + k] = v[k];
}

struct DirectCArgs {
  int64_t N, chunk, ldp, ldc;
  const double* tgt;   // 8N: x y z n A B
  const double* tg;    // 3N: grad_G a / (2 pi)
  const double* c;     // N
  const double* rows;
  double* part;        // part[chunk][rhs][i]
  int kernel;          // 0: remainder, 1: parametrix (representation)
};

template <int NR>
__global__ void __launch_bounds__(kBlock) k_direct64_c(DirectCArgs A) {
  constexpr int RL = row_len_c<NR>();
  const int64_t N = A.N;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < N ? i0 : N - 1;
  const int64_t j0 = (int64_t)blockIdx.y * A.chunk;
  const int64_t j1 = j0 + A.chunk < N ? j0 + A.chunk : N;
  const double xi = A.tgt[i], yi = A.tgt[N + i], zi = A.tgt[2 * N + i];
  const double nx = A.tgt[3 * N + i], ny = A.tgt[4 * N + i], nz = A.tgt[5 * N + i];
  const double at2 = 0.5 * A.tgt[6 * N + i], B = A.tgt[7 * N + i];
  const double gx = A.tg[i], gy = A.tg[N + i], gz = A.tg[2 * N + i];
  const double ct2 = A.c[i] * 0.15915494309189533577;
  const sdp S = (sdp)A.rows;
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  // e = a' F(x_i, x_j) from K0, K1 at kappa r
  auto term = [&](double dx, double dy, double dz, double ir, double kap, double k0, double k1) {
    if (A.kernel == 0) {
      const double snr = (nx * dx + ny * dy + nz * dz) * ir;
      const double gr = gx * dx + gy * dy + gz * dz;
      const double bra = fma(ir, fma(2.0 * at2 * snr, snr, gr), -B * snr);
      return kap * k1 * bra + at2 * kap * kap * k0 * fma(snr, snr, -1.0) - ct2 * k0;
    }
    return -k0 * 0.15915494309189533577;
  };
  // sources two at a time, their Bessel functions sharing coefficients (bessel_k01_x2)
  int64_t j = j0;
  for (; j + 1 < j1; j += 2) {
    double d[2][3], ir[2], kap[2], z[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const sdp row = S + (j + m) * RL;
      d[m][0] = xi - row[0];
      d[m][1] = yi - row[1];
      d[m][2] = zi - row[2];
      const double rr = fma(d[m][0], d[m][0], fma(d[m][1], d[m][1], fma(d[m][2], d[m][2], 1e-300)));
      ir[m] = rsqrt(rr);
      kap[m] = row[3];
      z[m] = fmax(kap[m] * (rr * ir[m]), 1e-150);
    }
    double k0[2], k1[2];
    bessel_k01_x2(z, k0, k1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      double e = term(d[m][0], d[m][1], d[m][2], ir[m], kap[m], k0[m], k1[m]);
      e = j + m == i ? 0.0 : e;
      const sdp row = S + (j + m) * RL;
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = fma(row[4 + r], e, acc[r]);
    }
  }
  if (j < j1) {
    const sdp row = S + j * RL;
    const double dx = xi - row[0], dy = yi - row[1], dz = zi - row[2];
    const double rr = fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-300)));
    const double ir = rsqrt(rr);
    const double kap = row[3];
    double k0, k1;
    bessel_k01(fmax(kap * (rr * ir), 1e-150), k0, k1);
    double e = term(dx, dy, dz, ir, kap, k0, k1);
    e = j == i ? 0.0 : e;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = fma(row[4 + r], e, acc[r]);
  }
  if (i0 < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) A.part[(int64_t)blockIdx.y * A.ldc + r * A.ldp + i0] = acc[r];
  }
}

// c > 0 (the Helmholtz type): G = -(i / 4a') H0(k r), k = sqrt(c'/a'), is complex, and so are
// sigma and the sums.  A complex density is two real columns (real parts, then imaginary parts);
// packed source rows are (x, y, z, k, re qt_1, im qt_1, .., re qt_NP, im qt_NP).  With z = k r and
// J0, J1, Y0, Y1 at z, a' times the remainder is (i pi / 2) {k H1 bra - m H0} with bra as for c < 0
// and m = at2 k^2 ((n.r)^2/r^2 - 1) + ct2:
//   e = (pi/2) [(m Y0 - k Y1 bra) + i (k J1 bra - m J0)];
// a' times the parametrix is (Y0 - i J0) / 4.  Each pair adds e times the complex qt_j.
template <int NP>
constexpr int row_len_cz() { return 4 + 2 * NP; }

template <int NP>
__global__ void __launch_bounds__(kBlock) k_pack_sources_cz(PackCArgs A) {
  constexpr int RL = row_len_cz<NP>();
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= A.N) return;
  const int64_t N = A.N;
  double v[RL];
  v[0] = A.X[j];
  v[1] = A.X[N + j];
  v[2] = A.X[2 * N + j];
  v[3] = sqrt(A.c[j] / A.a[j]);
#pragma unroll
  for (int r = 0; r < 2 * NP; ++r) v[4 + r] = A.q[r * A.ldq + j];   // columns re_1, im_1, re_2, ..
#pragma unroll
  for (int k = 0; k < RL; ++k) A.rows[j * RL + k] = v[k];
}

// Target quantities of the complex direct sum.
struct CzTarget {
  double x, y, z, nx, ny, nz, at2, B, gx, gy, gz, ct2;
  int kernel;
};

// e = a' F(x_i, x_j) (real and imaginary parts) for one source, from J0, J1, Y0, Y1 at k r.
__device__ __forceinline__ void cz_term(const CzTarget& T, double dx, double dy, double dz, double ir, double k,
                                        double bj0, double bj1, double by0, double by1, double& er, double& ei) {
  if (T.kernel == 0) {
    const double snr = (T.nx * dx + T.ny * dy + T.nz * dz) * ir;
    const double gr = T.gx * dx + T.gy * dy + T.gz * dz;
    const double bra = fma(ir, fma(2.0 * T.at2 * snr, snr, gr), -T.B * snr);
    const double m = fma(T.at2 * k * k, fma(snr, snr, -1.0), T.ct2);
    er = 1.5707963267948966192 * fma(m, by0, -k * by1 * bra);
    ei = 1.5707963267948966192 * fma(k * bj1, bra, -m * bj0);
  } else {
    er = 0.25 * by0;
    ei = -0.25 * bj0;
  }
}

// Sources two at a time: the Bessel functions of the two pairs share their coefficients
// (bessel_jy01_x2); an odd chunk ends with one source.
template <int NP>
__global__ void __launch_bounds__(kBlock) k_direct64_cz(DirectCArgs A) {
  constexpr int RL = row_len_cz<NP>();
  const int64_t N = A.N;
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = i0 < N ? i0 : N - 1;
  const int64_t j0 = (int64_t)blockIdx.y * A.chunk;
  const int64_t j1 = j0 + A.chunk < N ? j0 + A.chunk : N;
  CzTarget T;
  T.x = A.tgt[i];
  T.y = A.tgt[N + i];
  T.z = A.tgt[2 * N + i];
  T.nx = A.tgt[3 * N + i];
  T.ny = A.tgt[4 * N + i];
  T.nz = A.tgt[5 * N + i];
  T.at2 = 0.5 * A.tgt[6 * N + i];
  T.B = A.tgt[7 * N + i];
  T.gx = A.tg[i];
  T.gy = A.tg[N + i];
  T.gz = A.tg[2 * N + i];
  T.ct2 = A.c[i] * 0.15915494309189533577;
  T.kernel = A.kernel;
  const sdp S = (sdp)A.rows;
  double ar[NP], ai[NP];
#pragma unroll
  for (int r = 0; r < NP; ++r) ar[r] = ai[r] = 0.0;
  auto accumulate = [&](const sdp row, double er, double ei) {
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      const double qr = row[4 + 2 * r], qi = row[5 + 2 * r];
      ar[r] = fma(qr, er, fma(-qi, ei, ar[r]));
      ai[r] = fma(qr, ei, fma(qi, er, ai[r]));
    }
  };
  int64_t j = j0;
  for (; j + 1 < j1; j += 2) {
    double d[2][3], ir[2], k[2], z[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const sdp row = S + (j + m) * RL;
      d[m][0] = T.x - row[0];
      d[m][1] = T.y - row[1];
      d[m][2] = T.z - row[2];
      const double rr = fma(d[m][0], d[m][0], fma(d[m][1], d[m][1], fma(d[m][2], d[m][2], 1e-300)));
      ir[m] = rsqrt(rr);
      k[m] = row[3];
      z[m] = fmax(k[m] * (rr * ir[m]), 1e-150);
    }
    double bj0[2], bj1[2], by0[2], by1[2];
    bessel_jy01_x2(z, bj0, bj1, by0, by1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      double er, ei;
      cz_term(T, d[m][0], d[m][1], d[m][2], ir[m], k[m], bj0[m], bj1[m], by0[m], by1[m], er, ei);
      er = j + m == i ? 0.0 : er;
      ei = j + m == i ? 0.0 : ei;
      accumulate(S + (j + m) * RL, er, ei);
    }
  }
  if (j < j1) {
    const sdp row = S + j * RL;
    const double dx = T.x - row[0], dy = T.y - row[1], dz = T.z - row[2];
    const double rr = fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-300)));
    const double ir = rsqrt(rr);
    const double k = row[3];
    double bj0, bj1, by0, by1;
    bessel_jy01(fmax(k * (rr * ir), 1e-150), bj0, bj1, by0, by1);
    double er, ei;
    cz_term(T, dx, dy, dz, ir, k, bj0, bj1, by0, by1, er, ei);
    er = j == i ? 0.0 : er;
    ei = j == i ? 0.0 : ei;
    accumulate(row, er, ei);
  }
  if (i0 < N) {
#pragma unroll
    for (int r = 0; r < NP; ++r) {
      A.part[(int64_t)blockIdx.y * A.ldc + (2 * r) * A.ldp + i0] = ar[r];
      A.part[(int64_t)blockIdx.y * A.ldc + (2 * r + 1) * A.ldp + i0] = ai[r];
    }
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

template <int NR, typename T>
void pack_launch(const std::vector<PackArgs<T>>& recs, hipStream_t st) {
  std::vector<int64_t> nb;
  for (const auto& r : recs) nb.push_back((r.N + kBlock - 1) / kBlock);
  launch_grouped(recs, nb, [&](const Group<PackArgs<T>>& g, int64_t nblk) {
    hipLaunchKernelGGL((k_pack_sources<NR, T>), dim3((unsigned)nblk), dim3(kBlock), 0, st, g);
    PMX_HIP(hipGetLastError());
  });
}

// FP64 remainder sums of one group of NR right-hand sides (from r0) for several operators.
// Caller scratch (ApplyScratch) replaces the operator's buffers where given.
template <int NR>
void direct64_group(const std::vector<pmx_operator*>& ops, const std::vector<const ApplyScratch*>& scs, int n_rhs,
                    int r0, hipStream_t st) {
  constexpr int RL = row_len<NR, double>();
  constexpr int TPL = 1;   // one target per lane: more waves in flight beat reuse of a source row
  std::vector<PackArgs<double>> pk;
  std::vector<Direct64Args> da;
  std::vector<int64_t> nb;
  for (size_t k = 0; k < ops.size(); ++k) {
    pmx_operator* op = ops[k];
    const ApplyScratch* sc = scs[k];
    const int64_t N = op->s->g.N;
    const int64_t nc = n_chunks_for(N);
    if (!sc && op->rows64.n < (size_t)N * RL) op->rows64.alloc(&op->s->ctx->c, (size_t)N * RL);
    double* rows = sc ? sc->rows : op->rows64.p;
    const double* qt = sc ? sc->qt64 : op->qt64.p;
    double* part = sc ? sc->part : op->part.p;
    pk.push_back({N, op->s->g.x.p, qt + (int64_t)r0 * N, N, rows});
    const int64_t nbx = (N + TPL * kBlock - 1) / (TPL * kBlock);
    da.push_back({N, (N + nc - 1) / nc, nbx, N, (int64_t)n_rhs * N, op->co.tf64.p, rows, part + (int64_t)r0 * N});
    nb.push_back(nbx * nc);
  }
  pack_launch<NR, double>(pk, st);
  launch_grouped(da, nb, [&](const Group<Direct64Args>& g, int64_t nblk) {
    hipLaunchKernelGGL((k_direct64<NR, TPL>), dim3((unsigned)nblk), dim3(kBlock), 0, st, g);
    PMX_HIP(hipGetLastError());
  });
}

// c < 0: one operator, right-hand-side groups of NR; kernel 0 remainder, 1 parametrix.
template <int NR>
void direct_c_group(pmx_operator* op, const ApplyScratch* sc, int kernel, int n_rhs, int r0, hipStream_t st) {
  constexpr int RL = row_len_c<NR>();
  const int64_t N = op->s->g.N;
  const int64_t nc = n_chunks_for(N);
  if (!sc && op->rows64.n < (size_t)N * RL) op->rows64.alloc(&op->s->ctx->c, (size_t)N * RL);
  double* rows = sc ? sc->rows : op->rows64.p;
  const double* qt = sc ? sc->qt64 : op->qt64.p;
  double* part = sc ? sc->part : op->part.p;
  const unsigned nbx = (unsigned)((N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pack_sources_c<NR>, dim3(nbx), dim3(kBlock), 0, st,
                     PackCArgs{N, op->s->g.x.p, op->co.a.p, op->co.c.p, qt + (int64_t)r0 * N, N, rows});
  PMX_HIP(hipGetLastError());
  const DirectCArgs da{N, (N + nc - 1) / nc, N, (int64_t)n_rhs * N, op->co.tgt.p, op->co.tg.p, op->co.c.p, rows,
                       part + (int64_t)r0 * N, kernel};
  hipLaunchKernelGGL(k_direct64_c<NR>, dim3(nbx, (unsigned)nc), dim3(kBlock), 0, st, da);
  PMX_HIP(hipGetLastError());
}

// c > 0: complex densities NP at a time (columns c0 .. c0 + 2 NP - 1 of the n_cols real columns).
template <int NP>
void direct_cz_group(pmx_operator* op, const ApplyScratch* sc, int kernel, int n_cols, int c0, hipStream_t st) {
  constexpr int RL = row_len_cz<NP>();
  const int64_t N = op->s->g.N;
  const int64_t nc = n_chunks_for(N);
  if (!sc && op->rows64.n < (size_t)N * RL) op->rows64.alloc(&op->s->ctx->c, (size_t)N * RL);
  double* rows = sc ? sc->rows : op->rows64.p;
  const double* qt = sc ? sc->qt64 : op->qt64.p;
  double* part = sc ? sc->part : op->part.p;
  const unsigned nbx = (unsigned)((N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_pack_sources_cz<NP>, dim3(nbx), dim3(kBlock), 0, st,
                     PackCArgs{N, op->s->g.x.p, op->co.a.p, op->co.c.p, qt + (int64_t)c0 * N, N, rows});
  PMX_HIP(hipGetLastError());
  const DirectCArgs da{N, (N + nc - 1) / nc, N, (int64_t)n_cols * N, op->co.tgt.p, op->co.tg.p, op->co.c.p, rows,
                       part + (int64_t)c0 * N, kernel};
  hipLaunchKernelGGL(k_direct64_cz<NP>, dim3(nbx, (unsigned)nc), dim3(kBlock), 0, st, da);
  PMX_HIP(hipGetLastError());
}

// n_rhs: real columns (for c > 0, twice the number of complex densities).
void direct_c_all(pmx_operator* op, const ApplyScratch* sc, int kernel, int n_rhs, hipStream_t st) {
  const int64_t N = op->s->g.N;
  const size_t need = (size_t)n_chunks_for(N) * n_rhs * N;
  if (!sc && op->part.n < need) op->part.alloc(&op->s->ctx->c, need);
  if (op->cplx()) {
    const int nv = n_rhs / 2;
    int v0 = 0;
    while (v0 < nv) {
      const int left = nv - v0;
      if (left >= 8) { direct_cz_group<8>(op, sc, kernel, n_rhs, 2 * v0, st); v0 += 8; }
      else if (left >= 4) { direct_cz_group<4>(op, sc, kernel, n_rhs, 2 * v0, st); v0 += 4; }
      else if (left >= 2) { direct_cz_group<2>(op, sc, kernel, n_rhs, 2 * v0, st); v0 += 2; }
      else { direct_cz_group<1>(op, sc, kernel, n_rhs, 2 * v0, st); v0 += 1; }
    }
    return;
  }
  int r0 = 0;
  while (r0 < n_rhs) {
    const int left = n_rhs - r0;
    if (left >= 16) { direct_c_group<16>(op, sc, kernel, n_rhs, r0, st); r0 += 16; }
    else if (left >= 8) { direct_c_group<8>(op, sc, kernel, n_rhs, r0, st); r0 += 8; }
    else if (left >= 4) { direct_c_group<4>(op, sc, kernel, n_rhs, r0, st); r0 += 4; }
    else if (left >= 2) { direct_c_group<2>(op, sc, kernel, n_rhs, r0, st); r0 += 2; }
    else { direct_c_group<1>(op, sc, kernel, n_rhs, r0, st); r0 += 1; }
  }
}

void direct64_all(const std::vector<pmx_operator*>& ops_in, const std::vector<const ApplyScratch*>& scs_in,
                  int n_rhs, hipStream_t st) {
  // operators with c != 0 take their own kernels, one operator at a time
  std::vector<pmx_operator*> ops;
  std::vector<const ApplyScratch*> scs;
  for (size_t k = 0; k < ops_in.size(); ++k) {
    if (ops_in[k]->co.has_c()) direct_c_all(ops_in[k], scs_in[k], 0, n_rhs, st);
    else {
      ops.push_back(ops_in[k]);
      scs.push_back(scs_in[k]);
    }
  }
  if (ops.empty()) return;
  for (size_t k = 0; k < ops.size(); ++k) {
    if (scs[k]) continue;
    pmx_operator* op = ops[k];
    const int64_t N = op->s->g.N;
    const size_t need = (size_t)n_chunks_for(N) * n_rhs * N;
    if (op->part.n < need) op->part.alloc(&op->s->ctx->c, need);
  }
  int r0 = 0;
  while (r0 < n_rhs) {
    const int left = n_rhs - r0;
    if (left >= 16) { direct64_group<16>(ops, scs, n_rhs, r0, st); r0 += 16; }
    else if (left >= 8) { direct64_group<8>(ops, scs, n_rhs, r0, st); r0 += 8; }
    else if (left >= 4) { direct64_group<4>(ops, scs, n_rhs, r0, st); r0 += 4; }
    else if (left >= 2) { direct64_group<2>(ops, scs, n_rhs, r0, st); r0 += 2; }
    else { direct64_group<1>(ops, scs, n_rhs, r0, st); r0 += 1; }
  }
}

// mode 1: FP32 remainder, 2: FP64 log kernel (single operator).
template <int NR>
void launch_group(pmx_operator* op, int mode, int n_rhs, int r0, int64_t nc, hipStream_t st) {
  const int64_t N = op->s->g.N;
  const int64_t chunk = (N + nc - 1) / nc;
  const dim3 grid((unsigned)((N + kBlock - 1) / kBlock), (unsigned)nc);
  double* part = op->part.p + (int64_t)r0 * N;
  const int64_t ldc = (int64_t)n_rhs * N;
  if (mode == 1) {
    constexpr int RL = row_len<NR, float>();
    if (op->rows32.n < (size_t)N * RL) op->rows32.alloc(&op->s->ctx->c, (size_t)N * RL);
    pack_launch<NR, float>({{N, op->co.tgt32.p, op->qt32.p + (int64_t)r0 * N, N, op->rows32.p}}, st);
    hipLaunchKernelGGL(k_direct32<NR>, grid, dim3(kBlock), 0, st, N, op->co.tgt32.p, op->rows32.p, chunk, part, N,
                       ldc);
  } else {
    constexpr int RL = row_len<NR, double>();
    if (op->rows64.n < (size_t)N * RL) op->rows64.alloc(&op->s->ctx->c, (size_t)N * RL);
    pack_launch<NR, double>({{N, op->s->g.x.p, op->qt64.p + (int64_t)r0 * N, N, op->rows64.p}}, st);
    hipLaunchKernelGGL(k_direct_log<NR>, grid, dim3(kBlock), 0, st, N, op->s->g.x.p, op->rows64.p, chunk, part, N,
                       ldc);
  }
  PMX_HIP(hipGetLastError());
}

void far_direct_mode(pmx_operator* op, int mode, int n_rhs, hipStream_t st) {
  if (mode == 0) {
    direct64_all({op}, {nullptr}, n_rhs, st);
    return;
  }
  if (op->co.has_c()) {
    PMX_REQUIRE(mode == 2, PMX_ERR_INVALID, "with c != 0 only the FP64 direct far field is available");
    direct_c_all(op, nullptr, 1, n_rhs, st);
    return;
  }
  const int64_t N = op->s->g.N;
  const int64_t nc = n_chunks_for(N);
  const size_t need = (size_t)nc * n_rhs * N;
  if (op->part.n < need) op->part.alloc(&op->s->ctx->c, need);
  int r0 = 0;
  while (r0 < n_rhs) {
    const int left = n_rhs - r0;
    if (left >= 16) { launch_group<16>(op, mode, n_rhs, r0, nc, st); r0 += 16; }
    else if (left >= 8) { launch_group<8>(op, mode, n_rhs, r0, nc, st); r0 += 8; }
    else if (left >= 4) { launch_group<4>(op, mode, n_rhs, r0, nc, st); r0 += 4; }
    else if (left >= 2) { launch_group<2>(op, mode, n_rhs, r0, nc, st); r0 += 2; }
    else { launch_group<1>(op, mode, n_rhs, r0, nc, st); r0 += 1; }
  }
}
}  // namespace

int far_direct_chunks(const pmx_operator* op, bool) { return (int)n_chunks_for(op->s->g.N); }

void far_direct(pmx_operator* op, bool fp64, int n_rhs, hipStream_t st) { far_direct_mode(op, fp64 ? 0 : 1, n_rhs, st); }

void far_direct64_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st) {
  std::vector<pmx_operator*> ops;
  std::vector<const ApplyScratch*> scs;
  for (const ApplyJob& j : jobs) {
    ops.push_back(j.op);
    scs.push_back(j.sc);
  }
  direct64_all(ops, scs, n_rhs, st);
}

size_t direct64_scratch_doubles(int64_t N, int n_rhs) {
  auto up = [](size_t n) { return (n + 31) / 32 * 32; };
  const size_t nr = (size_t)n_rhs;
  const size_t nb = (size_t)((N + kBlock - 1) / kBlock);
  const int g = n_rhs >= 16 ? 16 : (n_rhs >= 8 ? 8 : (n_rhs >= 4 ? 4 : (n_rhs >= 2 ? 2 : 1)));
  const size_t rl = (size_t)((4 + g + 1) / 2) * 2;   // widest packed row of the groups used (c rows too)
  return up(nr * N) + up(nr * nb) + up(nr) + up(rl * N) + up((size_t)n_chunks_for(N) * nr * N);
}

void far_direct_log(pmx_operator* op, int n_rhs, hipStream_t st) { far_direct_mode(op, 2, n_rhs, st); }

}  // namespace pmx
