// Edge operators of the open-surface problems (Section 5): boundary-curve sources, surface targets.
//
// For a density mu on the boundary gamma of an open surface Gamma and a target x in Gamma:
//   K_gamma[mu](x) = int_gamma K(x, x') mu(x') ds(x')                       (representation, Neumann)
//   N_gamma[mu](x) = int_gamma nu(x') . grad'_G K(x, x') mu(x') ds(x')       (representation, Dirichlet)
//   R_gamma[mu](x) = int_gamma R(x, x') mu(x') ds(x')                       (Neumann system)
//   T_gamma[mu](x) = int_gamma nu(x') . grad'_G R(x, x') mu(x') ds(x')       (Dirichlet system)
// with nu the unit conormal at x' (tangent to Gamma, normal to gamma, out of Gamma) and the primed
// derivative acting on the source point, which enters through r = x - x' and through a(x').
// c = 0: K = log r / (2 pi a(x')), and with the target factors of the far-field sums
//   a(x') R(x, x') = Phi(r) = rho ((n'.r)^2 rho + h.r),  rho = 1 / r^2,  n' = sqrt(a / pi) n,
//   h = grad_G a / (2 pi) - (a H / pi) n,
// so that, with beta = nu . grad a(x') / a(x') and dr/dx' = -I,
//   a' nu.grad' K = (-(nu.r) rho - log(r) beta) / (2 pi)
//   a' nu.grad' R = -nu.grad_r Phi - Phi beta,
//   nu.grad_r Phi = rho (h.nu + rho (2 (n'.r)(n'.nu) - 2 (h.r)(nu.r) - 4 (n'.r)^2 (nu.r) rho)).
//
// Discretization (Section 6.1.4): each curve is given at n equispaced samples of a periodic
// parameter t in [0, 2 pi).  Every sampled quantity is replaced by its trigonometric interpolant at
// m n equispaced points, f(t_k) = sum_j f_j D(t_k - t_j), with the periodic Dirichlet kernel
//   D(tau) = sin(n tau / 2) cot(tau / 2) / n  (n even: the Nyquist mode split evenly),
//   D(tau) = sin(n tau / 2) / (n sin(tau / 2))  (n odd),
// which takes only the m n values tau = 2 pi k / (m n), tabulated once per curve.  The trapezoid rule
// on the fine points then has weights (2 pi / (m n)) |dgamma/dt|.
//
// K'_gamma, the conormal derivative at a target on gamma of the potential of K (the boundary rows of
// the Neumann and Dirichlet systems), has the smooth kernel nu(x) . (x - x') / (2 pi a(x') |x - x'|^2),
// and so has the double layer D_gamma (the conormal at the source) when nu . grad a = 0 on gamma:
// the trapezoid rule runs on the samples themselves, and at x' = x the kernel takes its limit
// -(nu . gamma'') / (4 pi a |gamma'|^2), with gamma'' the derivative of the interpolant of the sampled
// dgamma/dt at the samples, sum_k D1(j - k) gamma'_k with D1(l) = (-1)^l cot(pi l / n) / 2 (n even)
// or (-1)^l / (2 sin(pi l / n)) (n odd), D1(0) = 0.
//
// Layout: fine points in structure-of-arrays form, pts[c * Mf + p] for c = y (3), nu (3), beta,
// w / a, w, a (the last two for export only).  An apply interpolates mu, packs source rows (y, nu,
// beta, w mu / a per right-hand side) that every lane of a wavefront reads alike (through the scalar
// data cache), and sums over a chunk of fine points per workgroup row; the chunks' partial sums are
// added in a fixed order.
#include "pmx_internal.hpp"

namespace pmx {

namespace {
constexpr int kBlock = 256;
constexpr int kUpCh = 4;   // channels per pass of the interpolation kernel

typedef const __attribute__((address_space(4))) double* sdp;

__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

struct CurveIdx {
  const int64_t* off;    // coarse sample offsets, n_curves + 1
  const int64_t* foff;   // fine point offsets, n_curves + 1
  int nc;
  int m;
};

__device__ __forceinline__ int curve_of(const CurveIdx& c, int64_t g) {
  int k = 0;
  while (k + 1 < c.nc && g >= c.foff[k + 1]) ++k;
  return k;
}

__global__ void __launch_bounds__(kBlock) k_edge_table(CurveIdx c, int64_t Mf, double* __restrict__ D) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= Mf) return;
  const int k = curve_of(c, g);
  const int64_t i = g - c.foff[k];
  const int64_t n = c.off[k + 1] - c.off[k];
  const int m = c.m;
  // D is even in tau: evaluate at the smaller of i and m n - i, so that tau / (2 pi) <= 1/2 and sinpi
  // of it keeps its relative accuracy (near tau = 2 pi the rounding of i / (m n) would cost about
  // eps m n relative in the weights of the nearest samples)
  const int64_t ie = i <= m * n - i ? i : m * n - i;
  double v;
  if (ie % m == 0) {
    v = ie == 0 ? 1.0 : 0.0;
  } else {
    const double s = sinpi((double)(ie % (2 * m)) / m);         // sin(n tau / 2), tau = 2 pi ie / (m n)
    const double h = (double)ie / (double)(m * n);               // tau / (2 pi)
    v = (n % 2 == 0) ? s * cospi(h) / (n * sinpi(h)) : s / (n * sinpi(h));
  }
  D[g] = v;
}

struct UpArgs {
  CurveIdx c;
  int64_t Mf;
  int nch;
  const double* src;   // nch rows of M coarse values
  int64_t lds;
  double* dst;         // nch rows of Mf fine values
  int64_t ldd;
  const double* D;
};

// kUpLanes lanes per fine point, lane l summing the samples j = l (mod kUpLanes); the lanes' partial
// sums are combined by a fixed shuffle tree (deterministic), and lane 0 writes.
constexpr int kUpLanes = 8;

__global__ void __launch_bounds__(kBlock) k_edge_upsample(UpArgs A) {
  const int64_t g = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kUpLanes;
  const int l = threadIdx.x % kUpLanes;
  const bool live = g < A.Mf;
  const int k = live ? curve_of(A.c, g) : 0;
  const int64_t i = live ? g - A.c.foff[k] : 0;
  const int64_t base = A.c.off[k], n = live ? A.c.off[k + 1] - base : 0;
  const int64_t mn = (int64_t)A.c.m * (A.c.off[k + 1] - base);
  const int64_t step = ((int64_t)A.c.m * kUpLanes) % mn;
  const double* __restrict__ Dk = A.D + A.c.foff[k];
  for (int c0 = 0; c0 < A.nch; c0 += kUpCh) {
    double acc[kUpCh] = {0.0, 0.0, 0.0, 0.0};
    int64_t idx = i - (int64_t)A.c.m * l;   // i - m j, wrapped into [0, m n)
    while (idx < 0) idx += mn;
    for (int64_t j = l; j < n; j += kUpLanes) {
      const double d = Dk[idx];
#pragma unroll
      for (int c = 0; c < kUpCh; ++c)
        if (c0 + c < A.nch) acc[c] = fma(A.src[(c0 + c) * A.lds + base + j], d, acc[c]);
      idx -= step;
      if (idx < 0) idx += mn;
    }
#pragma unroll
    for (int c = 0; c < kUpCh; ++c) {
      double v = acc[c];
      v += __shfl_xor(v, 4, kUpLanes);
      v += __shfl_xor(v, 2, kUpLanes);
      v += __shfl_xor(v, 1, kUpLanes);
      if (live && l == 0 && c0 + c < A.nch) A.dst[(c0 + c) * A.ldd + g] = v;
    }
  }
}

// Fine geometry channels in: y (3), dy/dt (3), d (3), a, grad a (3).  Out: y, nu, beta, w / a, w, a.
__global__ void __launch_bounds__(kBlock) k_edge_geom(CurveIdx c, int64_t Mf, const double* __restrict__ F,
                                                      double* __restrict__ P, int* __restrict__ bad) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= Mf) return;
  const int k = curve_of(c, g);
  const int64_t n = c.off[k + 1] - c.off[k];
  double f[13];
#pragma unroll
  for (int q = 0; q < 13; ++q) f[q] = F[q * Mf + g];
  const double L = sqrt(f[3] * f[3] + f[4] * f[4] + f[5] * f[5]);
  const double t0 = f[3] / L, t1 = f[4] / L, t2 = f[5] / L;
  const double dt = f[6] * t0 + f[7] * t1 + f[8] * t2;
  double v0 = f[6] - dt * t0, v1 = f[7] - dt * t1, v2 = f[8] - dt * t2;
  const double vl = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
  const double dl = sqrt(f[6] * f[6] + f[7] * f[7] + f[8] * f[8]);
  v0 /= vl; v1 /= vl; v2 /= vl;
  const double a = f[9];
  const double w = (2.0 * M_PI / ((double)c.m * (double)n)) * L;
  const bool ok = L > 0.0 && isfinite(L) && vl > 1e-8 * dl && a > 0.0 && isfinite(a) &&
                  isfinite(f[0] + f[1] + f[2] + f[10] + f[11] + f[12]);
  if (!ok) atomicOr(bad, 1);
  P[0 * Mf + g] = f[0];
  P[1 * Mf + g] = f[1];
  P[2 * Mf + g] = f[2];
  P[3 * Mf + g] = v0;
  P[4 * Mf + g] = v1;
  P[5 * Mf + g] = v2;
  P[6 * Mf + g] = (v0 * f[10] + v1 * f[11] + v2 * f[12]) / a;
  P[7 * Mf + g] = w / a;
  P[8 * Mf + g] = w;
  P[9 * Mf + g] = a;
}

// Per sample (coarse geometry rows in: y (3), dy/dt (3), d (3), a, grad a (3)): x (3), nu (3), a, the
// trapezoid weight (2 pi / n) |dgamma/dt| and the diagonal limit of the K'_gamma kernel.
__global__ void __launch_bounds__(kBlock) k_edge_samples(CurveIdx c, int64_t M, const double* __restrict__ F,
                                                         double* __restrict__ S) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= M) return;
  int k = 0;
  while (k + 1 < c.nc && j >= c.off[k + 1]) ++k;
  const int64_t base = c.off[k], n = c.off[k + 1] - base, jl = j - base;
  double tt[3] = {0.0, 0.0, 0.0};   // gamma'' at the sample
  for (int64_t q = 0; q < n; ++q) {
    const int64_t l = (jl - q + n) % n;
    if (l == 0) continue;
    // D1 is odd in l (D1(n - l) = -D1(l)): evaluate at the smaller of l and n - l (as for D above)
    const int64_t le = l <= n - l ? l : n - l;
    const double h = (double)le / (double)n;
    const double sgn = ((le & 1) ? -0.5 : 0.5) * (le == l ? 1.0 : -1.0);
    const double wd = (n % 2 == 0) ? sgn * cospi(h) / sinpi(h) : sgn / sinpi(h);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) tt[cc] = fma(wd, F[(3 + cc) * M + base + q], tt[cc]);
  }
  const double t0 = F[3 * M + j], t1 = F[4 * M + j], t2 = F[5 * M + j];
  const double L2 = t0 * t0 + t1 * t1 + t2 * t2, L = sqrt(L2);
  const double u0 = t0 / L, u1 = t1 / L, u2 = t2 / L;
  const double d0 = F[6 * M + j], d1 = F[7 * M + j], d2 = F[8 * M + j];
  const double dt = d0 * u0 + d1 * u1 + d2 * u2;
  double v0 = d0 - dt * u0, v1 = d1 - dt * u1, v2 = d2 - dt * u2;
  const double vl = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
  v0 /= vl; v1 /= vl; v2 /= vl;
  const double a = F[9 * M + j];
  S[0 * M + j] = F[0 * M + j];
  S[1 * M + j] = F[1 * M + j];
  S[2 * M + j] = F[2 * M + j];
  S[3 * M + j] = v0;
  S[4 * M + j] = v1;
  S[5 * M + j] = v2;
  S[6 * M + j] = a;
  S[7 * M + j] = (2.0 * M_PI / (double)n) * L;
  S[8 * M + j] = -(v0 * tt[0] + v1 * tt[1] + v2 * tt[2]) / (4.0 * M_PI * a * L2);
}

// y[r][i] = sum_j w_j k(x_i, x_j) mu[r][j] over all samples with the smooth on-curve kernel
//   DL = false: K'_gamma, nu(x_i) . (x_i - x_j) / (2 pi a_j r^2)  (the conormal at the target),
//   DL = true:  D_gamma,  nu(x_j) . (x_j - x_i) / (2 pi a_j r^2)  (at the source; nu . grad a = 0),
// both with the limit -(nu . gamma'') / (4 pi a |gamma'|^2) at j = i.
// One wavefront per (target sample, right-hand side), four per workgroup, grid y the right-hand side:
// lane l takes the samples j = l (mod 64) and a fixed shuffle tree adds the lanes' sums.
template <bool DL>
__global__ void __launch_bounds__(kBlock) k_edge_on_curve(int64_t M, const double* __restrict__ S,
                                                          const double* __restrict__ mu, double* __restrict__ y) {
  constexpr double kInv2Pi = 0.15915494309189533577;
  const int64_t i = (int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  const int64_t r = blockIdx.y;
  if (i >= M) return;   // whole wavefronts leave together
  const double xi = S[i], yi = S[M + i], zi = S[2 * M + i];
  const double n0 = S[3 * M + i], n1 = S[4 * M + i], n2 = S[5 * M + i];
  const double* __restrict__ m = mu + r * M;
  double acc = 0.0;
  for (int64_t j = lane; j < M; j += 64) {
    double val;
    if (j == i) {
      val = S[8 * M + i];
    } else {
      const double dx = xi - S[j], dy = yi - S[M + j], dz = zi - S[2 * M + j];
      const double den = S[6 * M + j] * fma(dx, dx, fma(dy, dy, dz * dz));
      const double num = DL ? -fma(S[3 * M + j], dx, fma(S[4 * M + j], dy, S[5 * M + j] * dz))
                            : fma(n0, dx, fma(n1, dy, n2 * dz));
      val = kInv2Pi * num * rcp_nr(den);
    }
    acc = fma(S[7 * M + j] * m[j], val, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) y[r * M + i] = acc;
}

// Row of a packed source: y (3), nu (3), beta, NR weighted densities, padded to an even length.
template <int NR>
constexpr int edge_row_len() { return ((7 + NR + 1) / 2) * 2; }

template <int NR>
__global__ void __launch_bounds__(kBlock) k_edge_pack(int64_t Mf, const double* __restrict__ P,
                                                      const double* __restrict__ muf, double* __restrict__ rows) {
  constexpr int RL = edge_row_len<NR>();
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= Mf) return;
  double* row = rows + p * RL;
#pragma unroll
  for (int q = 0; q < 7; ++q) row[q] = P[q * Mf + p];
  const double wa = P[7 * Mf + p];
#pragma unroll
  for (int r = 0; r < NR; ++r) row[7 + r] = wa * muf[r * Mf + p];
#pragma unroll
  for (int q = 7 + NR; q < RL; ++q) row[q] = 0.0;
}

struct EdgePairArgs {
  int64_t N, Mf, chunk, nbx;
  const double* tf;    // 9N target factors: x y z n' h
  const double* rows;
  double* part;        // part[chunk][rhs][i]
  int64_t ldc;         // NR * N
};

// KIND: 0 K, 1 N, 2 R, 3 T.
template <int KIND, int NR>
__global__ void __launch_bounds__(kBlock) k_edge_pairs(EdgePairArgs A) {
  constexpr int RL = edge_row_len<NR>();
  constexpr double kInv2Pi = 0.15915494309189533577;
  const int64_t N = A.N;
  const int64_t by = blockIdx.x / A.nbx, bx = blockIdx.x - by * A.nbx;
  const int64_t p0 = by * A.chunk;
  const int64_t p1 = p0 + A.chunk < A.Mf ? p0 + A.chunk : A.Mf;
  const int64_t it = bx * kBlock + threadIdx.x;
  const int64_t i = it < N ? it : N - 1;
  const double* __restrict__ tf = A.tf;
  const double xi = tf[i], yi = tf[N + i], zi = tf[2 * N + i];
  double px = 0, py = 0, pz = 0, hx = 0, hy = 0, hz = 0;
  if (KIND >= 2) {
    px = tf[3 * N + i]; py = tf[4 * N + i]; pz = tf[5 * N + i];
    hx = tf[6 * N + i]; hy = tf[7 * N + i]; hz = tf[8 * N + i];
  }
  const sdp S = (sdp)A.rows;
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
#pragma unroll 4
  for (int64_t p = p0; p < p1; ++p) {
    const sdp row = S + p * RL;
    const double dx = xi - row[0], dy = yi - row[1], dz = zi - row[2];
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-300)));
    double val;
    if (KIND == 0) {
      val = (0.5 * kInv2Pi) * log_pair(r2);
    } else if (KIND == 1) {
      const double rho = rcp_nr(r2);
      const double v = fma(row[3], dx, fma(row[4], dy, row[5] * dz));
      val = -kInv2Pi * fma(v, rho, 0.5 * log_pair(r2) * row[6]);
    } else {
      const double rho = rcp_nr(r2);
      const double u = fma(px, dx, fma(py, dy, pz * dz));
      const double hr = fma(hx, dx, fma(hy, dy, hz * dz));
      const double phi = fma(u * rho, u, hr) * rho;
      if (KIND == 2) {
        val = phi;
      } else {
        const double nx = row[3], ny = row[4], nz = row[5];
        const double v = fma(nx, dx, fma(ny, dy, nz * dz));
        const double un = fma(px, nx, fma(py, ny, pz * nz));
        const double hn = fma(hx, nx, fma(hy, ny, hz * nz));
        const double in = fma(2.0 * u, un, -2.0 * hr * v) - 4.0 * u * u * v * rho;
        const double dphi = rho * fma(rho, in, hn);
        val = -fma(phi, row[6], dphi);
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = fma(row[7 + r], val, acc[r]);
  }
  if (it < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) A.part[by * A.ldc + r * N + it] = acc[r];
  }
}

__global__ void __launch_bounds__(kBlock) k_edge_reduce(int64_t len, int64_t nchunk, int64_t ldc,
                                                        const double* __restrict__ part, double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) s += part[c * ldc + e];
  y[e] = s;
}

int64_t nblk(int64_t n) { return (n + kBlock - 1) / kBlock; }

CurveIdx curve_idx(const EdgeSet& E) { return {E.doff.p, E.dfoff.p, E.n_curves, E.m}; }

template <int KIND, int NR>
void launch_pairs(const EdgePairArgs& a, int64_t blocks, hipStream_t st) {
  hipLaunchKernelGGL((k_edge_pairs<KIND, NR>), dim3(blocks), dim3(kBlock), 0, st, a);
}

template <int NR>
void pairs_kind(int kind, const EdgePairArgs& a, int64_t blocks, hipStream_t st) {
  switch (kind) {
    case 0: launch_pairs<0, NR>(a, blocks, st); break;
    case 1: launch_pairs<1, NR>(a, blocks, st); break;
    case 2: launch_pairs<2, NR>(a, blocks, st); break;
    default: launch_pairs<3, NR>(a, blocks, st); break;
  }
}
}  // namespace

void edge_build(Ctx* ctx, EdgeSet& E, const std::vector<int64_t>& off, const std::vector<double>& soa, int m,
                hipStream_t st) {
  E.n_curves = (int)off.size() - 1;
  E.m = m;
  E.off = off;
  E.M = off.back();
  E.foff.assign(off.size(), 0);
  for (size_t k = 0; k < off.size(); ++k) E.foff[k] = off[k] * m;
  E.Mf = E.foff.back();
  E.doff.alloc(ctx, off.size());
  E.dfoff.alloc(ctx, off.size());
  PMX_HIP(hipMemcpyAsync(E.doff.p, E.off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  PMX_HIP(hipMemcpyAsync(E.dfoff.p, E.foff.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
  DBuf<double> coarse, fine;
  DBuf<int> bad;
  coarse.alloc(ctx, 13 * E.M);
  fine.alloc(ctx, 13 * E.Mf);
  bad.alloc(ctx, 1);
  PMX_HIP(hipMemcpyAsync(coarse.p, soa.data(), 13 * E.M * sizeof(double), hipMemcpyHostToDevice, st));
  E.table.alloc(ctx, E.Mf);
  E.pts.alloc(ctx, 10 * E.Mf);
  const CurveIdx c = curve_idx(E);
  hipLaunchKernelGGL(k_edge_table, dim3(nblk(E.Mf)), dim3(kBlock), 0, st, c, E.Mf, E.table.p);
  UpArgs u{c, E.Mf, 13, coarse.p, E.M, fine.p, E.Mf, E.table.p};
  hipLaunchKernelGGL(k_edge_upsample, dim3(nblk(E.Mf * kUpLanes)), dim3(kBlock), 0, st, u);
  const int zero = 0;
  PMX_HIP(hipMemcpyAsync(bad.p, &zero, sizeof(int), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_edge_geom, dim3(nblk(E.Mf)), dim3(kBlock), 0, st, c, E.Mf, fine.p, E.pts.p, bad.p);
  E.samp.alloc(ctx, 9 * E.M);
  hipLaunchKernelGGL(k_edge_samples, dim3(nblk(E.M)), dim3(kBlock), 0, st, c, E.M, coarse.p, E.samp.p);
  PMX_HIP(hipGetLastError());
  int flag = 0;
  PMX_HIP(hipMemcpyAsync(&flag, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  PMX_REQUIRE(flag == 0, PMX_ERR_INVALID,
              "edge: an interpolated point has a vanishing curve derivative, a direction d along the curve, "
              "a <= 0 or non-finite data");
}

void edge_apply(pmx_operator* op, EdgeSet& E, int kind, int n_rhs, const double* mu, double* y, hipStream_t st) {
  Ctx* ctx = E.ctx;
  const int64_t N = op->s->g.N, Mf = E.Mf;
  if (E.muf.n < (size_t)n_rhs * Mf) E.muf.alloc(ctx, (size_t)n_rhs * Mf);
  const CurveIdx c = curve_idx(E);
  UpArgs u{c, Mf, n_rhs, mu, E.M, E.muf.p, Mf, E.table.p};
  hipLaunchKernelGGL(k_edge_upsample, dim3(nblk(Mf * kUpLanes)), dim3(kBlock), 0, st, u);
  // source chunks: enough workgroups to fill the chip several times over
  const int64_t nbx = nblk(N);
  int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>((4096 + nbx - 1) / nbx, (Mf + 127) / 128));
  const int64_t chunk = (Mf + nchunk - 1) / nchunk;
  nchunk = (Mf + chunk - 1) / chunk;
  const int nr_max = n_rhs >= 4 ? 4 : 1;
  if (E.rows.n < (size_t)edge_row_len<4>() * Mf) E.rows.alloc(ctx, (size_t)edge_row_len<4>() * Mf);
  if (E.part.n < (size_t)nchunk * nr_max * N) E.part.alloc(ctx, (size_t)nchunk * nr_max * N);
  for (int r0 = 0; r0 < n_rhs;) {
    const int nr = n_rhs - r0 >= 4 ? 4 : 1;
    EdgePairArgs a{N, Mf, chunk, nbx, op->co.tf64.p, E.rows.p, E.part.p, (int64_t)nr * N};
    if (nr == 4) {
      hipLaunchKernelGGL(k_edge_pack<4>, dim3(nblk(Mf)), dim3(kBlock), 0, st, Mf, E.pts.p, E.muf.p + r0 * Mf, E.rows.p);
      const int t = op->prof.begin(PMX_PHASE_EDGE, st);
      pairs_kind<4>(kind, a, nbx * nchunk, st);
      op->prof.end(t, st);
    } else {
      hipLaunchKernelGGL(k_edge_pack<1>, dim3(nblk(Mf)), dim3(kBlock), 0, st, Mf, E.pts.p, E.muf.p + r0 * Mf, E.rows.p);
      const int t = op->prof.begin(PMX_PHASE_EDGE, st);
      pairs_kind<1>(kind, a, nbx * nchunk, st);
      op->prof.end(t, st);
    }
    hipLaunchKernelGGL(k_edge_reduce, dim3(nblk((int64_t)nr * N)), dim3(kBlock), 0, st, (int64_t)nr * N, nchunk,
                       (int64_t)nr * N, E.part.p, y + (int64_t)r0 * N);
    r0 += nr;
  }
  PMX_HIP(hipGetLastError());
}

void edge_apply_on_curve(EdgeSet& E, bool double_layer, int n_rhs, const double* mu, double* y, hipStream_t st) {
  const dim3 grid((E.M + kBlock / 64 - 1) / (kBlock / 64), n_rhs);
  if (double_layer)
    hipLaunchKernelGGL(k_edge_on_curve<true>, grid, dim3(kBlock), 0, st, E.M, E.samp.p, mu, y);
  else
    hipLaunchKernelGGL(k_edge_on_curve<false>, grid, dim3(kBlock), 0, st, E.M, E.samp.p, mu, y);
  PMX_HIP(hipGetLastError());
}

}  // namespace pmx
