// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <functional>
#include <vector>

#include "../../include/pmx.h"

struct pmx_batcher;

namespace pmx {

// ----------------------------------------------------------------------------- errors
struct Error : std::runtime_error {
  pmx_status code;
  Error(pmx_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);

#define PMX_HIP(call)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      throw ::pmx::Error(e_ == hipErrorOutOfMemory ? PMX_ERR_OOM : PMX_ERR_DEVICE,              \
                         std::string(#call) + ": " + hipGetErrorString(e_));                    \
  } while (0)

#define PMX_REQUIRE(cond, code, msg) \
  do {                               \
    if (!(cond)) throw ::pmx::Error((code), (msg)); \
  } while (0)

// ----------------------------------------------------------------------------- device buffers
// Owning device allocation; the context tracks bytes against its HBM budget.
struct Ctx;
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  Ctx* ctx = nullptr;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { swap(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    swap(o);
    return *this;
  }
  ~DBuf() { release(); }
  void swap(DBuf& o) {
    std::swap(p, o.p);
    std::swap(n, o.n);
    std::swap(ctx, o.ctx);
  }
  void alloc(Ctx* c, size_t count);
  void release();
  size_t bytes() const { return n * sizeof(T); }
  T* get() const { return p; }
};

// Device memory accounting of a context (shared by the server's worker threads).  A server
// request allocates from a context of its own whose bytes are also charged to the server's
// context (parent) without that context's budget check: the server admits requests by
// footprint, so a running request is never failed by another request's size.
struct Ctx {
  int device = 0;
  uint64_t budget = 0;   // 0 = unbounded
  std::atomic<uint64_t> in_use{0};
  std::atomic<uint64_t> peak{0};
  Ctx* parent = nullptr;
  int n_cu = 256;
  void reserve(uint64_t bytes) {
    uint64_t cur = in_use.load();
    do {
      if (budget && cur + bytes > budget)
        throw Error(PMX_ERR_TOO_LARGE, "device footprint exceeds the context's HBM budget");
    } while (!in_use.compare_exchange_weak(cur, cur + bytes));
    const uint64_t now = cur + bytes;
    uint64_t pk = peak.load();
    while (now > pk && !peak.compare_exchange_weak(pk, now)) {
    }
    if (parent) parent->in_use.fetch_add(bytes);
  }
  void unreserve(uint64_t bytes) {
    in_use.fetch_sub(bytes);
    if (parent) parent->in_use.fetch_sub(bytes);
  }
};

template <class T>
void DBuf<T>::alloc(Ctx* c, size_t count) {
  release();
  if (count == 0) return;
  c->reserve(count * sizeof(T));
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) {
    c->unreserve(count * sizeof(T));
    p = nullptr;
    throw Error(PMX_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  n = count;
  ctx = c;
}

template <class T>
void DBuf<T>::release() {
  if (p) {
    (void)hipFree(p);
    if (ctx) ctx->unreserve(n * sizeof(T));
  }
  p = nullptr;
  n = 0;
}

// ----------------------------------------------------------------------------- data on the device
// Node-wise geometry in structure-of-arrays layout.  Target factors of the
// factored c = 0 remainder:
//   R(x_i, x_j) = (1/a_j) [ g_i . r / r^2 + A_i (n_i.r)^2 / r^4 - B_i (n_i.r) / r^2 ],
//   A_i = a_i / pi, B_i = a_i H_i / pi, g_i = grad_G a_i / (2 pi), r = x_i - x_j.
struct Geometry {
  int64_t N = 0, M = 0;
  int q = 0;
  DBuf<double> x;       // 3N  (x | y | z)
  DBuf<double> n;       // 3N
  DBuf<double> J, w, H; // N each
  DBuf<double> corner;  // M * 12  (4 corner images)
  DBuf<double> cent;    // M * 4   (centroid xyz, radius)
  DBuf<double> xu_p, xv_p;  // patch-local copies of x_u, x_v (3N each) for the local rules
  DBuf<double> tnodes;  // q Gauss-Legendre nodes
  DBuf<double> tweights;
  double area = 0.0;
};

// The far-field kernels use the equivalent form
//   R(x_i, x_j) a_j = (1/r^2) [ (n'_i . r)^2 / r^2 + h_i . r ],  n' = sqrt(A) n,  h = g - B n.
struct Coeff {
  DBuf<double> a;       // N
  DBuf<double> gs;      // 3N surface gradient
  DBuf<double> tgt;     // 8N: x y z nx ny nz A B | (g stored below)
  DBuf<double> tg;      // 3N: g = (grad_G a + b_t) / (2 pi), b_t the tangential advection field (0 without b)
  DBuf<double> tf64;    // 9N: x y z n'x n'y n'z hx hy hz (h = g - B n)
  DBuf<float> tgt32;    // 9N: the same in FP32
  DBuf<double> w_over_a;  // N
  DBuf<double> c;       // N: the zero-order coefficient (c < 0 or c > 0 at every node); empty for c = 0
  bool has_b = false;   // an advection field is folded into g and h
  bool complex_ = false;  // c > 0: the complex Helmholtz-type kernel
  bool has_c() const { return c.p != nullptr; }
};

struct NearLists {
  int64_t nnz = 0;
  DBuf<int64_t> ptr;        // N + 1
  DBuf<int32_t> patch;      // nnz
  DBuf<int32_t> target;     // nnz (pair -> target node)
  DBuf<double> C;           // nnz * q*q (remainder)
  DBuf<double> D;           // nnz * q*q (parametrix), built on demand
  DBuf<double> Ci, Di;      // imaginary parts of C and D (c > 0 only)
  bool have_D = false;
  // by target patch (for several right-hand sides): the union of the near patches of the
  // patch's targets, [tile_ptr[T], tile_ptr[T + 1]) into tile_patch, and for union entry u
  // the pair of each of the patch's targets with that patch, tile_pair[u * q*q + t] (-1: none)
  DBuf<int32_t> tile_ptr, tile_patch, tile_pair;
  bool have_tiles = false;
};

// Boundary curves of an open surface, Fourier-oversampled for the edge quadrature (edge.hip):
// curve k owns coarse samples [off[k], off[k+1]) and fine points [m off[k], m off[k+1]).
struct EdgeSet {
  Ctx* ctx = nullptr;
  int n_curves = 0, m = 1;
  bool nu_grad_a_zero = false;   // nu . grad a = 0 at every sample (D_gamma is then smooth)
  int64_t M = 0, Mf = 0;
  std::vector<int64_t> off, foff;
  DBuf<int64_t> doff, dfoff;
  DBuf<double> table;   // Mf: periodic Dirichlet kernel of each curve at its m n offsets
  DBuf<double> pts;     // 10 Mf: y (3), nu (3), beta = nu . grad a / a, w / a, w, a
  DBuf<double> samp;    // 9 M: per sample x (3), nu (3), a, trapezoid weight, K'_gamma diagonal limit
  DBuf<double> muf, rows, part;   // scratch of an apply
};

struct FMM;  // fmm.hip

// ----------------------------------------------------------------------------- grouped launches
// One launch serves up to kMaxSeg operators: segment s owns the blocks
// [off[s], off[s + 1]) of the grid and its own argument record.  A single-operator
// launch is a group of one.  The arguments travel by value in the kernel
// arguments, so forming a group needs no device memory.
constexpr int kMaxSeg = 8;

template <class A>
struct Group {
  int n = 0;
  int64_t off[kMaxSeg + 1] = {};
  A a[kMaxSeg];
};

// Segment of block b and the block's index inside it.
template <class A>
__device__ __forceinline__ const A& seg_of(const Group<A>& g, int64_t b, int64_t& local) {
  int s = 0;
  while (s + 1 < g.n && b >= g.off[s + 1]) ++s;
  local = b - g.off[s];
  return g.a[s];
}

// Natural logarithm of a positive normal x (log-kernel sums and quadrature), from the artanh series: with
// x = 2^e m, m in [sqrt(1/2), sqrt(2)) (hardware frexp), log x = e ln 2 + 2 artanh(s) where
// s = (m - 1) / (m + 1), |s| <= 0.1716, and artanh(s) = sum_k s^(2k+1) / (2k+1) (Taylor series).
// Ten terms (through s^19 / 19) leave a truncation error below 1e-17; the reciprocal takes two
// Newton steps, and e ln 2 is one rounding (|e| <= 60 here: error below 3e-15 absolute, about one
// ulp of the result).  About 30 FP64 instructions, against about 90 for the library's log, whose
// extra precision the sums and quadratures do not need.
__device__ __forceinline__ double log_pair(double x) {
  constexpr double kSqrtHalf = 0.70710678118654752440;
  constexpr double kLn2 = 0.69314718055994530942;
  double m = __builtin_amdgcn_frexp_mant(x);      // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < kSqrtHalf;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double d = m + 1.0;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  const double sv = (m - 1.0) * r;
  const double s2 = sv * sv;
  double p = 1.0 / 19.0;
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  p = fma(p, s2, 1.0);
  return fma((double)e, kLn2, 2.0 * sv * p);
}

// Modified Bessel functions K0(z) and K1(z) of a positive argument (FP64): the Green's function
// of (a Delta + c) G = delta with c < 0 is G = -K0(kappa r) / (2 pi a), kappa = sqrt(-c / a).
//  * z <= 2: the power series in t = z^2 / 4 (Abramowitz & Stegun 9.6.13 for K0, 9.6.11 with
//    n = 1 for K1), with I0 = sum t^k / (k!)^2, I1 = sum t^k / (k! (k+1)!) and harmonic
//    numbers H_k:  K0 = -(ln(z/2) + gamma) I0 + sum H_k t^k / (k!)^2,
//    K1 = 1/z + (ln(z/2) + gamma) (z/2) I1 - (z/4) sum (H_k + H_{k+1}) t^k / (k! (k+1)!),
//    each sum as a polynomial of degree 12 in t by Horner's rule (coefficients computed at
//    compile time; truncation below 5e-18 at t = 1).  The cancellation in K0 near z = 2 costs
//    about one decimal digit (relative error up to 4e-15).
//  * z > 2: sqrt(z) e^z K_nu(z) is smooth in s = 2/z on (0, 1]; its interpolant of degree 22 in
//    x = 4/z - 1 (interpolation at the Chebyshev points at 40 digits, converted to the power form,
//    bessel_k_table.py) has relative error 1.2e-16, evaluated by Horner's rule.
constexpr double kEulerGamma = 0.57721566490153286061;

struct KSeries {
  double i0[13], s0[13], i1[13], s1[13];
};
constexpr KSeries make_kseries() {
  KSeries r{};
  double f = 1.0, g = 1.0, h = 0.0;   // 1/(k!)^2, 1/(k!(k+1)!), H_k
  for (int k = 0; k < 13; ++k) {
    const double hn = h + 1.0 / (double)(k + 1);
    r.i0[k] = f;
    r.s0[k] = h * f;
    r.i1[k] = g;
    r.s1[k] = (h + hn) * g;
    f /= (double)(k + 1) * (double)(k + 1);
    g /= (double)(k + 1) * (double)(k + 2);
    h = hn;
  }
  return r;
}

constexpr double kPolyK0[23] = {
    1.21859533851339052e+00, -3.10714618248898629e-02, 3.03289181027414315e-03,
    -4.79769056735349661e-04, 9.95605474680700934e-05, -2.47352053744823634e-05,
    7.00224489119246702e-06, -2.19116792521650616e-06, 7.42786224915629391e-07,
    -2.68973007185193227e-07, 1.02925573280657489e-07, -4.10665802711522117e-08,
    1.71318560067890199e-08, -8.00485151596186128e-09, 3.64970419674587604e-09,
    -6.90944553209526845e-10, 2.39282475774540067e-10, -1.21546469253292140e-09,
    6.69690967735319141e-10, 4.29782283193599083e-10, -2.51158362375080098e-10,
    -1.74157926367135482e-10, 9.81540200885952561e-11};
constexpr double kPolyK1[23] = {
    1.36315189037134199e+00, 1.03349737753865606e-01, -5.56672988007330879e-03,
    7.35724154874510560e-04, -1.39590219614627790e-04, 3.28438664438236949e-05,
    -8.96120656800817468e-06, 2.73003069116461256e-06, -9.06715391779199444e-07,
    3.23053491198630796e-07, -1.22000639091108527e-07, 4.81650114775029143e-08,
    -1.99091691254213902e-08, 9.19183829361296321e-09, -4.15956404449566279e-09,
    8.25400261129896233e-10, -2.91588972545863801e-10, 1.33858499774653138e-09,
    -7.34780754419483894e-10, -4.67158267076234187e-10, 2.72604009952142169e-10,
    1.90768996505765517e-10, -1.07243915727052585e-10};

// The coefficients of bessel_k01 in one table: the four series (13 each), then the two
// interpolants' power forms (23 each).  (Staging the table in LDS for the direct sum, instead of the
// register-resident constants, was measured no faster: 152 vs 150 ms on 153,600 nodes.)
constexpr int kKTable = 4 * 13 + 2 * 23;
struct KTable {
  double v[kKTable];
};
constexpr KTable make_ktable() {
  KTable t{};
  const KSeries s = make_kseries();
  for (int k = 0; k < 13; ++k) {
    t.v[k] = s.i0[k];
    t.v[13 + k] = s.s0[k];
    t.v[26 + k] = s.i1[k];
    t.v[39 + k] = s.s1[k];
  }
  for (int k = 0; k < 23; ++k) {
    t.v[52 + k] = kPolyK0[k];
    t.v[75 + k] = kPolyK1[k];
  }
  return t;
}

// c: compile-time constants.  Each passes through an empty asm that takes it in scalar registers,
// so that it is materialised where it is used (scalar moves, issued beside the vector arithmetic)
// rather than hoisted out of the caller's loop into vector registers (98 constants, 196 VGPRs).
__device__ __forceinline__ double sconst(double v) {
  asm volatile("" : "+s"(v));
  return v;
}

template <int N, class C>
__device__ __forceinline__ double horner(C c, int o, double t) {
  double p = c[o + N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) p = fma(p, t, sconst(c[o + k]));
  return p;
}


// c: the coefficient table (make_ktable's order), compile-time constants
template <class C>
__device__ __forceinline__ void bessel_k01_t(double z, double& k0, double& k1, C c) {
  if (z <= 2.0) {
    const double t = 0.25 * z * z;
    const double L = 0.5 * log_pair(t) + kEulerGamma;   // ln(z/2) + gamma
    k0 = fma(-L, horner<13>(c, 0, t), horner<13>(c, 13, t));
    k1 = 1.0 / z + L * (0.5 * z * horner<13>(c, 26, t)) - 0.25 * z * horner<13>(c, 39, t);
  } else {
    const double x = 4.0 / z - 1.0;
    const double e = exp(-z) * rsqrt(z);
    k0 = horner<23>(c, 52, x) * e;
    k1 = horner<23>(c, 75, x) * e;
  }
}

__device__ __forceinline__ void bessel_k01(double z, double& k0, double& k1) {
  constexpr KTable kt = make_ktable();
  bessel_k01_t(z, k0, k1, kt.v);
}

// K0, K1 at two arguments on the same side of z = 2 (else one at a time), with each coefficient
// materialised once for both (the scalar moves of a 64-bit constant, shared by two FMAs, keep the
// vector unit busy: see poly).
__device__ __forceinline__ void bessel_k01_x2(const double (&z)[2], double (&k0)[2], double (&k1)[2]) {
  constexpr KTable kt = make_ktable();
  const bool sa = z[0] <= 2.0, sb = z[1] <= 2.0;
  if (sa != sb) {
    bessel_k01_t(z[0], k0[0], k1[0], kt.v);
    bessel_k01_t(z[1], k0[1], k1[1], kt.v);
    return;
  }
  if (sa) {
    double t[2], i0[2], s0[2], i1[2], s1[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) t[m] = 0.25 * z[m] * z[m];
#pragma unroll
    for (int m = 0; m < 2; ++m) i0[m] = s0[m] = i1[m] = s1[m] = 0.0;
#pragma unroll
    for (int k = 12; k >= 0; --k) {
      const double c0 = sconst(kt.v[k]), c1 = sconst(kt.v[13 + k]), c2 = sconst(kt.v[26 + k]),
                   c3 = sconst(kt.v[39 + k]);
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        i0[m] = fma(i0[m], t[m], c0);
        s0[m] = fma(s0[m], t[m], c1);
        i1[m] = fma(i1[m], t[m], c2);
        s1[m] = fma(s1[m], t[m], c3);
      }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double L = 0.5 * log_pair(t[m]) + kEulerGamma;   // ln(z/2) + gamma
      k0[m] = fma(-L, i0[m], s0[m]);
      k1[m] = 1.0 / z[m] + L * (0.5 * z[m] * i1[m]) - 0.25 * z[m] * s1[m];
    }
  } else {
    double x[2], p0[2], p1[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      x[m] = 4.0 / z[m] - 1.0;
      p0[m] = kt.v[52 + 22];
      p1[m] = kt.v[75 + 22];
    }
#pragma unroll
    for (int k = 21; k >= 0; --k) {
      const double c0 = sconst(kt.v[52 + k]), c1 = sconst(kt.v[75 + k]);
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        p0[m] = fma(p0[m], x[m], c0);
        p1[m] = fma(p1[m], x[m], c1);
      }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const double e = exp(-z[m]) * rsqrt(z[m]);
      k0[m] = p0[m] * e;
      k1[m] = p1[m] * e;
    }
  }
}


// Bessel functions J0, J1, Y0, Y1 of a real argument z > 0 (FP64): the Green's function of
// (a Delta + c) G = delta with c > 0 is the complex G = -(i / 4a) H0(k r), k = sqrt(c / a), with
// H0 = J0 + i Y0 and H0' = -H1 = -(J1 + i Y1).
//  * z <= 8: interpolants of degree 16 in x = z^2 / 32 - 1 of the entire functions J0, J1 / z,
//    S0 = Y0 - (2/pi) ln(z/2) J0 and S1 = (Y1 - (2/pi) ln(z/2) J1 + 2/(pi z)) / z (the power
//    series of Y0 and Y1 split into their log and entire parts);
//  * z > 8: Hankel's form H_nu = sqrt(2/(pi z)) (P_nu + i Q_nu) e^{i chi}, chi = z - nu pi/2 - pi/4,
//    with P_nu, Q_nu as interpolants of degree 14 in x = 16 / z - 1.
// Interpolation at the Chebyshev points at 40 digits, converted to the power form in x
// (bessel_jy_table.py) and evaluated by Horner's rule, one FMA per degree: absolute error below
// 1e-15 for z <= 8, and below 4e-16 times the envelope sqrt(2/(pi z)) beyond (plus the rounding of
// chi for large z).
constexpr double kPolyJ0[17] = {
    4.58296648598137679e-02, 9.30301247295857170e-01, -6.48469283087183657e-01,
    -8.08088807669687159e-01, 1.03837946114372115e+00, -5.07468045847100035e-01,
    1.45988848567592672e-01, -2.84727186108820439e-02, 4.05807898914080541e-03,
    -4.43545922431152020e-04, 3.84731978563400856e-05, -2.71774922362980731e-06,
    1.59561090577813045e-07, -7.91532308447919211e-09, 3.36345045686666908e-10,
    -1.24330113054980572e-11, 4.00304376406281128e-13};
constexpr double kPolyJ1z[17] = {
    -5.81438279559910731e-02, 8.10586603858979571e-02, 1.51516651438066335e-01,
    -2.59594865285930287e-01, 1.58583764327219379e-01, -5.47458182128472207e-02,
    1.24568143922554383e-02, -2.02903949457059959e-03, 2.49494581390904936e-04,
    -2.40457486596869831e-05, 1.86845253720572723e-06, -1.19670818678721719e-07,
    6.43126878575308811e-09, -2.94301379839091608e-10, 1.16105979140429647e-11,
    -4.00457273878614694e-13, 1.20936133963382890e-14};
constexpr double kPolyS0[17] = {
    -3.62027343237145194e-01, -4.17920742320695204e-01, 1.36094565996554562e+00,
    -2.12459994420659437e-01, -6.19340782630335762e-01, 4.48246044635631391e-01,
    -1.54536796523105618e-01, 3.38028569639960627e-02, -5.23502767079865160e-03,
    6.10434564379922656e-04, -5.58183046277945538e-05, 4.12205434835447046e-06,
    -2.51441069429675456e-07, 1.28980708993269862e-08, -5.64627421985713677e-10,
    2.14406072878012710e-11, -7.07204046766636683e-13};
constexpr double kPolyS1[17] = {
    4.51026620686948293e-02, -2.07608578428306018e-01, 9.02275063673093486e-02,
    1.20520354268881608e-01, -1.26419950565698824e-01, 5.43901163079462957e-02,
    -1.41319233942484926e-02, 2.52713404668281549e-03, -3.33722570111453490e-04,
    3.40636337531640451e-05, -2.77650558057605094e-06, 1.85242018405127545e-07,
    -1.03153888256016932e-08, 4.87102079864533318e-10, -1.97641052412663956e-11,
    6.99289828231632531e-13, -2.16103723343110078e-14};
constexpr double kPolyP0[15] = {
    9.99727020301939828e-01, -5.42665503949395678e-04, -2.64866539289064355e-04,
    6.23184838001214216e-06, 1.28155708141464465e-06, -1.44524821291491504e-07,
    -8.80919465124196836e-09, 4.45943034178490071e-09, -3.81665406833019405e-10,
    -1.07890896493245268e-10, 4.10756541653177263e-11, -3.62131059299667937e-12,
    -1.73902812765271616e-12, 6.37411548713499982e-13, -4.39309326982531792e-14};
constexpr double kPolyQ0[15] = {
    -7.79482908425647904e-03, -7.75989659340645989e-03, 5.16021657488700038e-05,
    1.59152491104618754e-05, -8.94214634126615001e-07, -1.15381323682373488e-07,
    2.50981519373035109e-08, -1.94087802054372866e-10, -7.58734439105768389e-10,
    1.43728795502030351e-10, 6.09196974193538222e-12, -9.87165862986276619e-12,
    2.22028605433867113e-12, 2.39896545073495687e-13, -1.98465580381616246e-13};
constexpr double kPolyP1[15] = {
    1.00045560224791075e+00, 9.06956476934860523e-04, 4.45126548017375789e-04,
    -8.07300631462911114e-06, -1.68879546695778430e-06, 1.73280276454166754e-07,
    1.13300715437623104e-08, -5.18167022293861879e-09, 4.11062102139095498e-10,
    1.25818334752817792e-10, -4.55330908338268183e-11, 3.71435715929805041e-12,
    1.96536245438344920e-12, -6.89141700418685567e-13, 4.28804015873852303e-14};
constexpr double kPolyQ1[15] = {
    2.34127237061823069e-02, 2.33636729886258498e-02, -7.25979678504675048e-05,
    -2.26180699758607612e-05, 1.10466539706616358e-06, 1.46908715443831984e-07,
    -2.95134732397787612e-08, 7.78233745253638928e-11, 8.77454843969775786e-10,
    -1.58370507852874116e-10, -8.01147751758117773e-12, 1.09912169075559172e-11,
    -2.38300056190567776e-12, -2.77205766752182690e-13, 2.16277330670697672e-13};

// Horner's rule on compile-time coefficients at M points, each coefficient materialised once at its
// use (sconst) and shared by the M points.  On this hardware a 64-bit constant operand takes two
// scalar moves, and scalar and vector instructions each issue at most once per four cycles per
// SIMD, so one point per coefficient leaves the vector unit half idle; two points balance them.
// (Hoisted out of the caller's loops, the 128 constants of bessel_jy01 would take 256 VGPRs.)
template <int N, int M>
__device__ __forceinline__ void poly(const double (&a)[N], const double (&x)[M], double (&p)[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) p[m] = a[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) {
    const double c = sconst(a[k]);
#pragma unroll
    for (int m = 0; m < M; ++m) p[m] = fma(p[m], x[m], c);
  }
}

// J0, J1, Y0, Y1 at M arguments that lie on the same side of z = 8 (the caller checks).
template <int M>
__device__ __forceinline__ void bessel_jy01_same(const double (&z)[M], bool small, double (&j0)[M],
                                                 double (&j1)[M], double (&y0)[M], double (&y1)[M]) {
  constexpr double k2OverPi = 0.63661977236758134308;   // 2 / pi
  double x[M], a0[M], a1[M], s0[M], s1[M];
  if (small) {
    double w[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      w[m] = z[m] * z[m];
      x[m] = fma(w[m], 1.0 / 32.0, -1.0);
    }
    poly(kPolyJ0, x, a0);
    poly(kPolyJ1z, x, a1);
    poly(kPolyS0, x, s0);
    poly(kPolyS1, x, s1);
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const double L = 0.5 * k2OverPi * log_pair(0.25 * w[m]);   // (2/pi) ln(z/2)
      j0[m] = a0[m];
      j1[m] = z[m] * a1[m];
      y0[m] = fma(L, a0[m], s0[m]);
      y1[m] = fma(L, j1[m], fma(z[m], s1[m], -k2OverPi / z[m]));
    }
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] = 16.0 / z[m] - 1.0;
    poly(kPolyP0, x, a0);   // P0
    poly(kPolyQ0, x, s0);   // Q0
    poly(kPolyP1, x, a1);   // P1
    poly(kPolyQ1, x, s1);   // Q1
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double sn, cs;
      sincos(z[m], &sn, &cs);
      const double env = sqrt(k2OverPi / z[m]);
      const double c0 = (cs + sn) * 0.70710678118654752440;   // cos(z - pi/4)
      const double s0m = (sn - cs) * 0.70710678118654752440;  // sin(z - pi/4)
      // chi_1 = chi_0 - pi/2: cos chi_1 = sin chi_0, sin chi_1 = -cos chi_0
      j0[m] = env * fma(a0[m], c0, -s0[m] * s0m);
      y0[m] = env * fma(a0[m], s0m, s0[m] * c0);
      j1[m] = env * fma(a1[m], s0m, s1[m] * c0);
      y1[m] = env * fma(s1[m], s0m, -a1[m] * c0);
    }
  }
}

__device__ __forceinline__ void bessel_jy01(double z, double& j0, double& j1, double& y0, double& y1) {
  double zz[1] = {z}, a[1], b[1], c[1], d[1];
  bessel_jy01_same<1>(zz, z <= 8.0, a, b, c, d);
  j0 = a[0];
  j1 = b[0];
  y0 = c[0];
  y1 = d[0];
}

// Two arguments at once (the direct sum's pairs of sources): shared coefficients when both lie on
// the same side of z = 8, else one at a time.
__device__ __forceinline__ void bessel_jy01_x2(const double (&z)[2], double (&j0)[2], double (&j1)[2],
                                               double (&y0)[2], double (&y1)[2]) {
  const bool sa = z[0] <= 8.0, sb = z[1] <= 8.0;
  if (sa == sb) {
    bessel_jy01_same<2>(z, sa, j0, j1, y0, y1);
  } else {
    bessel_jy01(z[0], j0[0], j1[0], y0[0], y1[0]);
    bessel_jy01(z[1], j0[1], j1[1], y0[1], y1[1]);
  }
}

// Launch `fn(group, total_blocks)` for the records in chunks of kMaxSeg; segments
// with no blocks are left out.
template <class A, class F>
void launch_grouped(const std::vector<A>& recs, const std::vector<int64_t>& blocks, F fn) {
  Group<A> g;
  int64_t total = 0;
  auto flush = [&]() {
    if (g.n > 0 && total > 0) fn(g, total);
    g = Group<A>();
    total = 0;
  };
  for (size_t k = 0; k < recs.size(); ++k) {
    if (blocks[k] <= 0) continue;
    if (g.n == kMaxSeg) flush();
    g.a[g.n] = recs[k];
    g.off[g.n] = total;
    total += blocks[k];
    g.off[++g.n] = total;
  }
  flush();
}

// Optional per-phase timing with HIP events on the launch stream.
struct Profiler {
  bool on = false;
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    PMX_HIP(hipEventCreate(&e));
    return e;
  }
  int begin(int phase, hipStream_t st) {
    if (!on) return -1;
    Rec r{phase, get(), get()};
    PMX_HIP(hipEventRecord(r.a, st));
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int id, hipStream_t st) {
    if (id >= 0) PMX_HIP(hipEventRecord(recs[id].b, st));
  }
  ~Profiler() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace pmx

// Handles hold references on what they were created from (surface -> context, operator ->
// surface, server -> context), so the caller may destroy handles in any order: a context or
// surface is freed when its own destroy call and the last handle using it have both gone.
// refs counts the caller's handle (1 until its destroy call) plus the dependent handles.
struct pmx_ctx {
  pmx::Ctx c;
  std::atomic<int> refs{1};
  bool owned = true;   // false for a context on the stack (a serving request's accounting)
};

struct pmx_surface {
  pmx_ctx* ctx = nullptr;
  pmx::Geometry g;
  std::atomic<int> refs{1};
};

inline void ctx_retain(pmx_ctx* c) { c->refs.fetch_add(1, std::memory_order_relaxed); }
inline void ctx_release(pmx_ctx* c) {
  if (c->refs.fetch_sub(1, std::memory_order_acq_rel) == 1 && c->owned) delete c;
}
inline void surface_retain(pmx_surface* s) { s->refs.fetch_add(1, std::memory_order_relaxed); }
inline void surface_release(pmx_surface* s) {
  if (s->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) {
    pmx_ctx* c = s->ctx;
    delete s;   // its buffers return their bytes to the context, which is still alive
    ctx_release(c);
  }
}

struct pmx_operator {
  pmx_surface* s = nullptr;
  pmx_options opts{};
  pmx::Coeff co;
  pmx::NearLists nl;
  pmx::FMM* fmm = nullptr;
  double t_setup = 0.0;
  // scratch reused across applies
  pmx::DBuf<double> part;      // far-field partial sums
  pmx::DBuf<double> qt64;      // w sigma / a (FP64)
  pmx::DBuf<float> qt32;       // same in FP32
  pmx::DBuf<double> rows64;    // packed source rows (x, y, z, densities) of the direct sums
  pmx::DBuf<float> rows32;
  pmx::DBuf<double> ssum_part; // partial sums of w sigma
  pmx::DBuf<double> ssum;      // s_r = sum_j w_j sigma_rj
  pmx::DBuf<double> io_a, io_b;  // staging for host arrays
  pmx::Profiler prof;
  const std::atomic<int>* cancel = nullptr;   // set by the server: abandon the solve when nonzero
  struct pmx_batcher* batcher = nullptr;      // set by the server: applies join shared launches
  hipEvent_t ev_ready = nullptr, ev_done = nullptr;   // hand-over events of batched applies
  // second stream of the mixed apply: the near correction and the P2P sums run on it while
  // the FMM's M2L chain runs on the caller's stream (fork after the source preparation,
  // join before L2P); default priority, created on first use
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // c > 0 makes the operator complex: a complex vector of N values is stored as two real
  // columns of N (real parts, then imaginary parts), so n complex vectors are 2 n real columns
  bool cplx() const { return co.complex_; }
  int cols(int n_vec) const { return co.complex_ ? 2 * n_vec : n_vec; }
};

// Boundary curves of an open surface (pmx_edge_create); holds a reference on its context.
struct pmx_edge {
  pmx_ctx* ctx = nullptr;
  pmx::EdgeSet e;
};

namespace pmx {

// Scratch of the FP64 direct apply carved out of memory the caller supplies (the
// allocation-free entry point); every buffer is written before it is read.
struct ApplyScratch {
  double* qt64;    // n_rhs * N: w sigma / a
  double* spart;   // n_rhs * ceil(N / 256): block partials of sum w sigma
  double* ssum;    // n_rhs
  double* rows;    // N * row length: packed source rows
  double* part;    // chunks * n_rhs * N: far-field partial sums
};

// One operator apply y = A sigma of a batch (device arrays).  sc == nullptr: the
// operator's own scratch (sized, and allocated if needed, by the apply).
struct ApplyJob {
  pmx_operator* op;
  const double* sigma;
  double* y;
  const ApplyScratch* sc = nullptr;
};

// geometry.hip
void build_geometry(Ctx* ctx, Geometry& g, const double* x, const double* xu, const double* xv, const double* xuu,
                    const double* xuv, const double* xvv, hipStream_t st);
// c: nullptr for c = 0, else N values, each negative and finite (checked).
void build_coeff(Ctx* ctx, const Geometry& g, Coeff& co, const double* a, const double* grad_a, const double* c,
                 const double* b, hipStream_t st);
void build_near_lists(Ctx* ctx, const Geometry& g, double eta, NearLists& nl, hipStream_t st);
// nearweights.hip
void build_near_weights(Ctx* ctx, const Geometry& g, const Coeff& co, NearLists& nl, const pmx_options& o,
                        bool parametrix, hipStream_t st);
// direct.hip
void far_direct(pmx_operator* op, bool fp64, int n_rhs, hipStream_t st);   // fills op->part + chunk count
int far_direct_chunks(const pmx_operator* op, bool fp64);
// Doubles of scratch the FP64 direct apply of n_rhs densities needs (ApplyScratch, each
// buffer rounded up to 32 doubles).
size_t direct64_scratch_doubles(int64_t N, int n_rhs);
void far_direct_log(pmx_operator* op, int n_rhs, hipStream_t st);          // representation far field (FP64)
// nearapply.hip
void source_prep(pmx_operator* op, const double* sigma, int n_rhs, bool need32, hipStream_t st);
// y = sigma + C sigma + (sum_j w_j sigma_j) + the n_part far-field partials in op->part
// (parametrix: y = D sigma + partials)
void near_combine(pmx_operator* op, const double* sigma, double* y, int n_rhs, int n_part, bool parametrix,
                  hipStream_t st);
void source_prep_batch(const std::vector<ApplyJob>& jobs, int n_rhs, bool need32, hipStream_t st);
void near_combine_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st);   // FP64 direct partials
// c > 0: y += i Ci sigma for the n_cols / 2 complex densities (Di for the parametrix)
void near_cross(pmx_operator* op, const double* sigma, double* y, int n_cols, bool parametrix, hipStream_t st);
// y = sigma + C sigma + (sum_j w_j sigma_j): everything but the far field, which the FMM adds later.
void near_only_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st);
// Builds the by-target-patch view of the near lists (host, once per operator).
void build_near_tiles(Ctx* ctx, const Geometry& g, NearLists& nl, hipStream_t st);
void far_direct64_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st);
void weighted_mean_remove(pmx_operator* op, double* u, int n_rhs, hipStream_t st);
// capi.hip
// One operator apply y = A sigma (device arrays); through the server's batcher when one is set.
void apply_device(pmx_operator* op, int precision, int n_rhs, const double* sigma_d, double* y_d, hipStream_t st);
// Applies of several operators (same precision and n_rhs) whose every kernel is one shared launch.
void apply_batch(const std::vector<ApplyJob>& jobs, int precision, int n_rhs, hipStream_t st);
// Sizes the per-operator scratch of the apply path (no allocation happens in later applies).
void prepare_apply(pmx_operator* op, int precision, int n_rhs, hipStream_t st);
// serve.cpp: hands one apply to the server's batcher, which runs it inside a shared launch
// on its own stream; the caller's stream then waits for that launch.
void batcher_apply(pmx_batcher* b, pmx_operator* op, int precision, int n_rhs, const double* sigma, double* y,
                   hipStream_t st);
void represent_device(pmx_operator* op, int n_rhs, const double* sigma_d, double* u_d, hipStream_t st);
// krylov.hip
struct SolveResult {
  std::vector<int> iters;
  std::vector<double> relres;
  int ir_steps = 0, applies64 = 0, applies_low = 0;
  bool converged = true;
};
SolveResult solve_device(pmx_operator* op, const pmx_options& o, int n_rhs, const double* f_d, double* sigma_d,
                         bool warm, hipStream_t st, std::vector<double>& removed_mean);
// edge.hip
// soa: 13 rows of M values (y, dy/dt, d, a, grad a); validates the fine points (INVALID).
void edge_build(Ctx* ctx, EdgeSet& E, const std::vector<int64_t>& off, const std::vector<double>& soa, int m,
                hipStream_t st);
// y (n_rhs rows of N) = edge operator `kind` (0 K, 1 N, 2 R, 3 T) of mu (n_rhs rows of M), device arrays.
void edge_apply(pmx_operator* op, EdgeSet& E, int kind, int n_rhs, const double* mu, double* y, hipStream_t st);
// y (n_rhs rows of M) = K'_gamma (double_layer false) or D_gamma (true) of mu (n_rhs rows of M) at the
// samples, device arrays.
void edge_apply_on_curve(EdgeSet& E, bool double_layer, int n_rhs, const double* mu, double* y, hipStream_t st);
// fmm.hip
void fmm_build(pmx_operator* op, hipStream_t st);
void fmm_destroy(FMM* f);
// y_r += far field of sigma_r for every job.  After the source permutation of each rhs,
// the P2P sums run on `side` while P2M, M2M, M2L, its slot sum and L2L run on st;
// side_work(side) is called once, before the first P2P launch, and st waits for side
// before each L2P launch (which adds into y), so side_work may write y.  side == st runs
// everything on one stream in the same order (events unused).
void fmm_far_batch(const std::vector<ApplyJob>& jobs, int n_rhs, hipStream_t st, hipStream_t side,
                   hipEvent_t ev_fork, hipEvent_t ev_join, const std::function<void(hipStream_t)>& side_work);
void side_stream(pmx_operator* op);   // creates op->side, op->ev_fork, op->ev_join once
void fmm_reserve(pmx_operator* op, int n_rhs);   // multi-rhs P2P buffers (no-op for one rhs)
void fmm_stats(const FMM* f, pmx_operator_stats* s);
uint64_t fmm_bytes(const FMM* f);

double now_seconds();
void gauss_legendre_host(int n, double* t, double* w);
void lagrange_host(int q, const double* t, double s, double* out);

}  // namespace pmx
