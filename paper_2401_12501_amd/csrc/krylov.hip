// GMRES (Saad-Schultz) on the Nystrom system and mixed-precision iterative refinement.
//
// The paper solves the discretized eq:IE with GMRES (Section 6, Section 7).
// Here the Krylov basis stays in device memory (FP64); each Arnoldi step is one
// batched operator apply for all right-hand sides, two classical Gram-Schmidt
// passes (CGS2) and a normalisation.  Dot products are reduced in a fixed order,
// so the iteration is deterministic.  The host keeps the small Hessenberg
// matrices and applies Givens rotations; per step it reads back (j+1)*2 + 1
// numbers per right-hand side.
//
// Mixed path: sigma_0 = 0 (or a warm start); r_k = f - A64 sigma_k with the FP64
// direct operator; stop when ||r_k|| <= ir_tol ||f||; else d = GMRES(A32, r_k) to
// the relative tolerance inner_tol with the FP32 far field, sigma_{k+1} = sigma_k + d.
#include <cmath>
#include <complex>

#include "pmx_internal.hpp"

namespace pmx {

namespace {
constexpr int kBlock = 256;
constexpr int kPer = 2;   // elements per thread in the dot kernels

// partial[r][k][b] = sum over block b's elements of V[k][r][.] * w[r][.].  SWAP (complex vectors of
// hN values stored as real parts then imaginary parts, N = 2 hN): w is read as (Im w, -Re w), so the
// sum is Im <V_k, w> = sum (Re v Im w - Im v Re w); the plain sum is Re <V_k, w>.
template <bool SWAP>
__global__ void __launch_bounds__(kBlock) k_multidot(int64_t N, int n_rhs, int nk, const double* __restrict__ V,
                                                     int64_t ldk, const double* __restrict__ w,
                                                     double* __restrict__ part, int64_t hN) {
  const int r = blockIdx.y;
  const int64_t base = (int64_t)blockIdx.x * kBlock * kPer;
  double wv[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int64_t i = base + t * kBlock + threadIdx.x;
    if (!SWAP) wv[t] = i < N ? w[(int64_t)r * N + i] : 0.0;
    else wv[t] = i < N ? (i < hN ? w[(int64_t)r * N + i + hN] : -w[(int64_t)r * N + i - hN]) : 0.0;
  }
  __shared__ double red[kBlock / 64];
  for (int k = 0; k < nk; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int64_t i = base + t * kBlock + threadIdx.x;
      if (i < N) acc = fma(V[k * ldk + (int64_t)r * N + i], wv[t], acc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int t = 0; t < kBlock / 64; ++t) s += red[t];
      part[((int64_t)r * nk + k) * gridDim.x + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[r][k] = sum_b part[r][k][b] (one block per (k, r), fixed order)
__global__ void __launch_bounds__(kBlock) k_reduce_parts(int64_t nb, int nk, const double* __restrict__ part,
                                                         double* __restrict__ out) {
  const int k = blockIdx.x, r = blockIdx.y;
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kBlock) acc += part[((int64_t)r * nk + k) * nb + b];
  __shared__ double red[kBlock];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)r * nk + k] = red[0];
}

// w[r] += sign * sum_k V[k][r] c[r][k]
__global__ void __launch_bounds__(kBlock) k_gemv(int64_t N, int nk, const double* __restrict__ V, int64_t ldk,
                                                 const double* __restrict__ c, double sign, double* __restrict__ w) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int k = 0; k < nk; ++k) acc = fma(V[k * ldk + (int64_t)r * N + i], c[(int64_t)r * nk + k], acc);
  w[(int64_t)r * N + i] += sign * acc;
}

// Complex vectors (hN values, real parts then imaginary parts): w[r] += sign * sum_k c[r][k] V[k][r] with
// complex c (real parts cr, imaginary parts ci), i.e. cr V + ci J V with J v = (-Im v, Re v).
__global__ void __launch_bounds__(kBlock) k_gemv_c(int64_t N, int64_t hN, int nk, const double* __restrict__ V,
                                                   int64_t ldk, const double* __restrict__ cr,
                                                   const double* __restrict__ ci, double sign,
                                                   double* __restrict__ w) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const int64_t j = i < hN ? i + hN : i - hN;
  const double sj = i < hN ? -1.0 : 1.0;
  double acc = 0.0;
  for (int k = 0; k < nk; ++k) {
    const double* v = V + k * ldk + (int64_t)r * N;
    acc = fma(v[i], cr[(int64_t)r * nk + k], acc);
    acc = fma(sj * v[j], ci[(int64_t)r * nk + k], acc);
  }
  w[(int64_t)r * N + i] += sign * acc;
}

// v[r] = w[r] / sqrt(nrm2[r]) (zero if the norm vanishes)
__global__ void k_scale_inv_norm(int64_t N, const double* __restrict__ w, const double* __restrict__ nrm2,
                                 double* __restrict__ v) {
  const int r = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const double nn = nrm2[r];
  v[(int64_t)r * N + i] = nn > 0.0 ? w[(int64_t)r * N + i] / sqrt(nn) : 0.0;
}

// y = a - b (elementwise)
__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = a[i] - b[i];
}

__global__ void k_add(int64_t n, const double* __restrict__ a, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] += a[i];
}

struct Dots {
  int64_t N;
  int n_rhs;
  int64_t nb;
  DBuf<double> part, out;
  void init(Ctx* ctx, int64_t N_, int n_rhs_, int max_k) {
    N = N_;
    n_rhs = n_rhs_;
    nb = (N + kBlock * kPer - 1) / (kBlock * kPer);
    part.alloc(ctx, (size_t)n_rhs * max_k * nb);
    out.alloc(ctx, (size_t)n_rhs * max_k);
  }
  // out[r][k] = V[k][r] . w[r], k < nk; swap_half > 0: the imaginary parts of the complex products
  // <V[k][r], w[r]> of vectors with swap_half values each (k_multidot<true>)
  void run(const double* V, int64_t ldk, int nk, const double* w, double* dst, hipStream_t st,
           int64_t swap_half = 0) {
    if (swap_half > 0)
      hipLaunchKernelGGL(k_multidot<true>, dim3(nb, n_rhs), dim3(kBlock), 0, st, N, n_rhs, nk, V, ldk, w, part.p,
                         swap_half);
    else
      hipLaunchKernelGGL(k_multidot<false>, dim3(nb, n_rhs), dim3(kBlock), 0, st, N, n_rhs, nk, V, ldk, w, part.p,
                         (int64_t)0);
    PMX_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_parts, dim3(nk, n_rhs), dim3(kBlock), 0, st, nb, nk, part.p, dst);
    PMX_HIP(hipGetLastError());
  }
};

inline dim3 grid_n(int64_t N, int n_rhs) { return dim3((unsigned)((N + kBlock - 1) / kBlock), (unsigned)n_rhs); }

// Norms ||v_r||_2 for n_rhs vectors (host result).
std::vector<double> norms(Dots& D, const double* v, hipStream_t st) {
  D.run(v, 0, 1, v, D.out.p, st);
  std::vector<double> h(D.n_rhs);
  PMX_HIP(hipMemcpyAsync(h.data(), D.out.p, D.n_rhs * sizeof(double), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  for (auto& x : h) x = std::sqrt(x);
  return h;
}

struct GmresOut {
  std::vector<int> iters;
  std::vector<double> est;   // final relative residual estimate per rhs
  int applies = 0;
  bool converged = true;
};

// GMRES for a complex operator (c > 0): the same lockstep restarted GMRES(m) with complex arithmetic.
// Vectors hold N complex values as 2N reals (real parts, then imaginary parts); inner products are
// the Hermitian <v, w> = sum conj(v) w (real parts by the plain dot of the 2N reals, imaginary parts
// by the swapped dot), the basis update takes complex coefficients (k_gemv_c), and the host applies
// complex Givens rotations to the complex Hessenberg matrix.  It needs fewer steps than GMRES on the
// equivalent real system of size 2N, whose Krylov space grows by one real dimension per step.
GmresOut gmres_complex(pmx_operator* op, int precision, int n_rhs, const double* b, double* x, bool x_zero,
                       double tol, int m, int max_iter, hipStream_t st) {
  typedef std::complex<double> cd;
  Ctx* ctx = &op->s->ctx->c;
  const int64_t hN = op->s->g.N;
  const int64_t N = 2 * hN;
  const int nc = op->cols(n_rhs);
  const int64_t ldk = (int64_t)n_rhs * N;
  DBuf<double> V, W;
  V.alloc(ctx, (size_t)(m + 1) * ldk);
  W.alloc(ctx, (size_t)ldk);
  Dots D;
  D.init(ctx, N, n_rhs, m + 1);
  DBuf<double> h1r, h1i, h2r, h2i, nn, yr, yi;
  for (DBuf<double>* d : {&h1r, &h1i, &h2r, &h2i}) d->alloc(ctx, (size_t)n_rhs * (m + 1));
  nn.alloc(ctx, n_rhs);
  yr.alloc(ctx, (size_t)n_rhs * m);
  yi.alloc(ctx, (size_t)n_rhs * m);
  GmresOut res;
  res.iters.assign(n_rhs, 0);
  res.est.assign(n_rhs, 1.0);
  if (x_zero) PMX_HIP(hipMemsetAsync(x, 0, ldk * sizeof(double), st));
  std::vector<double> bnorm = norms(D, b, st);
  for (auto& v : bnorm)
    if (v == 0.0) v = 1.0;
  std::vector<char> done(n_rhs, 0);
  int total = 0;
  const dim3 gN = grid_n(N, n_rhs);
  const dim3 g1((unsigned)((ldk + kBlock - 1) / kBlock));
  while (true) {
    if (x_zero && total == 0) {
      PMX_HIP(hipMemcpyAsync(W.p, b, ldk * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
      apply_device(op, precision, nc, x, W.p, st);
      res.applies++;
      hipLaunchKernelGGL(k_sub, g1, dim3(kBlock), 0, st, ldk, b, W.p, W.p);
      PMX_HIP(hipGetLastError());
    }
    D.run(W.p, 0, 1, W.p, nn.p, st);
    hipLaunchKernelGGL(k_scale_inv_norm, gN, dim3(kBlock), 0, st, N, W.p, nn.p, V.p);
    PMX_HIP(hipGetLastError());
    std::vector<double> beta(n_rhs);
    PMX_HIP(hipMemcpyAsync(beta.data(), nn.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
    bool all_done = true;
    for (int r = 0; r < n_rhs; ++r) {
      beta[r] = std::sqrt(beta[r]);
      res.est[r] = beta[r] / bnorm[r];
      done[r] = res.est[r] <= tol;
      all_done = all_done && done[r];
    }
    if (all_done || total >= max_iter) {
      res.converged = all_done;
      break;
    }
    std::vector<std::vector<cd>> H(n_rhs, std::vector<cd>((size_t)(m + 1) * m, cd(0.0)));
    std::vector<std::vector<double>> cs(n_rhs, std::vector<double>(m));
    std::vector<std::vector<cd>> sn(n_rhs, std::vector<cd>(m)), g(n_rhs, std::vector<cd>(m + 1, cd(0.0)));
    for (int r = 0; r < n_rhs; ++r) g[r][0] = beta[r];
    int j = 0;
    const size_t nh = (size_t)n_rhs * (m + 1);
    std::vector<double> a1r(nh), a1i(nh), a2r(nh), a2i(nh), hn(n_rhs);
    for (; j < m && total < max_iter; ++j) {
      if (op->cancel && op->cancel->load()) throw Error(PMX_ERR_CANCELLED, "solve cancelled");
      apply_device(op, precision, nc, V.p + (int64_t)j * ldk, W.p, st);
      res.applies++;
      const int nk = j + 1;
      // classical Gram-Schmidt twice with Hermitian products
      D.run(V.p, ldk, nk, W.p, h1r.p, st);
      D.run(V.p, ldk, nk, W.p, h1i.p, st, hN);
      hipLaunchKernelGGL(k_gemv_c, gN, dim3(kBlock), 0, st, N, hN, nk, V.p, ldk, h1r.p, h1i.p, -1.0, W.p);
      PMX_HIP(hipGetLastError());
      D.run(V.p, ldk, nk, W.p, h2r.p, st);
      D.run(V.p, ldk, nk, W.p, h2i.p, st, hN);
      hipLaunchKernelGGL(k_gemv_c, gN, dim3(kBlock), 0, st, N, hN, nk, V.p, ldk, h2r.p, h2i.p, -1.0, W.p);
      PMX_HIP(hipGetLastError());
      D.run(W.p, 0, 1, W.p, nn.p, st);
      hipLaunchKernelGGL(k_scale_inv_norm, gN, dim3(kBlock), 0, st, N, W.p, nn.p, V.p + (int64_t)(j + 1) * ldk);
      PMX_HIP(hipGetLastError());
      const size_t nb = (size_t)n_rhs * nk * sizeof(double);
      PMX_HIP(hipMemcpyAsync(a1r.data(), h1r.p, nb, hipMemcpyDeviceToHost, st));
      PMX_HIP(hipMemcpyAsync(a1i.data(), h1i.p, nb, hipMemcpyDeviceToHost, st));
      PMX_HIP(hipMemcpyAsync(a2r.data(), h2r.p, nb, hipMemcpyDeviceToHost, st));
      PMX_HIP(hipMemcpyAsync(a2i.data(), h2i.p, nb, hipMemcpyDeviceToHost, st));
      PMX_HIP(hipMemcpyAsync(hn.data(), nn.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, st));
      PMX_HIP(hipStreamSynchronize(st));
      ++total;
      bool all = true;
      for (int r = 0; r < n_rhs; ++r) {
        cd* col = H[r].data() + (size_t)j * (m + 1);
        for (int k = 0; k < nk; ++k) {
          const size_t e = (size_t)r * nk + k;
          col[k] = cd(a1r[e] + a2r[e], a1i[e] + a2i[e]);
        }
        col[j + 1] = cd(std::sqrt(hn[r]), 0.0);
        // earlier rotations: (x, y) -> (c x + s y, -conj(s) x + c y)
        for (int k = 0; k < j; ++k) {
          const cd t = cs[r][k] * col[k] + sn[r][k] * col[k + 1];
          col[k + 1] = -std::conj(sn[r][k]) * col[k] + cs[r][k] * col[k + 1];
          col[k] = t;
        }
        // the rotation that zeroes col[j + 1]
        const cd a = col[j], bb = col[j + 1];
        const double den = std::sqrt(std::norm(a) + std::norm(bb));
        if (den > 0.0) {
          const double aa = std::abs(a);
          cs[r][j] = aa / den;
          sn[r][j] = aa > 0.0 ? (a / aa) * std::conj(bb) / den : cd(1.0, 0.0);
        } else {
          cs[r][j] = 1.0;
          sn[r][j] = cd(0.0);
        }
        col[j] = cs[r][j] * a + sn[r][j] * bb;
        col[j + 1] = cd(0.0);
        g[r][j + 1] = -std::conj(sn[r][j]) * g[r][j];
        g[r][j] = cs[r][j] * g[r][j];
        if (!done[r]) res.iters[r]++;
        res.est[r] = std::abs(g[r][j + 1]) / bnorm[r];
        if (res.est[r] <= tol) done[r] = 1;
        all = all && done[r];
      }
      if (all) {
        ++j;
        break;
      }
    }
    // x += V y with H(1:j,1:j) y = g(1:j)
    std::vector<double> ywr((size_t)n_rhs * j, 0.0), ywi((size_t)n_rhs * j, 0.0);
    for (int r = 0; r < n_rhs; ++r) {
      std::vector<cd> y(j);
      for (int k = j - 1; k >= 0; --k) {
        cd sum = g[r][k];
        for (int c = k + 1; c < j; ++c) sum -= H[r][(size_t)c * (m + 1) + k] * y[c];
        const cd d = H[r][(size_t)k * (m + 1) + k];
        y[k] = std::abs(d) != 0.0 ? sum / d : cd(0.0);
      }
      for (int k = 0; k < j; ++k) {
        ywr[(size_t)r * j + k] = y[k].real();
        ywi[(size_t)r * j + k] = y[k].imag();
      }
    }
    if (j > 0) {
      PMX_HIP(hipMemcpyAsync(yr.p, ywr.data(), ywr.size() * sizeof(double), hipMemcpyHostToDevice, st));
      PMX_HIP(hipMemcpyAsync(yi.p, ywi.data(), ywi.size() * sizeof(double), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_gemv_c, gN, dim3(kBlock), 0, st, N, hN, j, V.p, ldk, yr.p, yi.p, 1.0, x);
      PMX_HIP(hipGetLastError());
      PMX_HIP(hipStreamSynchronize(st));   // the coefficients live on the host stack
    }
    x_zero = false;
    bool all = true;
    for (int r = 0; r < n_rhs; ++r) all = all && done[r];
    if (all) {
      res.converged = true;
      break;
    }
  }
  return res;
}

// Solve A x = b (n_rhs systems, lockstep) from the initial x; restarted GMRES(m).
GmresOut gmres(pmx_operator* op, int precision, int n_rhs, const double* b, double* x, bool x_zero, double tol,
               int m, int max_iter, hipStream_t st) {
  if (op->cplx()) return gmres_complex(op, precision, n_rhs, b, x, x_zero, tol, m, max_iter, st);
  Ctx* ctx = &op->s->ctx->c;
  const int64_t N = op->s->g.N;
  const int nc = op->cols(n_rhs);   // real columns of N nodes per apply
  const int64_t ldk = (int64_t)n_rhs * N;
  DBuf<double> V, W;
  V.alloc(ctx, (size_t)(m + 1) * ldk);
  W.alloc(ctx, (size_t)ldk);
  Dots D;
  D.init(ctx, N, n_rhs, m + 1);
  DBuf<double> h1, h2, nn;
  h1.alloc(ctx, (size_t)n_rhs * (m + 1));
  h2.alloc(ctx, (size_t)n_rhs * (m + 1));
  nn.alloc(ctx, n_rhs);
  DBuf<double> ydev;
  ydev.alloc(ctx, (size_t)n_rhs * m);
  GmresOut res;
  res.iters.assign(n_rhs, 0);
  res.est.assign(n_rhs, 1.0);

  // a zero initial guess is taken literally: x is cleared, not assumed clear
  if (x_zero) PMX_HIP(hipMemsetAsync(x, 0, ldk * sizeof(double), st));
  std::vector<double> bnorm = norms(D, b, st);
  for (auto& v : bnorm)
    if (v == 0.0) v = 1.0;
  std::vector<char> done(n_rhs, 0);
  int total = 0;
  const dim3 gN = grid_n(N, n_rhs);
  const dim3 g1((unsigned)((ldk + kBlock - 1) / kBlock));
  while (true) {
    // r0 = b - A x  -> V[0] (unnormalised) in W
    if (x_zero && total == 0) {
      PMX_HIP(hipMemcpyAsync(W.p, b, ldk * sizeof(double), hipMemcpyDeviceToDevice, st));
    } else {
      apply_device(op, precision, nc, x, W.p, st);
      res.applies++;
      hipLaunchKernelGGL(k_sub, g1, dim3(kBlock), 0, st, ldk, b, W.p, W.p);
      PMX_HIP(hipGetLastError());
    }
    D.run(W.p, 0, 1, W.p, nn.p, st);
    hipLaunchKernelGGL(k_scale_inv_norm, gN, dim3(kBlock), 0, st, N, W.p, nn.p, V.p);
    PMX_HIP(hipGetLastError());
    std::vector<double> beta(n_rhs);
    PMX_HIP(hipMemcpyAsync(beta.data(), nn.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
    bool all_done = true;
    for (int r = 0; r < n_rhs; ++r) {
      beta[r] = std::sqrt(beta[r]);
      res.est[r] = beta[r] / bnorm[r];
      done[r] = res.est[r] <= tol;
      all_done = all_done && done[r];
    }
    if (all_done || total >= max_iter) {
      res.converged = all_done;
      break;
    }
    // Arnoldi with Givens rotations (column-major Hessenberg per rhs)
    std::vector<std::vector<double>> H(n_rhs, std::vector<double>((size_t)(m + 1) * m, 0.0));
    std::vector<std::vector<double>> cs(n_rhs, std::vector<double>(m)), sn(n_rhs, std::vector<double>(m));
    std::vector<std::vector<double>> g(n_rhs, std::vector<double>(m + 1, 0.0));
    for (int r = 0; r < n_rhs; ++r) g[r][0] = beta[r];
    int j = 0;
    std::vector<double> hh1((size_t)n_rhs * (m + 1)), hh2((size_t)n_rhs * (m + 1)), hn(n_rhs);
    for (; j < m && total < max_iter; ++j) {
      if (op->cancel && op->cancel->load()) throw Error(PMX_ERR_CANCELLED, "solve cancelled");
      apply_device(op, precision, nc, V.p + (int64_t)j * ldk, W.p, st);
      res.applies++;
      const int nk = j + 1;
      D.run(V.p, ldk, nk, W.p, h1.p, st);
      hipLaunchKernelGGL(k_gemv, gN, dim3(kBlock), 0, st, N, nk, V.p, ldk, h1.p, -1.0, W.p);
      PMX_HIP(hipGetLastError());
      D.run(V.p, ldk, nk, W.p, h2.p, st);
      hipLaunchKernelGGL(k_gemv, gN, dim3(kBlock), 0, st, N, nk, V.p, ldk, h2.p, -1.0, W.p);
      PMX_HIP(hipGetLastError());
      D.run(W.p, 0, 1, W.p, nn.p, st);
      hipLaunchKernelGGL(k_scale_inv_norm, gN, dim3(kBlock), 0, st, N, W.p, nn.p, V.p + (int64_t)(j + 1) * ldk);
      PMX_HIP(hipGetLastError());
      PMX_HIP(hipMemcpyAsync(hh1.data(), h1.p, (size_t)n_rhs * nk * sizeof(double), hipMemcpyDeviceToHost, st));
      PMX_HIP(hipMemcpyAsync(hh2.data(), h2.p, (size_t)n_rhs * nk * sizeof(double), hipMemcpyDeviceToHost, st));
      PMX_HIP(hipMemcpyAsync(hn.data(), nn.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, st));
      PMX_HIP(hipStreamSynchronize(st));
      ++total;
      bool all = true;
      for (int r = 0; r < n_rhs; ++r) {
        double* col = H[r].data() + (size_t)j * (m + 1);
        for (int k = 0; k < nk; ++k) col[k] = hh1[(size_t)r * nk + k] + hh2[(size_t)r * nk + k];
        col[j + 1] = std::sqrt(hn[r]);
        for (int k = 0; k < j; ++k) {
          const double t = cs[r][k] * col[k] + sn[r][k] * col[k + 1];
          col[k + 1] = -sn[r][k] * col[k] + cs[r][k] * col[k + 1];
          col[k] = t;
        }
        const double a = col[j], bb = col[j + 1];
        const double den = std::hypot(a, bb);
        cs[r][j] = den > 0 ? a / den : 1.0;
        sn[r][j] = den > 0 ? bb / den : 0.0;
        col[j] = den;
        col[j + 1] = 0.0;
        g[r][j + 1] = -sn[r][j] * g[r][j];
        g[r][j] = cs[r][j] * g[r][j];
        if (!done[r]) res.iters[r]++;
        res.est[r] = std::fabs(g[r][j + 1]) / bnorm[r];
        if (res.est[r] <= tol) done[r] = 1;
        all = all && done[r];
      }
      if (all) {
        ++j;
        break;
      }
    }
    // x += V y with H(1:j,1:j) y = g(1:j)
    std::vector<double> y((size_t)n_rhs * j, 0.0);
    for (int r = 0; r < n_rhs; ++r) {
      for (int k = j - 1; k >= 0; --k) {
        double s = g[r][k];
        for (int c = k + 1; c < j; ++c) s -= H[r][(size_t)c * (m + 1) + k] * y[(size_t)r * j + c];
        const double d = H[r][(size_t)k * (m + 1) + k];
        y[(size_t)r * j + k] = d != 0.0 ? s / d : 0.0;
      }
    }
    if (j > 0) {
      PMX_HIP(hipMemcpyAsync(ydev.p, y.data(), y.size() * sizeof(double), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_gemv, gN, dim3(kBlock), 0, st, N, j, V.p, ldk, ydev.p, 1.0, x);
      PMX_HIP(hipGetLastError());
      PMX_HIP(hipStreamSynchronize(st));   // y lives on the host stack
    }
    x_zero = false;
    bool all = true;
    for (int r = 0; r < n_rhs; ++r) all = all && done[r];
    if (all) {
      // confirm with the true residual at the top of the loop only when restarting;
      // here the Arnoldi estimate is exact in exact arithmetic
      res.converged = true;
      break;
    }
  }
  return res;
}
}  // namespace

SolveResult solve_device(pmx_operator* op, const pmx_options& o, int n_rhs, const double* f_in, double* sigma,
                         bool warm, hipStream_t st, std::vector<double>& removed_mean) {
  Ctx* ctx = &op->s->ctx->c;
  const int64_t N = op->cplx() ? 2 * op->s->g.N : op->s->g.N;   // vector length (complex: 2N reals)
  const int nc = op->cols(n_rhs);
  const int64_t ld = (int64_t)n_rhs * N;
  SolveResult out;
  out.iters.assign(n_rhs, 0);
  out.relres.assign(n_rhs, 0.0);
  // f projected to mean zero (the c = 0 problem needs mean-zero data)
  DBuf<double> f, r;
  f.alloc(ctx, ld);
  r.alloc(ctx, ld);
  PMX_HIP(hipMemcpyAsync(f.p, f_in, ld * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (op->co.has_c()) {
    removed_mean.assign(n_rhs, 0.0);   // c != 0: no null space, f is used as given
  } else {
    // removed mean = (sum w f) / area, computed by weighted_mean_remove on a copy
    PMX_HIP(hipMemcpyAsync(r.p, f.p, ld * sizeof(double), hipMemcpyDeviceToDevice, st));
    weighted_mean_remove(op, f.p, n_rhs, st);
    const dim3 g1((unsigned)((ld + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_sub, g1, dim3(kBlock), 0, st, ld, r.p, f.p, r.p);   // r = f_in - f_z = mean
    PMX_HIP(hipGetLastError());
    removed_mean.assign(n_rhs, 0.0);
    for (int k = 0; k < n_rhs; ++k)
      PMX_HIP(hipMemcpyAsync(&removed_mean[k], r.p + (int64_t)k * N, sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
  }
  if (!warm) PMX_HIP(hipMemsetAsync(sigma, 0, ld * sizeof(double), st));
  Dots D;
  D.init(ctx, N, n_rhs, 1);
  const std::vector<double> fn = norms(D, f.p, st);
  const dim3 g1((unsigned)((ld + kBlock - 1) / kBlock));

  if (o.precision == PMX_PREC_FP64_DIRECT || o.precision == PMX_PREC_FP32_DIRECT) {
    GmresOut g = gmres(op, o.precision, n_rhs, f.p, sigma, !warm, o.gmres_tol, o.gmres_restart, o.max_iter, st);
    if (o.precision == PMX_PREC_FP64_DIRECT) out.applies64 += g.applies; else out.applies_low += g.applies;
    out.iters = g.iters;
    out.converged = g.converged;
  } else {
    // iterative refinement: residuals with A64, corrections with A32; the loop ends
    // with r = f - A64 sigma for the returned sigma, so no extra apply is needed
    DBuf<double> d;
    d.alloc(ctx, ld);
    for (int k = 0;; ++k) {
      if (k == 0 && !warm) {
        PMX_HIP(hipMemcpyAsync(r.p, f.p, ld * sizeof(double), hipMemcpyDeviceToDevice, st));
      } else {
        apply_device(op, PMX_PREC_FP64_DIRECT, nc, sigma, r.p, st);
        out.applies64++;
        hipLaunchKernelGGL(k_sub, g1, dim3(kBlock), 0, st, ld, f.p, r.p, r.p);
        PMX_HIP(hipGetLastError());
      }
      const std::vector<double> rn = norms(D, r.p, st);
      bool all = true;
      for (int q = 0; q < n_rhs; ++q) {
        out.relres[q] = rn[q] / (fn[q] > 0 ? fn[q] : 1.0);
        all = all && out.relres[q] <= o.ir_tol;
      }
      if (all) break;
      if (k >= o.max_ir) {
        out.converged = false;
        break;
      }
      GmresOut g = gmres(op, PMX_PREC_MIXED_FMM, n_rhs, r.p, d.p, true, o.inner_tol, o.gmres_restart,
                         o.max_iter, st);
      out.applies_low += g.applies;
      for (int q = 0; q < n_rhs; ++q) out.iters[q] += g.iters[q];
      hipLaunchKernelGGL(k_add, g1, dim3(kBlock), 0, st, ld, d.p, sigma);
      PMX_HIP(hipGetLastError());
      out.ir_steps++;
    }
    return out;
  }
  // FP64 / FP32 path: report the true residual with the FP64 operator
  apply_device(op, PMX_PREC_FP64_DIRECT, nc, sigma, r.p, st);
  out.applies64++;
  hipLaunchKernelGGL(k_sub, g1, dim3(kBlock), 0, st, ld, f.p, r.p, r.p);
  PMX_HIP(hipGetLastError());
  const std::vector<double> rn = norms(D, r.p, st);
  for (int q = 0; q < n_rhs; ++q) out.relres[q] = rn[q] / (fn[q] > 0 ? fn[q] : 1.0);
  return out;
}

}  // namespace pmx
