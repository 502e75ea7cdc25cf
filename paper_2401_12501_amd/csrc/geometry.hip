// Surface geometry, coefficient factors and near lists (FP64).
//
// Node geometry (Section 2.2): unit normal n = x_u x x_v / |x_u x x_v|, area
// element J = sqrt(det g) = |x_u x x_v|, mean curvature H = (1/2) div_G n for the
// outward normal, H = -(e G - 2 f F + g E) / (2 (E G - F^2)) with the first (E, F,
// G) and second (e, f, g) fundamental forms.  Nystrom weight w = w_a w_b J
// (Section 6.1).  Patch centroid = mean of the four corner images, radius = the
// largest centroid-corner distance; a target is near a patch when it lies
// within eta radii of the centroid (Section 6.1.2), and always near its own.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "pmx_internal.hpp"

namespace pmx {

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n (host, FP64).
void gauss_legendre_host(int n, double* t, double* w) {
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = x; p0 = 1.0; }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) {
        // one more pass to settle the derivative at the converged root
        p0 = 1.0; p1 = x;
        for (int k = 2; k <= n; ++k) {
          double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1; p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        break;
      }
    }
    t[n - 1 - i] = x;   // increasing order
    w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
}

// Lagrange basis values l_j(s) for nodes t (product form, no division by s - t_j).
void lagrange_host(int q, const double* t, double s, double* out) {
  for (int j = 0; j < q; ++j) {
    double v = 1.0;
    for (int k = 0; k < q; ++k)
      if (k != j) v *= (s - t[k]) / (t[j] - t[k]);
    out[j] = v;
  }
}

__global__ void k_geometry(int64_t N, int q, const double* __restrict__ x, const double* __restrict__ xu,
                           const double* __restrict__ xv, const double* __restrict__ xuu,
                           const double* __restrict__ xuv, const double* __restrict__ xvv,
                           const double* __restrict__ wgl, double* __restrict__ X, double* __restrict__ Nn,
                           double* __restrict__ J, double* __restrict__ W, double* __restrict__ H,
                           double* __restrict__ XU, double* __restrict__ XV, double* __restrict__ red,
                           int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double wn_dot_x = 0.0, wsum = 0.0;
  if (i < N) {
    double au = xu[3 * i], bu = xu[3 * i + 1], cu = xu[3 * i + 2];
    double av = xv[3 * i], bv = xv[3 * i + 1], cv = xv[3 * i + 2];
    double c0 = bu * cv - cu * bv, c1 = cu * av - au * cv, c2 = au * bv - bu * av;
    double jac = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    double n0 = c0 / jac, n1 = c1 / jac, n2 = c2 / jac;
    double E = au * au + bu * bu + cu * cu;
    double F = au * av + bu * bv + cu * cv;
    double G = av * av + bv * bv + cv * cv;
    double e = xuu[3 * i] * n0 + xuu[3 * i + 1] * n1 + xuu[3 * i + 2] * n2;
    double f = xuv[3 * i] * n0 + xuv[3 * i + 1] * n1 + xuv[3 * i + 2] * n2;
    double g = xvv[3 * i] * n0 + xvv[3 * i + 1] * n1 + xvv[3 * i + 2] * n2;
    double h = -(e * G - 2.0 * f * F + g * E) / (2.0 * (E * G - F * F));
    int loc = (int)(i % (q * q));
    double wi = wgl[loc / q] * wgl[loc % q] * jac;
    double px = x[3 * i], py = x[3 * i + 1], pz = x[3 * i + 2];
    if (!(jac > 0.0) || !isfinite(h) || !isfinite(px) || !isfinite(py) || !isfinite(pz)) atomicOr(bad, 1);
    X[i] = px; X[N + i] = py; X[2 * N + i] = pz;
    Nn[i] = n0; Nn[N + i] = n1; Nn[2 * N + i] = n2;
    J[i] = jac; W[i] = wi; H[i] = h;
    XU[i] = au; XU[N + i] = bu; XU[2 * N + i] = cu;
    XV[i] = av; XV[N + i] = bv; XV[2 * N + i] = cv;
    wn_dot_x = wi * (n0 * px + n1 * py + n2 * pz);
    wsum = wi;
  }
  // block partial sums (fixed order tree) of sum w n.x and sum w
  __shared__ double s0[256], s1[256];
  s0[threadIdx.x] = wn_dot_x;
  s1[threadIdx.x] = wsum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = s0[0];
    red[2 * blockIdx.x + 1] = s1[0];
  }
}

// Corner images (Lagrange at +-1), centroid and radius of every patch.
__global__ void k_patch_bounds(int64_t M, int q, const double* __restrict__ X, int64_t N,
                               const double* __restrict__ Lm, const double* __restrict__ Lp,
                               double* __restrict__ corner, double* __restrict__ cent) {
  int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= M) return;
  const int q2 = q * q;
  double cx[4], cy[4], cz[4];
  for (int k = 0; k < 4; ++k) {
    const double* Lu = (k == 1 || k == 2) ? Lp : Lm;   // corners (-1,-1) (1,-1) (1,1) (-1,1)
    const double* Lv = (k >= 2) ? Lp : Lm;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int a = 0; a < q; ++a) {
      double tx = 0.0, ty = 0.0, tz = 0.0;
      for (int b = 0; b < q; ++b) {
        int64_t j = P * q2 + a * q + b;
        tx += Lv[b] * X[j];
        ty += Lv[b] * X[N + j];
        tz += Lv[b] * X[2 * N + j];
      }
      sx += Lu[a] * tx; sy += Lu[a] * ty; sz += Lu[a] * tz;
    }
    cx[k] = sx; cy[k] = sy; cz[k] = sz;
    corner[P * 12 + 3 * k] = sx;
    corner[P * 12 + 3 * k + 1] = sy;
    corner[P * 12 + 3 * k + 2] = sz;
  }
  double mx = 0.25 * (cx[0] + cx[1] + cx[2] + cx[3]);
  double my = 0.25 * (cy[0] + cy[1] + cy[2] + cy[3]);
  double mz = 0.25 * (cz[0] + cz[1] + cz[2] + cz[3]);
  double rad = 0.0;
  for (int k = 0; k < 4; ++k) {
    double dx = cx[k] - mx, dy = cy[k] - my, dz = cz[k] - mz;
    rad = fmax(rad, sqrt(dx * dx + dy * dy + dz * dz));
  }
  cent[P * 4] = mx; cent[P * 4 + 1] = my; cent[P * 4 + 2] = mz; cent[P * 4 + 3] = rad;
}

__global__ void k_coeff(int64_t N, const double* __restrict__ a_in, const double* __restrict__ ga_in,
                        const double* __restrict__ X, const double* __restrict__ Nn, const double* __restrict__ H,
                        const double* __restrict__ W, double* __restrict__ a, double* __restrict__ gs,
                        double* __restrict__ tgt, double* __restrict__ tg, double* __restrict__ tf,
                        float* __restrict__ t32, double* __restrict__ woa, int* __restrict__ bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double ai = a_in[i];
  double g0 = ga_in[3 * i], g1 = ga_in[3 * i + 1], g2 = ga_in[3 * i + 2];
  if (!(ai > 0.0) || !isfinite(ai) || !isfinite(g0) || !isfinite(g1) || !isfinite(g2)) atomicOr(bad, 1);
  double n0 = Nn[i], n1 = Nn[N + i], n2 = Nn[2 * N + i];
  double nd = n0 * g0 + n1 * g1 + n2 * g2;
  double s0 = g0 - n0 * nd, s1 = g1 - n1 * nd, s2 = g2 - n2 * nd;
  a[i] = ai;
  gs[i] = s0; gs[N + i] = s1; gs[2 * N + i] = s2;
  const double inv_pi = 0.31830988618379067154;
  const double inv_2pi = 0.15915494309189533577;
  double A = ai * inv_pi, B = ai * H[i] * inv_pi;
  double x0 = X[i], x1 = X[N + i], x2 = X[2 * N + i];
  double v[8] = {x0, x1, x2, n0, n1, n2, A, B};
  for (int k = 0; k < 8; ++k) tgt[k * N + i] = v[k];
  tg[i] = s0 * inv_2pi; tg[N + i] = s1 * inv_2pi; tg[2 * N + i] = s2 * inv_2pi;
  // n' = sqrt(A) n and h = g - B n: A (n.r)^2 - B (n.r) r^2 + (g.r) r^2 = (n'.r)^2 + (h.r) r^2
  const double sa = sqrt(A);
  double v9[9] = {x0, x1, x2, sa * n0, sa * n1, sa * n2, s0 * inv_2pi - B * n0, s1 * inv_2pi - B * n1,
                  s2 * inv_2pi - B * n2};
  for (int k = 0; k < 9; ++k) {
    tf[k * N + i] = v9[k];
    t32[k * N + i] = (float)v9[k];
  }
  woa[i] = W[i] / ai;
}

// Near lists: pass 0 counts, pass 1 fills (patch ids ascending).
template <bool FILL>
__global__ void k_near(int64_t N, int64_t M, int q, double eta, const double* __restrict__ X,
                       const double* __restrict__ cent, const int64_t* __restrict__ ptr, int32_t* __restrict__ cnt,
                       int32_t* __restrict__ patch, int32_t* __restrict__ target) {
  __shared__ double sc[4 * 256];
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double px = 0, py = 0, pz = 0;
  int64_t own = -1;
  if (i < N) {
    px = X[i]; py = X[N + i]; pz = X[2 * N + i];
    own = i / (q * q);
  }
  int c = 0;
  int64_t base = FILL && i < N ? ptr[i] : 0;
  for (int64_t P0 = 0; P0 < M; P0 += 256) {
    __syncthreads();
    int64_t P = P0 + threadIdx.x;
    if (P < M) {
      for (int k = 0; k < 4; ++k) sc[4 * threadIdx.x + k] = cent[4 * P + k];
    }
    __syncthreads();
    int64_t lim = M - P0 < 256 ? M - P0 : 256;
    if (i < N) {
      for (int t = 0; t < lim; ++t) {
        double dx = px - sc[4 * t], dy = py - sc[4 * t + 1], dz = pz - sc[4 * t + 2];
        bool near = sqrt(dx * dx + dy * dy + dz * dz) < eta * sc[4 * t + 3] || (P0 + t) == own;
        if (near) {
          if (FILL) {
            patch[base + c] = (int32_t)(P0 + t);
            target[base + c] = (int32_t)i;
          }
          ++c;
        }
      }
    }
  }
  if (!FILL && i < N) cnt[i] = c;
}

__global__ void k_widen(const int32_t* __restrict__ c, int64_t* __restrict__ o, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = c[i];
}

void build_geometry(Ctx* ctx, Geometry& g, const double* x, const double* xu, const double* xv, const double* xuu,
                    const double* xuv, const double* xvv, hipStream_t st) {
  const int64_t N = g.N, M = g.M;
  const int q = g.q;
  std::vector<double> t(q), w(q);
  gauss_legendre_host(q, t.data(), w.data());
  g.tnodes.alloc(ctx, q);
  g.tweights.alloc(ctx, q);
  PMX_HIP(hipMemcpyAsync(g.tnodes.p, t.data(), q * sizeof(double), hipMemcpyHostToDevice, st));
  PMX_HIP(hipMemcpyAsync(g.tweights.p, w.data(), q * sizeof(double), hipMemcpyHostToDevice, st));
  g.x.alloc(ctx, 3 * N);
  g.n.alloc(ctx, 3 * N);
  g.J.alloc(ctx, N);
  g.w.alloc(ctx, N);
  g.H.alloc(ctx, N);
  g.xu_p.alloc(ctx, 3 * N);
  g.xv_p.alloc(ctx, 3 * N);
  g.corner.alloc(ctx, 12 * M);
  g.cent.alloc(ctx, 4 * M);
  const int B = 256;
  const int64_t nb = (N + B - 1) / B;
  DBuf<double> red;
  red.alloc(ctx, 2 * nb);
  DBuf<int> bad;
  bad.alloc(ctx, 1);
  PMX_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_geometry, dim3(nb), dim3(B), 0, st, N, q, x, xu, xv, xuu, xuv, xvv, g.tweights.p, g.x.p,
                     g.n.p, g.J.p, g.w.p, g.H.p, g.xu_p.p, g.xv_p.p, red.p, bad.p);
  PMX_HIP(hipGetLastError());
  std::vector<double> Lm(q), Lp(q);
  lagrange_host(q, t.data(), -1.0, Lm.data());
  lagrange_host(q, t.data(), 1.0, Lp.data());
  DBuf<double> L;
  L.alloc(ctx, 2 * q);
  PMX_HIP(hipMemcpyAsync(L.p, Lm.data(), q * sizeof(double), hipMemcpyHostToDevice, st));
  PMX_HIP(hipMemcpyAsync(L.p + q, Lp.data(), q * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_patch_bounds, dim3((M + 127) / 128), dim3(128), 0, st, M, q, g.x.p, N, L.p, L.p + q,
                     g.corner.p, g.cent.p);
  PMX_HIP(hipGetLastError());
  std::vector<double> hred(2 * nb);
  int hbad = 0;
  PMX_HIP(hipMemcpyAsync(hred.data(), red.p, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  PMX_REQUIRE(!hbad, PMX_ERR_INVALID, "surface data is non-finite or has a degenerate metric");
  double wnx = 0.0, area = 0.0;
  for (int64_t b = 0; b < nb; ++b) {
    wnx += hred[2 * b];
    area += hred[2 * b + 1];
  }
  g.area = area;
  // Divergence theorem: sum w n.x = 3 |volume| > 0 for outward normals.
  PMX_REQUIRE(wnx > 0.0, PMX_ERR_ORIENTATION, "surface normals point inward (sum w n.x <= 0)");
}

// c at the nodes: flag 2 for a zero or non-finite value; the signs present are reported once per
// wave (8: some c > 0, 16: some c < 0), since c must keep one sign.
__global__ void k_coeff_c(int64_t N, const double* __restrict__ c_in, double* __restrict__ c, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double v = c_in[i];
  if (!(v != 0.0) || !isfinite(v)) atomicOr(bad, 2);
  const uint64_t pos = __ballot(v > 0.0), neg = __ballot(v < 0.0);
  if ((threadIdx.x & 63) == 0) {
    const int f = (pos ? 8 : 0) | (neg ? 16 : 0);
    if (f) atomicOr(bad, f);
  }
  c[i] = v;
}

// Advection (eq:adv_remainder): b . grad_G K = G' (b_t . r_hat) for the tangential part b_t of b,
// the same form as the grad_G a . r_hat G' term, so b_t / (2 pi) joins g = grad_G a / (2 pi) in
// the target vectors (g, and h = g - B n).
__global__ void k_coeff_b(int64_t N, const double* __restrict__ b_in, const double* __restrict__ Nn,
                          double* __restrict__ tg, double* __restrict__ tf, float* __restrict__ t32,
                          int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double b0 = b_in[3 * i], b1 = b_in[3 * i + 1], b2 = b_in[3 * i + 2];
  if (!isfinite(b0) || !isfinite(b1) || !isfinite(b2)) atomicOr(bad, 4);
  const double n0 = Nn[i], n1 = Nn[N + i], n2 = Nn[2 * N + i];
  const double nd = n0 * b0 + n1 * b1 + n2 * b2;
  const double inv_2pi = 0.15915494309189533577;
  const double t[3] = {(b0 - n0 * nd) * inv_2pi, (b1 - n1 * nd) * inv_2pi, (b2 - n2 * nd) * inv_2pi};
  for (int k = 0; k < 3; ++k) {
    tg[k * N + i] += t[k];
    const double h = tf[(6 + k) * N + i] + t[k];
    tf[(6 + k) * N + i] = h;
    t32[(6 + k) * N + i] = (float)h;
  }
}

void build_coeff(Ctx* ctx, const Geometry& g, Coeff& co, const double* a, const double* grad_a, const double* c,
                 const double* b, hipStream_t st) {
  const int64_t N = g.N;
  co.a.alloc(ctx, N);
  co.gs.alloc(ctx, 3 * N);
  co.tgt.alloc(ctx, 8 * N);
  co.tg.alloc(ctx, 3 * N);
  co.tf64.alloc(ctx, 9 * N);
  co.tgt32.alloc(ctx, 9 * N);
  co.w_over_a.alloc(ctx, N);
  DBuf<int> bad;
  bad.alloc(ctx, 1);
  PMX_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_coeff, dim3((N + 255) / 256), dim3(256), 0, st, N, a, grad_a, g.x.p, g.n.p, g.H.p, g.w.p,
                     co.a.p, co.gs.p, co.tgt.p, co.tg.p, co.tf64.p, co.tgt32.p, co.w_over_a.p, bad.p);
  PMX_HIP(hipGetLastError());
  if (c) {
    co.c.alloc(ctx, N);
    hipLaunchKernelGGL(k_coeff_c, dim3((N + 255) / 256), dim3(256), 0, st, N, c, co.c.p, bad.p);
    PMX_HIP(hipGetLastError());
  }
  if (b) {
    hipLaunchKernelGGL(k_coeff_b, dim3((N + 255) / 256), dim3(256), 0, st, N, b, g.n.p, co.tg.p, co.tf64.p,
                       co.tgt32.p, bad.p);
    PMX_HIP(hipGetLastError());
    co.has_b = true;
  }
  int hbad = 0;
  PMX_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  PMX_REQUIRE(!(hbad & 1), PMX_ERR_INVALID, "coefficient a must be positive and finite, grad a finite");
  PMX_REQUIRE(!(hbad & 2), PMX_ERR_INVALID, "coefficient c must be nonzero and finite at every node");
  PMX_REQUIRE((hbad & 24) != 24, PMX_ERR_INVALID, "coefficient c must have one sign at every node");
  co.complex_ = c && (hbad & 8);
  PMX_REQUIRE(!(hbad & 4), PMX_ERR_INVALID, "advection field b must be finite");
}

void build_near_lists(Ctx* ctx, const Geometry& g, double eta, NearLists& nl, hipStream_t st) {
  const int64_t N = g.N, M = g.M;
  DBuf<int32_t> cnt;
  cnt.alloc(ctx, N);
  nl.ptr.alloc(ctx, N + 1);
  const int64_t nb = (N + 255) / 256;
  hipLaunchKernelGGL((k_near<false>), dim3(nb), dim3(256), 0, st, N, M, g.q, eta, g.x.p, g.cent.p,
                     (const int64_t*)nullptr, cnt.p, (int32_t*)nullptr, (int32_t*)nullptr);
  PMX_HIP(hipGetLastError());
  // exclusive scan of the counts into ptr (int64)
  DBuf<int64_t> cnt64;
  cnt64.alloc(ctx, N + 1);
  PMX_HIP(hipMemsetAsync(cnt64.p + N, 0, sizeof(int64_t), st));
  // widen, then scan N+1 entries so that ptr[N] = nnz
  hipLaunchKernelGGL(k_widen, dim3(nb), dim3(256), 0, st, (const int32_t*)cnt.p, cnt64.p, N);
  PMX_HIP(hipGetLastError());
  size_t tmp_bytes = 0;
  PMX_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt64.p, nl.ptr.p, N + 1, st));
  DBuf<unsigned char> tmp;
  tmp.alloc(ctx, tmp_bytes);
  PMX_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, cnt64.p, nl.ptr.p, N + 1, st));
  int64_t nnz = 0;
  PMX_HIP(hipMemcpyAsync(&nnz, nl.ptr.p + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  PMX_HIP(hipStreamSynchronize(st));
  nl.nnz = nnz;
  nl.patch.alloc(ctx, nnz);
  nl.target.alloc(ctx, nnz);
  hipLaunchKernelGGL((k_near<true>), dim3(nb), dim3(256), 0, st, N, M, g.q, eta, g.x.p, g.cent.p,
                     (const int64_t*)nl.ptr.p, (int32_t*)nullptr, nl.patch.p, nl.target.p);
  PMX_HIP(hipGetLastError());
}

}  // namespace pmx
