// Periodic pseudo-spectral problems (Sec. 4.1, 4.2 and 5.1) in mu-mode form: the
// Fourier differentiation matrices and the exponentials of the extracted operator are
// circulant along each axis, so every derivative and every exponential action is a mode
// product with a dense n x n circulant factor (the same GEMMs as the finite-difference
// path) instead of an FFT. This file holds the element-wise passes of the spectral
// remainder and the circulant builder; the GEMMs are the contraction kernels.
//
// The remainder of a periodic problem is evaluated in four kinds of passes, each axis mu
// accumulating into its own G_mu:
//   G_0 = r(u) (spec_react), G_mu = 0 for mu > 0 (fill)
//   per axis mu:  T1 = D_mu x_mu u  (D1 for the flux form, D2 for the non-divergence form)
//                 flux:   T2 = (a_mu - lam a^max_mu) T1 + (b_mu - beta_bar_mu) u
//                 nondiv: G_mu += (a_mu - lam a^max_mu) T1,  T2 = (b_mu - beta_bar_mu) u
//                                                            (spec_mid)
//                 G_mu += D1_mu x_mu T2                      (GEMM with accumulation)
//                 [F: G_mu += A_mu x_mu u]
//   outputs of the stage update from G_0 + G_1 [+ G_2]       (spec_combine)
// b_mu is the velocity field of the problem or, without one, its constant velocity.
#include "mm_internal.h"

#include <cfloat>

namespace mm {

__global__ __launch_bounds__(256) void build_circulant_kernel(double* __restrict__ M, int n,
                                                              const double* __restrict__ col) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int i = (int)(e / n);
  const int j = (int)(e - (int64_t)i * n);
  int k = i - j;
  if (k < 0) k += n;
  M[e] = col[k];   // (M v)_i = sum_j c_{(i - j) mod n} v_j
}

hipError_t launch_build_circulant(double* M, int n, const double* col, hipStream_t s) {
  const int64_t nn = (int64_t)n * n;
  build_circulant_kernel<<<dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s>>>(M, n, col);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void spec_react_kernel(double* __restrict__ G, const double* __restrict__ u,
                                                         int64_t n, double r0, double r1, double r2, double r3) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const double v = u[e];
  G[e] = r0 + v * (r1 + v * (r2 + v * r3));
}

hipError_t launch_spec_react(double* G, const double* u, int64_t n, const double* r, hipStream_t s) {
  spec_react_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(G, u, n, r[0], r[1], r[2], r[3]);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void spec_mid_kernel(SpecMidArgs p) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= p.n) return;
  const double u = p.u[e];
  const double adv = p.vel ? p.vel[e] - p.beta_bar : p.beta - p.beta_bar;
  const double c = p.a[e] - p.lam_amax;
  if (p.nondiv) {
    p.G[e] += c * p.T1[e];
    p.T2[e] = adv * u;
  } else {
    p.T2[e] = c * p.T1[e] + adv * u;
  }
}

hipError_t launch_spec_mid(const SpecMidArgs& a, hipStream_t s) {
  spec_mid_kernel<<<dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s>>>(a);
  return hipGetLastError();
}

// the output contract of the stencil: s = G_0 + G_1 + G_2 - sub (absent terms skipped);
// out0 = base0 + c0 s (0 + c0 s without base0), out1 likewise; the sticky flag is raised
// when out0 is not finite
__global__ __launch_bounds__(256) void spec_combine_kernel(const double* __restrict__ G0, const double* __restrict__ G1,
                                                           const double* __restrict__ G2, StencilArgs p, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  double g = G0[e];
  if (G1) g += G1[e];
  if (G2) g += G2[e];
  if (p.sub) g -= p.sub[e];
  const double o0 = (p.base0 ? p.base0[e] : 0.0) + p.c0 * g;
  double o1 = 0.0;
  const bool two = p.out1 || p.out1f;
  if (two) o1 = (p.base1 ? p.base1[e] : 0.0) + p.c1 * g;
  if (p.flag && !(fabs(o0) <= DBL_MAX)) p.flag[0] = 1;
  if (p.out0f)
    p.out0f[e] = (float)o0;
  else
    p.out0[e] = o0;
  if (two) {
    if (p.out1f)
      p.out1f[e] = (float)o1;
    else
      p.out1[e] = o1;
  }
}

hipError_t launch_spec_combine(const double* const (&G)[3], const StencilArgs& a, int64_t n, hipStream_t s) {
  // out0 (or its FP32 form) is written unconditionally; out1 when either form is set
  if ((!a.out0 && !a.out0f) || !G[0]) return hipErrorInvalidValue;
  spec_combine_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(G[0], G[1], G[2], a, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- exact phi, periodic axes
// In the real orthonormal Fourier basis of an axis (transform index 0: the constant;
// 2m - 1 and 2m: cos and sin of wavenumber m, 1 <= m < n/2; n - 1 for even n: the Nyquist
// mode) a real circulant with symbol sigma(m) = alpha(m) + i omega(m) (alpha even and
// omega odd in m) is block diagonal: a (cos, sin) coefficient pair (a, b) is the complex
// amplitude c+ = (a - i b)/2 of e^{i theta} and c- = (a + i b)/2 of e^{-i theta}, which it
// multiplies by sigma(m) and by its conjugate. So a function f of tau A = tau (A_1 (+)
// A_2 (+) A_3) acts on the (up to eight) coefficients of one wavenumber triple through
// these amplitudes: every sign pattern of the modes is multiplied by f(tau sum sigma_mu^+-),
// and the pairs are assembled back, a = c+ + c-, b = i (c+ - c-).
namespace {

struct cplx {
  double re, im;
};

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cscale(cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// f(z) for f = exp, phi1(z) = (e^z - 1)/z, phi2(z) = (e^z - 1 - z)/z^2 (series below |z| = 1/2,
// where the closed forms cancel), or 1
__device__ cplx cfun(int f, cplx z) {
  if (f == MM_EIG_ONE) return {1.0, 0.0};
  double sn, cs;
  sincos(z.im, &sn, &cs);
  const double ex = exp(z.re);
  const cplx e = {ex * cs, ex * sn};
  if (f == MM_EIG_EXP) return e;
  const int k = (f == MM_EIG_PHI1) ? 1 : 2;
  if (z.re * z.re + z.im * z.im < 0.25) {
    cplx acc = {0.0, 0.0}, term = {k == 1 ? 1.0 : 0.5, 0.0};   // z^j / (j + k)!
#pragma unroll 1
    for (int j = 0; j < 25; ++j) {
      acc = cadd(acc, term);
      term = cscale(cmul(term, z), 1.0 / (j + k + 1));
    }
    return acc;
  }
  cplx num = {expm1(z.re) * cs - 2.0 * sin(0.5 * z.im) * sin(0.5 * z.im), ex * sn};   // e^z - 1
  if (k == 1) return cdiv(num, z);
  num = csub(num, z);
  return cdiv(num, cmul(z, z));
}

// transform indices of wavenumber m on an axis of n points; returns whether it is a pair
__device__ __forceinline__ bool mode_index(int m, int n, int& i0) {
  if (m == 0) {
    i0 = 0;
    return false;
  }
  if ((n & 1) == 0 && m == n / 2) {
    i0 = n - 1;
    return false;
  }
  i0 = 2 * m - 1;
  return true;
}

}  // namespace

__global__ __launch_bounds__(256) void spec_eig_scale_kernel(double* __restrict__ out, const double* __restrict__ a,
                                                             double ca, int fa, const double* __restrict__ b,
                                                             double cb, int fb, const double* __restrict__ sym1,
                                                             const double* __restrict__ sym2,
                                                             const double* __restrict__ sym3, int n1, int n2, int n3,
                                                             int M1, int M2, int M3, double tau) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M1 * M2 * M3) return;
  const int m1 = (int)(e % M1);
  const int64_t r = e / M1;
  const int m2 = (int)(r % M2), m3 = (int)(r / M2);
  int i1, i2, i3;
  const bool p1 = mode_index(m1, n1, i1), p2 = mode_index(m2, n2, i2);
  const bool p3 = n3 > 1 ? mode_index(m3, n3, i3) : (i3 = 0, false);
  const bool pair[3] = {p1, p2, p3};
  const double al[3] = {sym1[2 * m1], sym2[2 * m2], sym3 ? sym3[2 * m3] : 0.0};
  const double om[3] = {sym1[2 * m1 + 1], sym2[2 * m2 + 1], sym3 ? sym3[2 * m3 + 1] : 0.0};
  // slot t = t1 + 2 t2 + 4 t3 (t_mu = 1: the sin member of a pair)
  int64_t idx[8];
  bool used[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int t1 = t & 1, t2 = (t >> 1) & 1, t3 = t >> 2;
    used[t] = (!t1 || p1) && (!t2 || p2) && (!t3 || p3);
    idx[t] = used[t] ? (int64_t)(i3 + t3) * n2 * n1 + (int64_t)(i2 + t2) * n1 + (i1 + t1) : 0;
  }
  auto apply = [&](const double* src, int f, cplx (&res)[8]) {
    cplx v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = {used[t] ? src[idx[t]] : 0.0, 0.0};
    // to amplitudes: (a, b) -> ((a - i b)/2, (a + i b)/2) along every pair axis
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (!pair[ax]) continue;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (t & (1 << ax)) continue;
        const cplx x = v[t], y = v[t | (1 << ax)];
        const cplx iy = {-y.im, y.re};
        v[t] = cscale(csub(x, iy), 0.5);
        v[t | (1 << ax)] = cscale(cadd(x, iy), 0.5);
      }
    }
    // amplitude of sign pattern t (bit set: the conjugate mode) times f(tau sum sigma)
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (!used[t]) continue;
      cplx z = {0.0, 0.0};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        z.re += al[ax];
        z.im += (t & (1 << ax)) ? -om[ax] : om[ax];
      }
      v[t] = cmul(v[t], cfun(f, cscale(z, tau)));
    }
    // back: a = c+ + c-, b = i (c+ - c-)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (!pair[ax]) continue;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (t & (1 << ax)) continue;
        const cplx cp = v[t], cm = v[t | (1 << ax)];
        const cplx d = csub(cp, cm);
        v[t] = cadd(cp, cm);
        v[t | (1 << ax)] = {-d.im, d.re};
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) res[t] = v[t];
  };
  cplx ra[8], rb[8];
  apply(a, fa, ra);
  if (b) apply(b, fb, rb);
#pragma unroll
  for (int t = 0; t < 8; ++t)
    if (used[t]) out[idx[t]] = ca * ra[t].re + (b ? cb * rb[t].re : 0.0);
}

hipError_t launch_spec_eig_scale(double* out, const double* a, double ca, int fa, const double* b, double cb, int fb,
                                 const double* sym1, const double* sym2, const double* sym3, int n1, int n2, int n3,
                                 double tau, hipStream_t s) {
  if (!out || !a || !sym1 || !sym2 || (n3 > 1 && !sym3) || n1 < 1 || n2 < 1 || n3 < 1) return hipErrorInvalidValue;
  const int M1 = n1 / 2 + 1, M2 = n2 / 2 + 1, M3 = n3 > 1 ? n3 / 2 + 1 : 1;
  const int64_t cnt = (int64_t)M1 * M2 * M3;
  spec_eig_scale_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(out, a, ca, fa, b, cb, fb, sym1, sym2, sym3,
                                                                      n1, n2, n3, M1, M2, M3, tau);
  return hipGetLastError();
}

}  // namespace mm
