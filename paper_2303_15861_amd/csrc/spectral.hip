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

}  // namespace mm
