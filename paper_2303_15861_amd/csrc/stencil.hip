// Remainder stencil and small helper kernels.
//
// g(u) of eq. (eq:nonlin) on the tensor grid (Sec. 5.2 discretisation, flux form):
//   g = sum_mu [(abar+ - lam a_max)(u+ - u) - (abar- - lam a_max)(u - u-)] / h_mu^2
//     + sum_mu (beta_mu - beta_bar_mu)(u+ - u-)/(2 h_mu) + r0 + r1 u + r2 u^2 + r3 u^3,
// abar = mean of the two nodal coefficients at a face, zero Dirichlet ghosts. With
// lam_amax = 0 and the full velocity the same kernel yields F(u) (Appendix, u' = F(u)).
// The stage updates of the schemes are fused as out0 = base0 + c0 (g - sub) and
// out1 = base1 + c1 (g - sub), so each remainder evaluation is one pass over HBM.
// Threads run along x1 (coalesced); neighbours along x2/x3 come from L2.
#include <cfloat>

#include "mm_internal.h"

namespace mm {

template <int D>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs p) {
  const int i1 = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i2 = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int i3 = blockIdx.z;
  const int n1 = p.n1, n2 = p.n2, n3 = p.n3;
  if (i1 >= n1 || i2 >= n2 || i3 >= n3) return;
  const int s2 = n1, s3 = n1 * n2;                      // strides of u
  const int t2 = n1 + 2, t3 = (n1 + 2) * (n2 + 2);      // strides of a
  const int idx = i1 + s2 * i2 + s3 * i3;
  const int ia = (i1 + 1) + t2 * (i2 + 1) + (D == 3 ? t3 * (i3 + 1) : 0);
  const double* __restrict__ u = p.u;
  const double* __restrict__ a = p.a;
  const double uc = u[idx];
  const double ac = a[ia];
  const double la = p.lam_amax;

  // axis 1
  const double um1 = (i1 > 0) ? u[idx - 1] : 0.0;
  const double up1 = (i1 + 1 < n1) ? u[idx + 1] : 0.0;
  double g = ((0.5 * (ac + a[ia + 1]) - la) * (up1 - uc) - (0.5 * (ac + a[ia - 1]) - la) * (uc - um1)) * p.ih2[0] +
             p.cadv[0] * (up1 - um1);
  // axis 2
  const double um2 = (i2 > 0) ? u[idx - s2] : 0.0;
  const double up2 = (i2 + 1 < n2) ? u[idx + s2] : 0.0;
  g += ((0.5 * (ac + a[ia + t2]) - la) * (up2 - uc) - (0.5 * (ac + a[ia - t2]) - la) * (uc - um2)) * p.ih2[1] +
       p.cadv[1] * (up2 - um2);
  if (D == 3) {
    const double um3 = (i3 > 0) ? u[idx - s3] : 0.0;
    const double up3 = (i3 + 1 < n3) ? u[idx + s3] : 0.0;
    g += ((0.5 * (ac + a[ia + t3]) - la) * (up3 - uc) - (0.5 * (ac + a[ia - t3]) - la) * (uc - um3)) * p.ih2[2] +
         p.cadv[2] * (up3 - um3);
  }
  g += p.r0 + uc * (p.r1 + uc * (p.r2 + uc * p.r3));
  if (p.sub) g -= p.sub[idx];
  const double o0 = (p.base0 ? p.base0[idx] : 0.0) + p.c0 * g;
  p.out0[idx] = o0;
  if (p.out1) p.out1[idx] = (p.base1 ? p.base1[idx] : 0.0) + p.c1 * g;
  if (p.flag && !(fabs(o0) <= DBL_MAX)) p.flag[0] = 1;
}

hipError_t launch_stencil(int d, const StencilArgs& a, hipStream_t s) {
  const dim3 block(256);
  const dim3 grid((a.n1 + 63) / 64, (a.n2 + 3) / 4, d == 3 ? a.n3 : 1);
  if (d == 3)
    stencil_kernel<3><<<grid, block, 0, s>>>(a);
  else
    stencil_kernel<2><<<grid, block, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- max reduction
__global__ __launch_bounds__(256) void max_partial(const double* __restrict__ x, int64_t n,
                                                   double* __restrict__ part) {
  __shared__ double sm[256];
  double m = -DBL_MAX;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    m = fmax(m, x[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

hipError_t launch_max_reduce(const double* x, int64_t n, double* partial, int nparts, double* out,
                             hipStream_t s) {
  max_partial<<<nparts, 256, 0, s>>>(x, n, partial);
  max_partial<<<1, 256, 0, s>>>(partial, nparts, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dense helpers
__global__ void build_tridiag(double* M, int n, double sub, double diag, double sup) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  M[e] = (c == r) ? diag : (c == r - 1) ? sub : (c == r + 1) ? sup : 0.0;
}

hipError_t launch_build_tridiag(double* M, int n, double sub, double diag, double sup, hipStream_t s) {
  const int64_t cnt = (int64_t)n * n;
  build_tridiag<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(M, n, sub, diag, sup);
  return hipGetLastError();
}

__global__ void combo_kernel(double* out, int n, double c0, const double* X0, double c1, const double* X1,
                             double c2, const double* X2, double c3, const double* X3, double cI) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  double v = (r == c) ? cI : 0.0;
  if (X0) v += c0 * X0[e];
  if (X1) v += c1 * X1[e];
  if (X2) v += c2 * X2[e];
  if (X3) v += c3 * X3[e];
  out[e] = v;
}

hipError_t launch_combo(double* out, int n, double c0, const double* X0, double c1, const double* X1,
                        double c2, const double* X2, double c3, const double* X3, double cI,
                        hipStream_t s) {
  const int64_t cnt = (int64_t)n * n;
  combo_kernel<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(out, n, c0, X0, c1, X1, c2, X2, c3, X3, cI);
  return hipGetLastError();
}

__global__ void axpy_kernel(double* out, const double* X, double s, const double* Y, int64_t cnt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < cnt) out[e] = X[e] + s * Y[e];
}

hipError_t launch_axpy(double* out, const double* X, double s, const double* Y, int64_t count,
                       hipStream_t st) {
  axpy_kernel<<<(unsigned)((count + 255) / 256), 256, 0, st>>>(out, X, s, Y, count);
  return hipGetLastError();
}

__global__ void fill_kernel(double* d, double v, int64_t cnt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < cnt) d[e] = v;
}

hipError_t launch_fill(double* dst, double v, int64_t count, hipStream_t s) {
  fill_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(dst, v, count);
  return hipGetLastError();
}

__global__ void place_scaled(double* dst, int ldd, int col0, const double* src, int n, double w) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  dst[(int64_t)r * ldd + col0 + c] = w * src[e];
}

hipError_t launch_place_scaled(double* dst, int ldd, int col0, const double* src, int n, double w,
                               hipStream_t s) {
  const int64_t cnt = (int64_t)n * n;
  place_scaled<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(dst, ldd, col0, src, n, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dense solve
// Gaussian elimination with partial pivoting on [Q | P] (n x 2n), one workgroup per
// system, followed by back substitution; P is overwritten with Q^{-1} P.
__global__ __launch_bounds__(1024) void lu_solve_kernel(double* Qall, double* Pall, int n) {
  double* Q = Qall + (int64_t)blockIdx.x * n * n;
  double* P = Pall + (int64_t)blockIdx.x * n * n;
  __shared__ double sval[1024];
  __shared__ int sidx[1024];
  __shared__ double pivrow_inv;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int col = 0; col < n; ++col) {
    // pivot search over rows col..n-1
    double best = -1.0;
    int bi = col;
    for (int r = col + tid; r < n; r += nt) {
      const double v = fabs(Q[(int64_t)r * n + col]);
      if (v > best) { best = v; bi = r; }
    }
    sval[tid] = best;
    sidx[tid] = bi;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w && (sval[tid + w] > sval[tid] ||
                      (sval[tid + w] == sval[tid] && sidx[tid + w] < sidx[tid]))) {
        sval[tid] = sval[tid + w];
        sidx[tid] = sidx[tid + w];
      }
      __syncthreads();
    }
    const int piv = sidx[0];
    __syncthreads();
    if (piv != col) {
      for (int c = tid; c < n; c += nt) {
        const double t0 = Q[(int64_t)col * n + c];
        Q[(int64_t)col * n + c] = Q[(int64_t)piv * n + c];
        Q[(int64_t)piv * n + c] = t0;
        const double t1 = P[(int64_t)col * n + c];
        P[(int64_t)col * n + c] = P[(int64_t)piv * n + c];
        P[(int64_t)piv * n + c] = t1;
      }
    }
    __syncthreads();
    if (tid == 0) pivrow_inv = 1.0 / Q[(int64_t)col * n + col];
    __syncthreads();
    // eliminate below the pivot: rows col+1..n-1, columns col..n-1 of Q and all of P
    const int rows = n - col - 1;
    const int qcols = n - col;
    const int width = qcols + n;
    const int work = rows * width;
    for (int e = tid; e < work; e += nt) {
      const int rr = e / width;
      const int cc = e - rr * width;
      const int r = col + 1 + rr;
      const double f = Q[(int64_t)r * n + col] * pivrow_inv;
      if (cc < qcols) {
        if (cc > 0) Q[(int64_t)r * n + col + cc] -= f * Q[(int64_t)col * n + col + cc];
      } else {
        const int pc = cc - qcols;
        P[(int64_t)r * n + pc] -= f * P[(int64_t)col * n + pc];
      }
    }
    __syncthreads();
    // the multipliers in column col are consumed; zero them last
    for (int r = col + 1 + tid; r < n; r += nt) Q[(int64_t)r * n + col] = 0.0;
    __syncthreads();
  }
  // back substitution, one column of P per thread group
  for (int row = n - 1; row >= 0; --row) {
    const double inv = 1.0 / Q[(int64_t)row * n + row];
    for (int c = tid; c < n; c += nt) P[(int64_t)row * n + c] *= inv;
    __syncthreads();
    const int work = row * n;
    for (int e = tid; e < work; e += nt) {
      const int r = e / n, c = e - r * n;
      P[(int64_t)r * n + c] -= Q[(int64_t)r * n + row] * P[(int64_t)row * n + c];
    }
    __syncthreads();
  }
}

hipError_t launch_lu_solve(double* Q, double* P, int n, int count, hipStream_t s) {
  lu_solve_kernel<<<count, 1024, 0, s>>>(Q, P, n);
  return hipGetLastError();
}

}  // namespace mm
