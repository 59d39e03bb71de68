// Remainder stencil and small helper kernels.
//
// g(u) of eq. (eq:nonlin) on the tensor grid (Sec. 5.2 discretisation, flux form):
//   g = sum_mu [(abar+ - lam a_max)(u+ - u) - (abar- - lam a_max)(u - u-)] / h_mu^2
//     + sum_mu (beta_mu - beta_bar_mu)(u+ - u-)/(2 h_mu) + r0 + r1 u + r2 u^2 + r3 u^3,
// abar = mean of the two nodal coefficients at a face, zero Dirichlet ghosts. With
// lam_amax = 0 and the full velocity the same kernel yields F(u) (Appendix, u' = F(u)).
// The stage updates of the schemes are fused as out0 = base0 + c0 (g - sub) and
// out1 = base1 + c1 (g - sub), so each remainder evaluation is one pass over HBM.
#include <cfloat>

#include "mm_internal.h"

namespace mm {

// Each thread owns one x1 column of a YT (x2) x ZT (x3) patch of grid points and keeps
// the patch with a one-point halo in registers, so the x2/x3 neighbours of u and a are
// loaded once per patch instead of once per point; x1 neighbours come from the same
// cache lines as the neighbouring lanes' centres. A wave covers 64 consecutive x1, so
// every access is a coalesced row segment. No LDS and no barriers.
constexpr int SX = 64, SY = 4, YT = 2, ZT = 4;

// Block order: workgroups are dealt round-robin over the eight XCDs (id % 8), each with
// its own L2. XCD k takes a contiguous band of x2-blocks and walks it x1-fastest, then
// x2, then x3, so the x2 and x3 halos a block reads were (or are about to be) fetched
// into the same L2 by its neighbours.
struct StencilGrid {
  int nxb, nyb, nzb, ybx;
};

template <int D>
__global__ __launch_bounds__(SX * SY) void stencil_kernel(StencilArgs p, StencilGrid sg) {
  constexpr int ZP = (D == 3) ? ZT : 1;   // points per thread along x3
  const int L = blockIdx.x;
  const int xcd = L & 7, j = L >> 3;
  const int bx = j % sg.nxb;
  const int r = j / sg.nxb;
  const int by = xcd * sg.ybx + r % sg.ybx;
  const int bz = r / sg.ybx;
  if (by >= sg.nyb || bz >= sg.nzb) return;
  const int tx = threadIdx.x & (SX - 1), ty = threadIdx.x / SX;
  const int i1 = bx * SX + tx;
  const int y0 = (by * SY + ty) * YT;
  const int z0 = (D == 3) ? bz * ZT : 0;
  const int n1 = p.n1, n2 = p.n2, n3 = p.n3;
  if (i1 >= n1) return;
  const int s2 = n1, s3 = n1 * n2;                    // strides of u
  const int t2 = n1 + 2, t3 = (n1 + 2) * (n2 + 2);    // strides of a (padded)
  const double* __restrict__ u = p.u;
  const double* __restrict__ a = p.a;
  // patch with halo: uu[y][z] holds u at (i1, y0 - 1 + y, z0 - 1 + z); corners unused
  double uu[YT + 2][ZP + 2], aa[YT + 2][ZP + 2];
#pragma unroll
  for (int y = 0; y < YT + 2; ++y)
#pragma unroll
    for (int z = 0; z < ZP + 2; ++z) {
      const int i2 = y0 - 1 + y;
      const int i3 = (D == 3) ? z0 - 1 + z : 0;
      const bool need = (D == 3) ? !((y == 0 || y == YT + 1) && (z == 0 || z == ZP + 1)) : (z == 1);
      const bool uin = need && i2 >= 0 && i2 < n2 && i3 >= 0 && i3 < n3;
      const bool ain = need && i2 >= -1 && i2 <= n2 && (D == 2 || (i3 >= -1 && i3 <= n3));
      uu[y][z] = uin ? u[i1 + s2 * i2 + s3 * i3] : 0.0;
      aa[y][z] = ain ? a[(i1 + 1) + t2 * (i2 + 1) + (D == 3 ? t3 * (i3 + 1) : 0)] : 0.0;
    }
  const double la = p.lam_amax;
#pragma unroll
  for (int y = 1; y <= YT; ++y)
#pragma unroll
    for (int z = 1; z <= ZP; ++z) {
      const int i2 = y0 - 1 + y;
      const int i3 = (D == 3) ? z0 - 1 + z : 0;
      if (i2 >= n2 || i3 >= n3) continue;
      const int idx = i1 + s2 * i2 + s3 * i3;
      const int ia = (i1 + 1) + t2 * (i2 + 1) + (D == 3 ? t3 * (i3 + 1) : 0);
      const double uc = uu[y][z], ac = aa[y][z];
      const double uxm = (i1 > 0) ? u[idx - 1] : 0.0;
      const double uxp = (i1 + 1 < n1) ? u[idx + 1] : 0.0;
      const double axm = a[ia - 1], axp = a[ia + 1];
      double g = ((0.5 * (ac + axp) - la) * (uxp - uc) - (0.5 * (ac + axm) - la) * (uc - uxm)) * p.ih2[0] +
                 p.cadv[0] * (uxp - uxm);
      g += ((0.5 * (ac + aa[y + 1][z]) - la) * (uu[y + 1][z] - uc) -
            (0.5 * (ac + aa[y - 1][z]) - la) * (uc - uu[y - 1][z])) * p.ih2[1] +
           p.cadv[1] * (uu[y + 1][z] - uu[y - 1][z]);
      if (D == 3)
        g += ((0.5 * (ac + aa[y][z + 1]) - la) * (uu[y][z + 1] - uc) -
              (0.5 * (ac + aa[y][z - 1]) - la) * (uc - uu[y][z - 1])) * p.ih2[2] +
             p.cadv[2] * (uu[y][z + 1] - uu[y][z - 1]);
      g += p.r0 + uc * (p.r1 + uc * (p.r2 + uc * p.r3));
      if (p.sub) g -= p.sub[idx];
      const double o0 = (p.base0 ? p.base0[idx] : 0.0) + p.c0 * g;
      if (p.out0f)
        p.out0f[idx] = (float)o0;
      else
        p.out0[idx] = o0;
      if (p.out1 || p.out1f) {
        const double o1 = (p.base1 ? p.base1[idx] : 0.0) + p.c1 * g;
        if (p.out1f)
          p.out1f[idx] = (float)o1;
        else
          p.out1[idx] = o1;
      }
      if (p.flag && !(fabs(o0) <= DBL_MAX)) p.flag[0] = 1;
    }
}

hipError_t launch_stencil(int d, const StencilArgs& a, hipStream_t s) {
  StencilGrid sg;
  sg.nxb = (a.n1 + SX - 1) / SX;
  sg.nyb = (a.n2 + SY * YT - 1) / (SY * YT);
  sg.nzb = (d == 3) ? (a.n3 + ZT - 1) / ZT : 1;
  sg.ybx = (sg.nyb + 7) / 8;
  const int64_t blocks = 8LL * sg.nxb * sg.ybx * sg.nzb;
  if (blocks >= (1LL << 31)) return hipErrorInvalidValue;
  if (d == 3)
    stencil_kernel<3><<<dim3((unsigned)blocks), dim3(SX * SY), 0, s>>>(a, sg);
  else
    stencil_kernel<2><<<dim3((unsigned)blocks), dim3(SX * SY), 0, s>>>(a, sg);
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

// ---------------------------------------------------------------- eigenbasis scaling
// In the joint eigenbasis of A = A_1 (+) A_2 (+) A_3 every function of tau A is diagonal:
// the entry (k3, k2, k1) is scaled by f(tau (ev1[k1] + ev2[k2] + ev3[k3])).
// phi2(z) = (e^z - 1 - z)/z^2 = sum_k z^k/(k+2)!; the series for |z| < 1/2 (where the
// closed form cancels), the closed form through expm1 elsewhere.
__device__ __forceinline__ double phi2_fn(double z) {
  if (fabs(z) < 0.5) {
    double term = 0.5, acc = 0.0;   // term = z^k/(k+2)!
#pragma unroll 1
    for (int k = 0; k < 24; ++k) {
      acc += term;
      term *= z / (k + 3);
    }
    return acc;
  }
  return (expm1(z) - z) / (z * z);
}

__device__ __forceinline__ double eig_fn(int f, double z) {
  if (f == MM_EIG_EXP) return exp(z);
  if (f == MM_EIG_PHI1) return (z == 0.0) ? 1.0 : expm1(z) / z;   // phi1(z) = (e^z - 1)/z
  if (f == MM_EIG_PHI2) return phi2_fn(z);
  return 1.0;
}

__global__ void eig_scale(double* out, const double* a, double ca, int fa, const double* b, double cb, int fb,
                          const double* ev1, const double* ev2, const double* ev3, int n1, int n2, int64_t cnt,
                          double tau) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= cnt) return;
  const int k1 = (int)(e % n1);
  const int64_t r = e / n1;
  const int k2 = (int)(r % n2);
  const int k3 = (int)(r / n2);
  const double z = tau * (ev1[k1] + ev2[k2] + (ev3 ? ev3[k3] : 0.0));
  double v = ca * eig_fn(fa, z) * a[e];
  if (b) v += cb * eig_fn(fb, z) * b[e];
  out[e] = v;
}

hipError_t launch_eig_scale(double* out, const double* a, double ca, int fa, const double* b, double cb, int fb,
                            const double* ev1, const double* ev2, const double* ev3, int n1, int n2, int n3,
                            double tau, hipStream_t s) {
  const int64_t cnt = (int64_t)n1 * n2 * n3;
  eig_scale<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(out, a, ca, fa, b, cb, fb, ev1, ev2, ev3, n1, n2, cnt,
                                                          tau);
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

// out[0] = max column sum of |Q| (1-norm), out[1] = max row sum (inf-norm); one block
__global__ __launch_bounds__(1024) void norms_kernel(const double* Q, int n, double* out) {
  __shared__ double s1[1024], si[1024];
  double c1 = 0.0, ci = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double col = 0.0, row = 0.0;
    for (int i = 0; i < n; ++i) {
      col += fabs(Q[(int64_t)i * n + j]);
      row += fabs(Q[(int64_t)j * n + i]);
    }
    c1 = fmax(c1, col);
    ci = fmax(ci, row);
  }
  s1[threadIdx.x] = c1;
  si[threadIdx.x] = ci;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
      si[threadIdx.x] = fmax(si[threadIdx.x], si[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s1[0];
    out[1] = si[0];
  }
}

hipError_t launch_norms(const double* Q, int n, double* out, hipStream_t s) {
  norms_kernel<<<1, 1024, 0, s>>>(Q, n, out);
  return hipGetLastError();
}

__global__ void scaled_transpose(double* X, const double* Q, int n, double alpha) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  X[e] = alpha * Q[(int64_t)c * n + r];
}

hipError_t launch_scaled_transpose(double* X, const double* Q, int n, double alpha, hipStream_t s) {
  const int64_t cnt = (int64_t)n * n;
  scaled_transpose<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(X, Q, n, alpha);
  return hipGetLastError();
}

// out[0] = max |R - I|; one block
__global__ __launch_bounds__(1024) void resid_kernel(const double* R, int n, double* out) {
  __shared__ double sm[1024];
  double m = 0.0;
  const int64_t cnt = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int r = (int)(e / n), c = (int)(e % n);
    m = fmax(m, fabs(R[e] - (r == c ? 1.0 : 0.0)));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

hipError_t launch_resid(const double* R, int n, double* out, hipStream_t s) {
  resid_kernel<<<1, 1024, 0, s>>>(R, n, out);
  return hipGetLastError();
}

hipError_t launch_lu_solve(double* Q, double* P, int n, int count, hipStream_t s) {
  lu_solve_kernel<<<count, 1024, 0, s>>>(Q, P, n);
  return hipGetLastError();
}

}  // namespace mm
