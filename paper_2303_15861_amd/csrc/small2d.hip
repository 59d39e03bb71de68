// Whole Lawson solves of small 2D problems in one workgroup (the time loop on the
// device). For n1, n2 <= 64 a step is ~1 MFLOP: launched kernel by kernel it is bound
// by launch latency, so one workgroup keeps the state, the stage vectors
// and the coefficient a in LDS and each lane's factor operands in registers for the
// whole solve, and runs every step -- the remainder stencil (eq. (eq:nonlin), flux
// form, the same arithmetic as the grid kernel), the two mode products (FP64 MFMA) and
// the stage combinations -- with workgroup barriers between the phases. Sixteen waves:
// one 16 x 16 output tile of the 64 x 64 padded grid each.
#include <cfloat>

#include "mm_internal.h"

namespace mm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NS = 64;        // largest n1, n2
constexpr int PS = NS + 1;    // LDS row pitch in doubles
constexpr int THS = 1024;     // sixteen waves, one 16 x 16 output tile each

constexpr int PA = NS + 2;    // pitch of the LDS copy of a

// g at interior point (i2, i1) from the LDS grid U (zero outside [0,n2) x [0,n1)) and
// the LDS copy of a ((n2+2) x (n1+2) nodes, pitch PA).
__device__ __forceinline__ double g_small(const SmallArgs& p, const double* U, const double* A, int i2, int i1) {
  const int n1 = p.n1, n2 = p.n2;
  const double uc = U[i2 * PS + i1];
  const double uxm = (i1 > 0) ? U[i2 * PS + i1 - 1] : 0.0;
  const double uxp = (i1 + 1 < n1) ? U[i2 * PS + i1 + 1] : 0.0;
  const double uym = (i2 > 0) ? U[(i2 - 1) * PS + i1] : 0.0;
  const double uyp = (i2 + 1 < n2) ? U[(i2 + 1) * PS + i1] : 0.0;
  const int ia = (i1 + 1) + PA * (i2 + 1);
  const double ac = A[ia], axm = A[ia - 1], axp = A[ia + 1], aym = A[ia - PA], ayp = A[ia + PA];
  const double la = p.lam_amax;
  double g = ((0.5 * (ac + axp) - la) * (uxp - uc) - (0.5 * (ac + axm) - la) * (uc - uxm)) * p.ih2[0] +
             p.cadv[0] * (uxp - uxm);
  g += ((0.5 * (ac + ayp) - la) * (uyp - uc) - (0.5 * (ac + aym) - la) * (uc - uym)) * p.ih2[1] +
       p.cadv[1] * (uyp - uym);
  g += p.r0 + uc * (p.r1 + uc * (p.r2 + uc * p.r3));
  return g;
}

// The factor operand of this lane for all 16 k-steps of a 64-long contraction (zero
// beyond n), loaded once per solve: f[kk] = E[r0 + lane%16][4 kk + lane/16].
struct FactorFrags {
  double f[16];
};

__device__ __forceinline__ void load_frags(FactorFrags& F, const double* __restrict__ E, int n, int r0) {
  const int lane = threadIdx.x & 63, lg = lane >> 4, lr = lane & 15;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int r = r0 + lr, k = 4 * kk + lg;
    F.f[kk] = (r < n && k < n) ? E[r * n + k] : 0.0;
  }
}

// the 16 x 16 output tile of this wave
__device__ __forceinline__ int tile_row() { return ((threadIdx.x >> 6) >> 2) * 16; }
__device__ __forceinline__ int tile_col() { return ((threadIdx.x >> 6) & 3) * 16; }

// Mode products of one workgroup on 64 x 64 LDS tiles (zero beyond n), factor operands
// from registers:
//   mode 1:  X[i2][j1] <- sum_k X[i2][k] E1[j1][k]      (F = E1 rows j1 of this wave)
//   mode 2:  X[j2][i1] <- sum_k E2[j2][k] X[k][i1]      (F = E2 rows j2 of this wave)
// Each wave computes its 16 x 16 tile into registers; the barrier before the write-back
// lets the product overwrite its own input.
template <int MODE>
__device__ __forceinline__ void mode_product(double* X, const FactorFrags& F, int m1, int m2) {
  const int lane = threadIdx.x & 63;
  const int wm = tile_row(), wn = tile_col();
  const int lg = lane >> 4, lr = lane & 15;
  // two independent accumulators over alternate k-steps keep the matrix pipe busy
  d4 acc[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
  // v_mfma_f64_16x16x4: lane (lg, lr) supplies A[lr][lg] and B[lg][lr] of each 16x16x4 step
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int k = 4 * kk + lg;
    const double av = (MODE == 1) ? X[(wm + lr) * PS + k] : F.f[kk];   // X[i2][k] or E2[j2][k]
    const double bv = (MODE == 1) ? F.f[kk] : X[k * PS + wn + lr];     // E1[j1][k] or X[k][i1]
    acc[kk & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[kk & 1], 0, 0, 0);
  }
  __syncthreads();   // every wave has read X
  // f64 16x16 layout: lane l, element t holds row 4t + l/16, column l%16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = wm + 4 * t + lg, c = wn + lr;
    X[r * PS + c] = (r < m2 && c < m1) ? acc[0][t] + acc[1][t] : 0.0;
  }
  __syncthreads();
}

}  // namespace

// LE (L2B = 0) or Lawson2b (L2B = 1), nsteps steps of u (global, n2 x n1) in place.
template <int L2B>
__device__ __forceinline__ void lawson_small2d_body(const SmallArgs& p) {
  __shared__ double Us[NS * PS], V1[NS * PS], V2[L2B ? NS * PS : 1], As[PA * PA];
  const int n1 = p.n1, n2 = p.n2, tid = threadIdx.x;
  // factor fragments for the whole solve: mode 1 uses E1 rows of the wave's columns,
  // mode 2 E2 rows of the wave's rows
  FactorFrags F1, F2;
  load_frags(F1, p.E1, n1, tile_col());
  load_frags(F2, p.E2, n2, tile_row());
  for (int e = tid; e < NS * PS; e += THS) {
    const int i2 = e / PS, i1 = e % PS;
    Us[e] = (i2 < n2 && i1 < n1) ? p.u[i2 * n1 + i1] : 0.0;
    V1[e] = 0.0;
    if (L2B) V2[e] = 0.0;
  }
  for (int e = tid; e < (n2 + 2) * (n1 + 2); e += THS) {
    const int j2 = e / (n1 + 2), j1 = e % (n1 + 2);
    As[j2 * PA + j1] = p.a[e];
  }
  __syncthreads();
  const double tau = p.tau;
  bool bad = false;
  for (int it = 0; it < p.nsteps; ++it) {
    // first stage vectors: v1 = u + tau g(u) (LE and L2b), v2 = u + tau/2 g(u) (L2b)
    for (int e = tid; e < n1 * n2; e += THS) {
      const int i2 = e / n1, i1 = e % n1;
      const double g = g_small(p, Us, As, i2, i1);
      const double u = Us[i2 * PS + i1];
      V1[i2 * PS + i1] = u + tau * g;
      if (L2B) V2[i2 * PS + i1] = u + 0.5 * tau * g;
    }
    __syncthreads();
    mode_product<1>(V1, F1, n1, n2);
    mode_product<2>(V1, F2, n1, n2);
    if (!L2B) {
      // u+ = e^{tau A} v1
      for (int e = tid; e < NS * PS; e += THS) Us[e] = V1[e];
      __syncthreads();
      for (int e = tid; e < n1 * n2; e += THS) bad |= !(fabs(Us[(e / n1) * PS + e % n1]) <= DBL_MAX);
    } else {
      // U = e^{tau A} v1, W = e^{tau A} v2; u+ = W + tau/2 g(U)
      mode_product<1>(V2, F1, n1, n2);
      mode_product<2>(V2, F2, n1, n2);
      for (int e = tid; e < n1 * n2; e += THS) {
        const int i2 = e / n1, i1 = e % n1;
        const double o = V2[i2 * PS + i1] + 0.5 * tau * g_small(p, V1, As, i2, i1);
        bad |= !(fabs(o) <= DBL_MAX);
        Us[i2 * PS + i1] = o;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < n1 * n2; e += THS) p.u[e] = Us[(e / n1) * PS + e % n1];
  if (bad && p.flag) p.flag[0] = 1;
}

// One solve per workgroup: blockIdx.x selects the problem (its own sizes, factors,
// coefficients and step count). A single solve is launched the same way with one entry,
// so a problem's result does not depend on whether it ran alone or in a group.
template <int L2B>
__global__ __launch_bounds__(THS) void lawson_small2d_batch(SmallBatch b) {
  lawson_small2d_body<L2B>(b.a[blockIdx.x]);
}

bool small2d_fits(int d, int n1, int n2) { return d == 2 && n1 >= 1 && n2 >= 1 && n1 <= NS && n2 <= NS; }

hipError_t launch_lawson_small2d(const SmallArgs& a, bool l2b, hipStream_t s) {
  return launch_lawson_small2d_batch(&a, 1, l2b, s);
}

hipError_t launch_lawson_small2d_batch(const SmallArgs* a, int count, bool l2b, hipStream_t s) {
  if (count < 1 || count > kMaxSmallBatch) return hipErrorInvalidValue;
  SmallBatch b;
  for (int i = 0; i < count; ++i) {
    if (a[i].n1 < 1 || a[i].n2 < 1 || a[i].n1 > NS || a[i].n2 > NS || a[i].nsteps < 0) return hipErrorInvalidValue;
    b.a[i] = a[i];
  }
  if (l2b)
    lawson_small2d_batch<1><<<count, THS, 0, s>>>(b);
  else
    lawson_small2d_batch<0><<<count, THS, 0, s>>>(b);
  return hipGetLastError();
}

}  // namespace mm
