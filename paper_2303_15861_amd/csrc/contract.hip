// mu-mode contraction kernels for gfx950 (Sec. 1 and Sec. 5.2: the action of the
// exponential of a Kronecker sum is a sequence of mode products V x_mu E_mu, each a
// dense GEMM with one small n x n factor and one large grid-shaped operand).
//
// Every mode product is cast as a batched row-major GEMM C = A . B' with
//   mode 1 (x1, fastest):  A = V viewed (n2 n3) x n1,  B'[n][k] = E1[n][k],   C = (n2 n3) x n1
//   mode 2:                A = E2,  B'[n][k] = V_slab[k][n] (slab = one x3 plane), C = n2 x n1
//   mode 3 (2D: mode 2):   A = E3,  B'[n][k] = V[k][n] with V viewed n3 x (n1 n2)
// so A is always read along k (row-major) and B' either along k (factor, mode 1) or
// along n (grid operand, modes 2/3, "b_trans"). Workgroup tile 128 x 128, four waves of
// 64 x 64, K staged through LDS in chunks; ragged edges are zero-filled on load and
// masked on store. The linear workgroup id is remapped so that tiles sharing the large
// operand are dispatched to the same XCD (workgroups are dealt round-robin over the
// eight XCDs, each with its own L2).
//
// Precisions (operands are FP64 in memory in every mode; conversion happens while
// staging into LDS):
//   FP64   v_mfma_f64_16x16x4 with FP64 accumulation.
//   FP32   operands rounded to FP32, v_mfma_f32_16x16x4, each 16-long K-chunk summed
//          in FP32 and added into FP64 accumulators.
//   BF16xS operands split into S BF16 slices (x = s0 + s1 [+ s2], each the nearest-even
//          BF16 of the remaining residual); all slice products s_i s_j with i + j < S on
//          v_mfma_f32_16x16x32_bf16, FP32 accumulation per 32-long K-chunk, chunk sums
//          added into FP32 accumulators.
#include "mm_internal.h"

namespace mm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int MT = 128, NT = 128, THREADS = 256;

__device__ __forceinline__ void decode_tile(const GemmArgs& p, int P, int& g, int& b, int& m0,
                                            int& n0) {
  const int tiles = p.tiles_m * p.tiles_n;
  const int gb = P / tiles;
  const int t = P - gb * tiles;
  g = gb / p.inner;
  b = gb - g * p.inner;
  int tm, tn;
  if (p.b_trans) {  // large operand is B': neighbouring ids share the n-tile
    tm = t % p.tiles_m;
    tn = t / p.tiles_m;
  } else {          // large operand is A: neighbouring ids share the m-tile
    tn = t % p.tiles_n;
    tm = t / p.tiles_n;
  }
  m0 = tm * MT;
  n0 = tn * NT;
}

// ------------------------------------------------------------------------------------
// FP64 and FP32: v_mfma_*_16x16x4. K-chunk of 16; within a chunk the four lane groups
// g = lane/16 take k = 4g + s at MFMA step s, so A and B use one consistent permutation.
// ------------------------------------------------------------------------------------
constexpr int KC4 = 16;
constexpr int P4 = KC4 + 1;  // LDS row pitch (elements), odd to spread banks

template <typename T, int BT>
struct Stage4 {
  // global -> registers for one 128 x 16 tile of A (rows m0.., k0..) and B'
  __device__ __forceinline__ static void loadA(double (&ra)[8], const double* __restrict__ A, int lda,
                                               int m0, int M, int k0, int K, int tid) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = i * THREADS + tid;
      const int row = e >> 4, kk = e & 15;
      const int m = m0 + row, k = k0 + kk;
      ra[i] = (m < M && k < K) ? A[m * lda + k] : 0.0;
    }
  }
  __device__ __forceinline__ static void loadB(double (&rb)[8], const double* __restrict__ B, int ldb,
                                               int n0, int N, int k0, int K, int tid) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = i * THREADS + tid;
      if (BT) {
        const int kk = e >> 7, nn = e & 127;
        const int n = n0 + nn, k = k0 + kk;
        rb[i] = (n < N && k < K) ? B[k * ldb + n] : 0.0;
      } else {
        const int row = e >> 4, kk = e & 15;
        const int n = n0 + row, k = k0 + kk;
        rb[i] = (n < N && k < K) ? B[n * ldb + k] : 0.0;
      }
    }
  }
  __device__ __forceinline__ static void storeA(T* s, const double (&ra)[8], int tid) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = i * THREADS + tid;
      s[(e >> 4) * P4 + (e & 15)] = (T)ra[i];
    }
  }
  __device__ __forceinline__ static void storeB(T* s, const double (&rb)[8], int tid) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = i * THREADS + tid;
      if (BT)
        s[(e & 127) * P4 + (e >> 7)] = (T)rb[i];
      else
        s[(e >> 4) * P4 + (e & 15)] = (T)rb[i];
    }
  }
};

template <int BT>
__global__ __launch_bounds__(THREADS, 2) void gemm_f64(GemmArgs p) {
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  int g, b, m0, n0;
  decode_tile(p, P, g, b, m0, n0);
  const double* __restrict__ A = p.A[g] + b * p.sA;
  const double* __restrict__ B = p.B[g] + b * p.sB;
  double* __restrict__ C = p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;

  __shared__ double As[2][MT * P4];
  __shared__ double Bs[2][NT * P4];
  using S = Stage4<double, BT>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lg = lane >> 4, lr = lane & 15;
  const int M = p.M, N = p.N, K = p.K;

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[8], rb[8];
  S::loadA(ra, A, p.lda, m0, M, 0, K, tid);
  S::loadB(rb, B, p.ldb, n0, N, 0, K, tid);
  S::storeA(As[0], ra, tid);
  S::storeB(Bs[0], rb, tid);
  __syncthreads();
  const int nch = (K + KC4 - 1) / KC4;
  for (int c = 0; c < nch; ++c) {
    const int cur = c & 1;
    if (c + 1 < nch) {
      S::loadA(ra, A, p.lda, m0, M, (c + 1) * KC4, K, tid);
      S::loadB(rb, B, p.ldb, n0, N, (c + 1) * KC4, K, tid);
    }
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 4 * lg + s;
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = as[(wm + 16 * i + lr) * P4 + kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = bs[(wn + 16 * j + lr) * P4 + kk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (c + 1 < nch) {
      S::storeA(As[cur ^ 1], ra, tid);
      S::storeB(Bs[cur ^ 1], rb, tid);
    }
    __syncthreads();
  }
  // f64 16x16 layout: lane l, element t holds row 4t + l/16, column l%16
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * t + lg;
        const int n = n0 + wn + 16 * j + lr;
        if (m < M && n < N) {
          double v = alpha * acc[i][j][t];
          if (Cadd) v += beta * Cadd[m * p.ldc + n];
          C[m * p.ldc + n] = v;
        }
      }
}

template <int BT>
__global__ __launch_bounds__(THREADS, 1) void gemm_f32(GemmArgs p) {
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  int g, b, m0, n0;
  decode_tile(p, P, g, b, m0, n0);
  const double* __restrict__ A = p.A[g] + b * p.sA;
  const double* __restrict__ B = p.B[g] + b * p.sB;
  double* __restrict__ C = p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;

  __shared__ float As[2][MT * P4];
  __shared__ float Bs[2][NT * P4];
  using S = Stage4<float, BT>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lg = lane >> 4, lr = lane & 15;
  const int M = p.M, N = p.N, K = p.K;

  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[8], rb[8];
  S::loadA(ra, A, p.lda, m0, M, 0, K, tid);
  S::loadB(rb, B, p.ldb, n0, N, 0, K, tid);
  S::storeA(As[0], ra, tid);
  S::storeB(Bs[0], rb, tid);
  __syncthreads();
  const int nch = (K + KC4 - 1) / KC4;
  for (int c = 0; c < nch; ++c) {
    const int cur = c & 1;
    if (c + 1 < nch) {
      S::loadA(ra, A, p.lda, m0, M, (c + 1) * KC4, K, tid);
      S::loadB(rb, B, p.ldb, n0, N, (c + 1) * KC4, K, tid);
    }
    const float* as = As[cur];
    const float* bs = Bs[cur];
    f4 part[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) part[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 4 * lg + s;
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = as[(wm + 16 * i + lr) * P4 + kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = bs[(wn + 16 * j + lr) * P4 + kk];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], part[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[i][j][t] += (double)part[i][j][t];
    if (c + 1 < nch) {
      S::storeA(As[cur ^ 1], ra, tid);
      S::storeB(Bs[cur ^ 1], rb, tid);
    }
    __syncthreads();
  }
  // f32 16x16 layout: lane l, element t holds row 4(l/16) + t, column l%16
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * lg + t;
        const int n = n0 + wn + 16 * j + lr;
        if (m < M && n < N) {
          double v = alpha * acc[i][j][t];
          if (Cadd) v += beta * Cadd[m * p.ldc + n];
          C[m * p.ldc + n] = v;
        }
      }
}

// ------------------------------------------------------------------------------------
// Split BF16: K-chunk of 32 (one v_mfma_f32_16x16x32_bf16 per tile and product). LDS
// holds S slices of each operand, rows of 32 k (+8 pad) so that lane group g reads its
// eight consecutive k (8g .. 8g+7) as one 16-byte access.
// ------------------------------------------------------------------------------------
constexpr int KCB = 32;
constexpr int PB = 40;

template <int S>
__device__ __forceinline__ void split_bf16(double x, __bf16 (&out)[S]) {
  double rem = x;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const __bf16 h = (__bf16)(float)rem;
    out[s] = h;
    rem -= (double)(float)h;
  }
}

template <int BT, int S>
__global__ __launch_bounds__(THREADS, 2) void gemm_bf16(GemmArgs p) {
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  int g, b, m0, n0;
  decode_tile(p, P, g, b, m0, n0);
  const double* __restrict__ A = p.A[g] + b * p.sA;
  const double* __restrict__ B = p.B[g] + b * p.sB;
  double* __restrict__ C = p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;

  __shared__ __attribute__((aligned(16))) __bf16 As[S][MT * PB];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[S][NT * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int lg = lane >> 4, lr = lane & 15;
  const int M = p.M, N = p.N, K = p.K;

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // each thread stages two runs of 8 consecutive k for A and for B'
  double ra[2][8], rb[2][8];
  auto load = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = h * THREADS + tid;
      {  // A: row = e/4, k run = 8*(e%4)
        const int row = e >> 2, k8 = (e & 3) * 8;
        const int m = m0 + row;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = k0 + k8 + j;
          ra[h][j] = (m < M && k < K) ? A[m * p.lda + k] : 0.0;
        }
      }
      if (BT) {  // B'[n][k] = B[k*ldb + n]: lanes take consecutive n
        const int nn = e & 127, k8 = (e >> 7) * 8;
        const int n = n0 + nn;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = k0 + k8 + j;
          rb[h][j] = (n < N && k < K) ? B[k * p.ldb + n] : 0.0;
        }
      } else {
        const int row = e >> 2, k8 = (e & 3) * 8;
        const int n = n0 + row;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = k0 + k8 + j;
          rb[h][j] = (n < N && k < K) ? B[n * p.ldb + k] : 0.0;
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = h * THREADS + tid;
      bf8 va[S], vb[S];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 sa[S], sb[S];
        split_bf16<S>(ra[h][j], sa);
        split_bf16<S>(rb[h][j], sb);
#pragma unroll
        for (int s = 0; s < S; ++s) {
          va[s][j] = sa[s];
          vb[s][j] = sb[s];
        }
      }
      const int rowA = e >> 2, kA = (e & 3) * 8;
      int rowB, kB;
      if (BT) {
        rowB = e & 127;
        kB = (e >> 7) * 8;
      } else {
        rowB = e >> 2;
        kB = (e & 3) * 8;
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        *reinterpret_cast<bf8*>(&As[s][rowA * PB + kA]) = va[s];
        *reinterpret_cast<bf8*>(&Bs[s][rowB * PB + kB]) = vb[s];
      }
    }
  };

  const int nch = (K + KCB - 1) / KCB;
  load(0);
  for (int c = 0; c < nch; ++c) {
    store();
    __syncthreads();
    if (c + 1 < nch) load((c + 1) * KCB);
    bf8 av[S][4], bv[S][4];
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        av[s][i] = *reinterpret_cast<const bf8*>(&As[s][(wm + 16 * i + lr) * PB + 8 * lg]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        bv[s][j] = *reinterpret_cast<const bf8*>(&Bs[s][(wn + 16 * j + lr) * PB + 8 * lg]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int sa = 0; sa < S; ++sa)
#pragma unroll
          for (int sb = 0; sb + sa < S; ++sb)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[sa][i], bv[sb][j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * lg + t;
        const int n = n0 + wn + 16 * j + lr;
        if (m < M && n < N) {
          double v = alpha * (double)acc[i][j][t];
          if (Cadd) v += beta * Cadd[m * p.ldc + n];
          C[m * p.ldc + n] = v;
        }
      }
}

hipError_t launch_gemm(int prec, GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.inner <= 0 || g.groups <= 0 || g.groups > kMaxGroups)
    return hipErrorInvalidValue;
  // in-batch offsets are 32-bit
  const int64_t lim = (int64_t)1 << 31;
  if ((int64_t)g.M * g.lda >= lim || (int64_t)g.M * g.ldc >= lim ||
      (int64_t)(g.b_trans ? g.K : g.N) * g.ldb >= lim)
    return hipErrorInvalidValue;
  g.tiles_m = (g.M + MT - 1) / MT;
  g.tiles_n = (g.N + NT - 1) / NT;
  const int64_t total = (int64_t)g.tiles_m * g.tiles_n * g.inner * g.groups;
  if (total >= lim / 8) return hipErrorInvalidValue;
  g.total = (int)total;
  g.per_xcd = (g.total + 7) / 8;
  const dim3 grid(8 * g.per_xcd), block(THREADS);
  switch (prec) {
    case MM_FP64:
      if (g.b_trans) gemm_f64<1><<<grid, block, 0, s>>>(g);
      else gemm_f64<0><<<grid, block, 0, s>>>(g);
      break;
    case MM_FP32:
      if (g.b_trans) gemm_f32<1><<<grid, block, 0, s>>>(g);
      else gemm_f32<0><<<grid, block, 0, s>>>(g);
      break;
    case MM_BF16X3:
      if (g.b_trans) gemm_bf16<1, 2><<<grid, block, 0, s>>>(g);
      else gemm_bf16<0, 2><<<grid, block, 0, s>>>(g);
      break;
    case MM_BF16X6:
      if (g.b_trans) gemm_bf16<1, 3><<<grid, block, 0, s>>>(g);
      else gemm_bf16<0, 3><<<grid, block, 0, s>>>(g);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mm
