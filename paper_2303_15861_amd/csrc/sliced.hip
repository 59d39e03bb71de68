// Exact-slice mode products on the int8 matrix cores (v_mfma_i32_16x16x64_i8).
//
// Every operand row r (along the contracted index k) gets a power-of-two scale: e_r with
// max_k |x_rk| < 2^e_r. A value becomes Y = round(x 2^(8S-2-e_r)) (|Y| <= 2^(8S-2))
// written with S balanced base-256 digits b_i in [-128, 127] (int8 exactly):
//     x ~ 2^(e_r + 2 - 8S) sum_i b_i 256^i.
// The digits are the bytes of Y + 0x80..80 each minus 128 (an XOR with 0x80 per byte),
// so one 64-bit add and two XORs give all of them, packed. Then
//     sum_k A_mk B'_nk ~= 2^(e_m + e_n - 12) sum_(l<S) 2^(-8l) P_l,
//     P_l = sum_(s+t=l) sum_k dA_s dB_t     (digit planes s, t most significant first),
// where every partial sum of P_l is an integer below S 2^14 K < 2^31 (checked at launch),
// so the int32 accumulation is exact; the levels are combined in FP64 in the epilogue.
// Products with s + t >= S are dropped; with the rounding of Y they set the error,
// ~2^(-8S) relative to the row scales whatever the summation order.
//
// The factor (n x n, or stacked quadrature factors) is split once at setup into S digit
// planes with per-row exponents (rows zero-padded to a multiple of 64 in k). The grid
// operand stays FP64 in memory: each workgroup first finds the exponents of its 64 grid
// rows (mode 1) or columns (modes 2/3) over the whole k range, then splits values into
// digits while staging them into LDS, four consecutive k at a time (a 4 x 4 byte
// transpose turns four packed values into one dword per digit plane). Workgroup tile
// 64 x 64, four waves of 32 x 32, one accumulator per digit level.
#include "mm_internal.h"

namespace mm {

typedef int i4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int T8 = 64;      // workgroup tile
constexpr int KC8 = 64;     // k per chunk (one int8 MFMA)
constexpr int PI8 = 80;     // LDS row pitch in bytes (16 lanes of 16-byte reads hit all 64 banks once)
constexpr int TH = 256;

// Balanced base-256 digits of x relative to exponent e, packed: byte i of (lo, hi) is
// b_i (least significant first) as a two's-complement int8.
template <int S>
__device__ __forceinline__ void slice_bytes(double x, int e, unsigned& lo, unsigned& hi) {
  const double y = __builtin_rint(__builtin_ldexp(x, 8 * S - 2 - e));   // |y| <= 2^(8S-2)
  const double hf = __builtin_floor(y * 0x1p-32);
  const unsigned l = (unsigned)__builtin_fma(-hf, 0x1p32, y);           // exact, in [0, 2^32)
  const int h = (int)hf;
  constexpr unsigned long long C = 0x8080808080808080ull >> (64 - 8 * S);
  const unsigned long long Y = ((((unsigned long long)(unsigned)h) << 32) | l) + C;
  lo = (unsigned)Y ^ 0x80808080u;
  hi = (unsigned)(Y >> 32) ^ 0x80808080u;
}

// o[j] = byte j of w0, w1, w2, w3 (in that order, lowest byte first)
__device__ __forceinline__ void transpose4(unsigned w0, unsigned w1, unsigned w2, unsigned w3, unsigned (&o)[4]) {
  const unsigned t0 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);   // w0.b0 w1.b0 w0.b1 w1.b1
  const unsigned t1 = __builtin_amdgcn_perm(w1, w0, 0x07030602u);   // w0.b2 w1.b2 w0.b3 w1.b3
  const unsigned t2 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
  const unsigned t3 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
  o[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
  o[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
  o[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
  o[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// Digit planes (most significant first) of four consecutive values: pl[s] holds digit
// S-1-s of v0..v3 in its bytes 0..3.
template <int S>
__device__ __forceinline__ void slice4(double v0, double v1, double v2, double v3, int e, unsigned (&pl)[S]) {
  unsigned lo[4], hi[4];
  slice_bytes<S>(v0, e, lo[0], hi[0]);
  slice_bytes<S>(v1, e, lo[1], hi[1]);
  slice_bytes<S>(v2, e, lo[2], hi[2]);
  slice_bytes<S>(v3, e, lo[3], hi[3]);
  unsigned o[4];
  transpose4(lo[0], lo[1], lo[2], lo[3], o);
#pragma unroll
  for (int i = 0; i < 4 && i < S; ++i) pl[S - 1 - i] = o[i];
  if (S > 4) {
    transpose4(hi[0], hi[1], hi[2], hi[3], o);
#pragma unroll
    for (int i = 4; i < S; ++i) pl[S - 1 - i] = o[i - 4];
  }
}

__device__ __forceinline__ int row_exponent(double mx) {
  int e = 0;
  __builtin_frexp(mx, &e);                   // mx < 2^e (e = 0 for mx = 0)
  return e;
}

}  // namespace

template <int BT, int S>
__global__ __launch_bounds__(TH, 2) void gemm_i8(GemmArgs p) {
  constexpr int FI = 2;                      // 16 x 16 fragments per wave and dimension
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  int g, b, m0, n0;
  {
    const int tiles = p.tiles_m * p.tiles_n;
    const int gb = P / tiles;
    const int t = P - gb * tiles;
    g = gb / p.inner;
    b = gb - g * p.inner;
    int tm, tn;
    if (p.b_trans) {
      tm = t % p.tiles_m;
      tn = t / p.tiles_m;
    } else {
      tn = t % p.tiles_n;
      tm = t / p.tiles_n;
    }
    m0 = tm * T8;
    n0 = tn * T8;
  }
  const signed char* __restrict__ F =
      BT ? (const signed char*)p.A[g] + b * p.sA : (const signed char*)p.B[g] + b * p.sB;
  const double* __restrict__ V = BT ? (const double*)p.B[g] + b * p.sB : (const double*)p.A[g] + b * p.sA;
  const int* __restrict__ Fexp = p.fexp[g];
  double* __restrict__ C = (double*)p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;
  const int M = p.M, N = p.N, K = p.K;
  const int ldf = BT ? p.lda : p.ldb;        // digit-plane row stride (multiple of 64)
  const int ldv = BT ? p.ldb : p.lda;
  const int fr0 = BT ? m0 : n0, frows = BT ? M : N;
  const int vr0 = BT ? n0 : m0, vrows = BT ? N : M;
  const int64_t fsl = p.fac_slice;

  __shared__ __attribute__((aligned(16))) signed char Fs[S][T8 * PI8];
  __shared__ __attribute__((aligned(16))) signed char Vs[S][T8 * PI8];
  __shared__ int Fe[T8], Ve[T8];
  __shared__ double red[4][T8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lg = lane >> 4, lr = lane & 15;
  const int nch = (K + KC8 - 1) / KC8;

  // grid staging map. !BT: k quad kq = tid & 15 (k = 4kq..4kq+3), rows r16 + 16j.
  //                    BT: column n = tid & 63, k run 16 kg..16 kg+15.
  const int kq = tid & 15, r16 = tid >> 4;
  const int cn = tid & 63, kg = tid >> 6;

  // ---- exponents: factor rows from setup, grid rows/columns over the whole k range
  if (tid < T8) Fe[tid] = Fexp[min(fr0 + tid, frows - 1)];
  if (!BT) {
    double mx[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < nch; ++c) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned row = (unsigned)min(vr0 + r16 + 16 * j, vrows - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const unsigned k = (unsigned)min(c * KC8 + 4 * kq + q, K - 1);
          mx[j] = __builtin_fmax(mx[j], __builtin_fabs(V[row * (unsigned)ldv + k]));
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) mx[j] = __builtin_fmax(mx[j], __shfl_xor(mx[j], off, 16));
      if (kq == 0) Ve[r16 + 16 * j] = row_exponent(mx[j]);
    }
  } else {
    double mx = 0.0;
    const unsigned col = (unsigned)min(vr0 + cn, vrows - 1);
    for (int c = 0; c < nch; ++c) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const unsigned k = (unsigned)min(c * KC8 + 16 * kg + i, K - 1);
        mx = __builtin_fmax(mx, __builtin_fabs(V[k * (unsigned)ldv + col]));
      }
    }
    red[kg][cn] = mx;
    __syncthreads();
    if (tid < T8)
      Ve[tid] = row_exponent(__builtin_fmax(__builtin_fmax(red[0][tid], red[1][tid]),
                                            __builtin_fmax(red[2][tid], red[3][tid])));
  }
  __syncthreads();

  i4 acc[S][FI][FI];
#pragma unroll
  for (int l = 0; l < S; ++l)
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
      for (int j = 0; j < FI; ++j) acc[l][i][j] = i4{0, 0, 0, 0};

  // factor digits: 64 rows x 64 bytes per plane, one 16-byte vector per thread
  const int frow = tid >> 2, fk = (tid & 3) * 16;
  const int64_t foff = (int64_t)min(fr0 + frow, frows - 1) * ldf + fk;

  for (int c = 0; c < nch; ++c) {
    const int k0 = c * KC8;
    i4 rf[S];
#pragma unroll
    for (int s = 0; s < S; ++s) rf[s] = *reinterpret_cast<const i4*>(F + s * fsl + foff + k0);
    double rv[16];
    if (!BT) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const unsigned row = (unsigned)min(vr0 + r16 + 16 * j, vrows - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const unsigned k = (unsigned)min(k0 + 4 * kq + q, K - 1);
          rv[4 * j + q] = V[row * (unsigned)ldv + k];
        }
      }
    } else {
      const unsigned col = (unsigned)min(vr0 + cn, vrows - 1);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const unsigned k = (unsigned)min(k0 + 16 * kg + i, K - 1);
        rv[i] = V[k * (unsigned)ldv + col];
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) *reinterpret_cast<i4*>(&Fs[s][frow * PI8 + fk]) = rf[s];
    // k >= K: clamped grid values meet zero factor digits, so no masking is needed
    if (!BT) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rloc = r16 + 16 * j;
        unsigned pl[S];
        slice4<S>(rv[4 * j + 0], rv[4 * j + 1], rv[4 * j + 2], rv[4 * j + 3], Ve[rloc], pl);
#pragma unroll
        for (int s = 0; s < S; ++s) *reinterpret_cast<unsigned*>(&Vs[s][rloc * PI8 + 4 * kq]) = pl[s];
      }
    } else {
      const int e = Ve[cn];
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        unsigned pl[S];
        slice4<S>(rv[4 * qd + 0], rv[4 * qd + 1], rv[4 * qd + 2], rv[4 * qd + 3], e, pl);
#pragma unroll
        for (int s = 0; s < S; ++s) *reinterpret_cast<unsigned*>(&Vs[s][cn * PI8 + 16 * kg + 4 * qd]) = pl[s];
      }
    }
    __syncthreads();
    // A rows: grid (!BT) or factor (BT); B' rows: factor (!BT) or grid (BT)
    i4 af[S][FI];
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int i = 0; i < FI; ++i)
        af[s][i] = *reinterpret_cast<const i4*>(&(BT ? Fs : Vs)[s][(wm + 16 * i + lr) * PI8 + 16 * lg]);
#pragma unroll
    for (int sb = 0; sb < S; ++sb) {
      i4 bfr[FI];
#pragma unroll
      for (int j = 0; j < FI; ++j)
        bfr[j] = *reinterpret_cast<const i4*>(&(BT ? Vs : Fs)[sb][(wn + 16 * j + lr) * PI8 + 16 * lg]);
#pragma unroll
      for (int sa = 0; sa + sb < S; ++sa)
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FI; ++j)
            acc[sa + sb][i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[sa][i], bfr[j], acc[sa + sb][i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // 16x16 integer accumulator layout: lane l, element t holds row 4(l/16) + t, column l%16
  const double alpha = p.alpha * (p.galpha[g] != 0.0 ? p.galpha[g] : 1.0), beta = p.beta;
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FI; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ml = wm + 16 * i + 4 * lg + t, nl = wn + 16 * j + lr;
        const int m = m0 + ml, n = n0 + nl;
        if (m < M && n < N) {
          double v = (double)acc[S - 1][i][j][t];
#pragma unroll
          for (int l = S - 2; l >= 0; --l) v = __builtin_fma(v, 0x1p-8, (double)acc[l][i][j][t]);
          const int e = (BT ? Fe[ml] + Ve[nl] : Ve[ml] + Fe[nl]) - 12;
          double o = alpha * __builtin_ldexp(v, e);
          if (Cadd) o += beta * Cadd[m * p.ldc + n];
          C[m * p.ldc + n] = o;
        }
      }
}

// Split `rows` rows of an FP64 matrix (row stride lds, k columns) into S digit planes of
// row stride ldd (zero for k <= c < ldd) and per-row exponents. One workgroup per row.
__global__ __launch_bounds__(TH) void slice_rows(signed char* dst, int* exps, const double* src, int rows, int k,
                                                 int lds, int ldd, int S) {
  __shared__ double red[TH];
  const int r = blockIdx.x;
  if (r >= rows) return;
  const double* row = src + (int64_t)r * lds;
  double mx = 0.0;
  for (int c = threadIdx.x; c < k; c += TH) mx = __builtin_fmax(mx, __builtin_fabs(row[c]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = TH / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = __builtin_fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const int e = row_exponent(red[0]);
  if (threadIdx.x == 0) exps[r] = e;
  const int64_t plane = (int64_t)rows * ldd;
  for (int c = threadIdx.x; c < ldd; c += TH) {
    // Y = round(x 2^(8S-2-e)) as a 64-bit integer; its balanced base-256 digits follow
    // from the bytes of Y + 0x80..80
    const double x = (c < k) ? row[c] : 0.0;
    const double y = __builtin_rint(__builtin_ldexp(x, 8 * S - 2 - e));
    long long Y = (long long)__builtin_floor(y * 0x1p-32) * 4294967296ll +
                  (long long)(unsigned)__builtin_fma(-__builtin_floor(y * 0x1p-32), 0x1p32, y);
    const unsigned long long U = (unsigned long long)Y + (0x8080808080808080ull >> (64 - 8 * S));
    for (int s = 0; s < S; ++s) {
      const int i = S - 1 - s;                                  // digit i, plane s
      const int byte = (int)((U >> (8 * i)) & 255ull);
      dst[s * plane + (int64_t)r * ldd + c] = (signed char)(byte - 128);
    }
  }
}

hipError_t launch_slice_rows(signed char* dst, int* exps, const double* src, int rows, int k, int lds, int ldd,
                             int S, hipStream_t s) {
  if (rows <= 0 || k <= 0 || ldd < k || S < kMinSlices || S > kMaxSlices) return hipErrorInvalidValue;
  slice_rows<<<rows, TH, 0, s>>>(dst, exps, src, rows, k, lds, ldd, S);
  return hipGetLastError();
}

hipError_t launch_gemm_sliced(GemmArgs& g, hipStream_t s) {
  // every level sum must stay an exact int32: S products of at most 2^14 per k
  if ((int64_t)g.K * g.slices * 16384 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  g.tiles_m = (g.M + T8 - 1) / T8;
  g.tiles_n = (g.N + T8 - 1) / T8;
  const int64_t total = (int64_t)g.tiles_m * g.tiles_n * g.inner * g.groups;
  if (total >= ((int64_t)1 << 28)) return hipErrorInvalidValue;
  g.total = (int)total;
  g.per_xcd = (g.total + 7) / 8;
  const dim3 grid(8 * g.per_xcd), block(TH);
#define MM_SLICED_CASE(SS)                                  \
  case SS:                                                  \
    if (g.b_trans) gemm_i8<1, SS><<<grid, block, 0, s>>>(g); \
    else gemm_i8<0, SS><<<grid, block, 0, s>>>(g);           \
    break;
  switch (g.slices) {
    MM_SLICED_CASE(3)
    MM_SLICED_CASE(4)
    MM_SLICED_CASE(5)
    MM_SLICED_CASE(6)
    MM_SLICED_CASE(7)
    default: return hipErrorInvalidValue;
  }
#undef MM_SLICED_CASE
  return hipGetLastError();
}

}  // namespace mm
