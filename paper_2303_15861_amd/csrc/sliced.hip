// Exact-slice mode products on the int8 matrix cores (v_mfma_i32_32x32x32_i8).
//
// Every operand row r (along the contracted index k) gets a power-of-two scale: e_r with
// max_k |x_rk| (1 + 2^-7) < 2^e_r. A value becomes Y = round(x 2^(8S-1-e_r))
// (|Y| < 0.4963 256^S) written with S balanced base-256 digits b_i in [-128, 127] (int8
// exactly; they cover [-0.502, 0.498] 256^S):
//     x ~ 2^(e_r + 1 - 8S) sum_i b_i 256^i.
// The digits are the bytes of Y + 0x80..80 each minus 128 (an XOR with 0x80 per byte),
// so one 64-bit add and two XORs give all of them, packed. Then
//     sum_k A_mk B'_nk ~= 2^(e_m + e_n - 14) sum_(l<S) 2^(-8l) P_l,
//     P_l = sum_(s+t=l) sum_k dA_s dB_t     (digit planes s, t most significant first),
// where every partial sum of P_l is an integer below S 2^14 K < 2^31 (checked at launch),
// so the int32 accumulation is exact; the levels are combined in FP64 in the epilogue.
// Products with s + t >= S are dropped; with the rounding of Y they set the error,
// ~2^(-8S) relative to the row scales whatever the summation order.
//
// The factor (n x n, or stacked quadrature factors) is split once at setup into S digit
// planes with per-row exponents (rows zero-padded to a multiple of 64 in k). The grid
// operand is split once per launch by slice_grid, a streaming pass that finds the
// exponent of every grid fiber (a row of the operand in mode 1, a column in modes 2/3,
// over the whole k range) and writes its digit planes (k-contiguous rows in mode 1, runs
// of 16 k of adjacent fibers in modes 2/3). The product kernel then stages both operands
// into LDS with
// 16-byte loads only (splitting inside the product kernel would repeat the work once
// per 64-row output tile). Workgroup tile 64 x 64, four waves of 32 x 32, one
// accumulator per digit level.
#include "mm_internal.h"
#include "slice_digits.h"
#include "wave_ops.h"

#include <type_traits>

namespace mm {

typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int T8 = 64;      // workgroup tile
constexpr int KC8 = 64;     // k per chunk (two int8 MFMA k-steps)
constexpr int PI8 = 80;     // LDS row pitch in bytes (chosen so that 16 lanes of 16-byte reads from
                            // consecutive rows would hit 64 banks once; gfx950's bank-conflict
                            // counter still counts conflicts on this kernel's LDS accesses)
constexpr int TH = 256;

__device__ __forceinline__ int row_exponent(double mx) { return digits::digit_exponent(mx); }

}  // namespace

// Grid digits of group g, plane s (plane = fibers * slice_ld(K) bytes, group stride
// S * plane):
//   mode 1 (rows):     base + fiber * slice_ld(K) + k                 (k contiguous)
//   modes 2/3 (cols):  base + (k / 16) * (fibers * 16) + fiber * 16 + k % 16
// (16 consecutive k of one fiber per 16-byte vector, consecutive fibers adjacent, so
// that the column split writes, and the product stages, whole 1 KB runs).
template <int BT, int S>
__global__ __launch_bounds__(TH) void slice_grid(GemmArgs p, int fblocks) {
  const int g = blockIdx.x / fblocks;
  const int fb = blockIdx.x - g * fblocks;
  const int K = p.K, kp = slice_ld(K);
  const int64_t F = sliced_fibers(p);
  const int64_t plane = F * kp;
  signed char* __restrict__ D = p.vdig + g * (S * plane);
  int* __restrict__ X = p.vexp + g * F;
  const int tid = threadIdx.x;
  if (!BT) {
    // one wave per row, four consecutive k per lane (coalesced row reads and writes)
    const int row = fb * (TH / 64) + (tid >> 6), lane = tid & 63;
    if (row >= p.M) return;   // whole waves
    const double* __restrict__ vr = (const double*)p.A[g] + (int64_t)row * p.lda;
    double mx = 0.0;
    for (int k0 = 4 * lane; k0 < K; k0 += 256)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (k0 + i < K) mx = __builtin_fmax(mx, __builtin_fabs(vr[k0 + i]));
    mx = wave::wave_max(mx);
    const int e = row_exponent(mx);
    if (lane == 0) X[row] = e;
    signed char* __restrict__ dr = D + (int64_t)row * kp;
    for (int k0 = 4 * lane; k0 < kp; k0 += 256) {
      double v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (k0 + i < K) ? vr[k0 + i] : 0.0;
      unsigned pl[S];
      digits::slice4<S>(v[0], v[1], v[2], v[3], e, pl);
#pragma unroll
      for (int t = 0; t < S; ++t) *reinterpret_cast<unsigned*>(dr + t * plane + k0) = pl[t];
    }
  } else {
    // 64 columns of one batch per workgroup; lane = column, the four waves take every
    // fourth 16-run of k; for K <= 256 the values stay in registers between the
    // exponent scan and the split
    const int nb = (p.N + T8 - 1) / T8;
    const int b = fb / nb, n = (fb - b * nb) * T8 + (tid & 63), kg = tid >> 6;
    const bool live = n < p.N;
    const double* __restrict__ V = (const double*)p.B[g] + b * p.sB + (live ? n : 0);
    __shared__ double red[4][T8];
    const int64_t f = (int64_t)b * p.N + n;
    auto store = [&](int k0, const double (&v)[16], int e) {
      unsigned pl[4][S];
#pragma unroll
      for (int q = 0; q < 4; ++q) digits::slice4<S>(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3], e, pl[q]);
#pragma unroll
      for (int t = 0; t < S; ++t)
        *reinterpret_cast<i4*>(D + t * plane + (int64_t)(k0 >> 4) * (F * 16) + f * 16) =
            i4{(int)pl[0][t], (int)pl[1][t], (int)pl[2][t], (int)pl[3][t]};
    };
    if (K <= 256) {
      double v[4][16];
      double mx = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int k = 16 * kg + 64 * j + i;
          v[j][i] = (k < K) ? V[(int64_t)k * p.ldb] : 0.0;
          mx = __builtin_fmax(mx, __builtin_fabs(v[j][i]));
        }
      red[kg][tid & 63] = mx;
      __syncthreads();
      const int c = tid & 63;
      const int e =
          row_exponent(__builtin_fmax(__builtin_fmax(red[0][c], red[1][c]), __builtin_fmax(red[2][c], red[3][c])));
      if (!live) return;
      if (kg == 0) X[f] = e;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (16 * kg + 64 * j < kp) store(16 * kg + 64 * j, v[j], e);
    } else {
      double mx = 0.0;
      for (int k0 = 16 * kg; k0 < K; k0 += 64)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (k0 + i < K) mx = __builtin_fmax(mx, __builtin_fabs(V[(int64_t)(k0 + i) * p.ldb]));
      red[kg][tid & 63] = mx;
      __syncthreads();
      const int c = tid & 63;
      const int e =
          row_exponent(__builtin_fmax(__builtin_fmax(red[0][c], red[1][c]), __builtin_fmax(red[2][c], red[3][c])));
      if (!live) return;
      if (kg == 0) X[f] = e;
      for (int k0 = 16 * kg; k0 < kp; k0 += 64) {
        double v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = (k0 + i < K) ? V[(int64_t)(k0 + i) * p.ldb] : 0.0;
        store(k0, v, e);
      }
    }
  }
}

template <int BT, int S>
__global__ __launch_bounds__(TH, 2) void gemm_i8(GemmArgs p) {
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
  const int* __restrict__ Fexp = p.fexp[g];
  double* __restrict__ C = (double*)p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;
  const int M = p.M, N = p.N, K = p.K;
  const int ldf = BT ? p.lda : p.ldb;        // digit-plane row stride (multiple of 64)
  const int fr0 = BT ? m0 : n0, frows = BT ? M : N;
  const int vr0 = BT ? n0 : m0, vrows = BT ? N : M;
  const int64_t fsl = p.fac_slice;
  // grid digits of this group and the fiber of this thread's staging column
  const int64_t nfib = sliced_fibers(p);
  const int64_t vplane = nfib * slice_ld(K);
  const signed char* __restrict__ Vd = p.vdig + g * (S * vplane);
  const int* __restrict__ Vx = p.vexp + g * nfib;
  const int64_t vfib0 = BT ? (int64_t)b * N : 0;

  __shared__ __attribute__((aligned(16))) signed char Fs[S][T8 * PI8];
  __shared__ __attribute__((aligned(16))) signed char Vs[S][T8 * PI8];
  __shared__ int Fe[T8], Ve[T8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int nch = (K + KC8 - 1) / KC8;

  // exponents of the factor rows and the grid fibers of this tile (fibers past the end
  // repeat the last one; their outputs are not stored)
  if (tid < T8) {
    Fe[tid] = Fexp[min(fr0 + tid, frows - 1)];
    Ve[tid] = Vx[vfib0 + min(vr0 + tid, vrows - 1)];
  }

  // one 32 x 32 accumulator per digit level (v_mfma_i32_32x32x32_i8: the 32x32x32 form
  // runs at about twice the int8 rate of the 16x16x64 form on this chip)
  i16 acc[S];
#pragma unroll
  for (int l = 0; l < S; ++l)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[l][j] = 0;

  // factor digits: 64 rows x 64 bytes per plane, one 16-byte vector per thread
  const int frow = tid >> 2, fk = (tid & 3) * 16;
  const int64_t foff = (int64_t)min(fr0 + frow, frows - 1) * ldf + fk;
  // grid digits, one 16-byte vector per thread: modes 2/3 fiber cn = tid & 63, k run
  // kg = tid >> 6 of the chunk; mode 1 like the factor (fiber tid >> 2, k 16 (tid & 3))
  const int cn = BT ? (tid & 63) : (tid >> 2);
  const int vk = BT ? 16 * (tid >> 6) : 16 * (tid & 3);
  const int64_t vfib = vfib0 + min(vr0 + cn, vrows - 1);
  const int64_t voff = BT ? vfib * 16 + (int64_t)(vk >> 4) * (nfib * 16) : vfib * slice_ld(K) + vk;
  const int64_t vstep = BT ? 4 * (nfib * 16) : KC8;   // per chunk

  // chunk c's digits into registers (the next chunk's loads overlap this chunk's products)
  i4 rf[S], rv[S];
  auto load = [&](int c) {
#pragma unroll
    for (int s = 0; s < S; ++s) rf[s] = *reinterpret_cast<const i4*>(F + s * fsl + foff + c * KC8);
#pragma unroll
    for (int s = 0; s < S; ++s) rv[s] = *reinterpret_cast<const i4*>(Vd + s * vplane + voff + c * vstep);
  };
  load(0);
  for (int c = 0; c < nch; ++c) {
#pragma unroll
    for (int s = 0; s < S; ++s) *reinterpret_cast<i4*>(&Fs[s][frow * PI8 + fk]) = rf[s];
#pragma unroll
    for (int s = 0; s < S; ++s) *reinterpret_cast<i4*>(&Vs[s][cn * PI8 + vk]) = rv[s];
    __syncthreads();
    if (c + 1 < nch) load(c + 1);
    // A rows: grid (!BT) or factor (BT); B' rows: factor (!BT) or grid (BT). Lane l
    // supplies row l % 32 of its operand, k bytes 16 (l / 32) .. +15 of each 32-k step.
    // All 2S fragments of a 32-k step are read before its products, so one LDS wait
    // covers the step; the S(S+1)/2 products then go round-robin over the levels (round r
    // takes digit sa = r of A against sb = l - r for every level l >= r), so consecutive
    // MFMAs update different accumulators; odd steps run the levels upwards so that the
    // step boundary does not chain two updates of one level. Integer sums: the order does
    // not change the result.
    const int rl = lane & 31, kh = 16 * (lane >> 5);
#pragma unroll
    for (int ks = 0; ks < KC8 / 32; ++ks) {
      i4 af[S], bf[S];
#pragma unroll
      for (int s = 0; s < S; ++s)
        af[s] = *reinterpret_cast<const i4*>(&(BT ? Fs : Vs)[s][(wm + rl) * PI8 + 32 * ks + kh]);
#pragma unroll
      for (int s = 0; s < S; ++s)
        bf[s] = *reinterpret_cast<const i4*>(&(BT ? Vs : Fs)[s][(wn + rl) * PI8 + 32 * ks + kh]);
#pragma unroll
      for (int r = 0; r < S; ++r)
#pragma unroll
        for (int i = 0; i < S - r; ++i) {
          const int l = (ks & 1) ? r + i : S - 1 - i;   // level of this product
          acc[l] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[r], bf[l - r], acc[l], 0, 0, 0);
        }
    }
    __syncthreads();
  }

  // 32x32 integer accumulator layout: lane l, element j holds row 8(j/4) + 4(l/32) + j%4,
  // column l%32
  const double alpha = p.alpha * (p.galpha[g] != 0.0 ? p.galpha[g] : 1.0), beta = p.beta;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int ml = wm + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3), nl = wn + (lane & 31);
    const int m = m0 + ml, n = n0 + nl;
    if (m < M && n < N) {
      double v = (double)acc[S - 1][j];
#pragma unroll
      for (int l = S - 2; l >= 0; --l) v = __builtin_fma(v, 0x1p-8, (double)acc[l][j]);
      const int e = (BT ? Fe[ml] + Ve[nl] : Ve[ml] + Fe[nl]) - 14;
      double o = alpha * __builtin_ldexp(v, e);
      if (Cadd) o += beta * Cadd[m * p.ldc + n];
      C[m * p.ldc + n] = o;
    }
  }
}

// ---------------------------------------------------------------- chained products
// A tile: 32 factor rows (m) against the F <= 256 fibers of one fiber group (j), all K.
// The factor digits are staged through LDS (shared by every wave); each wave streams the
// digits of its own WN fibers straight from memory into MFMA fragment registers, one
// 2 KB block per pair of load instructions (the chain layout of slice_digits.h). At MFMA
// step ks of a 64-k chunk, lane half h supplies chunk bytes [32h + 16ks, +16) of both
// operands (a fixed permutation of k; integer sums do not depend on the order).
// The epilogue combines the digit levels in FP64 exactly as gemm_i8 does; for a middle
// mode it stages the 32 x 256 result tile in LDS, takes each row's maximum (a whole fiber
// of the next product) and writes the row's digit planes and exponent in the chain layout,
// the digits that slice_grid would produce for the same values. Its stores are
// nontemporal: their reader is the next launch, and L2 is kept for the digits being read.
// Workgroups are persistent (one per compute unit, each walking tiles of its XCD's range;
// the eight factor-row tiles of a fiber group run side by side on one XCD and share its
// digits in L2), and the last chunk of a tile already loads the next tile's first factor
// chunk, grid fragments and exponents, so that their latency and the epilogue overlap.
namespace {
constexpr int CM = 32;        // factor rows per tile
constexpr int CF = 256;       // fibers per tile
constexpr int CPI = 80;       // LDS row pitch (bytes) of the staged factor digits
constexpr int CPD = CF + 32;  // LDS row pitch (doubles) of the staged result tile: two
                              // doubles of padding after every 16, so that the 16 lanes
                              // reading one row's 16-value segments hit distinct banks
constexpr int CSLOTS = 32;    // persistent workgroups per XCD (one per compute unit)
__device__ __forceinline__ int cs_col(int j) { return j + 2 * (j >> 4); }
}  // namespace

template <int S, int WN>
__global__ __launch_bounds__(64 * (CF / WN), 1) void gemm_i8_chain(ChainArgs p) {
  constexpr int NW = CF / WN;      // waves
  constexpr int NT = 64 * NW;      // threads
  constexpr int NB = WN / 32;      // 32-fiber MFMA blocks per wave
  const int xcd = blockIdx.x & 7, nslot = gridDim.x >> 3;
  const int Pend = min(p.total, (xcd + 1) * p.per_xcd);
  int P = xcd * p.per_xcd + (blockIdx.x >> 3);
  if (P >= Pend) return;
  const int M = p.M, K = p.K, F = p.F;
  const int kp = slice_ld(K);
  const int nch = kp / 64;

  constexpr int ABYTES = 2 * S * CM * CPI;
  __shared__ __attribute__((aligned(16))) unsigned char As[ABYTES];
  __shared__ __attribute__((aligned(16))) double Cs[CM * CPD];
  __shared__ __attribute__((aligned(16))) int Fe[2][CM];
  __shared__ __attribute__((aligned(16))) int Junk[256];   // target of the L2 prefetch loads

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int half = lane >> 5, rl = lane & 31;

  // factor staging: piece q = (plane, row, 16-byte part) -> registers -> LDS
  constexpr int APIECES = S * CM * 4;
  constexpr int AREG = (APIECES + NT - 1) / NT;
  i4 ra[AREG];
  auto aload = [&](int m0, int c) {
#pragma unroll
    for (int i = 0; i < AREG; ++i) {
      const int q = tid + i * NT;
      if (q < APIECES) {
        const int s = q / (4 * CM), r = (q >> 2) % CM, part = q & 3;
        ra[i] = *reinterpret_cast<const i4*>(p.fdig + s * p.fplane + (int64_t)min(m0 + r, M - 1) * kp + c * 64 +
                                             16 * part);
      }
    }
  };
  auto astore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AREG; ++i) {
      const int q = tid + i * NT;
      if (q < APIECES) {
        const int s = q / (4 * CM), r = (q >> 2) % CM, part = q & 3;
        *reinterpret_cast<i4*>(As + ((buf * S + s) * CM + r) * CPI + 16 * part) = ra[i];
      }
    }
  };

  // grid fragments of the two MFMA steps of a chunk: slot ks holds step ks and is
  // refilled with step ks of the next chunk (of this tile, else the next tile's first)
  // right after that step's products
  i4 bq[NB][S][2];
  auto gbase = [&](int g, int b) {
    return p.vdig + ((int64_t)(g * 8 + wave * NB + b) * nch) * (S * 2048) + rl * 64 + 32 * half;
  };
  auto bload_plane = [&](const signed char* const (&base)[NB], int c, int ks, int s) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
      bq[b][s][ks] = *reinterpret_cast<const i4*>(base[b] + (c * S + s) * 2048 + ks * 16);
  };
  auto bload = [&](const signed char* const (&base)[NB], int c, int ks) {
#pragma unroll
    for (int s = 0; s < S; ++s) bload_plane(base, c, ks, s);
  };

  // the first tile's prefetch
  const signed char* vbn[NB];
  int ve_n[NB], fe_n = 0;
  {
    const int g = P / p.tiles_m, m0 = (P % p.tiles_m) * CM;
#pragma unroll
    for (int b = 0; b < NB; ++b) vbn[b] = gbase(g, b);
    aload(m0, 0);
    bload(vbn, 0, 0);
    bload(vbn, 0, 1);
#pragma unroll
    for (int b = 0; b < NB; ++b) ve_n[b] = p.vexp[g * 256 + wave * WN + 32 * b + rl];
    if (tid < CM) fe_n = p.fexp[min(m0 + tid, M - 1)];
  }

  for (int it = 0;; ++it) {
    const int m0 = (P % p.tiles_m) * CM, grp = P / p.tiles_m;
    const int v = grp / p.Gv, gi = grp - v * p.Gv;
    const int Pn = P + nslot;
    const bool next = Pn < Pend;
    const int m0n = next ? (Pn % p.tiles_m) * CM : m0, grpn = next ? Pn / p.tiles_m : grp;
    const signed char* vb[NB];
    int ve[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      vb[b] = vbn[b];
      vbn[b] = gbase(grpn, b);
      ve[b] = ve_n[b];
    }
    const int fe = it & 1;
    if (tid < CM) Fe[fe][tid] = fe_n;
    astore(0);

    __syncthreads();

    // the next tile's grid digits into L2 while this tile runs: its eight factor-row tiles
    // run on eight compute units of this XCD, each of which brings one 32-fiber block (one
    // contiguous run of nch S 2 KB) with loads straight into a junk LDS block (no
    // registers; issued after the step loads they must not delay)
    const int64_t pf_base = ((int64_t)grpn * 8 + (Pn % p.tiles_m)) * nch * (S * 2048);
    const bool pf = next && (Pn % p.tiles_m) < 8;
    auto prefetch = [&](int c) {
      constexpr int Q = (S + 3) / 4;   // 1 KB units per wave and chunk: 8 nch Q >= 2 nch S
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int u = wave + 8 * (c * Q + q);
        if (u < 2 * nch * S)
          __builtin_amdgcn_global_load_lds(
              (const __attribute__((address_space(1))) void*)(p.vdig + pf_base + (int64_t)u * 1024 + lane * 16),
              (__attribute__((address_space(3))) void*)Junk, 16, 0, 0);
      }
    };

    i16 acc[NB][S];
    // one 64-k chunk: two MFMA steps; Z: the tile's first chunk, whose first product of
    // every level starts from zero instead of an accumulator
    auto chunk = [&](auto zinit, int c) {
      constexpr bool Z = decltype(zinit)::value;
      const int buf = c & 1;
      const bool more = c + 1 < nch;
      const bool pre = more || next;   // a chunk to prefetch (this tile's or the next's)
      if (pre) aload(more ? m0 : m0n, more ? c + 1 : 0);
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        i4 af[S];
#pragma unroll
        for (int s = 0; s < S; ++s)
          af[s] = *reinterpret_cast<const i4*>(As + ((buf * S + s) * CM + rl) * CPI + 32 * half + 16 * ks);
        // round t: grid digit t against factor digit s for every level l = s + t < S (the
        // factor digits alternate direction between steps, blocks innermost, so that
        // consecutive products update different accumulators). Grid plane t is read in
        // round t only: right after it, the plane's slot is refilled with the same step
        // of the next chunk, two steps ahead of its use.
#pragma unroll
        for (int t = 0; t < S; ++t) {
#pragma unroll
          for (int i = 0; i < S - t; ++i) {
            const int sa = ks ? i : S - 1 - t - i, l = sa + t;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              if (Z && ks == 0 && t == 0)
                acc[b][l] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[sa], bq[b][t][ks], i16{}, 0, 0, 0);
              else
                acc[b][l] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[sa], bq[b][t][ks], acc[b][l], 0, 0, 0);
            }
          }
          if (pre) bload_plane(more ? vb : vbn, more ? c + 1 : 0, ks, t);
        }
      }
      if (pf && more) prefetch(c);
      if (more) astore(buf ^ 1);
      __syncthreads();
    };
    chunk(std::true_type{}, 0);
    for (int c = 1; c < nch; ++c) chunk(std::false_type{}, c);
    if (next) {
#pragma unroll
      for (int b = 0; b < NB; ++b) ve_n[b] = p.vexp[grpn * 256 + wave * WN + 32 * b + rl];
      if (tid < CM) fe_n = p.fexp[min(m0n + tid, M - 1)];
    }

    // accumulator element e of lane l: factor row 8(e/4) + 4(l/32) + e%4, fiber l%32 of
    // the block; the factor-row exponents of four consecutive elements in one 16-byte read
    auto value = [&](int b, int e, int ex) {
      double x = (double)acc[b][S - 1][e];
#pragma unroll
      for (int l = S - 2; l >= 0; --l) x = __builtin_fma(x, 0x1p-8, (double)acc[b][l][e]);
      return __builtin_ldexp(x, ex - 14);
    };
    if (!p.odig) {
      // FP64 rows m0 + 4 half + 8 q + e4 of output row block (v, gi): element offsets from
      // the lane's first row by multiples of the row stride Gv ldo
      const int64_t rs = (int64_t)p.Gv * p.ldo;
      double* const ob = p.out + (int64_t)v * p.ovs + ((int64_t)(m0 + 4 * half) * p.Gv + gi) * p.ldo;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const i4 fq = *reinterpret_cast<const i4*>(&Fe[fe][8 * q + 4 * half]);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int j = wave * WN + 32 * b + rl;
#pragma unroll
          for (int e4 = 0; e4 < 4; ++e4) {
            const double x = value(b, 4 * q + e4, fq[e4] + ve[b]);
            if (m0 + 4 * half + 8 * q + e4 < M && j < F) __builtin_nontemporal_store(x, ob + (8 * q + e4) * rs + j);
          }
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const i4 fq = *reinterpret_cast<const i4*>(&Fe[fe][8 * q + 4 * half]);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int j = wave * WN + 32 * b + rl;
#pragma unroll
          for (int e4 = 0; e4 < 4; ++e4) {
            const int ml = 8 * q + 4 * half + e4;
            const double x = value(b, 4 * q + e4, fq[e4] + ve[b]);
            Cs[ml * CPD + cs_col(j)] = (m0 + ml < M && j < F) ? x : 0.0;
          }
        }
      }
    }
    if (p.odig) {
      __syncthreads();
      // row r of the tile in 16-value segments, one per thread; the 16 segments of a row
      // are 16 consecutive lanes
      const int kq = slice_ld(F), nchq = kq / 64;
#pragma unroll
      for (int itm = tid; itm < CM * 16; itm += NT) {
        const int r = itm >> 4, sg = itm & 15;
        double x[16];
        double mx = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          x[i] = Cs[r * CPD + cs_col(16 * sg) + i];
          mx = __builtin_fmax(mx, __builtin_fabs(x[i]));
        }
        mx = wave::row16_max(mx);
        const int e = row_exponent(mx);
        const int m = m0 + r;
        if (m < M && 16 * sg < kq) {
          // the next product's fiber: group go, fiber jn (fewer than 2^31 fibers: checked
          // at launch)
          const unsigned lin = ((unsigned)v * M + m) * p.Gv + gi;
          const unsigned go = lin / (unsigned)p.Fn;
          const int jn = (int)(lin - go * p.Fn);
          unsigned pl[4][S];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            digits::slice4<S>(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3], e, pl[q]);
          signed char* o = p.odig + digits::chain_offset(go, jn, 16 * sg, 0, nchq, S);
#pragma unroll
          for (int s = 0; s < S; ++s)
            __builtin_nontemporal_store(i4{(int)pl[0][s], (int)pl[1][s], (int)pl[2][s], (int)pl[3][s]},
                                        reinterpret_cast<i4*>(o + s * 2048));
          if (sg == 0) __builtin_nontemporal_store(e, p.oexp + (int64_t)go * 256 + jn);
        }
      }
    }
    if (!next) break;
    P = Pn;
  }
}

hipError_t launch_gemm_sliced_chain(ChainArgs& c, hipStream_t s) {
  if (c.M < 1 || c.K < 1 || c.F < 1 || c.F > CF || c.Gv < 1 || c.Gv > CF || c.nvec < 1) return hipErrorInvalidValue;
  if ((int64_t)c.K * c.slices * 16384 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  if (!c.fdig || !c.fexp || !c.vdig || !c.vexp || (c.odig ? !c.oexp : !c.out)) return hipErrorInvalidValue;
  c.tiles_m = (c.M + CM - 1) / CM;
  const int64_t total = (int64_t)c.tiles_m * c.Gv * c.nvec;
  if (total >= ((int64_t)1 << 28)) return hipErrorInvalidValue;
  // chain-layout extents: groups of 256 fibers, positions padded to 64
  const int64_t gin = (int64_t)c.nvec * c.Gv;
  if (gin * 256 * c.slices * slice_ld(c.K) > c.vcap || gin * 256 > c.vexp_cap) return hipErrorInvalidValue;
  if (c.odig) {
    const int64_t fibers = (int64_t)c.nvec * c.M * c.Gv;   // the next product's fibers
    if (c.Fn < 1 || c.Fn > CF || fibers % c.Fn != 0 || fibers >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const int64_t gout = fibers / c.Fn;
    if (gout * 256 * c.slices * slice_ld(c.F) > c.ocap || gout * 256 > c.oexp_cap) return hipErrorInvalidValue;
  }
  c.total = (int)total;
  c.per_xcd = (c.total + 7) / 8;
  // one workgroup per compute unit (eight XCDs of 32), fewer for small launches
  const dim3 grid(8 * std::min(CSLOTS, c.per_xcd));
#define MM_CHAIN_CASE(SS)                                                             \
  case SS:                                                                            \
    if (c.wide)                                                                       \
      gemm_i8_chain<SS, 64><<<grid, dim3(256), 0, s>>>(c);                            \
    else                                                                              \
      gemm_i8_chain<SS, 32><<<grid, dim3(512), 0, s>>>(c);                            \
    break;
  switch (c.slices) {
    MM_CHAIN_CASE(3)
    MM_CHAIN_CASE(4)
    MM_CHAIN_CASE(5)
    MM_CHAIN_CASE(6)
    MM_CHAIN_CASE(7)
    default: return hipErrorInvalidValue;
  }
#undef MM_CHAIN_CASE
  return hipGetLastError();
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
    // Y = round(x 2^(8S-1-e)) as a 64-bit integer; its balanced base-256 digits follow
    // from the bytes of Y + 0x80..80
    const double x = (c < k) ? row[c] : 0.0;
    const double y = __builtin_rint(__builtin_ldexp(x, 8 * S - 1 - e));
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
  if (g.M < 1 || g.N < 1 || g.K < 1 || g.inner < 1 || g.groups < 1 || g.groups > kMaxGroups)
    return hipErrorInvalidValue;
  // the grid operand's digits and fiber exponents go to the caller's workspace
  if (!g.vdig || !g.vexp || sliced_digit_bytes(g) > g.vdig_cap ||
      (int64_t)g.groups * sliced_fibers(g) > g.vexp_cap)
    return hipErrorInvalidValue;
  g.tiles_m = (g.M + T8 - 1) / T8;
  g.tiles_n = (g.N + T8 - 1) / T8;
  const int64_t total = (int64_t)g.tiles_m * g.tiles_n * g.inner * g.groups;
  if (total >= ((int64_t)1 << 28)) return hipErrorInvalidValue;
  g.total = (int)total;
  g.per_xcd = (g.total + 7) / 8;
  const int64_t fblocks = g.b_trans ? (int64_t)g.inner * ((g.N + T8 - 1) / T8) : ((int64_t)g.M + 3) / 4;
  if (fblocks * g.groups >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const dim3 sgrid((unsigned)(fblocks * g.groups)), grid(8 * g.per_xcd), block(TH);
#define MM_SLICED_CASE(SS)                                                \
  case SS:                                                                \
    if (g.b_trans) {                                                      \
      if (!g.vready) slice_grid<1, SS><<<sgrid, block, 0, s>>>(g, (int)fblocks); \
      gemm_i8<1, SS><<<grid, block, 0, s>>>(g);                           \
    } else {                                                              \
      if (!g.vready) slice_grid<0, SS><<<sgrid, block, 0, s>>>(g, (int)fblocks); \
      gemm_i8<0, SS><<<grid, block, 0, s>>>(g);                           \
    }                                                                     \
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
