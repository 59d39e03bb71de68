// mu-mode contraction kernels for gfx950 (Sec. 1 and Sec. 5.2: the action of the
// exponential of a Kronecker sum is a sequence of mode products V x_mu E_mu, each a
// dense GEMM with one small n x n factor and one large grid-shaped operand).
//
// Every mode product is cast as a batched row-major GEMM C = A . B' with
//   mode 1 (x1, fastest):  A = V viewed (n2 n3) x n1,  B'[n][k] = E1[n][k],   C = (n2 n3) x n1
//   mode 2:                A = E2,  B'[n][k] = V_slab[k][n] (slab = one x3 plane), C = n2 x n1
//   mode 3 (2D: mode 2):   A = E3,  B'[n][k] = V[k][n] with V viewed n3 x (n1 n2)
// so A is always read along k (row-major) and B' either along k (factor, mode 1) or
// along n (grid operand, modes 2/3, "b_trans"). Square workgroup tiles of T = 128 or 64
// (four waves of T/2 x T/2, or for FP64 128-tiles eight waves of 32 x 64; the launcher
// takes 64 when 128-tiles would not fill the chip once), K staged through LDS in chunks; ragged edges are zero-filled on load and
// masked on store. The linear workgroup id is remapped so that tiles sharing the large
// operand are dispatched to the same XCD (workgroups are dealt round-robin over the
// eight XCDs, each with its own L2).
//
// Precisions:
//   FP64   v_mfma_f64_16x16x4 with FP64 accumulation; all operands FP64.
//   FP32   factor pre-rounded to FP32 at setup, grid operand rounded to FP32 (nearest
//          even) while staging, v_mfma_f32_16x16x4 with FP32 accumulation.
//   BF16xS factor pre-split at setup, grid operand split while staging into S BF16
//          slices (x = s0 + s1 [+ s2], each the nearest-even BF16 of the remaining
//          residual); all slice products s_i s_j with i + j < S on
//          v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
// In the mixed modes the grid operand may be FP32 or FP64 in memory and C may be
// written as FP32 (intermediate passes) or FP64 (last pass of an action).
#include "mm_internal.h"

#include <algorithm>
#include <type_traits>

namespace mm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));   // 8-byte aligned pair
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int THREADS = 256;

template <int T>
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
  m0 = tm * T;
  n0 = tn * T;
}

template <typename TOut>
__device__ __forceinline__ void store_out(TOut* C, const double* Cadd, int idx, double v, double beta) {
  if (Cadd) v += beta * Cadd[idx];
  C[idx] = (TOut)v;
}

// ------------------------------------------------------------------------------------
// FP64: v_mfma_f64_16x16x4. K-chunk of 16; within a chunk the four lane groups
// g = lane/16 take k = 4g + s at MFMA step s, so A and B use one consistent
// permutation. Rows of A (and of B' when it is read along k) sit in LDS as [row][k]
// and a lane reads two k values of a fragment row with one 16-byte access; the grid
// operand of modes 2/3 stays in its [k][n] order in LDS (pitch 132 doubles: a wave's
// four k rows of sixteen n hit every bank exactly twice) and is read one value at a
// time. Global loads are branch-free: out-of-range rows of A or B' are clamped into
// the matrix (they only feed outputs that are masked at the store) and only the last
// K-chunk zeroes k >= K.
// ------------------------------------------------------------------------------------
constexpr int KC4 = 16;
constexpr int P64 = KC4 + 2;   // [row][k] pitch in doubles (144 B: 16-byte aligned rows)
// [k][n] pitch T + 4 doubles: 8 * pitch = 32 mod 64 banks for both tile sizes

template <int T>
constexpr int occupancy() { return T == 128 ? 2 : 4; }

// FP64 workgroups: 128-tiles run eight waves (4 x 2 waves of 32 x 64), so that two
// workgroups per compute unit put four waves on every SIMD (more waves to cover the
// per-chunk barrier and load waits than four waves of 64 x 64 at two per SIMD; the
// accumulation order per output is the same); 64-tiles run four waves of 32 x 32.
template <int T>
constexpr int f64_waves() { return T == 128 ? 8 : 4; }

template <int BT, int T>
__global__ __launch_bounds__(64 * f64_waves<T>(), 4) void gemm_f64(GemmArgs p) {
  constexpr int NT = 64 * f64_waves<T>();       // threads
  constexpr int WM = T / (f64_waves<T>() / 2);  // wave tile: WM x T/2
  constexpr int FIM = WM / 16, FIN = T / 32;    // 16 x 16 fragments per wave
  constexpr int NL = T * KC4 / NT;    // tile elements per thread and operand per chunk
  constexpr int RS = NT / 16;         // rows of a [row][k] tile covered by one pass
  constexpr int PKN = T + 4;
  constexpr int KR = NT / T;          // k rows of the [k][n] tile covered by one pass
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  int g, b, m0, n0;
  decode_tile<T>(p, P, g, b, m0, n0);
  const double* __restrict__ A = (const double*)p.A[g] + b * p.sA;
  const double* __restrict__ B = (const double*)p.B[g] + b * p.sB;
  double* __restrict__ C = (double*)p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;

  constexpr int BSZ = BT ? KC4 * PKN : T * P64;
  __shared__ __attribute__((aligned(16))) double As[2][T * P64];
  __shared__ __attribute__((aligned(16))) double Bs[2][BSZ];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * (T / 2);
  const int lg = lane >> 4, lr = lane & 15;
  const int M = p.M, N = p.N, K = p.K, lda = p.lda, ldb = p.ldb;

  d4 acc[FIM][FIN];
#pragma unroll
  for (int i = 0; i < FIM; ++i)
#pragma unroll
    for (int j = 0; j < FIN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // element e = i*NT + tid of a tile: A and B' read along k: row = e/16 = RS*i + tid/16,
  // k = tid%16;  B' read along n: k = e/T = KR*i + tid/T, n = tid%T
  const int r16 = tid >> 4, k16 = tid & 15;
  const int nB = min(n0 + (tid % T), N - 1), kB = tid / T;
  double ra[NL], rb[NL];
  // loads are unconditional (clamped indices, unsigned 32-bit offsets from the uniform
  // base) so that the loads of a chunk stay in flight through the MFMA phase. Only the
  // last K-chunk can reach past K: it alone clamps k into the matrix and zeroes k >= K
  // when the registers are written to LDS (tail = true_type); the other chunks skip
  // both, which takes about a third of the loop's vector-ALU instructions off the
  // MFMA issue slots.
  auto load = [&](int k0, auto tail) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const unsigned arow = (unsigned)min(m0 + RS * i + r16, M - 1);
      const int kb = BT ? KR * i + kB : k16;
      const unsigned brow = (unsigned)(BT ? nB : min(n0 + RS * i + r16, N - 1));
      const unsigned ka = (unsigned)(tail ? min(k0 + k16, K - 1) : k0 + k16);
      const unsigned kbb = (unsigned)(tail ? min(k0 + kb, K - 1) : k0 + kb);
      ra[i] = A[arow * (unsigned)lda + ka];
      rb[i] = BT ? B[kbb * (unsigned)ldb + brow] : B[brow * (unsigned)ldb + kbb];
    }
  };
  auto store = [&](double* as, double* bs, int k0, auto tail) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = i * NT + tid;
      const int kb = BT ? KR * i + kB : k16;
      as[(e >> 4) * P64 + (e & 15)] = (!tail || k0 + k16 < K) ? ra[i] : 0.0;
      const double y = (!tail || k0 + kb < K) ? rb[i] : 0.0;
      if (BT)
        bs[(e / T) * PKN + (e % T)] = y;
      else
        bs[(e >> 4) * P64 + (e & 15)] = y;
    }
  };
  using Tail = std::true_type;
  using Body = std::false_type;
  const int nch = (K + KC4 - 1) / KC4;
  if (nch > 1) {
    load(0, Body());
    store(As[0], Bs[0], 0, Body());
  } else {
    load(0, Tail());
    store(As[0], Bs[0], 0, Tail());
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int cur = c & 1;
    const bool last = c + 2 == nch;   // the chunk staged in this iteration is the last
    if (c + 1 < nch) {
      if (last) load((c + 1) * KC4, Tail());
      else load((c + 1) * KC4, Body());
    }
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // k = 4g + 2h + {0, 1}
      d2 af[FIM], bf[FIN];
#pragma unroll
      for (int i = 0; i < FIM; ++i)
        af[i] = *reinterpret_cast<const d2*>(as + (wm + 16 * i + lr) * P64 + 4 * lg + 2 * h);
#pragma unroll
      for (int i = 0; i < FIN; ++i) {
        if (BT) {
          const double* q = bs + (4 * lg + 2 * h) * PKN + wn + 16 * i + lr;
          bf[i] = d2{q[0], q[PKN]};
        } else {
          bf[i] = *reinterpret_cast<const d2*>(bs + (wn + 16 * i + lr) * P64 + 4 * lg + 2 * h);
        }
      }
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < FIM; ++i)
#pragma unroll
          for (int j = 0; j < FIN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][s], bf[j][s], acc[i][j], 0, 0, 0);
    }
    if (c + 1 < nch) {
      if (last) store(As[cur ^ 1], Bs[cur ^ 1], (c + 1) * KC4, Tail());
      else store(As[cur ^ 1], Bs[cur ^ 1], (c + 1) * KC4, Body());
    }
    __syncthreads();
  }
  // f64 16x16 layout: lane l, element t holds row 4t + l/16, column l%16
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < FIM; ++i)
#pragma unroll
    for (int j = 0; j < FIN; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * t + lg;
        const int n = n0 + wn + 16 * j + lr;
        if (m < M && n < N) store_out<double>(C, Cadd, m * p.ldc + n, alpha * acc[i][j][t], beta);
      }
}

// ------------------------------------------------------------------------------------
// FP64 mode products with a centrosymmetric factor (E = J E J with J the exchange matrix:
// exp(c tau A) of a symmetric Toeplitz A, i.e. Dirichlet ends and no advection in A).
// Along the contracted axis of n points (m = n/2 mirror pairs, f = n - m folded positions)
// a fiber x gives s_r = x_r + x_{n-1-r} and d_r = x_r - x_{n-1-r} for r < m (odd n: s_m =
// x_m, d_m = 0), and y = E x follows from the two f x f products a = Es s and b = Ed d:
// y_i = a_i + b_i and y_{n-1-i} = a_i - b_i (i < m; launch_fold_factor defines Es and
// Ed). This is half the multiply-adds of the plain product. A workgroup covers 128 grid
// rows (mode 1) or columns (modes 2/3) against 64 folded positions of both halves, with
// eight waves; k runs in chunks of 8 (two MFMA steps: lane group g supplies k = 2g + s at
// step s, in both operands) through double-buffered LDS tiles: the factor rows [Es; Ed]
// as [row][k], the grid's s and d tiles as [row][k] (mode 1) or [k][n] (modes 2/3).
// Each wave accumulates the Es and the Ed products of the same outputs, so the epilogue
// combines a and b in registers and writes both mirror rows (or columns).
// ------------------------------------------------------------------------------------
constexpr int PFN = 128 + 4;   // [k][n] pitch of the modes-2/3 grid tiles

template <int BT>
__global__ __launch_bounds__(512, 4) void gemm_f64_fold(GemmArgs p) {
  constexpr int KC = 8;        // folded k per chunk
  constexpr int PF = KC;       // [row][k] pitch in doubles: rows of four 16-byte units
  // [row][k] tiles: unit u = k/2 of row r sits at unit u ^ (r/4 mod 4), so that the 16-byte
  // stores (four threads per row) and the fragment reads (sixteen rows at one unit) both
  // spread over all banks (k even)
  auto rk = [](int r, int k) { return r * PF + ((((k >> 1) ^ (r >> 2)) & 3) << 1); };
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  const int tiles = p.tiles_m * p.tiles_n;
  const int gb = P / tiles, t = P - gb * tiles;
  const int g = gb / p.inner, b = gb - g * p.inner;
  int tm, tn;
  if (BT) {   // neighbouring ids share the grid tile
    tm = t % p.tiles_m;
    tn = t / p.tiles_m;
  } else {
    tn = t % p.tiles_n;
    tm = t / p.tiles_n;
  }
  // G = fold_blocks stacked factors along k (the grid operand's k axis holds G vectors of
  // n): folded position kk = g fl + r (fl = fold_ld(n); pad positions f <= r < fl are zero
  // in the folded factor)
  const int G = p.fold_blocks, n = p.K / G, m = n >> 1, f = n - m, fl = fold_ld(n), kf = G * fl;
  // BT: rows are folded positions (64 per tile), columns grid columns (128);
  // !BT: rows are grid rows (128), columns folded positions (64)
  const int r0 = tm * (BT ? 64 : 128), c0 = tn * (BT ? 128 : 64);
  const int fo = BT ? r0 : c0;   // first folded position of the tile
  const double* __restrict__ X = (const double*)(BT ? p.B[g] : p.A[g]) + b * (BT ? p.sB : p.sA);
  const double* __restrict__ Fq = p.Ff[g];
  double* __restrict__ C = (double*)p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;
  const int M = p.M, N = p.N, ldx = BT ? p.ldb : p.lda, ldf = p.ldf;

  __shared__ __attribute__((aligned(16))) double Fs[2][128 * PF];
  __shared__ __attribute__((aligned(16))) double Gs[2][2][BT ? KC * PFN : 128 * PF];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int lg = lane >> 4, lr = lane & 15;

  d4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // Chunk staging: every thread moves two consecutive values of each kind with 16-byte
  // accesses. Factor: row tid/4 of the tile's [Es; Ed] rows (rows past f clamped: they
  // feed masked outputs), k pair 2 (tid%4). Grid: modes 2/3 k = tid/64 and the column pair
  // 2 (tid%64) with the mirror row; mode 1 row tid/4 (rows past M clamped) and the k pair
  // 2 (tid%4) with its mirror pair (whose two values come in reverse order). The loads
  // only fill registers; the sums, differences and zeroing happen when the chunk is
  // written to LDS, after the current chunk's products, so that no wait for the loads
  // stands in front of them. Chunks whose positions are all below m (every chunk but the
  // last for odd n) need no clamping or zeroing; the tail chunk takes the elementwise path.
  const int fr = tid >> 2, kq = 2 * (tid & 3);
  const double* fbase = Fq + (min(fo + (fr & 63), f - 1) + (fr >> 6) * f) * ldf;
  const int gk = BT ? (tid >> 6) : kq;                          // grid k within the chunk
  const int gcol = BT ? c0 + 2 * (tid & 63) : 0;                // modes 2/3: first column
  const int grow = BT ? 0 : min(r0 + (tid >> 2), M - 1);        // mode 1: grid row
  // modes 2/3: the body chunks read the 16-byte column pair at gpc. Values that feed only
  // masked outputs may come from anywhere inside the operand, so that no lane of the last
  // column tile leaves the 16-byte path: the second column may be row padding (gcol + 1 <
  // ldx), a pair starting at the last column of an unpadded row takes the next row's first
  // value (not in the operand's last slab, where no row may follow), and a pair wholly
  // past the last column reads the last two columns
  int gpc = gcol;
  bool gpair = true;
  if (BT && gcol + 1 >= ldx) {
    if (gcol >= N && N >= 2)
      gpc = N - 2;
    else
      gpair = gcol + 1 == ldx && b + 1 < p.inner;
  }
  const int gc0 = min(gcol, N - 1), gc1 = min(gcol + 1, N - 1);
  d2 rf, q1, q2;   // raw factor pair; grid values and their mirror partners
  // modes 2/3: the block lg0 and in-block position lr0 of this thread's folded position
  // k0 + gk in the next chunk to load (past the end: the last block), advanced by KC per
  // chunk without a division; sr0 keeps the loaded chunk's position for its store
  int lg0 = min(gk / fl, G - 1), lr0 = gk - lg0 * fl, sr0 = 0;
  auto load = [&](int k0, auto tail) {
    constexpr bool T = decltype(tail)::value;
    // (an index past the factor row is clamped; its values are zeroed when stored)
    rf = *reinterpret_cast<const d2*>(fbase + (T ? min(k0 + kq, kf - 2) : k0 + kq));
    if (BT) {
      const int r = lr0, base = lg0 * n;
      sr0 = lr0;
      lr0 += KC;
      while (lr0 >= fl && lg0 < G - 1) {
        lr0 -= fl;
        ++lg0;
      }
      if (!T && gpair) {
        q1 = *reinterpret_cast<const d2u*>(X + (base + r) * ldx + gpc);
        q2 = *reinterpret_cast<const d2u*>(X + (base + n - 1 - r) * ldx + gpc);
      } else {
        const int rc = base + min(r, f - 1), rm = base + n - 1 - min(r, f - 1);   // rm >= rc
        q1 = d2{X[rc * ldx + gc0], X[rc * ldx + gc1]};
        q2 = d2{X[rm * ldx + gc0], X[rm * ldx + gc1]};
      }
    } else {
      const double* xr = X + grow * ldx;
      if (!T) {
        const int r = k0 + kq;
        q1 = *reinterpret_cast<const d2u*>(xr + r);
        q2 = *reinterpret_cast<const d2u*>(xr + n - 2 - r);   // x[n-2-r], x[n-1-r]
      } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int rc = min(k0 + kq + q, f - 1);
          q1[q] = xr[rc];
          q2[q] = xr[n - 1 - rc];
        }
      }
    }
  };
  auto store = [&](int buf, int k0, auto tail) {
    constexpr bool T = decltype(tail)::value;
    d2 sf = rf, rs, rd;
    if (T) {
      sf.x = k0 + kq < kf ? rf.x : 0.0;
      sf.y = k0 + kq + 1 < kf ? rf.y : 0.0;
    }
    if (BT) {
      const int rr = sr0;
      const bool live = k0 + gk < kf;
      if (!T || (live && rr < m)) {
        rs = q1 + q2;
        rd = q1 - q2;
      } else {
        rs = live && rr < f ? q1 : d2{0.0, 0.0};
        rd = d2{0.0, 0.0};
      }
    } else if (!T) {
      rs = d2{q1.x + q2.y, q1.y + q2.x};
      rd = d2{q1.x - q2.y, q1.y - q2.x};
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int rr = k0 + kq + q;
        rs[q] = rr < m ? q1[q] + q2[q] : rr < f ? q1[q] : 0.0;
        rd[q] = rr < m ? q1[q] - q2[q] : 0.0;
      }
    }
    *reinterpret_cast<d2*>(&Fs[buf][rk(fr, kq)]) = sf;
    const int gi = BT ? gk * PFN + 2 * (tid & 63) : rk(tid >> 2, kq);
    *reinterpret_cast<d2*>(&Gs[buf][0][gi]) = rs;
    *reinterpret_cast<d2*>(&Gs[buf][1][gi]) = rd;
  };
  using Tail = std::true_type;
  using Body = std::false_type;

  // a chunk needs no clamping or zeroing when its positions lie in one block, below m
  // (km: the first position of the next chunk modulo fl, advanced without a division)
  int km = 0;
  auto next_body = [&]() {
    const bool body = km + KC <= m;
    km += KC;
    while (km >= fl) km -= fl;
    return body;
  };
  const int nch = (kf + KC - 1) / KC;
  if (next_body()) {
    load(0, Body());
    store(0, 0, Body());
  } else {
    load(0, Tail());
    store(0, 0, Tail());
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int cur = c & 1;
    const int k1 = (c + 1) * KC;
    const bool body1 = next_body();
    if (c + 1 < nch) {
      if (body1) load(k1, Body());
      else load(k1, Tail());
    }
    const double* fs = Fs[cur];
    const double* gs = Gs[cur][0];
    const double* gd = Gs[cur][1];
#pragma unroll
    for (int h = 0; h < KC / 8; ++h) {   // k = (KC/4) g + 2 h + s at MFMA step (h, s)
      const int kb = (KC / 4) * lg + 2 * h;
      if (BT) {
        // wave: folded rows 16 wr + [0, 16) of Es and of Ed, columns 64 wc + [0, 64)
        const d2 as = *reinterpret_cast<const d2*>(fs + rk(16 * wr + lr, kb));
        const d2 ad = *reinterpret_cast<const d2*>(fs + rk(64 + 16 * wr + lr, kb));
        // the Es products against the s tile, then the Ed products against the d tile (one
        // set of grid fragments live at a time)
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const double* gt = h2 ? gd : gs;
          d2 bf[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int col = 64 * wc + 16 * j + lr;
            bf[j] = d2{gt[kb * PFN + col], gt[(kb + 1) * PFN + col]};
          }
#pragma unroll
          for (int st = 0; st < 2; ++st)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[h2][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(h2 ? ad[st] : as[st], bf[j][st], acc[h2][j], 0, 0, 0);
        }
      } else {
        // wave: grid rows 32 wr + [0, 32), folded columns 32 wc + [0, 32) of Es (j = 0, 1)
        // and of Ed (j = 2, 3)
        d2 as[2], ad[2], bf[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          as[i] = *reinterpret_cast<const d2*>(gs + rk(32 * wr + 16 * i + lr, kb));
          ad[i] = *reinterpret_cast<const d2*>(gd + rk(32 * wr + 16 * i + lr, kb));
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bf[j] = *reinterpret_cast<const d2*>(fs + rk((j >> 1) * 64 + 32 * wc + 16 * (j & 1) + lr, kb));
#pragma unroll
        for (int st = 0; st < 2; ++st)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(j < 2 ? as[i][st] : ad[i][st], bf[j][st], acc[i][j], 0,
                                                               0, 0);
      }
    }
    if (c + 1 < nch) {
      if (body1) store(cur ^ 1, k1, Body());
      else store(cur ^ 1, k1, Tail());
    }
    __syncthreads();
  }
  // f64 16x16 layout: lane l, element t holds row 4t + l/16, column l%16
  const double alpha = p.alpha, beta = p.beta;
  // (one loop without and one with the added term, so that the common case carries no
  // per-element test of Cadd)
  auto epilogue = [&](auto with_add) {
    constexpr bool ADD = decltype(with_add)::value;
    auto put = [&](int row, int col, double v) {
      const int idx = row * p.ldc + col;
      if (ADD) v += beta * Cadd[idx];
      C[idx] = v;
    };
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) {
      if (BT) {
        const int fr = r0 + 16 * wr + 4 * t4 + lg;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = c0 + 64 * wc + 16 * j + lr;
          if (fr < f && col < N) {
            const double a = acc[0][j][t4], bb = acc[1][j][t4];
            put(fr, col, alpha * (a + bb));
            if (fr < m) put(n - 1 - fr, col, alpha * (a - bb));
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int row = r0 + 32 * wr + 16 * i + 4 * t4 + lg;
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int fc = c0 + 32 * wc + 16 * j + lr;
            if (row < M && fc < f) {
              const double a = acc[i][j][t4], bb = acc[i][j + 2][t4];
              put(row, fc, alpha * (a + bb));
              if (fc < m) put(row, n - 1 - fc, alpha * (a - bb));
            }
          }
        }
      }
    }
  };
  if (Cadd)
    epilogue(std::true_type{});
  else
    epilogue(std::false_type{});
}

// Folds the n x n block q of E (row stride lde, blocks es apart) into Ff (row stride ldff,
// blocks fs apart): Es rows 0..f-1, Ed rows f..2f-1, fold_ld(n) columns (padding zero).
__global__ void fold_factor(double* __restrict__ Ff, int ldff, int64_t fs, const double* __restrict__ E, int lde,
                            int64_t es, int n) {
  const int m = n >> 1, f = n - m, ld = fold_ld(n);
  const int64_t q = (int64_t)blockIdx.y;
  const double* Eq = E + q * es;
  double* Fq = Ff + q * fs;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < f * ld; e += gridDim.x * blockDim.x) {
    const int i = e / ld, r = e - i * ld;
    if (r >= f) {   // row padding
      Fq[(int64_t)i * ldff + r] = 0.0;
      Fq[(int64_t)(f + i) * ldff + r] = 0.0;
      continue;
    }
    const double x = Eq[(int64_t)i * lde + r], y = Eq[(int64_t)i * lde + n - 1 - r];
    Fq[(int64_t)i * ldff + r] = r < m ? 0.5 * (x + y) : x;
    Fq[(int64_t)(f + i) * ldff + r] = r < m ? 0.5 * (x - y) : 0.0;
  }
}

hipError_t launch_fold_factor(double* Ff, const double* E, int n, int count, hipStream_t s) {
  if (!Ff || !E || n < 1 || count < 1 || count > 65535) return hipErrorInvalidValue;
  const int f = n - n / 2, ld = fold_ld(n);
  const int blocks = std::min(1024, (f * ld + 255) / 256);
  fold_factor<<<dim3(blocks, count), dim3(256), 0, s>>>(Ff, ld, (int64_t)2 * f * ld, E, n, (int64_t)n * n, n);
  return hipGetLastError();
}

hipError_t launch_fold_stacked(double* Ff, const double* E, int n, int G, hipStream_t s) {
  if (!Ff || !E || n < 1 || G < 1 || G > 65535) return hipErrorInvalidValue;
  const int f = n - n / 2, ld = fold_ld(n);
  const int blocks = std::min(1024, (f * ld + 255) / 256);
  fold_factor<<<dim3(blocks, G), dim3(256), 0, s>>>(Ff, G * ld, ld, E, G * n, n, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// FP32: same K permutation as FP64; the pre-converted factor arrives as 16-byte vectors
// of four k values, the grid operand as runs of eight k values per thread.
// ------------------------------------------------------------------------------------
constexpr int P32 = KC4 + 4;  // LDS row pitch in floats (80 B: 16-byte aligned rows)

template <int BT, int T, typename TIn, typename TOut>
__global__ __launch_bounds__(THREADS, occupancy<T>()) void gemm_f32(GemmArgs p) {
  constexpr int FI = T / 32;
  constexpr int NF = T / 64;          // factor float4 per thread and chunk
  constexpr int NV = T / 16;          // grid values per thread and chunk
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  int g, b, m0, n0;
  decode_tile<T>(p, P, g, b, m0, n0);
  // factor: A (BT) or B' (!BT), float rows of stride ld = fac_ld(K)
  const float* __restrict__ F = BT ? (const float*)p.A[g] + b * p.sA : (const float*)p.B[g] + b * p.sB;
  const TIn* __restrict__ V = BT ? (const TIn*)p.B[g] + b * p.sB : (const TIn*)p.A[g] + b * p.sA;
  TOut* __restrict__ C = (TOut*)p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;
  const int M = p.M, N = p.N, K = p.K;
  const int ldf = BT ? p.lda : p.ldb;           // factor row stride (padded)
  const int ldv = BT ? p.ldb : p.lda;           // grid operand stride
  const int fr0 = BT ? m0 : n0, frows = BT ? M : N;   // factor rows of this tile
  const int vr0 = BT ? n0 : m0, vrows = BT ? N : M;   // grid rows (n for BT, m otherwise)

  __shared__ __attribute__((aligned(16))) float Fs[2][T * P32];
  __shared__ __attribute__((aligned(16))) float Vs[2][T * P32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (T / 2), wn = (wave & 1) * (T / 2);
  const int lg = lane >> 4, lr = lane & 15;

  f4 acc[FI][FI];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FI; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  f4 rf[NF];
  TIn rv[NV];
  // factor: T rows x 16 k = 4T float4 (rows clamped into range)
  int foff[NF];
#pragma unroll
  for (int h = 0; h < NF; ++h) {
    const int e = h * THREADS + tid;
    foff[h] = min(fr0 + (e >> 2), frows - 1) * ldf + (e & 3) * 4;
  }
  // grid: BT: lanes take consecutive n, a run of NV k per thread;
  //       !BT: lanes take consecutive k (coalesced rows), NV rows per thread
  int voff[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (BT)
      voff[j] = ((tid / T) * NV + j) * ldv + min(vr0 + (tid % T), vrows - 1);
    else
      voff[j] = min(vr0 + (tid >> 4) + 16 * j, vrows - 1) * ldv + (tid & 15);
  }
  auto vk_of = [&](int j) { return BT ? (tid / T) * NV + j : (tid & 15); };
  auto load = [&](int k0) {
#pragma unroll
    for (int h = 0; h < NF; ++h) rf[h] = *reinterpret_cast<const f4*>(F + foff[h] + k0);
    // unconditional loads (k clamped); conversion and the k >= K zeroing happen at the
    // LDS store so that the loads stay in flight through the MFMA phase
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int kk = vk_of(j);
      const int kc = min(k0 + kk, K - 1) - kk;
      rv[j] = V[(unsigned)(voff[j] + kc * (BT ? ldv : 1))];
    }
  };
  auto cv = [&](int j, int k0) -> float { return (k0 + vk_of(j) < K) ? (float)rv[j] : 0.f; };
  auto store = [&](float* fs, float* vs, int k0) {
#pragma unroll
    for (int h = 0; h < NF; ++h) {
      const int e = h * THREADS + tid;
      *reinterpret_cast<f4*>(fs + (e >> 2) * P32 + (e & 3) * 4) = rf[h];
    }
    if (BT) {
      const int vrow = tid % T, vk = (tid / T) * NV;
#pragma unroll
      for (int q = 0; q < NV / 4; ++q)
        *reinterpret_cast<f4*>(vs + vrow * P32 + vk + 4 * q) =
            f4{cv(4 * q, k0), cv(4 * q + 1, k0), cv(4 * q + 2, k0), cv(4 * q + 3, k0)};
    } else {
#pragma unroll
      for (int j = 0; j < NV; ++j) vs[((tid >> 4) + 16 * j) * P32 + (tid & 15)] = cv(j, k0);
    }
  };
  load(0);
  store(Fs[0], Vs[0], 0);
  __syncthreads();
  const int nch = (K + KC4 - 1) / KC4;
  for (int c = 0; c < nch; ++c) {
    const int cur = c & 1;
    if (c + 1 < nch) load((c + 1) * KC4);
    const float* as = BT ? Fs[cur] : Vs[cur];
    const float* bs = BT ? Vs[cur] : Fs[cur];
    f4 af[FI], bf[FI];
#pragma unroll
    for (int i = 0; i < FI; ++i) {
      af[i] = *reinterpret_cast<const f4*>(as + (wm + 16 * i + lr) * P32 + 4 * lg);
      bf[i] = *reinterpret_cast<const f4*>(bs + (wn + 16 * i + lr) * P32 + 4 * lg);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s], bf[j][s], acc[i][j], 0, 0, 0);
    if (c + 1 < nch) store(Fs[cur ^ 1], Vs[cur ^ 1], (c + 1) * KC4);
    __syncthreads();
  }
  // f32 16x16 layout: lane l, element t holds row 4(l/16) + t, column l%16
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FI; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * lg + t;
        const int n = n0 + wn + 16 * j + lr;
        if (m < M && n < N) store_out<TOut>(C, Cadd, m * p.ldc + n, alpha * (double)acc[i][j][t], beta);
      }
}

// ------------------------------------------------------------------------------------
// Split BF16: K-chunk of 32 (one v_mfma_f32_16x16x32_bf16 per tile and slice product).
// LDS holds S slices of each operand in rows of 32 k (+8 pad); lane group g reads its
// eight consecutive k (8g .. 8g+7) as one 16-byte access.
// ------------------------------------------------------------------------------------
constexpr int KCB = 32;
constexpr int PB = 40;

template <int S>
__device__ __forceinline__ void split_bf16(float x, __bf16 (&out)[S]) {
  float rem = x;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const __bf16 h = (__bf16)rem;
    out[s] = h;
    rem -= (float)h;   // exact: rem and h agree in their leading bits
  }
}

template <int BT, int T, int S, typename TIn, typename TOut>
__global__ __launch_bounds__(THREADS, occupancy<T>()) void gemm_bf16(GemmArgs p) {
  constexpr int FI = T / 32;
  constexpr int NF = T / 64;          // factor bf8 vectors per thread, slice and chunk
  constexpr int NV = T / 8;           // grid values per thread and chunk
  const int L = blockIdx.x;
  const int P = (L & 7) * p.per_xcd + (L >> 3);
  if (P >= p.total) return;
  int g, b, m0, n0;
  decode_tile<T>(p, P, g, b, m0, n0);
  const __bf16* __restrict__ F = BT ? (const __bf16*)p.A[g] + b * p.sA : (const __bf16*)p.B[g] + b * p.sB;
  const TIn* __restrict__ V = BT ? (const TIn*)p.B[g] + b * p.sB : (const TIn*)p.A[g] + b * p.sA;
  TOut* __restrict__ C = (TOut*)p.C[g] + b * p.sC;
  const double* __restrict__ Cadd = p.Cadd[g] ? p.Cadd[g] + b * p.sC : nullptr;
  const int M = p.M, N = p.N, K = p.K;
  const int ldf = BT ? p.lda : p.ldb;
  const int ldv = BT ? p.ldb : p.lda;
  const int fr0 = BT ? m0 : n0, frows = BT ? M : N;
  const int vr0 = BT ? n0 : m0, vrows = BT ? N : M;
  const int64_t fsl = p.fac_slice;

  __shared__ __attribute__((aligned(16))) __bf16 Fs[S][T * PB];
  __shared__ __attribute__((aligned(16))) __bf16 Vs[S][T * PB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (T / 2), wn = (wave & 1) * (T / 2);
  const int lg = lane >> 4, lr = lane & 15;

  f4 acc[FI][FI];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FI; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  bf8 rf[S][NF];
  TIn rv[NV];
  int foff[NF];
#pragma unroll
  for (int h = 0; h < NF; ++h) {
    const int e = h * THREADS + tid;
    foff[h] = min(fr0 + (e >> 2), frows - 1) * ldf + (e & 3) * 8;
  }
  // grid: BT: lanes take consecutive n, a run of NV k per thread;
  //       !BT: lanes take consecutive k (coalesced rows), NV rows per thread
  int voff[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    if (BT)
      voff[j] = ((tid / T) * NV + j) * ldv + min(vr0 + (tid % T), vrows - 1);
    else
      voff[j] = min(vr0 + (tid >> 5) + 8 * j, vrows - 1) * ldv + (tid & 31);
  }
  auto vk_of = [&](int j) { return BT ? (tid / T) * NV + j : (tid & 31); };
  auto load = [&](int k0) {
#pragma unroll
    for (int h = 0; h < NF; ++h)
#pragma unroll
      for (int s = 0; s < S; ++s) rf[s][h] = *reinterpret_cast<const bf8*>(F + s * fsl + foff[h] + k0);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int kk = vk_of(j);
      const int kc = min(k0 + kk, K - 1) - kk;
      rv[j] = V[(unsigned)(voff[j] + kc * (BT ? ldv : 1))];
    }
  };
  auto cv = [&](int j, int k0) -> float { return (k0 + vk_of(j) < K) ? (float)rv[j] : 0.f; };
  auto store = [&](int k0) {
#pragma unroll
    for (int h = 0; h < NF; ++h) {
      const int e = h * THREADS + tid;
#pragma unroll
      for (int s = 0; s < S; ++s) *reinterpret_cast<bf8*>(&Fs[s][(e >> 2) * PB + (e & 3) * 8]) = rf[s][h];
    }
    if (BT) {
      const int vrow = tid % T, vk = (tid / T) * NV;
#pragma unroll
      for (int half = 0; half < NV / 8; ++half) {
        bf8 v[S];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 sl[S];
          split_bf16<S>(cv(8 * half + j, k0), sl);
#pragma unroll
          for (int s = 0; s < S; ++s) v[s][j] = sl[s];
        }
#pragma unroll
        for (int s = 0; s < S; ++s) *reinterpret_cast<bf8*>(&Vs[s][vrow * PB + vk + 8 * half]) = v[s];
      }
    } else {
#pragma unroll
      for (int j = 0; j < NV; ++j) {
        __bf16 sl[S];
        split_bf16<S>(cv(j, k0), sl);
#pragma unroll
        for (int s = 0; s < S; ++s) Vs[s][((tid >> 5) + 8 * j) * PB + (tid & 31)] = sl[s];
      }
    }
  };

  const int nch = (K + KCB - 1) / KCB;
  load(0);
  for (int c = 0; c < nch; ++c) {
    store(c * KCB);
    __syncthreads();
    if (c + 1 < nch) load((c + 1) * KCB);
#pragma unroll
    for (int sa = 0; sa < S; ++sa) {
      bf8 af[FI];
#pragma unroll
      for (int i = 0; i < FI; ++i) {
        const __bf16* base = BT ? &Fs[sa][0] : &Vs[sa][0];
        af[i] = *reinterpret_cast<const bf8*>(base + (wm + 16 * i + lr) * PB + 8 * lg);
      }
#pragma unroll
      for (int sb = 0; sa + sb < S; ++sb) {
        bf8 bfr[FI];
#pragma unroll
        for (int j = 0; j < FI; ++j) {
          const __bf16* base = BT ? &Vs[sb][0] : &Fs[sb][0];
          bfr[j] = *reinterpret_cast<const bf8*>(base + (wn + 16 * j + lr) * PB + 8 * lg);
        }
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FI; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = m0 + wm + 16 * i + 4 * lg + t;
        const int n = n0 + wn + 16 * j + lr;
        if (m < M && n < N) store_out<TOut>(C, Cadd, m * p.ldc + n, alpha * (double)acc[i][j][t], beta);
      }
}

// ------------------------------------------------------------------------------------
// factor pre-conversion for the mixed modes
// ------------------------------------------------------------------------------------
int factor_slices(int prec) { return prec == MM_BF16X3 ? 2 : prec == MM_BF16X6 ? 3 : 1; }

__global__ void convert_factor_f32(float* dst, const double* src, int rows, int k, int lds, int ldd) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * ldd) return;
  const int r = (int)(e / ldd), c = (int)(e % ldd);
  dst[e] = (c < k) ? (float)src[(int64_t)r * lds + c] : 0.f;
}

template <int S>
__global__ void convert_factor_bf16(__bf16* dst, const double* src, int rows, int k, int lds, int ldd) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t cnt = (int64_t)rows * ldd;
  if (e >= cnt) return;
  const int r = (int)(e / ldd), c = (int)(e % ldd);
  double rem = (c < k) ? src[(int64_t)r * lds + c] : 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const __bf16 h = (__bf16)(float)rem;
    dst[s * cnt + e] = h;
    rem -= (double)(float)h;
  }
}

hipError_t launch_convert_factor(int prec, void* dst, const double* src, int rows, int k, int lds,
                                 hipStream_t s) {
  const int ldd = fac_ld(k);
  const int64_t cnt = (int64_t)rows * ldd;
  const unsigned blocks = (unsigned)((cnt + 255) / 256);
  switch (prec) {
    case MM_FP32: convert_factor_f32<<<blocks, 256, 0, s>>>((float*)dst, src, rows, k, lds, ldd); break;
    case MM_BF16X3: convert_factor_bf16<2><<<blocks, 256, 0, s>>>((__bf16*)dst, src, rows, k, lds, ldd); break;
    case MM_BF16X6: convert_factor_bf16<3><<<blocks, 256, 0, s>>>((__bf16*)dst, src, rows, k, lds, ldd); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
template <int BT, int T>
hipError_t launch_mixed(int prec, GemmArgs& g, dim3 grid, dim3 block, hipStream_t s) {
  const int io = (g.in_f32 ? 1 : 0) | (g.out_f32 ? 2 : 0);
#define MM_LAUNCH_IO(KERNEL, ...)                                                     \
  switch (io) {                                                                     \
    case 0: KERNEL<__VA_ARGS__, double, double><<<grid, block, 0, s>>>(g); break;   \
    case 1: KERNEL<__VA_ARGS__, float, double><<<grid, block, 0, s>>>(g); break;    \
    case 2: KERNEL<__VA_ARGS__, double, float><<<grid, block, 0, s>>>(g); break;    \
    default: KERNEL<__VA_ARGS__, float, float><<<grid, block, 0, s>>>(g); break;    \
  }
  switch (prec) {
    case MM_FP32: MM_LAUNCH_IO(gemm_f32, BT, T) break;
    case MM_BF16X3: MM_LAUNCH_IO(gemm_bf16, BT, T, 2) break;
    case MM_BF16X6: MM_LAUNCH_IO(gemm_bf16, BT, T, 3) break;
    default: return hipErrorInvalidValue;
  }
#undef MM_LAUNCH_IO
  return hipGetLastError();
}

template <int T>
hipError_t launch_tile(int prec, GemmArgs& g, hipStream_t s) {
  g.tiles_m = (g.M + T - 1) / T;
  g.tiles_n = (g.N + T - 1) / T;
  const int64_t total = (int64_t)g.tiles_m * g.tiles_n * g.inner * g.groups;
  if (total >= ((int64_t)1 << 28)) return hipErrorInvalidValue;
  g.total = (int)total;
  g.per_xcd = (g.total + 7) / 8;
  const dim3 grid(8 * g.per_xcd), block(THREADS);
  if (prec == MM_FP64) {
    if (g.in_f32 || g.out_f32) return hipErrorInvalidValue;
    const dim3 fblock(64 * f64_waves<T>());
    if (g.b_trans) gemm_f64<1, T><<<grid, fblock, 0, s>>>(g);
    else gemm_f64<0, T><<<grid, fblock, 0, s>>>(g);
    return hipGetLastError();
  }
  if constexpr (T == 32) {
    return hipErrorInvalidValue;   // 32-tiles are FP64 only
  } else {
    return g.b_trans ? launch_mixed<1, T>(prec, g, grid, block, s) : launch_mixed<0, T>(prec, g, grid, block, s);
  }
}

// Workgroups of 128-tiles that fill every compute unit at their occupancy (256 CUs x 2).
constexpr int64_t kFillSlots = 512;
// FP64 launches with fewer 64-tiles than compute units take 32-tiles (four waves of
// 16 x 16): four times the workgroups, and a quarter of the serial MFMA chain per wave,
// which is what bounds such a launch (the small grids of the paper's own examples).
constexpr int64_t kComputeUnits = 256;

int choose_tile(const GemmArgs& g, int prec) {
  if (g.tile == 32) return prec == MM_FP64 ? 32 : 64;
  if (g.tile == 64 || g.tile == 128) return g.tile;
  const int64_t t128 = (int64_t)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.inner * g.groups;
  if (t128 >= kFillSlots) return 128;
  const int64_t t64 = (int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64) * g.inner * g.groups;
  return prec == MM_FP64 && t64 < kComputeUnits ? 32 : 64;
}

// stacked factor blocks of a folded launch (0 counts as one)
int fold_blocks(const GemmArgs& g) { return g.fold_blocks > 1 ? g.fold_blocks : 1; }

// Folded FP64 launch: 128 x 64 tiles (grid x folded positions).
hipError_t launch_fold(GemmArgs& g, hipStream_t s) {
  g.fold_blocks = fold_blocks(g);
  const int f = g.K / g.fold_blocks - g.K / g.fold_blocks / 2;
  g.tiles_m = g.b_trans ? (f + 63) / 64 : (g.M + 127) / 128;
  g.tiles_n = g.b_trans ? (g.N + 127) / 128 : (f + 63) / 64;
  const int64_t total = (int64_t)g.tiles_m * g.tiles_n * g.inner * g.groups;
  if (total >= ((int64_t)1 << 28)) return hipErrorInvalidValue;
  g.total = (int)total;
  g.per_xcd = (g.total + 7) / 8;
  const dim3 grid(8 * g.per_xcd), block(512);
  if (g.b_trans)
    gemm_f64_fold<1><<<grid, block, 0, s>>>(g);
  else
    gemm_f64_fold<0><<<grid, block, 0, s>>>(g);
  return hipGetLastError();
}

// Folded launches take over from the plain ones from this many 128 x 64 tiles per group:
// at 127^3 Lawson2b (254 tiles per pass) the folded step runs 109 against 121 us, while a
// single 127^3 vector (127 tiles) runs faster on the plain kernel's 64-tiles, which spread
// it over more compute units.
constexpr int64_t kFoldMinTiles = 192;

// Whether g runs folded: FP64, every group with a folded factor, a square factor, and
// (fold = 1) at least kFoldMinTiles tiles per group.
// The count excludes the group count, so that a problem's products take the same form
// alone and in a grouped launch with other problems (folded and plain products round
// differently).
int64_t fold_tiles(const GemmArgs& g) {
  const int n = g.K / fold_blocks(g), f = n - n / 2;
  return (int64_t)(g.b_trans ? (f + 63) / 64 * ((g.N + 127) / 128) : (g.M + 127) / 128 * ((f + 63) / 64)) * g.inner;
}

bool use_fold(const GemmArgs& g, int prec) {
  if (prec != MM_FP64 || g.fold == 0 || g.in_f32 || g.out_f32) return false;
  const int G = fold_blocks(g);
  if (g.K % G != 0 || (g.b_trans ? g.M : g.N) != g.K / G || (G > 1 && !g.b_trans)) return false;
  for (int i = 0; i < g.groups; ++i)
    if (!g.Ff[i]) return false;
  return g.fold == 2 || fold_tiles(g) >= kFoldMinTiles;
}

hipError_t launch_gemm(int prec, GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.inner <= 0 || g.groups <= 0 || g.groups > kMaxGroups)
    return hipErrorInvalidValue;
  if (g.fold < 0 || g.fold > 2) return hipErrorInvalidValue;
  if (g.tile != 0 && g.tile != 32 && g.tile != 64 && g.tile != 128) return hipErrorInvalidValue;
  if (prec == MM_SLICED && (g.in_f32 || g.out_f32)) return hipErrorInvalidValue;
  // in-batch offsets are 32-bit
  const int64_t lim = (int64_t)1 << 31;
  if ((int64_t)g.M * g.lda >= lim || (int64_t)g.M * g.ldc >= lim ||
      (int64_t)(g.b_trans ? g.K : g.N) * g.ldb >= lim)
    return hipErrorInvalidValue;
  if (prec != MM_SLICED)
    for (int i = 0; i < g.groups; ++i)
      if (g.galpha[i] != 0.0) return hipErrorInvalidValue;   // per-group scales: sliced mode only
  if (prec == MM_SLICED) {
    const int ldf = g.b_trans ? g.lda : g.ldb;
    if (ldf < slice_ld(g.K) || ldf % 64 != 0) return hipErrorInvalidValue;
    for (int i = 0; i < g.groups; ++i)
      if (!g.fexp[i]) return hipErrorInvalidValue;
    return launch_gemm_sliced(g, s);
  }
  if (use_fold(g, prec)) {
    const int G = fold_blocks(g), n = g.K / G, f = n - n / 2;
    if (g.ldf < G * fold_ld(n) || g.ldf % 2 != 0 || (int64_t)2 * f * g.ldf >= lim) return hipErrorInvalidValue;
    return launch_fold(g, s);
  }
  if (prec != MM_FP64) {
    // the pre-converted factor must have its padded row stride
    const int ldf = g.b_trans ? g.lda : g.ldb;
    if (ldf < fac_ld(g.K) || ldf % kFacPad != 0) return hipErrorInvalidValue;
  }
  switch (choose_tile(g, prec)) {
    case 32: return launch_tile<32>(prec, g, s);
    case 64: return launch_tile<64>(prec, g, s);
    default: return launch_tile<128>(prec, g, s);
  }
}

}  // namespace mm
