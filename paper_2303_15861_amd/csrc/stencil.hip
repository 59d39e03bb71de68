// Remainder stencil and small helper kernels.
//
// g(u) of eq. (eq:nonlin) on the tensor grid (Sec. 5.2 discretisation, flux form):
//   g = sum_mu [(abar+ - lam a_max)(u+ - u) - (abar- - lam a_max)(u - u-)] / h_mu^2
//     + sum_mu (beta_mu - beta_bar_mu)(u+ - u-)/(2 h_mu) + r0 + r1 u + r2 u^2 + r3 u^3,
// abar = mean of the two nodal coefficients at a face, zero Dirichlet ghosts. With
// lam_amax = 0 and the full velocity the same kernel yields F(u) (Appendix, u' = F(u)).
// Sec. 5.2, eq. (eq:adr3d): the diffusion may instead be in non-divergence form,
// (a - lam a_max) Lap_h u, and an axis may carry a zero normal derivative at x = 1,
// whose ghost beyond the last unknown is the mirror value: at that unknown the + and -
// neighbours along the axis are equal (u_{n+1} = u_{n-1}), so no extra loads.
// The stage updates of the schemes are fused as out0 = base0 + c0 (g - sub) and
// out1 = base1 + c1 (g - sub), so each remainder evaluation is one pass over HBM.
#include <cfloat>

#include "mm_internal.h"
#include "slice_digits.h"
#include "wave_ops.h"

namespace mm {

// Layout of the work. Each lane owns P consecutive x1 points (P = 1, 2 or 4), so one
// wave covers a 64 P-point segment of an x1 row with 8 P-byte loads per lane, and the
// x1 neighbours of its points come from its own registers or, at the lane edges, from
// the neighbouring lanes by shuffles; only the two ends of the segment need a load
// (lanes 0 and 63 together, one instruction per row). Each lane also keeps a YT (x2)
// x ZT (x3) patch of such rows with a one-row halo in registers (no corners), so the
// x2/x3 neighbours are loaded once per patch: 1 x 2 in 3D, 2 x 1 in 2D, and 1 x 1 for the
// 3D digit output, whose extra live values would otherwise cost a wave per SIMD (255^3:
// 144 us per pass at four waves per SIMD against 159 at three with the 1 x 2 patch). The cost of this kernel is the number
// of vector memory instructions per point more than its HBM bytes; this layout
// needs about 3 per point plus the stage operands, against 12 for one point per lane.
// Blocks are four waves stacked along x2 and are numbered x1 segment fastest, then x2,
// then x3. Outputs are written with nontemporal stores: the next reader is another
// kernel, much later than any cache would keep them.
typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float flt2u __attribute__((ext_vector_type(2), aligned(4)));
typedef float flt4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr int SW = 4;   // waves per block, stacked along x2

struct StencilGrid {
  int nxs, nyb, nzb;    // x1 segments, x2 blocks, x3 blocks
};

// P values at base[off..off+P) into v; element k is wanted for k < cnt (cnt may exceed
// P). One vector access when all P lie inside the row or at least inside the
// allocation [0, lim); elementwise otherwise (the last row of an array).
template <int P>
__device__ __forceinline__ void load_row(double (&v)[P], const double* __restrict__ base, int64_t off, int64_t lim,
                                         int cnt) {
  if (cnt >= P || off + P <= lim) {
    if constexpr (P == 1) {
      v[0] = base[off];
    } else {
#pragma unroll
      for (int k = 0; k < P; k += 2) {
        const dbl2u t = *(const dbl2u*)(base + off + k);
        v[k] = t.x;
        v[k + 1] = t.y;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = (k < cnt) ? base[off + k] : 0.0;
  }
}

template <int P>
__device__ __forceinline__ void store_row(double* __restrict__ base, int64_t off, const double (&v)[P], int cnt) {
  if (cnt >= P) {
    if constexpr (P == 1) {
      __builtin_nontemporal_store(v[0], base + off);
    } else {
#pragma unroll
      for (int k = 0; k < P; k += 2) __builtin_nontemporal_store(dbl2u{v[k], v[k + 1]}, (dbl2u*)(base + off + k));
    }
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (k < cnt) base[off + k] = v[k];
  }
}

template <int P>
__device__ __forceinline__ void store_row(float* __restrict__ base, int64_t off, const double (&v)[P], int cnt) {
  if (cnt >= P) {
    if constexpr (P == 1) {
      __builtin_nontemporal_store((float)v[0], base + off);
    } else if constexpr (P == 2) {
      __builtin_nontemporal_store(flt2u{(float)v[0], (float)v[1]}, (flt2u*)(base + off));
    } else {
      __builtin_nontemporal_store(flt4u{(float)v[0], (float)v[1], (float)v[2], (float)v[3]},
                                  (flt4u*)(base + off));
    }
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (k < cnt) base[off + k] = (float)v[k];
  }
}

// The exact-slice split of one stage vector's row (sliced.hip defines it for the mode
// products): the row's exponent e (max |v| (1 + 2^-7) < 2^e, from a wave maximum: the whole
// row is in this wave) and, per value, Y = rint(v 2^(8S-1-e)) written with S balanced base-256
// digits in [-128, 127], the bytes of Y + 0x80..80 each minus 128. Plane t holds digit
// S-1-t (most significant first) at row r, position x of a plane of rows kp bytes;
// values past n1 are zero digits. Every lane of the wave takes part (the reduction).
template <int P, int S>
__device__ __forceinline__ void write_row_digits(const double (&v)[P], int cnt, int x, int64_t row,
                                                 const StencilArgs& p, int kp) {
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < P; ++k)
    if (k < cnt) m = fmax(m, fabs(v[k]));
  m = wave::wave_max(m);
  const int e = digits::digit_exponent(m);
  // row layout: plane t at t dplane, row r at r kp; chain layout (slice_digits.h): fiber
  // r % n2 of group r / n2, the P values of a lane inside one 16-byte fragment, planes
  // 2048 bytes apart
  const int64_t g = p.dchain ? row / p.n2 : 0;
  const int j = p.dchain ? (int)(row - g * p.n2) : 0;
  if ((threadIdx.x & 63) == 0) p.dexp[p.dchain ? g * 256 + j : row] = e;
  if (x >= kp) return;
  signed char* base = p.dchain ? p.dig + digits::chain_offset(g, j, x, 0, kp / 64, S) : p.dig + row * kp + x;
  const int64_t pstride = p.dchain ? 2048 : p.dplane;
  if constexpr (P == 4) {
    // four consecutive values: one 4-byte word per plane through the byte transpose
    unsigned pl[S];
    digits::slice4<S>(cnt > 0 ? v[0] : 0.0, cnt > 1 ? v[1] : 0.0, cnt > 2 ? v[2] : 0.0, cnt > 3 ? v[3] : 0.0, e, pl);
#pragma unroll
    for (int t = 0; t < S; ++t) *(unsigned*)(base + t * pstride) = pl[t];
  } else {
    unsigned lo[P], hi[P];
#pragma unroll
    for (int k = 0; k < P; ++k) digits::slice_bytes<S>(k < cnt ? v[k] : 0.0, e, lo[k], hi[k]);
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int i = S - 1 - t;                       // digit i (least significant first) in plane t
      unsigned w = 0;
#pragma unroll
      for (int k = 0; k < P; ++k) w |= (((i < 4 ? lo[k] >> (8 * i) : hi[k] >> (8 * (i - 4))) & 255u) << (8 * k));
      if constexpr (P == 2)
        *(unsigned short*)(base + t * pstride) = (unsigned short)w;
      else
        *(base + t * pstride) = (signed char)w;
    }
  }
}

template <int D, int P, int S>
__device__ __forceinline__ void stencil_body(const StencilArgs& p, const StencilGrid& sg) {
  constexpr int YT = (D == 3) ? 1 : 2;   // rows per lane along x2
  constexpr int ZT = (D == 3 && S == 0) ? 2 : 1;   // rows per lane along x3
  constexpr int YH = YT + 2;             // with the x2 halo
  constexpr int ZH = (D == 3) ? ZT + 2 : 1;
  const int L = blockIdx.x;
  const int bx = L % sg.nxs;
  const int rb = L / sg.nxs;
  const int by = rb % sg.nyb;
  const int bz = rb / sg.nyb;
  const int tx = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n1 = p.n1, n2 = p.n2, n3 = p.n3;
  const int x0 = bx * 64 * P;            // first x1 of the wave's segment
  const int x = x0 + P * tx;             // first x1 of this lane
  const int y0 = (by * SW + w) * YT;
  const int z0 = (D == 3) ? bz * ZT : 0;
  // x1 row strides: u, sub and base* (input layout), out* (output layout); 0 = n1
  const int64_t ldi = p.ldi ? p.ldi : n1, ldo = p.ldo ? p.ldo : n1;
  const int64_t s2 = ldi, s3 = ldi * n2;                       // strides of u
  const int64_t o2 = ldo, o3 = ldo * n2;                       // strides of the outputs
  const int64_t t2 = n1 + 2, t3 = (int64_t)(n1 + 2) * (n2 + 2);   // strides of a (padded)
  const int64_t nu = s3 * n3, na = t3 * ((D == 3) ? n3 + 2 : 1);
  const int ucnt = n1 - x;               // u elements of this lane inside the row
  const int acnt = n1 + 1 - x;           // a elements with x1 <= n1 (the last is a boundary node)
  const double* __restrict__ u = p.u;
  const double* __restrict__ a = p.a;
  // uu[y][z][k] = u at (x + k, y0 - 1 + y, z0 - 1 + z) (2D: z0 + z); zero outside the grid
  double uu[YH][ZH][P], aa[YH][ZH][P];
  // the rows of u and a at (x2, x3) = (i2, i3) into cu, ca (zero outside the grid; the u
  // values of a lane past the row's end are zeroed by zero_tail once every row's loads
  // are in flight, so that no row waits for the one before)
  auto load_rows = [&](double (&cu)[P], double (&ca)[P], int i2, int i3, bool need) {
    const bool urow = need && ucnt > 0 && i2 >= 0 && i2 < n2 && i3 >= 0 && i3 < n3;
    const bool arow = need && acnt > 0 && i2 >= -1 && i2 <= n2 && (D == 2 || (i3 >= -1 && i3 <= n3));
    if (urow) {
      load_row<P>(cu, u, x + s2 * i2 + s3 * i3, nu, ucnt);
    } else {
#pragma unroll
      for (int k = 0; k < P; ++k) cu[k] = 0.0;
    }
    if (arow) {
      load_row<P>(ca, a, (x + 1) + t2 * (i2 + 1) + ((D == 3) ? t3 * (i3 + 1) : 0), na, acnt);
    } else {
#pragma unroll
      for (int k = 0; k < P; ++k) ca[k] = 0.0;
    }
  };
  auto zero_tail = [&](double (&cu)[P]) {
#pragma unroll
    for (int k = 0; k < P; ++k)
      if (k >= ucnt) cu[k] = 0.0;
  };
  // The x2 halo rows of a wave are centre rows of the waves beside it in the block, shared
  // through LDS (the 2 ZT rows just outside the block are brought by the first 2 ZT
  // waves). Per array and wave: 3D five row loads instead of eight (1 x 2 patch) or three
  // or four instead of five (1 x 1); 2D two or three instead of four.
  constexpr int ZB = (D == 3) ? 1 : 0;   // index in uu of the first centre plane
  // the row just outside the block that this wave brings (first 2 ZT waves), loaded first
  constexpr int BR = YT * SW;
  const bool outw = w < 2 * ZT;
  const int orr = (w < ZT) ? -1 : BR, ozi = w % ZT;
  double ou[P], oa[P];
  load_rows(ou, oa, by * BR + orr, (D == 3) ? z0 + ozi : 0, outw);
#pragma unroll
  for (int y = 1; y <= YT; ++y)
#pragma unroll
    for (int z = 0; z < ZH; ++z) {
      const bool need = (D == 3) ? !((y == 0 || y == YH - 1) && (z == 0 || z == ZH - 1)) : true;
      load_rows(uu[y][z], aa[y][z], y0 - 1 + y, (D == 3) ? z0 - 1 + z : 0, need);
    }
  // with the rows: the segment-end neighbours of the centre rows (lanes 0 and 63) and a
  // separate stage base (base0 other than u), so that no load is issued after the rows
  // have been waited for
  const bool edge = (tx == 0) || (tx == 63);
  const int xe = (tx == 0) ? x0 - 1 : x0 + 64 * P;   // the segment's outside neighbour
  const bool useg = sg.nxs > 1;                      // u beyond the segment can be nonzero
  const bool wpre = p.base0 != nullptr && p.base0 != u;
  double ue_c[YT][ZT], ae_c[YT][ZT], wb[YT][ZT][P];
#pragma unroll
  for (int y = 1; y <= YT; ++y)
#pragma unroll
    for (int zi = 0; zi < ZT; ++zi) {
      const int i2 = y0 - 1 + y;
      const int i3 = (D == 3) ? z0 + zi : 0;
      const bool live_row = i2 < n2 && i3 < n3;
      ue_c[y - 1][zi] = 0.0;
      ae_c[y - 1][zi] = 0.0;
      if (edge) {
        if (useg && live_row && xe >= 0 && xe < n1) ue_c[y - 1][zi] = u[s2 * i2 + s3 * i3 + xe];
        if (live_row && xe >= -1 && xe <= n1)
          ae_c[y - 1][zi] = a[t2 * (i2 + 1) + ((D == 3) ? t3 * (i3 + 1) : 0) + xe + 1];
      }
      if (wpre && live_row && ucnt > 0) load_row<P>(wb[y - 1][zi], p.base0, x + s2 * i2 + s3 * i3, nu, ucnt);
    }
#pragma unroll
  for (int y = 1; y <= YT; ++y)
#pragma unroll
    for (int z = 0; z < ZH; ++z) zero_tail(uu[y][z]);
  zero_tail(ou);
  // slot ZT (r + 1) + zi: block row r (-1..BR, x2 = by BR + r) at centre plane zi
  constexpr int NS = ZT * (BR + 2);
  __shared__ __attribute__((aligned(16))) double Lu[NS][64 * P], La[NS][64 * P];
  auto put = [&](double (&L)[NS][64 * P], int slot, const double (&v)[P]) {
#pragma unroll
    for (int k = 0; k < P; ++k) L[slot][P * tx + k] = v[k];
  };
  auto get = [&](double (&L)[NS][64 * P], int slot, double (&v)[P]) {
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = L[slot][P * tx + k];
  };
  if (outw) {
    put(Lu, ZT * (orr + 1) + ozi, ou);
    put(La, ZT * (orr + 1) + ozi, oa);
  }
#pragma unroll
  for (int y = 1; y <= YT; ++y)
#pragma unroll
    for (int zi = 0; zi < ZT; ++zi) {
      put(Lu, ZT * (w * YT + y) + zi, uu[y][ZB + zi]);
      put(La, ZT * (w * YT + y) + zi, aa[y][ZB + zi]);
    }
  __syncthreads();
  const double la = p.lam_amax;
#pragma unroll
  for (int y = 1; y <= YT; ++y)
#pragma unroll
    for (int z = (D == 3) ? 1 : 0; z < ((D == 3) ? ZT + 1 : 1); ++z) {
      const int i2 = y0 - 1 + y;
      const int i3 = (D == 3) ? z0 - 1 + z : 0;
      const bool live_row = i2 < n2 && i3 < n3;
      const int64_t urow = s2 * i2 + s3 * i3;
      // the x2 halo rows of this centre row from LDS (read where they are used, so that
      // only one centre row's halo is held at a time)
      if (y == 1) {
        get(Lu, ZT * (w * YT) + z - ZB, uu[0][z]);
        get(La, ZT * (w * YT) + z - ZB, aa[0][z]);
      }
      if (y == YT) {
        get(Lu, ZT * (w * YT + YT + 1) + z - ZB, uu[YT + 1][z]);
        get(La, ZT * (w * YT + YT + 1) + z - ZB, aa[YT + 1][z]);
      }
      const double* uc = uu[y][z];
      const double* ac = aa[y][z];
      // x1 neighbours across lanes (every lane takes part), then the segment ends
      double ul = wave::from_prev(uc[P - 1]), ur = wave::from_next(uc[0]);
      double al = wave::from_prev(ac[P - 1]), ar = wave::from_next(ac[0]);
      if (edge) {
        const double ue = ue_c[y - 1][z - ZB], ae = ae_c[y - 1][z - ZB];
        if (tx == 0) {
          ul = ue;
          al = ae;
        } else {
          ur = ue;
          ar = ae;
        }
      }
      // (the digit output needs every lane of the row's wave for its row maximum)
      if (!live_row || (ucnt <= 0 && S == 0)) continue;
      const int64_t idx = x + urow;
      const int64_t idxo = x + o2 * i2 + o3 * i3;
      // last unknown of an axis with a zero normal derivative at x = 1: mirror ghost
      const bool my = p.neu[1] && i2 == n2 - 1;
      const bool mz = (D == 3) && p.neu[2] && i3 == n3 - 1;
      double g[P];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const double u0 = uc[k], a0 = ac[k];
        const double uxm = (k == 0) ? ul : uc[k - 1];
        const double uxp = (p.neu[0] && x + k == n1 - 1) ? uxm : (k == P - 1) ? ur : uc[k + 1];
        const double uym = uu[y - 1][z][k], uyp = my ? uym : uu[y + 1][z][k];
        double v;
        if (p.nondiv) {
          const double c = a0 - la;
          v = c * (uxp - 2.0 * u0 + uxm) * p.ih2[0] + p.cadv[0] * (uxp - uxm);
          v += c * (uyp - 2.0 * u0 + uym) * p.ih2[1] + p.cadv[1] * (uyp - uym);
          if constexpr (D == 3) {
            const double uzm = uu[y][z - 1][k], uzp = mz ? uzm : uu[y][z + 1][k];
            v += c * (uzp - 2.0 * u0 + uzm) * p.ih2[2] + p.cadv[2] * (uzp - uzm);
          }
        } else {
          const double axm = (k == 0) ? al : ac[k - 1], axp = (k == P - 1) ? ar : ac[k + 1];
          v = ((0.5 * (a0 + axp) - la) * (uxp - u0) - (0.5 * (a0 + axm) - la) * (u0 - uxm)) * p.ih2[0] +
              p.cadv[0] * (uxp - uxm);
          v += ((0.5 * (a0 + aa[y + 1][z][k]) - la) * (uyp - u0) - (0.5 * (a0 + aa[y - 1][z][k]) - la) * (u0 - uym)) *
                   p.ih2[1] +
               p.cadv[1] * (uyp - uym);
          if constexpr (D == 3) {
            const double uzm = uu[y][z - 1][k], uzp = mz ? uzm : uu[y][z + 1][k];
            v += ((0.5 * (a0 + aa[y][z + 1][k]) - la) * (uzp - u0) - (0.5 * (a0 + aa[y][z - 1][k]) - la) * (u0 - uzm)) *
                     p.ih2[2] +
                 p.cadv[2] * (uzp - uzm);
          }
        }
        v += p.r0 + u0 * (p.r1 + u0 * (p.r2 + u0 * p.r3));
        g[k] = v;
      }
      if (p.sub) {
        double sv[P];
        load_row<P>(sv, p.sub, idx, nu, ucnt);
#pragma unroll
        for (int k = 0; k < P; ++k) g[k] -= sv[k];
      }
      // out0 = base0 + c0 g (base0 == u: from registers)
      double o[P];
      if (p.base0 == nullptr) {
#pragma unroll
        for (int k = 0; k < P; ++k) o[k] = p.c0 * g[k];
      } else if (p.base0 == u) {
#pragma unroll
        for (int k = 0; k < P; ++k) o[k] = uc[k] + p.c0 * g[k];
      } else {
#pragma unroll
        for (int k = 0; k < P; ++k) o[k] = wb[y - 1][z - ZB][k] + p.c0 * g[k];
      }
      if (p.flag) {
        bool bad = false;
#pragma unroll
        for (int k = 0; k < P; ++k) bad |= (k < ucnt) && !(fabs(o[k]) <= DBL_MAX);
        if (bad) p.flag[0] = 1;
      }
      if constexpr (S > 0) {
        // the stage vectors as digit planes of the mode-1 operand (rows of one wave)
        const int kp = slice_ld(n1);
        const int64_t row = i2 + (int64_t)n2 * i3;
        write_row_digits<P, S>(o, ucnt, x, row, p, kp);
        if (p.drow1) {   // base1 is u or null (checked at launch)
#pragma unroll
          for (int k = 0; k < P; ++k) o[k] = (p.base1 ? uc[k] : 0.0) + p.c1 * g[k];
          write_row_digits<P, S>(o, ucnt, x, p.drow1 + row, p, kp);
        }
        continue;
      }
      if (p.out0f)
        store_row<P>(p.out0f, idxo, o, ucnt);
      else
        store_row<P>(p.out0, idxo, o, ucnt);
      if (p.out1 || p.out1f) {
        if (p.base1 == nullptr) {
#pragma unroll
          for (int k = 0; k < P; ++k) o[k] = p.c1 * g[k];
        } else if (p.base1 == u) {
#pragma unroll
          for (int k = 0; k < P; ++k) o[k] = uc[k] + p.c1 * g[k];
        } else {
          load_row<P>(o, p.base1, idx, nu, ucnt);
#pragma unroll
          for (int k = 0; k < P; ++k) o[k] += p.c1 * g[k];
        }
        if (p.out1f)
          store_row<P>(p.out1f, idxo, o, ucnt);
        else
          store_row<P>(p.out1, idxo, o, ucnt);
      }
    }
}

// blockIdx.y selects one of up to kMaxGroups problems of the same grid shape (their own
// u, a, coefficients and outputs). A single problem is launched the same way with one
// entry, so one compiled kernel serves both, and a problem's results do not depend on
// whether it ran alone or in a group (two instantiations of the body may contract
// multiply-adds differently, which changes last bits).
template <int D, int P, int S>
__global__ __launch_bounds__(64 * SW, 3) void stencil_batch_kernel(StencilBatch b, StencilGrid sg) {
  stencil_body<D, P, S>(b.a[blockIdx.y], sg);
}

// Points per lane: the P in {4, 2, 1} that pads n1 least to whole 64 P-point segments,
// the larger P on ties. Measured per pass at n^3 (us, P = 1 / 2 / 4): n = 63: 5 / 7 / 8;
// 191: 54 / 71 / 59; 255: 129-149 / 141-146 / 132-134; 383: 510 / 481 / 591 -- idle lanes
// cost more than the extra instructions of narrower lanes.
static int points_per_lane(int n1) {
  int best = 4;
  int64_t width = 256LL * ((n1 + 255) / 256);
  for (int P : {2, 1}) {
    const int64_t wdt = 64LL * P * ((n1 + 64 * P - 1) / (64 * P));
    if (wdt < width) {
      width = wdt;
      best = P;
    }
  }
  return best;
}

template <int D, int S>
static void launch_batch_ds(int P, const StencilBatch& b, int count, StencilGrid sg, unsigned blocks,
                            hipStream_t s) {
  const dim3 grid(blocks, (unsigned)count);
  if (P == 4)
    stencil_batch_kernel<D, 4, S><<<grid, dim3(64 * SW), 0, s>>>(b, sg);
  else if (P == 2)
    stencil_batch_kernel<D, 2, S><<<grid, dim3(64 * SW), 0, s>>>(b, sg);
  else
    stencil_batch_kernel<D, 1, S><<<grid, dim3(64 * SW), 0, s>>>(b, sg);
}

template <int D>
static void launch_batch_d(int P, const StencilBatch& b, int count, StencilGrid sg, unsigned blocks, hipStream_t s) {
  switch (b.a[0].dig ? b.a[0].dS : 0) {
    case 3: launch_batch_ds<D, 3>(P, b, count, sg, blocks, s); break;
    case 4: launch_batch_ds<D, 4>(P, b, count, sg, blocks, s); break;
    case 5: launch_batch_ds<D, 5>(P, b, count, sg, blocks, s); break;
    case 6: launch_batch_ds<D, 6>(P, b, count, sg, blocks, s); break;
    case 7: launch_batch_ds<D, 7>(P, b, count, sg, blocks, s); break;
    default: launch_batch_ds<D, 0>(P, b, count, sg, blocks, s); break;
  }
}

// Work decomposition of one grid (blocks of four waves); false if it does not fit a grid.
static bool stencil_grid(int d, int n1, int n2, int n3, bool dig, int& P, StencilGrid& sg, int64_t& blocks) {
  if (n1 < 1 || n2 < 1 || n3 < 1) return false;
  P = points_per_lane(n1);
  sg.nxs = (n1 + 64 * P - 1) / (64 * P);
  const int yt = (d == 3) ? 1 : 2, zt = (d == 3 && !dig) ? 2 : 1;
  sg.nyb = (n2 + SW * yt - 1) / (SW * yt);
  sg.nzb = (d == 3) ? (n3 + zt - 1) / zt : 1;
  blocks = (int64_t)sg.nxs * sg.nyb * sg.nzb;
  return blocks < (1LL << 31);
}

hipError_t launch_stencil(int d, const StencilArgs& a, hipStream_t s) { return launch_stencil_batch(d, &a, 1, s); }

bool stencil_row_in_one_wave(int n1) { return n1 >= 1 && 64 * points_per_lane(n1) >= n1; }

hipError_t launch_stencil_batch(int d, const StencilArgs* a, int count, hipStream_t s) {
  if (count < 1 || count > kMaxGroups) return hipErrorInvalidValue;
  for (int i = 1; i < count; ++i)
    if (a[i].n1 != a[0].n1 || a[i].n2 != a[0].n2 || a[i].n3 != a[0].n3) return hipErrorInvalidValue;
  for (int i = 0; i < count; ++i)
    if (!a[i].u || !a[i].a || (!a[i].dig && !a[i].out0 && !a[i].out0f)) return hipErrorInvalidValue;
  for (int i = 1; i < count; ++i)   // one kernel for the group: the same output form
    if ((a[i].dig != nullptr) != (a[0].dig != nullptr) || (a[0].dig && a[i].dS != a[0].dS))
      return hipErrorInvalidValue;
  for (int i = 0; i < count; ++i)
    if (a[i].dig && (!a[i].dexp || a[i].dS < kMinSlices || a[i].dS > kMaxSlices || !stencil_row_in_one_wave(a[i].n1) ||
                     (a[i].base1 != a[i].u && a[i].base1 != nullptr && a[i].drow1) ||
                     (a[i].dchain && (a[i].n2 > 256 || (a[i].drow1 && a[i].drow1 % a[i].n2 != 0)))))
      return hipErrorInvalidValue;
  int P;
  StencilGrid sg;
  int64_t blocks;
  if (!stencil_grid(d, a[0].n1, a[0].n2, a[0].n3, a[0].dig != nullptr, P, sg, blocks)) return hipErrorInvalidValue;
  StencilBatch b;
  for (int i = 0; i < count; ++i) b.a[i] = a[i];
  if (d == 3)
    launch_batch_d<3>(P, b, count, sg, (unsigned)blocks, s);
  else
    launch_batch_d<2>(P, b, count, sg, (unsigned)blocks, s);
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
__global__ void build_tridiag(double* M, int n, double sub, double diag, double sup, double last_sub) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  M[e] = (c == r) ? diag : (c == r - 1) ? (r == n - 1 ? last_sub : sub) : (c == r + 1) ? sup : 0.0;
}

hipError_t launch_build_tridiag(double* M, int n, double sub, double diag, double sup, double last_sub,
                                hipStream_t s) {
  const int64_t cnt = (int64_t)n * n;
  build_tridiag<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(M, n, sub, diag, sup, last_sub);
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
