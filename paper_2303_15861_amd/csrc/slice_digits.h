// Exact-slice digits of FP64 values (device code shared by the grid split of the
// exact-slice mode products and the stencil that can write its stage vectors as digit
// planes). A row or fiber with maximum m gets the exponent e of m (1 + 2^-7) (so that
// m < 0.993 2^e); a value x becomes Y = rint(x 2^(8S-1-e)), |Y| < 0.4963 256^S, written
// with S balanced base-256 digits in [-128, 127] (they cover [-0.502, 0.498] 256^S): the
// bytes of Y + 0x80..80, each minus 128 (an XOR with 0x80 per byte).
#pragma once

#include <hip/hip_runtime.h>

namespace mm {
namespace digits {

// The exponent of a row or fiber with maximum m >= 0 (0 for m = 0).
__device__ __forceinline__ int digit_exponent(double m) {
  int e = 0;
  __builtin_frexp(m * (1.0 + 0x1p-7), &e);
  return e;
}

// Balanced base-256 digits of x relative to exponent e, packed: byte i of (lo, hi) is
// b_i (least significant first) as a two's-complement int8.
template <int S>
__device__ __forceinline__ void slice_bytes(double x, int e, unsigned& lo, unsigned& hi) {
  constexpr unsigned long long C = 0x8080808080808080ull >> (64 - 8 * S);
  unsigned long long Y;   // round(x 2^(8S-1-e)) + C
  if constexpr (S <= 6) {
    // z = x 2^(8S-1-e), |z| < 0.4963 2^(8S) <= 2^47. Adding the integer 2^52 + C (exact
    // in FP64) rounds z to the nearest integer, ties to even (the sum lies in
    // [2^52, 2^53), where FP64 values are the integers, and 2^52 + C is even), and
    // leaves round(z) + C in [0, 2^48) in the significand field.
    const double d = __builtin_ldexp(x, 8 * S - 1 - e) + (double)((1ull << 52) + C);
    Y = __builtin_bit_cast(unsigned long long, d) & ((1ull << 52) - 1);
  } else {
    const double y = __builtin_rint(__builtin_ldexp(x, 8 * S - 1 - e));   // |y| < 0.4963 2^(8S)
    const double hf = __builtin_floor(y * 0x1p-32);
    const unsigned l = (unsigned)__builtin_fma(-hf, 0x1p32, y);           // exact, in [0, 2^32)
    const int h = (int)hf;
    Y = ((((unsigned long long)(unsigned)h) << 32) | l) + C;
  }
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

// Chain layout of S digit planes, the grid operand of the chained mode products: fibers
// come in groups of at most 256 (fiber j of group g), positions k are padded to kp = 64 nch.
// Per (32-fiber block, 64-k chunk, plane) one 2 KB block holds the 32 fibers' 64-byte
// chunks one after another, so a writer of 16 consecutive positions of one fiber writes
// within one 64-byte run, and a load of MFMA fragments (lane j % 32 + 32 h: the chunk
// bytes [32 h + 16 ks, +16) at step ks) covers one 2 KB block. Offset of (g, j, k, s):
__host__ __device__ inline int64_t chain_offset(int64_t g, int j, int k, int s, int nch, int S) {
  return (((g * 8 + (j >> 5)) * nch + (k >> 6)) * S + s) * 2048 + (j & 31) * 64 + (k & 63);
}

}  // namespace digits
}  // namespace mm
