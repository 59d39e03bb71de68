// Cross-lane moves and reductions of FP64 values within a wave, on DPP (the data-parallel
// primitives of the vector ALU) instead of the LDS crossbar: no LDS round trip and no wait
// between the steps. Every lane of the wave must be active.
#pragma once

#include <hip/hip_runtime.h>

namespace mm {
namespace wave {

// DPP controls (gfx9 encoding): quad permutations, mirrors within 8 and 16 lanes, and
// whole-wave shifts by one lane.
constexpr int kQuadXor1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kWaveShl1 = 0x130;      // lane i reads lane i + 1
constexpr int kWaveShr1 = 0x138;      // lane i reads lane i - 1

// x of the lane that DPP control C selects; lanes without a source keep x.
template <int C>
__device__ __forceinline__ double dpp(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, C, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), C, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// maximum over each row of 16 lanes (lanes 16 r .. 16 r + 15), in every lane of the row
__device__ __forceinline__ double row16_max(double x) {
  x = __builtin_fmax(x, dpp<kQuadXor1>(x));
  x = __builtin_fmax(x, dpp<kQuadXor2>(x));
  x = __builtin_fmax(x, dpp<kRowHalfMirror>(x));
  x = __builtin_fmax(x, dpp<kRowMirror>(x));
  return x;
}

// maximum over the wave, in every lane
__device__ __forceinline__ double wave_max(double x) {
  x = row16_max(x);
  const long long b = __builtin_bit_cast(long long, x);
  double m = x;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int lo = __builtin_amdgcn_readlane((int)b, 16 * r);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * r);
    m = __builtin_fmax(m, __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo));
  }
  return m;
}

// x of lane i - 1 (lane 0: its own x) and of lane i + 1 (lane 63: its own x)
__device__ __forceinline__ double from_prev(double x) { return dpp<kWaveShr1>(x); }
__device__ __forceinline__ double from_next(double x) { return dpp<kWaveShl1>(x); }

}  // namespace wave
}  // namespace mm
