// Per-wave LDS ring of grid columns for the gridding passes.
//
// A wave walking the tiles of one row of tiles keeps the partial sums of the
// 16 grid rows of that row's regions (rows ty C - S/2 .. + 15) in a ring of
// kRing columns indexed by grid column modulo kRing.  When the walk moves on,
// ring columns that no later tile of the item can reach are added to the grid
// with hardware FP32 atomics (regions of neighbouring tiles and rows overlap,
// so other waves add to the same cells) and cleared.
#pragma once

#include "internal.h"

namespace sepw {

constexpr int kRing = 32;        // ring columns (power of two, >= 2 x 16)
constexpr int kRingPitch = 34;   // complex entries per ring row (spreads LDS banks)
constexpr int kRingFloats = 2 * 16 * kRingPitch;

// Flush ring columns [fx, fx + 16) (grid rows gy0 .. gy0 + 15) to the grid with
// atomics and clear them.  Lane L takes float L % 32 of a 16-column row
// segment (column (L % 32) / 2, real or imaginary part) of rows 2 k + L / 32.
// All eight ring reads are issued before the first use; the lane's rows all
// have the parity of gy0 + L / 32, so its checkerboard sign is computed once.
__device__ inline void ring_flush16(float* ring, int fx, float* g, int gy0, int N, int checker,
                                    int lane) {
  const int f = lane & 31, half = lane >> 5;
  const int gx = fx + (f >> 1);
  const int slot = gx & (kRing - 1);
  const bool col_ok = gx >= 0 && gx < N;
  float* p = ring + 2 * (half * kRingPitch + slot) + (f & 1);   // row half, then 2 rows apart
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = p[4 * k * kRingPitch];
#pragma unroll
  for (int k = 0; k < 8; ++k) p[4 * k * kRingPitch] = 0.f;
  const float sg = (checker && ((gx + gy0 + half) & 1)) ? -1.f : 1.f;
  float* gp = g + 2 * ((int64_t)(gy0 + half) * N + gx) + (f & 1);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int gy = gy0 + 2 * k + half;
    if (v[k] != 0.f && col_ok && gy >= 0 && gy < N)
      unsafeAtomicAdd(gp + (int64_t)4 * k * N, sg * v[k]);
  }
}

}  // namespace sepw
