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

// Register ring of the LDS-table gridding kernels.  With region column
// (c - x0) & 15 assigned to lane column c, lane c always holds grid columns
// congruent to c modulo 16, so a tile's region sums fall into one of two
// aligned blocks of 16 grid columns held in registers: block blk (lo) and
// block blk + 1 (hi), lane column c holding grid column 16 blk + c (lo) and
// 16 (blk + 1) + c (hi), rows 4 grp + r of the item's 16 rows.
typedef float ring_f32x4 __attribute__((ext_vector_type(4)));

struct RegRing {
  ring_f32x4 lo_re, lo_im, hi_re, hi_im;
  int blk;
};

// Add the lo block (grid columns 16 blk + col, rows y0 + 4 grp + r) times
// scale to the grid with atomics ((-1)^(x+y) when the grid feeds the centred
// FFT), then move hi down to lo and clear hi.
__device__ inline void reg_ring_shift(RegRing& rg, float* grid, int N, int checker, int y0,
                                      int col, int grp, float scale) {
  const int gx = 16 * rg.blk + col;
  if (gx >= 0 && gx < N) {
    const int gy0 = y0 + 4 * grp;
    float sg = (checker && ((gx + gy0) & 1)) ? -scale : scale;
    float* p = grid + 2 * ((int64_t)gy0 * N + gx);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gy = gy0 + r;
      if (gy >= 0 && gy < N) {
        if (rg.lo_re[r] != 0.f) unsafeAtomicAdd(p, sg * rg.lo_re[r]);
        if (rg.lo_im[r] != 0.f) unsafeAtomicAdd(p + 1, sg * rg.lo_im[r]);
      }
      p += 2 * (int64_t)N;
      if (checker) sg = -sg;
    }
  }
  rg.lo_re = rg.hi_re;
  rg.lo_im = rg.hi_im;
  rg.hi_re = ring_f32x4{0.f, 0.f, 0.f, 0.f};
  rg.hi_im = rg.hi_re;
  rg.blk += 1;
}

// Add a region's sums (re, im) for first grid column x0 into the block that
// holds this lane's column; selects, not a branch, so that the ring stays in
// registers (each lane adds to one block and 0 to the other).
__device__ inline void reg_ring_add(RegRing& rg, const ring_f32x4& re, const ring_f32x4& im, int x0,
                                    int col) {
  const int xa = x0 + ((col - x0) & 15);
  const bool hi = (xa >> 4) != rg.blk;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    rg.hi_re[r] += hi ? re[r] : 0.f;
    rg.hi_im[r] += hi ? im[r] : 0.f;
    rg.lo_re[r] += hi ? 0.f : re[r];
    rg.lo_im[r] += hi ? 0.f : im[r];
  }
}

// Make the ring hold the blocks a region starting at grid column x0 touches
// (x0 >> 4 and the next), flushing the blocks the walk has left.
__device__ inline void reg_ring_advance(RegRing& rg, int x0, float* grid, int N, int checker, int y0,
                                        int col, int grp, float scale) {
  const int b = x0 >> 4;   // floor(x0 / 16), also for x0 < 0
  if (b > rg.blk) {
    reg_ring_shift(rg, grid, N, checker, y0, col, grp, scale);
    if (b > rg.blk) {
      reg_ring_shift(rg, grid, N, checker, y0, col, grp, scale);
      rg.blk = b;
    }
  }
}

}  // namespace sepw
