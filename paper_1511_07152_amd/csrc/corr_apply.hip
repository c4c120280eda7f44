// The correction F_w - F~_w applied beside the separable GCF (Section 6):
// a small full 2D table C[k][fu][fv][sv][su] (S_c x S_c taps, oversampling
// O_c) added to the separable footprint when gridding, and its adjoint when
// degridding.
//
// A visibility's correction sample is the point of the 1/O_c lattice nearest
// to its quantised position cell + f/O, ties towards +: with r = O / O_c,
// g = floor((f + floor(r/2)) / r) in [-O_c/2, O_c/2]; g = O_c/2 moves to the
// next cell (cell_c = cell + 1, f_c = -O_c/2).  The correction footprint,
// S_c cells about cell_c, lies inside the separable footprint (the library
// enforces S_c <= S - 2 unless O_c is O or 1, where cell_c = cell), hence
// inside the tile's 16 x 16 region: both passes walk the plan's tile work
// items exactly like the separable kernels and decode everything from the
// slot records (plane, sub-cell rows and position in the tile).
//
// Lane layout: the S_c^2 taps of a visibility occupy an aligned group of Tp
// lanes (S_c^2 rounded up to a power of two): with Tp <= 64 one pass over the
// wave covers 64 / Tp visibilities, with Tp > 64 a visibility takes Tp / 64
// passes.  Table reads of a group are contiguous.
// Gridding adds y_i C into the wave's LDS ring of grid columns with LDS float
// atomics (taps of different visibilities of one pass can meet in a cell) and
// flushes the ring to the grid as the separable kernel does.  Degridding
// multiplies each tap's grid value by the conjugate table entry, sums the
// group's lanes with butterflies and adds the sum to the visibility's result,
// which the separable degridding kernel has already written.
#include "ring.h"
#include "walk.h"

namespace sepw {

namespace {

constexpr int kCorrWaves = 4;

struct TapPos {
  int col;   // region column (gridding) or grid column (degridding) of tap su = 0
  int row;   // band row (gridding) or grid row (degridding) of tap sv = 0
  int tb;    // table offset of the visibility's S_c x S_c block
};

// Slot record -> correction footprint origin relative to the tile's region
// (region column x = cell - (tx C - S/2)) and table block.
template <int S>
__device__ inline TapPos decode(const SlotRec& r, const CorrGeom& g) {
  constexpr int L = 32 - S, C = 17 - S, H = S / 2;
  const int row_u = r.x / L, ox = C - 1 - (r.x - row_u * L);
  const int row_v = r.y / L, oy = C - 1 - (r.y - row_v * L);
  const int k = row_u >> g.lo;
  const int fu = row_u & (g.O - 1), fv = row_v & (g.O - 1);
  const int half_r = (1 << g.lr) >> 1;
  const int gu = ((fu - g.O / 2 + half_r + g.O) >> g.lr) - g.Oc;   // floor((f + r/2) / r)
  const int gv = ((fv - g.O / 2 + half_r + g.O) >> g.lr) - g.Oc;
  const int shu = gu + g.Oc / 2 >= g.Oc ? 1 : 0, shv = gv + g.Oc / 2 >= g.Oc ? 1 : 0;
  const int fcu = gu + g.Oc / 2 - shu * g.Oc, fcv = gv + g.Oc / 2 - shv * g.Oc;
  TapPos t;
  t.col = ox + H + shu - g.hc;
  t.row = oy + H + shv - g.hc;
  t.tb = ((k * g.Oc + fcu) * g.Oc + fcv) * g.T2;
  return t;
}

__device__ inline int bperm_i(int src_lane, int v) {
  return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}
__device__ inline float bperm_f(int src_lane, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

// Tap t of a group -> (sv, su); t < T2 <= 225, so the float quotient is exact.
__device__ inline void tap_rc(int t, const CorrGeom& g, int& sv, int& su) {
  sv = (int)(((float)t + 0.5f) * g.inv_sc);
  su = t - sv * g.Sc;
}

// Tiles of one work item: calls body(tx, c0, re) for the real slots [c0, re)
// of each non-empty tile in order, and on_move(x0) before each tile after the first.
template <int S, class Body, class Move>
__device__ inline void walk_item(const int4& item, const uint2* tdesc, int ntx, int lane, Body&& body,
                                 Move&& on_move) {
  const int ty = uniform(item.x), s_end = uniform(item.z);
  TileWalk tw;
  tw.start(tdesc + (int64_t)ty * ntx, ntx, uniform(item.w), lane);
  int c0 = uniform(item.y);
  while (true) {
    const int pe = min(tw.padded_end(), s_end);
    body(tw.tx, c0, min(tw.real_end(), s_end));
    if (pe >= s_end || !tw.next(lane)) break;
    on_move(tw.tx);
    c0 = tw.first_slot();
  }
}

template <int S>
__global__ __launch_bounds__(64 * kCorrWaves) void corr_grid_kernel(CorrArgs a) {
  constexpr int C = 17 - S, H = S / 2;
  __shared__ float rings[kCorrWaves * kRingFloats];
  const int lane = threadIdx.x & 63;
  float* ring = rings + (threadIdx.x >> 6) * kRingFloats;
  for (int i = lane; i < kRingFloats; i += 64) ring[i] = 0.f;
  float* grid = reinterpret_cast<float*>(a.grid);
  const CorrGeom g = a.g;
  const int tp = 1 << g.lt;
  const int n_items = (int)*a.nitems;
  int stride;
  for (int it = uniform(wave_items(kCorrWaves, &stride)); it < n_items; it += stride) {
    const int4 item = a.items[it];
    const int by = uniform(item.x) * C - H;
    int fx = uniform(item.w) * C - H;
    walk_item<S>(
        item, a.tdesc, a.ntx, lane,
        [&](int tx, int c0, int re) {
          const int x0 = tx * C - H;
          for (int b0 = c0; b0 < re; b0 += 64) {
            const int nb = min(64, re - b0);
            TapPos mine{0, 0, 0};
            float2 y = make_float2(0.f, 0.f);
            if (lane < nb) {
              const SlotRec r = a.krec[b0 + lane];
              mine = decode<S>(r, g);
              y = a.yrow[r.z];
            }
            const int passes = (nb * tp + 63) >> 6;
            for (int p = 0; p < passes; ++p) {
              const int f = (p << 6) + lane;
              const int v = f >> g.lt, t = f & (tp - 1);
              const int src = v & 63;
              const int col = bperm_i(src, mine.col), row = bperm_i(src, mine.row);
              const int tb = bperm_i(src, mine.tb);
              const float yr = bperm_f(src, y.x), yi = bperm_f(src, y.y);
              if (v < nb && t < g.T2) {
                int sv, su;
                tap_rc(t, g, sv, su);
                const float2 cv = a.tab[tb + t];
                float* cell = ring + 2 * ((row + sv) * kRingPitch + ((x0 + col + su) & (kRing - 1)));
                atomicAdd(cell, yr * cv.x - yi * cv.y);
                atomicAdd(cell + 1, yr * cv.y + yi * cv.x);
              }
            }
          }
        },
        [&](int tx) {
          // ring columns [fx, fx + kRing) hold the band; make room for [x0, x0 + 16)
          const int x0 = tx * C - H;
          if (x0 >= fx + kRing) {
            ring_flush16(ring, fx, grid, by, a.N, a.checker, lane);
            ring_flush16(ring, fx + 16, grid, by, a.N, a.checker, lane);
            fx = x0;
          } else if (x0 + 16 > fx + kRing) {
            ring_flush16(ring, fx, grid, by, a.N, a.checker, lane);
            fx += 16;
          }
        });
    ring_flush16(ring, fx, grid, by, a.N, a.checker, lane);
    ring_flush16(ring, fx + 16, grid, by, a.N, a.checker, lane);
  }
}

template <int S>
__global__ __launch_bounds__(64 * kCorrWaves) void corr_degrid_kernel(CorrArgs a) {
  constexpr int C = 17 - S, H = S / 2;
  const int lane = threadIdx.x & 63;
  const CorrGeom g = a.g;
  const int tp = 1 << g.lt;
  const int gl = tp < 64 ? tp : 64;                 // lanes reduced together
  const int pv = tp > 64 ? tp >> 6 : 1;             // passes per visibility
  const int n_items = (int)*a.nitems;
  const float2* grid = a.grid;
  int stride;
  for (int it = uniform(wave_items(kCorrWaves, &stride)); it < n_items; it += stride) {
    const int4 item = a.items[it];
    const int by = uniform(item.x) * C - H;
    walk_item<S>(
        item, a.tdesc, a.ntx, lane,
        [&](int tx, int c0, int re) {
          const int x0 = tx * C - H;
          for (int b0 = c0; b0 < re; b0 += 64) {
            const int nb = min(64, re - b0);
            TapPos mine{0, 0, 0};
            int z = 0;
            if (lane < nb) {
              const SlotRec r = a.krec[b0 + lane];
              mine = decode<S>(r, g);
              z = r.z;
            }
            const int passes = (nb * tp + 63) >> 6;
            float sre = 0.f, sim = 0.f;
            for (int p = 0; p < passes; ++p) {
              const int f = (p << 6) + lane;
              const int v = f >> g.lt, t = f & (tp - 1);
              const int src = v & 63;
              const int col = bperm_i(src, mine.col), row = bperm_i(src, mine.row);
              const int tb = bperm_i(src, mine.tb);
              if (v < nb && t < g.T2) {
                int sv, su;
                tap_rc(t, g, sv, su);
                const int gx = x0 + col + su, gy = by + row + sv;
                float2 gv = grid[(int64_t)gy * a.N + gx];
                if (a.checker && ((gx + gy) & 1)) gv = make_float2(-gv.x, -gv.y);
                const float2 cv = a.tab[tb + t];
                sre += gv.x * cv.x + gv.y * cv.y;   // G conj(C)
                sim += gv.y * cv.x - gv.x * cv.y;
              }
              if ((p + 1) % pv == 0) {
                for (int o = gl >> 1; o > 0; o >>= 1) {
                  sre += __shfl_xor(sre, o, 64);
                  sim += __shfl_xor(sim, o, 64);
                }
                const int zv = bperm_i(src, z);
                if ((lane & (gl - 1)) == 0 && v < nb) {
                  float2* o = a.yrow + zv;
                  const float2 old = *o;
                  *o = make_float2(old.x + sre, old.y + sim);
                }
                sre = 0.f;
                sim = 0.f;
              }
            }
          }
        },
        [](int) {});
  }
}

inline int64_t corr_blocks(int64_t max_items) {
  int64_t b = (max_items + kCorrWaves - 1) / kCorrWaves;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return b;
}

template <int S>
hipError_t launch_s(bool degrid, const CorrArgs& a, int64_t max_items, hipStream_t s) {
  const dim3 grid((unsigned)corr_blocks(max_items)), block(64 * kCorrWaves);
  if (degrid)
    hipLaunchKernelGGL(corr_degrid_kernel<S>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(corr_grid_kernel<S>, grid, block, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_any(int S, bool degrid, const CorrArgs& a, int64_t max_items, hipStream_t s) {
  switch (S) {
    case 1: return launch_s<1>(degrid, a, max_items, s);
    case 3: return launch_s<3>(degrid, a, max_items, s);
    case 5: return launch_s<5>(degrid, a, max_items, s);
    case 7: return launch_s<7>(degrid, a, max_items, s);
    case 9: return launch_s<9>(degrid, a, max_items, s);
    case 11: return launch_s<11>(degrid, a, max_items, s);
    case 13: return launch_s<13>(degrid, a, max_items, s);
    case 15: return launch_s<15>(degrid, a, max_items, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_corr_grid(int S, const CorrArgs& a, int64_t max_items, hipStream_t s) {
  return launch_any(S, false, a, max_items, s);
}

hipError_t launch_corr_degrid(int S, const CorrArgs& a, int64_t max_items, hipStream_t s) {
  return launch_any(S, true, a, max_items, s);
}

}  // namespace sepw
