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
// Lane layout: every correction footprint of a tile's visibilities lies in a
// W x W window of the tile's region (W = C + S_c, or C + S_c - 1 when the
// coarse cell never moves), and each lane owns up to four fixed cells of that
// window, as the matrix-core kernels own their accumulator cells.  The slot
// records of a batch of up to 64 visibilities are decoded one per lane; then
// the visibilities go through one at a time (their data broadcast from the
// decoding lane with readlane), two at a time with all table loads issued
// before the first use, and every lane handles the taps that fall on its
// cells.  Gridding accumulates in registers and adds the window into the
// wave's LDS ring of grid columns when the walk leaves the tile (each lane
// its own cells, so no atomics), flushing the ring to the grid as the
// separable kernel does.  Degridding loads the window from the grid once per
// tile, multiplies each tap's value by the conjugate table entry, sums over
// the wave with DPP row operations and adds the sum to the visibility's
// result (already written by the separable degridding kernel) once per batch.
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

constexpr int kUnroll = 2;   // visibilities whose table loads are in flight together (more costs occupancy)
constexpr int kCells = 4;    // window cells per lane (W^2 <= 256)

// x + (x of the lane the DPP control selects), disabled rows adding 0
template <int CTRL, int ROWS>
__device__ inline float dpp_add(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xF, true));
}

// Sum over the wave, ending in lane 63 (inclusive scans within rows of 16,
// then row broadcasts).
__device__ inline float wave_sum63(float x) {
  x = dpp_add<0x111, 0xF>(x);   // row_shr:1
  x = dpp_add<0x112, 0xF>(x);   // row_shr:2
  x = dpp_add<0x114, 0xF>(x);   // row_shr:4
  x = dpp_add<0x118, 0xF>(x);   // row_shr:8
  x = dpp_add<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
  return x;
}

// The lane's window cells: cell c = lane + 64 r, at (c % W, c / W).
struct Cells {
  int wx[kCells], wy[kCells];
  bool ok[kCells];
  __device__ void init(int lane, int W) {
#pragma unroll
    for (int r = 0; r < kCells; ++r) {
      const int c = lane + 64 * r;
      ok[r] = c < W * W;
      wy[r] = c / W;
      wx[r] = c - wy[r] * W;
    }
  }
};

// Per-visibility data of a batch, one visibility per lane: footprint origin in
// window coordinates (column | row << 8), table block, and W V or result slot.
struct VisData {
  int pc, tb, a, b;
};

template <int S>
__device__ inline VisData load_vis(const CorrArgs& args, int slot, bool with_y) {
  const SlotRec r = args.krec[slot];
  const TapPos t = decode<S>(r, args.g);
  constexpr int H = S / 2;
  const int wo = H - args.g.hc;   // window origin in region coordinates
  VisData d;
  d.pc = (t.col - wo) | ((t.row - wo) << 8);
  d.tb = t.tb;
  if (with_y) {
    const float2 y = args.yrow[rec_pos(r)];
    d.a = __float_as_int(y.x);
    d.b = __float_as_int(y.y);
  } else {
    d.a = rec_pos(r);
    d.b = 0;
  }
  return d;
}

__device__ inline int rl(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Table taps of the group of kUnroll visibilities starting at v0 that fall on
// the lane's window cells (cells r < R only; R is uniform).
struct Group {
  float2 cv[kUnroll][kCells];
  bool in[kUnroll][kCells];
};

__device__ inline void fetch_group(const CorrArgs& a, const Cells& cl, int R, const VisData& mine,
                                   int v0, int nb, Group& gr) {
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int v = min(v0 + u, nb - 1);
    const int pc = rl(mine.pc, v), tb = rl(mine.tb, v);
#pragma unroll
    for (int r = 0; r < kCells; ++r) {
      gr.in[u][r] = false;
      if (r < R) {
        const int su = cl.wx[r] - (pc & 0xFF), sv = cl.wy[r] - (pc >> 8);
        gr.in[u][r] = cl.ok[r] && (unsigned)su < (unsigned)a.g.Sc && (unsigned)sv < (unsigned)a.g.Sc;
        if (gr.in[u][r]) gr.cv[u][r] = a.tab[tb + sv * a.g.Sc + su];
      }
    }
  }
}

// acc += y_v C over the group's taps on the lane's cells
__device__ inline void accumulate(const Group& gr, const VisData& mine, int v0, int nb, int R,
                                  float* acc_re, float* acc_im) {
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const int v = min(v0 + u, nb - 1);
    const float yr = v0 + u < nb ? __int_as_float(rl(mine.a, v)) : 0.f;
    const float yi = v0 + u < nb ? __int_as_float(rl(mine.b, v)) : 0.f;
#pragma unroll
    for (int r = 0; r < kCells; ++r)
      if (r < R && gr.in[u][r]) {
        acc_re[r] += yr * gr.cv[u][r].x - yi * gr.cv[u][r].y;
        acc_im[r] += yr * gr.cv[u][r].y + yi * gr.cv[u][r].x;
      }
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
  const int wo = H - g.hc;
  Cells cl;
  cl.init(lane, g.win);
  const int R = (g.win * g.win + 63) >> 6;   // window cells per lane in use
  const int n_items = (int)*a.nitems;
  int stride;
  for (int it = uniform(wave_items(kCorrWaves, &stride)); it < n_items; it += stride) {
    const int4 item = a.items[it];
    const int ty = uniform(item.x), s_end = uniform(item.z);
    const int by = ty * C - H;
    TileWalk tw;
    tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), lane);
    int fx = tw.tx * C - H;
    int c0 = uniform(item.y);
    float acc_re[kCells], acc_im[kCells];
    while (true) {
      const int x0 = tw.tx * C - H;
      const int re = min(tw.real_end(), s_end), pe = min(tw.padded_end(), s_end);
#pragma unroll
      for (int r = 0; r < kCells; ++r) acc_re[r] = acc_im[r] = 0.f;
      for (int b0 = c0; b0 < re; b0 += 64) {
        const int nb = min(64, re - b0);
        VisData mine{0, 0, 0, 0};
        if (lane < nb) mine = load_vis<S>(a, b0 + lane, true);
        for (int v0 = 0; v0 < nb; v0 += kUnroll) {
          Group gr;
          fetch_group(a, cl, R, mine, v0, nb, gr);
          accumulate(gr, mine, v0, nb, R, acc_re, acc_im);
        }
      }
      // bank the tile's window in the ring (each lane its own cells)
#pragma unroll
      for (int r = 0; r < kCells; ++r) {
        if (r >= R || !cl.ok[r]) continue;
        float2* p = reinterpret_cast<float2*>(ring) + (wo + cl.wy[r]) * kRingPitch +
                    ((x0 + wo + cl.wx[r]) & (kRing - 1));
        float2 o = *p;
        o.x += acc_re[r];
        o.y += acc_im[r];
        *p = o;
      }
      if (pe >= s_end || !tw.next(lane)) break;
      // ring columns [fx, fx + kRing) hold the band; make room for the next region
      const int nx0 = tw.tx * C - H;
      if (nx0 >= fx + kRing) {
        ring_flush16(ring, fx, grid, by, a.N, a.checker, lane);
        ring_flush16(ring, fx + 16, grid, by, a.N, a.checker, lane);
        fx = nx0;
      } else if (nx0 + 16 > fx + kRing) {
        ring_flush16(ring, fx, grid, by, a.N, a.checker, lane);
        fx += 16;
      }
      c0 = tw.first_slot();
    }
    ring_flush16(ring, fx, grid, by, a.N, a.checker, lane);
    ring_flush16(ring, fx + 16, grid, by, a.N, a.checker, lane);
  }
}

// Lane v0 + u of the batch receives sum over the wave of G conj(C) for its
// visibility (each lane's cells of the window G).
__device__ inline void reduce_group(const Group& gr, const float2* gw, int v0, int nb, int R,
                                    int lane, float& res_re, float& res_im) {
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    if (v0 + u >= nb) break;
    float pr = 0.f, pi = 0.f;
#pragma unroll
    for (int r = 0; r < kCells; ++r)
      if (r < R && gr.in[u][r]) {
        pr += gw[r].x * gr.cv[u][r].x + gw[r].y * gr.cv[u][r].y;
        pi += gw[r].y * gr.cv[u][r].x - gw[r].x * gr.cv[u][r].y;
      }
    pr = wave_sum63(pr);
    pi = wave_sum63(pi);
    const float sr = __int_as_float(rl(__float_as_int(pr), 63));
    const float si = __int_as_float(rl(__float_as_int(pi), 63));
    if (lane == v0 + u) {
      res_re = sr;
      res_im = si;
    }
  }
}

template <int S>
__global__ __launch_bounds__(64 * kCorrWaves) void corr_degrid_kernel(CorrArgs a) {
  constexpr int C = 17 - S, H = S / 2;
  const int lane = threadIdx.x & 63;
  const CorrGeom g = a.g;
  const int wo = H - g.hc;
  Cells cl;
  cl.init(lane, g.win);
  const int R = (g.win * g.win + 63) >> 6;
  const int n_items = (int)*a.nitems;
  const float2* grid = a.grid;
  int stride;
  for (int it = uniform(wave_items(kCorrWaves, &stride)); it < n_items; it += stride) {
    const int4 item = a.items[it];
    const int ty = uniform(item.x), s_end = uniform(item.z);
    const int gy0 = ty * C - H + wo;     // grid row of window row 0
    TileWalk tw;
    tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), lane);
    int c0 = uniform(item.y);
    while (true) {
      const int gx0 = tw.tx * C - H + wo;   // grid column of window column 0
      const int re = min(tw.real_end(), s_end), pe = min(tw.padded_end(), s_end);
      // the tile's window, signed for the centred transform (cells off the grid read 0)
      float2 gw[kCells];
#pragma unroll
      for (int r = 0; r < kCells; ++r) {
        const int gx = gx0 + cl.wx[r], gy = gy0 + cl.wy[r];
        gw[r] = make_float2(0.f, 0.f);
        if (r < R && cl.ok[r] && gx >= 0 && gx < a.N && gy >= 0 && gy < a.N) {
          gw[r] = grid[(int64_t)gy * a.N + gx];
          if (a.checker && ((gx + gy) & 1)) gw[r] = make_float2(-gw[r].x, -gw[r].y);
        }
      }
      for (int b0 = c0; b0 < re; b0 += 64) {
        const int nb = min(64, re - b0);
        VisData mine{0, 0, 0, 0};
        if (lane < nb) mine = load_vis<S>(a, b0 + lane, false);
        float res_re = 0.f, res_im = 0.f;   // lane v: result of visibility v of the batch
        for (int v0 = 0; v0 < nb; v0 += kUnroll) {
          Group gr;
          fetch_group(a, cl, R, mine, v0, nb, gr);
          reduce_group(gr, gw, v0, nb, R, lane, res_re, res_im);
        }
        if (lane < nb) {
          float2* o = a.yrow + mine.a;
          const float2 old = *o;
          *o = make_float2(old.x + res_re, old.y + res_im);
        }
      }
      if (pe >= s_end || !tw.next(lane)) break;
      c0 = tw.first_slot();
    }
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
