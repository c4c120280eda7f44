// Gridding on the matrix cores (FP32 MFMA).
//
// Section 5: with the separable GCF the update of cell (x, y) by visibility i
// is y_i Tu_i[x] Tv_i[y] (y_i = W_i V_i), and the partial product y_i Tu_i is
// formed once and reused for every row.  Over the visibilities binned into one
// c x c tile this is a complex rank-K update of the tile's 16 x 16 region,
//     R += A_v^T diag(y) A_u,   A_u[i][x] = Tu_i[x - ox_i],  A_v[i][y] = Tv_i[y - oy_i],
// an MFMA product with K = visibilities: the B operand carries the row product
// y_i Tu_i (the paper's reuse), the A operand the v-row Tv_i.  c = 17 - S makes
// the region exactly 16 cells (c = 2 at S = 15: 225 of 256 MACs useful).
// The complex product takes three real v_mfma_f32_16x16x4f32 per 4
// visibilities (Gauss's three-multiplication form):
//     P1 += Re A Re B,  P2 += Im A Im B,  P3 += (Re A + Im A)(Re B + Im B),
//     Re R = P1 - P2,   Im R = P3 - P1 - P2.
//
// Work item: a range of tile slots of one row of tiles, walked left to right.
// Tiles are padded to multiples of 4 slots (padding carries W V = 0), so each
// MFMA group of 4 slots belongs to one tile and needs no per-visibility test.
// Operand traffic is shaped for the memory pipeline: a slot record (table
// bases and the row-bin position of its W V) and its W V are loaded once, one
// slot per lane, 64 slots at a time and two batches ahead; ds_bpermute then
// hands each MFMA lane the record of its group's visibility, and the table
// taps come through the caches as buffer loads with 32-bit offsets.  Each
// step multiplies group g and then fetches group g + 2 into the registers it
// just consumed, so taps have two groups' time to arrive.
// Region accumulation: when the walk moves to another tile, the 16 x 16
// region sums are added (plain read-modify-write) into a per-wave ring of 32
// grid columns x 16 rows in LDS at their absolute columns, and the sums
// restart from zero.  Ring columns that no later tile of the item can touch
// are flushed to the grid 16 at a time with hardware FP32 atomics (regions of
// neighbouring tiles and rows overlap, so other waves add to the same cells),
// all 64 lanes active and each row segment contiguous.
// Lane layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 (l / 16) + r][l % 16],
// so region column x = l % 16 and region row y = 4 (l / 16) + r.
#include "ring.h"
#include "walk.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;   // waves per workgroup of the cache-table and batched launches

// Add the region sums (column x0 + col, rows 4 grp + r) into the ring.
__device__ inline void ring_add(float* ring, const f32x4& re, const f32x4& im, int x0, int col,
                                int grp) {
  const int slot = (x0 + col) & (kRing - 1);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float2* p = reinterpret_cast<float2*>(ring) + (4 * grp + r) * kRingPitch + slot;
    float2 v = *p;
    v.x += re[r];
    v.y += im[r];
    *p = v;
  }
}

// Operands of one MFMA group (4 slots) as one lane sees them.
struct GroupOps {
  float2 y;     // W V of the lane's slot
  float2 tu;    // u-table tap of the lane's column
  float2 tv;    // v-table tap of the lane's row
};

struct GridState {
  f32x4 p1, p2, p3;   // the three real sums of the region accumulator
  int tx;             // tile column of the region
  int pe;             // end of the current tile's slots
  int fx;             // first grid column not yet flushed from the ring
};

struct GridCtx {
  const SlotRec* krec;
  const float2* yrow;
  float* grid;
  float* ring;                  // this wave's LDS ring
  __amdgpu_buffer_rsrc_t tu;    // padded tables as buffer resources
  __amdgpu_buffer_rsrc_t tv;
  int N, checker;
  int s0, last, ng, by, lane, col, grp;
  int col8, grp4;               // col * 8 (tap byte offset), grp * 4 (bpermute lane offset)
};

// Buffer resource over n bytes at p (raw 32-bit dword loads; reads past n return 0).
__device__ inline __amdgpu_buffer_rsrc_t table_rsrc(const float2* p, int64_t n_entries) {
  const int64_t bytes = n_entries * (int64_t)sizeof(float2);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(p), (short)0,
                                           (int)(bytes < 0x7FFFFFFF ? bytes : 0x7FFFFFFF),
                                           0x00020000);
}

__device__ inline float2 tap(__amdgpu_buffer_rsrc_t r, int byte_off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
  return make_float2(__int_as_float(v[0]), __int_as_float(v[1]));
}

__device__ inline void region_parts(const GridState& st, f32x4& re, f32x4& im) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    re[r] = st.p1[r] - st.p2[r];
    im[r] = st.p3[r] - st.p1[r] - st.p2[r];
  }
}

__device__ inline float bperm(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// Operands of group j (slots s0 + 4 j ..): the record of slot 4 (j % 16) + grp
// of the batch (R, Y), moved to this lane, then its table taps.
__device__ __forceinline__ void fetch_group(const GridCtx& c, const SlotRec& R, const float2& Y,
                                            int j, GroupOps& o) {
  const int src = c.grp4 + ((j & 15) << 4);
  const int kx = __builtin_amdgcn_ds_bpermute(src, R.x);
  const int ky = __builtin_amdgcn_ds_bpermute(src, R.y);
  o.y = make_float2(bperm(src, Y.x), bperm(src, Y.y));
  o.tu = tap(c.tu, (kx << 3) + c.col8);
  o.tv = tap(c.tv, (ky << 3) + c.col8);
}

// One pipeline step: multiply group g from buf (fetched two steps earlier),
// then fetch group g + 2 (from batch registers R, Y) into the same registers.
// The fetch is unconditional (past the item's end it reads harmless repeats of
// valid records), so that every path leaves the same loads in flight.
template <int S>
__device__ __forceinline__ void grid_step(const GridCtx& c, int g, const SlotRec& R, const float2& Y,
                                          TileWalk& tw, GridState& st, GroupOps& buf) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  if (c.s0 + 4 * g >= st.pe) {
    // next non-empty tile of the row: bank the region sums in the ring,
    // flush ring columns the new region cannot reach, restart the sums
    if (tw.next(c.lane)) {
      f32x4 re, im;
      region_parts(st, re, im);
      ring_add(c.ring, re, im, st.tx * C - H, c.col, c.grp);
      const int x0 = tw.tx * C - H;
      if (x0 >= st.fx + kRing) {
        ring_flush16(c.ring, st.fx, c.grid, c.by - H, c.N, c.checker, c.lane);
        ring_flush16(c.ring, st.fx + 16, c.grid, c.by - H, c.N, c.checker, c.lane);
        st.fx = x0;
      } else if (x0 + 16 > st.fx + kRing) {
        ring_flush16(c.ring, st.fx, c.grid, c.by - H, c.N, c.checker, c.lane);
        st.fx += 16;
      }
      st.p1 = f32x4{0.f, 0.f, 0.f, 0.f};
      st.p2 = st.p1;
      st.p3 = st.p1;
      st.tx = tw.tx;
      st.pe = tw.padded_end();
    }
  }
  const float b_re = buf.y.x * buf.tu.x - buf.y.y * buf.tu.y;   // row product W V Tu
  const float b_im = buf.y.x * buf.tu.y + buf.y.y * buf.tu.x;
  st.p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(buf.tv.x, b_re, st.p1, 0, 0, 0);
  st.p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(buf.tv.y, b_im, st.p2, 0, 0, 0);
  st.p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(buf.tv.x + buf.tv.y, b_re + b_im, st.p3, 0, 0, 0);
  fetch_group(c, R, Y, g + 2, buf);
}

// One work item of one gridding job; tu_tab / tv_tab are the padded tables
// (in LDS or global memory).
template <int S>
__device__ __forceinline__ void grid_item(const GridArgs& a, float* ring, int it, int lane,
                                          int col, int grp) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  GridCtx c;
  c.krec = a.krec;
  c.yrow = a.yrow;
  c.grid = reinterpret_cast<float*>(a.grid);
  c.ring = ring;
  c.tu = table_rsrc(a.tab_u, a.tab_len);
  c.tv = table_rsrc(a.tab_v, a.tab_len);
  c.N = a.N;
  c.checker = a.checker;
  c.s0 = uniform(item.y);
  c.last = s_end - 1;
  c.ng = (s_end - c.s0) >> 2;
  c.by = ty * C;
  c.lane = lane;
  c.col = col;
  c.grp = grp;
  c.col8 = col << 3;
  c.grp4 = grp << 2;
  TileWalk tw;
  tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), lane);
  GridState st;
  st.tx = tw.tx;
  st.pe = tw.padded_end();
  st.fx = st.tx * C - H;
  st.p1 = f32x4{0.f, 0.f, 0.f, 0.f};
  st.p2 = st.p1;
  st.p3 = st.p1;

  // records of batches 0..2 and W V of batches 0 and 1, one slot per lane
  SlotRec r0 = load_rec(c.krec + min(c.s0 + lane, c.last));
  SlotRec r1 = load_rec(c.krec + min(c.s0 + 64 + lane, c.last));
  SlotRec r2 = load_rec(c.krec + min(c.s0 + 128 + lane, c.last));
  float2 y0 = c.yrow[rec_pos(r0)];
  float2 y1 = c.yrow[rec_pos(r1)];
  GroupOps A, B;   // groups of even / odd index
  fetch_group(c, r0, y0, 0, A);
  fetch_group(c, r0, y0, 1, B);
  int g = 0;
  while (true) {
    // the 16 groups of one batch; the last two fetch from the next batch
    for (int p = 0; p < 7; ++p) {
      grid_step<S>(c, g, r0, y0, tw, st, A);
      if (++g >= c.ng) goto done;
      grid_step<S>(c, g, r0, y0, tw, st, B);
      if (++g >= c.ng) goto done;
    }
    grid_step<S>(c, g, r1, y1, tw, st, A);
    if (++g >= c.ng) goto done;
    grid_step<S>(c, g, r1, y1, tw, st, B);
    if (++g >= c.ng) goto done;
    // next batch: W V one batch ahead (its records arrived a batch ago),
    // records two batches ahead
    r0 = r1;
    y0 = y1;
    r1 = r2;
    y1 = c.yrow[rec_pos(r1)];
    r2 = load_rec(c.krec + min(c.s0 + 4 * g + 128 + lane, c.last));
  }
done:
  f32x4 re, im;
  region_parts(st, re, im);
  ring_add(c.ring, re, im, st.tx * C - H, col, grp);
  ring_flush16(c.ring, st.fx, c.grid, c.by - H, c.N, c.checker, lane);
  ring_flush16(c.ring, st.fx + 16, c.grid, c.by - H, c.N, c.checker, lane);
}

template <int S>
__global__ __launch_bounds__(64 * kWaves) void grid_fp32_kernel(GridArgs a) {
  __shared__ float rings[kWaves * kRingFloats];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* ring = rings + wave * kRingFloats;
  for (int i = lane; i < kRingFloats; i += 64) ring[i] = 0.f;
  // plain grid-stride order (the per-XCD lists were measured slower for gridding)
  int stride;
  const int n_items = (int)*a.nitems;
  for (int it = uniform(wave_items(kWaves, &stride)); it < n_items; it += stride)
    grid_item<S>(a, ring, it, lane, lane & 15, lane >> 4);
}

// Persistent launch over the work items of many jobs (facets, snapshots):
// waves take (job, item) pairs from the concatenated item lists (jobs ordered
// by decreasing size on the host) through eight block counters, so uneven
// jobs share the GPU without a launch per job.
template <int S>
__global__ __launch_bounds__(64 * kWaves) void grid_fp32_batched_kernel(
    const GridArgs* __restrict__ jobs, const uint32_t* __restrict__ first, int njobs,
    uint32_t* __restrict__ counter) {
  __shared__ float rings[kWaves * kRingFloats];
  const int lane = threadIdx.x & 63;
  float* ring = rings + (threadIdx.x >> 6) * kRingFloats;
  for (int i = lane; i < kRingFloats; i += 64) ring[i] = 0.f;
  for_blocks8(counter, first[njobs], lane, [&](uint32_t gi) {
    int lo = 0, hi = njobs - 1;   // last job with first[job] <= gi
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const int job = uniform(lo);
    grid_item<S>(jobs[job], ring, (int)(gi - first[job]), lane, lane & 15, lane >> 4);
  });
}

// ------------------------------------------------ tables in LDS, ring in registers
//
// When the padded tables fit in LDS, one workgroup of 16 waves per CU stages
// them there and the table taps become LDS reads instead of buffer loads
// (whose per-lane address processing bounds the cache-table kernel above).
// The LDS then has no room for the accumulation rings, so each wave keeps its
// ring in registers.  That works because the accumulator's columns are tied
// to absolute grid columns modulo 16: lane column c holds the region column
// whose grid column x satisfies x = c (mod 16), i.e. region column
// rc = (c - x0) mod 16 for a region whose first column is x0.  A lane's sums
// therefore always belong to the same two ring columns (x mod 32 is c or
// c + 16), and banking a tile's sums is an add into one of two register
// halves, with no data exchanged between lanes.  The ring holds two aligned
// blocks of 16 grid columns (block b in half b & 1); when the walk reaches a
// region that starts in a later block, the blocks it has left are added to
// the grid with FP32 atomics.  The B operand of lane c for a group of tile T
// is y Tu at region column rc_T, so the operand fetch, two groups ahead of
// the arithmetic, walks the tiles as well (a second TileWalk) to know each
// group's x0; the tap address is then one add.

constexpr int kLdsWaves = 16;

struct LdsState {
  f32x4 p1, p2, p3;   // region sums of the current tile (three real products)
  int x0;             // first grid column of the current region
  int pe;             // end of the current tile's slots
};

struct FetchPos {
  int pe;             // end of the slots of the tile the tap reads are in
  int rc8;            // byte offset of this lane's region column in that tile: ((c - x0) & 15) * 8
};

struct LdsCtx {
  const float2* yrow;
  const char* tu;     // LDS tables (byte addressing)
  const char* tv;
  float* grid;
  int N, checker;
  int s0, last, ng, y0, lane, col, grp;
  int col8, grp4;
};

__device__ inline void ring_shift(RegRing& rg, const LdsCtx& c) {
  reg_ring_shift(rg, c.grid, c.N, c.checker, c.y0, c.col, c.grp, 1.f);
}

// Bank the current tile's region sums into the ring block of this lane's column.
__device__ inline void ring_bank(RegRing& rg, const LdsState& st, int col) {
  f32x4 re, im;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    re[r] = st.p1[r] - st.p2[r];
    im[r] = st.p3[r] - st.p1[r] - st.p2[r];
  }
  reg_ring_add(rg, re, im, st.x0, col);
}

// Record of group j (table bases and W V of slot 4 (j % 16) + grp of the
// batch R, Y) moved to this lane.
struct GroupKey {
  int kx, ky;
  float2 y;
};

__device__ __forceinline__ void key_group(const LdsCtx& c, const SlotRec& R, const float2& Y, int j,
                                          GroupKey& k) {
  const int src = c.grp4 + ((j & 15) << 4);
  k.kx = __builtin_amdgcn_ds_bpermute(src, R.x);
  k.ky = __builtin_amdgcn_ds_bpermute(src, R.y);
  k.y = make_float2(bperm(src, Y.x), bperm(src, Y.y));
}

// Taps of group j from the LDS tables, with its record k moved to this lane
// one step earlier.  The read position enters a new tile exactly when j
// reaches that tile's first group.
template <int S>
__device__ __forceinline__ void taps_group(const LdsCtx& c, const GroupKey& k, int j, TileWalk& fw,
                                           FetchPos& f, GroupOps& o) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  if (c.s0 + 4 * j >= f.pe && fw.next(c.lane)) {
    const int x0 = fw.tx * C - H;
    f.pe = fw.padded_end();
    f.rc8 = ((c.col - x0) & 15) << 3;
  }
  o.y = k.y;
  o.tu = *reinterpret_cast<const float2*>(c.tu + (k.kx << 3) + f.rc8);
  o.tv = *reinterpret_cast<const float2*>(c.tv + (k.ky << 3) + c.col8);
}

// Slot records and W V of the item, one slot per lane, in batches of 64:
// batch a (records ra, W V ya) holds the group whose record is moved next,
// batch a + 1 (rb, yb) follows, and the records of batch a + 2 (rc) are in
// flight.
struct Batches {
  SlotRec ra, rb, rc;
  float2 ya, yb;
  int nb;             // batch index of rc
};

// One pipeline step: multiply group g (operands in buf, read two steps
// earlier), move the record of group g + 3 to the lanes, then read the taps of
// group g + 2 (record moved one step earlier) into buf.  The record exchange
// is issued before the tap reads, so that its wait in the next step does not
// also wait for these reads (LDS operations complete in order).
template <int S>
__device__ __forceinline__ void grid_step_lds(const GridArgs& a, const LdsCtx& c, int g,
                                              Batches& bt, TileWalk& tw, TileWalk& fw,
                                              FetchPos& f, GroupKey& key, LdsState& st,
                                              RegRing& rg, GroupOps& buf) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  bool first = false;
  if (c.s0 + 4 * g >= st.pe && tw.next(c.lane)) {
    // next non-empty tile of the row: bank the sums, flush the ring blocks
    // the new region has left behind, restart the sums
    ring_bank(rg, st, c.col);
    const int x0 = tw.tx * C - H;
    reg_ring_advance(rg, x0, c.grid, c.N, c.checker, c.y0, c.col, c.grp, 1.f);
    st.x0 = x0;
    st.pe = tw.padded_end();
    first = true;
  }
  const float b_re = buf.y.x * buf.tu.x - buf.y.y * buf.tu.y;   // row product W V Tu
  const float b_im = buf.y.x * buf.tu.y + buf.y.y * buf.tu.x;
  const float a_s = buf.tv.x + buf.tv.y, b_s = b_re + b_im;
  if (first) {
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    st.p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(buf.tv.x, b_re, z, 0, 0, 0);
    st.p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(buf.tv.y, b_im, z, 0, 0, 0);
    st.p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a_s, b_s, z, 0, 0, 0);
  } else {
    st.p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(buf.tv.x, b_re, st.p1, 0, 0, 0);
    st.p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(buf.tv.y, b_im, st.p2, 0, 0, 0);
    st.p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a_s, b_s, st.p3, 0, 0, 0);
  }
  if (((g + 3) & 15) == 0) {
    // group g + 3 opens the next batch: W V one batch ahead (its records
    // arrived a batch ago), records two batches ahead
    bt.ra = bt.rb;
    bt.ya = bt.yb;
    bt.rb = bt.rc;
    bt.yb = c.yrow[rec_pos(bt.rb)];
    bt.nb += 1;
    bt.rc = load_rec(a.krec + min(c.s0 + 64 * bt.nb + c.lane, c.last));
  }
  GroupKey next;
  key_group(c, bt.ra, bt.ya, g + 3, next);
  taps_group<S>(c, key, g + 2, fw, f, buf);
  key = next;
}

template <int S>
__device__ __forceinline__ void grid_item_lds(const GridArgs& a, const char* tu, const char* tv,
                                              int it, int lane) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  LdsCtx c;
  c.yrow = a.yrow;
  c.tu = tu;
  c.tv = tv;
  c.grid = reinterpret_cast<float*>(a.grid);
  c.N = a.N;
  c.checker = a.checker;
  c.s0 = uniform(item.y);
  c.last = s_end - 1;
  c.ng = (s_end - c.s0) >> 2;
  c.y0 = ty * C - H;
  c.lane = lane;
  c.col = lane & 15;
  c.grp = lane >> 4;
  c.col8 = c.col << 3;
  c.grp4 = c.grp << 2;
  const int last = c.last;
  TileWalk tw;
  tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), lane);
  TileWalk fw = tw;
  LdsState st;
  st.x0 = tw.tx * C - H;
  st.pe = tw.padded_end();
  st.p1 = f32x4{0.f, 0.f, 0.f, 0.f};
  st.p2 = st.p1;
  st.p3 = st.p1;
  FetchPos f;
  f.pe = st.pe;
  f.rc8 = ((c.col - st.x0) & 15) << 3;
  RegRing rg;
  rg.lo_re = st.p1;
  rg.lo_im = st.p1;
  rg.hi_re = st.p1;
  rg.hi_im = st.p1;
  rg.blk = st.x0 >> 4;

  Batches bt;
  bt.ra = load_rec(a.krec + min(c.s0 + lane, last));
  bt.rb = load_rec(a.krec + min(c.s0 + 64 + lane, last));
  bt.rc = load_rec(a.krec + min(c.s0 + 128 + lane, last));
  bt.nb = 2;
  bt.ya = c.yrow[rec_pos(bt.ra)];
  bt.yb = c.yrow[rec_pos(bt.rb)];
  GroupOps A, B;   // groups of even / odd index
  GroupKey key;
  key_group(c, bt.ra, bt.ya, 0, key);
  taps_group<S>(c, key, 0, fw, f, A);
  key_group(c, bt.ra, bt.ya, 1, key);
  taps_group<S>(c, key, 1, fw, f, B);
  key_group(c, bt.ra, bt.ya, 2, key);
  for (int g = 0;;) {
    grid_step_lds<S>(a, c, g, bt, tw, fw, f, key, st, rg, A);
    if (++g >= c.ng) break;
    grid_step_lds<S>(a, c, g, bt, tw, fw, f, key, st, rg, B);
    if (++g >= c.ng) break;
  }
  ring_bank(rg, st, c.col);
  ring_shift(rg, c);
  ring_shift(rg, c);
}

// One workgroup of 16 waves per CU with the tables in LDS; waves take work
// items through the eight block counters (measured at array scale: 2.43 ms;
// one counter over all items 2.49 ms, the per-XCD lists 2.83 ms).
template <int S>
__global__ __launch_bounds__(64 * kLdsWaves) void grid_fp32_lds_kernel(GridArgs a) {
  extern __shared__ float2 smem[];
  const int n = a.tab_len;
  const bool two = a.tab_v != a.tab_u;
  for (int i = threadIdx.x; i < n; i += blockDim.x) smem[i] = a.tab_u[i];
  if (two)
    for (int i = threadIdx.x; i < n; i += blockDim.x) smem[n + i] = a.tab_v[i];
  __syncthreads();
  const char* tu = reinterpret_cast<const char*>(smem);
  const char* tv = reinterpret_cast<const char*>(two ? smem + n : smem);
  const int lane = threadIdx.x & 63;
  for_blocks8(a.qctr, (uint32_t)uniform((int)*a.nitems), lane,
              [&](uint32_t it) { grid_item_lds<S>(a, tu, tv, (int)it, lane); });
}

template <int S>
hipError_t launch_lds_s(const GridArgs& a, int lds_bytes, int n_cu, hipStream_t s) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&grid_fp32_lds_kernel<S>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  hipLaunchKernelGGL(grid_fp32_lds_kernel<S>, dim3((unsigned)n_cu), dim3(64 * kLdsWaves),
                     lds_bytes, s, a);
  return hipGetLastError();
}

template <int S>
hipError_t launch_s(const GridArgs& a, int64_t max_items, hipStream_t s) {
  int64_t b = (max_items + kWaves - 1) / kWaves;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(grid_fp32_kernel<S>, dim3((unsigned)b), dim3(64 * kWaves), 0, s, a);
  return hipGetLastError();
}

template <int S>
hipError_t launch_batched_s(const GridArgs* jobs, const uint32_t* first, int njobs,
                            uint32_t* counter, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(grid_fp32_batched_kernel<S>, dim3(blocks), dim3(64 * kWaves), 0, s, jobs,
                     first, njobs, counter);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_fp32_batched(int S, const GridArgs* jobs, const uint32_t* first, int njobs,
                                    uint32_t* counter, int blocks, hipStream_t s) {
  switch (S) {
    case 1: return launch_batched_s<1>(jobs, first, njobs, counter, blocks, s);
    case 3: return launch_batched_s<3>(jobs, first, njobs, counter, blocks, s);
    case 5: return launch_batched_s<5>(jobs, first, njobs, counter, blocks, s);
    case 7: return launch_batched_s<7>(jobs, first, njobs, counter, blocks, s);
    case 9: return launch_batched_s<9>(jobs, first, njobs, counter, blocks, s);
    case 11: return launch_batched_s<11>(jobs, first, njobs, counter, blocks, s);
    case 13: return launch_batched_s<13>(jobs, first, njobs, counter, blocks, s);
    case 15: return launch_batched_s<15>(jobs, first, njobs, counter, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grid_fp32_lds(int S, const GridArgs& a, int lds_bytes, int n_cu,
                                hipStream_t s) {
  switch (S) {
    case 1: return launch_lds_s<1>(a, lds_bytes, n_cu, s);
    case 3: return launch_lds_s<3>(a, lds_bytes, n_cu, s);
    case 5: return launch_lds_s<5>(a, lds_bytes, n_cu, s);
    case 7: return launch_lds_s<7>(a, lds_bytes, n_cu, s);
    case 9: return launch_lds_s<9>(a, lds_bytes, n_cu, s);
    case 11: return launch_lds_s<11>(a, lds_bytes, n_cu, s);
    case 13: return launch_lds_s<13>(a, lds_bytes, n_cu, s);
    case 15: return launch_lds_s<15>(a, lds_bytes, n_cu, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grid_fp32(int S, const GridArgs& a, int64_t max_items, hipStream_t s) {
  switch (S) {
    case 1: return launch_s<1>(a, max_items, s);
    case 3: return launch_s<3>(a, max_items, s);
    case 5: return launch_s<5>(a, max_items, s);
    case 7: return launch_s<7>(a, max_items, s);
    case 9: return launch_s<9>(a, max_items, s);
    case 11: return launch_s<11>(a, max_items, s);
    case 13: return launch_s<13>(a, max_items, s);
    case 15: return launch_s<15>(a, max_items, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sepw
