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
  float2 y0 = c.yrow[r0.z];
  float2 y1 = c.yrow[r1.z];
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
    y1 = c.yrow[r1.z];
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
// waves take (job, item) pairs from one atomic counter over the concatenated
// item lists (jobs ordered by decreasing size on the host), so uneven jobs
// share the GPU without a launch per job.
template <int S>
__global__ __launch_bounds__(64 * kWaves) void grid_fp32_batched_kernel(
    const GridArgs* __restrict__ jobs, const uint32_t* __restrict__ first, int njobs,
    uint32_t* __restrict__ counter) {
  __shared__ float rings[kWaves * kRingFloats];
  const int lane = threadIdx.x & 63;
  float* ring = rings + (threadIdx.x >> 6) * kRingFloats;
  for (int i = lane; i < kRingFloats; i += 64) ring[i] = 0.f;
  const uint32_t total = first[njobs];
  while (true) {
    uint32_t gi = 0;
    if (lane == 0) gi = atomicAdd(counter, 1u);
    gi = (uint32_t)uniform((int)__shfl(gi, 0, 64));
    if (gi >= total) break;
    int lo = 0, hi = njobs - 1;   // last job with first[job] <= gi
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const int job = uniform(lo);
    grid_item<S>(jobs[job], ring, (int)(gi - first[job]), lane, lane & 15, lane >> 4);
  }
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
