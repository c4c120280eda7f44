// Degridding on the matrix cores (FP32 MFMA).
//
// Degridding is the adjoint of gridding (Section 2, prediction equation;
// Section 6, prediction for major cycles):
//     V_i = sum_y conj(Tv_i[y - oy_i]) sum_x conj(Tu_i[x - ox_i]) R[y][x]
// over the 16 x 16 grid region R of the visibility's tile.  The inner sums for
// a chunk of 16 visibilities of one tile are the dense product Z = R conj(A_u)^T
// (M = 16 rows, N = 16 visibilities, K = 16 columns): four K-steps of
// v_mfma_f32_16x16x4f32, each complex product in Gauss's three-multiplication
// form (with B = conj(Tu)):
//     P1 += Re R Re Tu,  P2 += Im R Im Tu,  P3 += (Re R + Im R)(Re Tu - Im Tu),
//     Re Z = P1 + P2,    Im Z = P3 - P1 + P2.
// The outer sum is an S-term dot product per visibility on the vector unit
// from the accumulator layout, reduced across the four 16-lane groups.
//
// Work item: a range of tile slots of one row of tiles, processed in chunks of
// at most 16 slots that never cross a tile.  K-step q of the product takes
// region columns x = 4 k + q (k = lane group), so each lane reads four
// consecutive taps of a table row.  Table taps come from LDS when the tables
// fit there (staged once per workgroup) or from the caches otherwise.  Loads
// run ahead of the arithmetic: the slot records of chunk n + 2 and the taps
// and (on a tile change) the grid region of chunk n + 1 are in flight while
// chunk n is multiplied.  If the grid came from the FFT, the checkerboard
// (-1)^(x+y) of the centred transform is applied to the region.  Results of
// real visibilities go straight to their row-bin positions (held in the slot
// records); the placement map moves them to the caller's order and undoes the
// facet rotation afterwards.
// Lane layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 (l / 16) + r][l % 16].
#include "walk.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));


// Region operand for the tile at column tx: lane (col, grp) holds
// R[y = col][x = 4 grp + q], four consecutive cells of the lane's grid row.
// A region inside the grid is read as two 16-byte loads (8-byte aligned).  A
// region that reaches past a grid edge is read at clamped (always valid)
// addresses, and region_zero() sets its cells outside the grid to 0 once the
// data is needed (the taps there are 0, but a non-finite edge cell times 0
// would not be).  The checkerboard of the centred FFT is not applied here: the
// tables carry (-1)^s per tap and the result (-1)^(cu+cv) per visibility.
typedef float f4u __attribute__((ext_vector_type(4), aligned(8)));

template <int S>
__device__ inline bool edge_region(int tx, int y0, int N) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int x0 = tx * C - H;
  return x0 < 0 || x0 + kRegion > N || y0 < 0 || y0 + kRegion > N;
}

template <int S>
__device__ inline void load_region(const float2* __restrict__ grid, int N, int tx, int gy, int grp,
                                   bool edge, float2 (&r)[4]) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int x0 = tx * C - H + 4 * grp;
  if (!edge) {
    const f4u* p = reinterpret_cast<const f4u*>(grid + (int64_t)gy * N + x0);
    const f4u a = p[0], b = p[1];
    r[0] = make_float2(a[0], a[1]);
    r[1] = make_float2(a[2], a[3]);
    r[2] = make_float2(b[0], b[1]);
    r[3] = make_float2(b[2], b[3]);
  } else {
    const int64_t row = (int64_t)min(max(gy, 0), N - 1) * N;
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = grid[row + min(max(x0 + q, 0), N - 1)];
  }
}

template <int S>
__device__ inline void region_zero(int tx, int gy, int grp, int N, float2 (&r)[4]) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const bool row_ok = gy >= 0 && gy < N;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gx = tx * C - H + 4 * grp + q;
    if (!row_ok || gx < 0 || gx >= N) r[q] = make_float2(0.f, 0.f);
  }
}

// Operands of one chunk of 16 slots as one lane sees them.
struct ChunkBuf {
  SlotRec k;       // record of the lane's slot (column of Z), two chunks ahead
  float2 tu[4];    // u-table taps x = 4 grp + q of the lane's visibility
  float2 tv[4];    // v-table taps y = 4 grp + rr
  float2 reg[4];   // grid region R[y = col][x = 4 grp + q] of the chunk's tile
  bool fresh;      // region loaded for this chunk (edge regions: cells off the grid not yet zeroed)
  bool edge;       // the region reaches past a grid edge
};

struct DegridCtx {
  const DegridArgs* a;
  const float2* tu_tab;
  const float2* tv_tab;
  int s_end, s0, last, y0, gy, col, grp, lane;
  uint32_t smask;   // kRecSign when the result takes the record's sign (-1)^(cu+cv)
};

// Results of up to four chunks: lane (col, grp) holds V[col] of chunk grp of
// the group (every lane of a column has it after the cross-group sum), so the
// group goes out with one store instruction.
struct ResGroup {
  float2 v;
  int pos;    // row-bin position, -1: nothing to store
  int j;      // chunks in the group
};

__device__ __forceinline__ void res_flush(const DegridArgs& a, ResGroup& g) {
  if (g.pos >= 0) {
    float2 v = g.v;
    if (a.accum) {
      const float2 o = a.yrow[g.pos];
      v.x += o.x;
      v.y += o.y;
    }
    a.yrow[g.pos] = v;
  }
  g.pos = -1;
  g.j = 0;
}

__device__ __forceinline__ void fetch_taps(const DegridCtx& c, ChunkBuf& B) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    B.tu[q] = c.tu_tab[B.k.x + 4 * c.grp + q];
    B.tv[q] = c.tv_tab[B.k.y + 4 * c.grp + q];
  }
}

// One pipeline step: chunk cur from buffer X (taps and region in flight or
// ready; a region loaded for this chunk gets its sign / bounds factor here), while
// the record of chunk n2 goes into X.k and the taps (and, on a tile change, the
// region) of chunk n1 (record Y.k, loaded one step earlier) into Y.  Buffers
// alternate between steps.  Returns false after the item's last chunk.
template <int S>
__device__ __forceinline__ bool degrid_step(const DegridCtx& c, TileWalk& tw, RecBatch& bt,
                                            ResGroup& rg, ChunkPos& cur, ChunkPos& n1,
                                            ChunkPos& n2, ChunkBuf& X, ChunkBuf& Y) {
  const DegridArgs& a = *c.a;
  const SlotRec kx = X.k;   // this chunk's record (row-bin position of the result)
  X.k = rec_key(bt, a.krec, c.s0, c.last, n2.c0, c.col, c.lane);
  fetch_taps(c, Y);
  if (X.fresh && X.edge) region_zero<S>(cur.tx, c.gy, c.grp, a.N, X.reg);
  Y.fresh = n1.ok && n1.tx != cur.tx;
  if (Y.fresh) {
    Y.edge = edge_region<S>(n1.tx, c.y0, a.N);
    load_region<S>(a.grid, a.N, n1.tx, c.gy, c.grp, Y.edge, Y.reg);
  } else {
    Y.edge = X.edge;
#pragma unroll
    for (int q = 0; q < 4; ++q) Y.reg[q] = X.reg[q];
  }

  // chunk cur: Z = R conj(Tu)^T on the matrix cores
  f32x4 p1 = {0.f, 0.f, 0.f, 0.f}, p2 = p1, p3 = p1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(X.reg[q].x, X.tu[q].x, p1, 0, 0, 0);
    p2 = __builtin_amdgcn_mfma_f32_16x16x4f32(X.reg[q].y, X.tu[q].y, p2, 0, 0, 0);
    p3 = __builtin_amdgcn_mfma_f32_16x16x4f32(X.reg[q].x + X.reg[q].y, X.tu[q].x - X.tu[q].y, p3,
                                              0, 0, 0);
  }
  // V = sum_y conj(Tv[y]) Z[y] over this lane's rows y = 4 grp + rr
  float v_re = 0.f, v_im = 0.f;
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const float z_re = p1[rr] + p2[rr];
    const float z_im = p3[rr] - p1[rr] + p2[rr];
    v_re += X.tv[rr].x * z_re + X.tv[rr].y * z_im;
    v_im += X.tv[rr].x * z_im - X.tv[rr].y * z_re;
  }
  v_re += __shfl_xor(v_re, 16, 64);
  v_im += __shfl_xor(v_im, 16, 64);
  v_re += __shfl_xor(v_re, 32, 64);
  v_im += __shfl_xor(v_im, 32, 64);
  if (c.grp == rg.j) {
    const uint32_t sg = (uint32_t)kx.z & c.smask;
    rg.v = make_float2(__uint_as_float(__float_as_uint(v_re) ^ sg),
                       __uint_as_float(__float_as_uint(v_im) ^ sg));
    rg.pos = cur.c0 + c.col < cur.re ? rec_pos(kx) : -1;
  }
  if (++rg.j == 4) res_flush(a, rg);

  if (!n1.ok) return false;
  cur = n1;
  n1 = n2;
  n2 = next_chunk(n2, tw, c.s_end, c.lane);
  return true;
}

template <int S>
__device__ __forceinline__ void degrid_item(const DegridArgs& a, const float2* tu_tab,
                                            const float2* tv_tab, int it, int lane, int col,
                                            int grp) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  DegridCtx c;
  c.a = &a;
  c.tu_tab = tu_tab;
  c.tv_tab = tv_tab;
  c.s_end = s_end;
  c.s0 = uniform(item.y);
  c.last = s_end - 1;
  c.y0 = ty * C - H;                // first grid row of the item's regions
  c.gy = c.y0 + col;                // grid row of this lane's A operand
  c.smask = a.checker ? kRecSign : 0u;
  c.col = col;
  c.grp = grp;
  c.lane = lane;
  TileWalk tw;
  tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), lane);
  ChunkPos cur;
  cur.c0 = uniform(item.y);
  cur.pe = min(tw.padded_end(), s_end);
  cur.re = min(tw.real_end(), s_end);
  cur.tx = tw.tx;
  cur.ok = true;
  ChunkPos n1 = next_chunk(cur, tw, s_end, lane);
  ChunkPos n2 = next_chunk(n1, tw, s_end, lane);

  // prologue: chunk cur complete in A, record of chunk n1 in B
  RecBatch bt;
  rec_batch_start(bt, a.krec, c.s0, c.last, lane);
  ResGroup rg;
  rg.v = make_float2(0.f, 0.f);
  rg.pos = -1;
  rg.j = 0;
  ChunkBuf A, B;
  A.edge = edge_region<S>(cur.tx, c.y0, a.N);
  load_region<S>(a.grid, a.N, cur.tx, c.gy, grp, A.edge, A.reg);
  A.k = rec_key(bt, a.krec, c.s0, c.last, cur.c0, col, lane);
  fetch_taps(c, A);
  A.fresh = true;
  B.k = rec_key(bt, a.krec, c.s0, c.last, n1.c0, col, lane);
  while (degrid_step<S>(c, tw, bt, rg, cur, n1, n2, A, B) &&
         degrid_step<S>(c, tw, bt, rg, cur, n1, n2, B, A)) {
  }
  if (rg.j > 0) res_flush(a, rg);
}

// Tables staged in LDS (LDS = true, the workgroup owns a CU with 16 waves) or
// read through the caches.
template <int S, bool LDS>
__global__ __launch_bounds__(LDS ? 1024 : 256) void degrid_fp32_kernel(DegridArgs a) {
  extern __shared__ float2 smem[];
  constexpr int kW = LDS ? 16 : 4;
  const float2* tu_tab = a.tab_u;
  const float2* tv_tab = a.tab_v;
  if constexpr (LDS) {
    const int n = a.tab_len;
    const bool two = a.tab_v != a.tab_u;
    for (int i = threadIdx.x; i < n; i += blockDim.x) smem[i] = a.tab_u[i];
    if (two)
      for (int i = threadIdx.x; i < n; i += blockDim.x) smem[n + i] = a.tab_v[i];
    __syncthreads();
    tu_tab = smem;
    tv_tab = two ? smem + n : smem;
  }
  const int lane = threadIdx.x & 63;
  // per-XCD work lists: all items of a row of tiles write that row's results
  // through one L2 (measured faster than grid-stride order for degridding)
  for_items(a.lists, a.r8, a.qctr, lane,
            [&](int it) { degrid_item<S>(a, tu_tab, tv_tab, it, lane, lane & 15, lane >> 4); });
}

// Many jobs in one launch: a wave takes global item gi, the item
// gi - first[job] of the job with first[job] <= gi < first[job + 1].  With
// LDS every job uses jobs[0]'s tables (staged once); without, each job reads
// its own.
template <int S, bool LDS>
__global__ __launch_bounds__(LDS ? 1024 : 256) void degrid_fp32_batched_kernel(
    const DegridArgs* __restrict__ jobs, const uint32_t* __restrict__ first, int njobs,
    uint32_t* __restrict__ counter) {
  extern __shared__ float2 smem[];
  const float2* tu_tab = jobs[0].tab_u;
  const float2* tv_tab = jobs[0].tab_v;
  if constexpr (LDS) {
    const int n = jobs[0].tab_len;
    const bool two = tv_tab != tu_tab;
    for (int i = threadIdx.x; i < n; i += blockDim.x) smem[i] = tu_tab[i];
    if (two)
      for (int i = threadIdx.x; i < n; i += blockDim.x) smem[n + i] = tv_tab[i];
    __syncthreads();
    tv_tab = two ? smem + n : smem;
    tu_tab = smem;
  }
  const int lane = threadIdx.x & 63;
  for_blocks8(counter, first[njobs], lane, [&](uint32_t gi) {
    int lo = 0, hi = njobs - 1;   // last job with first[job] <= gi
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const int job = uniform(lo);
    const DegridArgs& a = jobs[job];
    degrid_item<S>(a, LDS ? tu_tab : a.tab_u, LDS ? tv_tab : a.tab_v, (int)(gi - first[job]), lane,
                   lane & 15, lane >> 4);
  });
}

template <int S>
hipError_t launch_batched_s(const DegridArgs* jobs, const uint32_t* first, int njobs,
                            uint32_t* counter, int lds_bytes, int n_cu, hipStream_t s) {
  if (lds_bytes > 0) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&degrid_fp32_batched_kernel<S, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    hipLaunchKernelGGL((degrid_fp32_batched_kernel<S, true>), dim3((unsigned)n_cu), dim3(1024),
                       lds_bytes, s, jobs, first, njobs, counter);
  } else {
    hipLaunchKernelGGL((degrid_fp32_batched_kernel<S, false>), dim3((unsigned)(4 * n_cu)),
                       dim3(256), 0, s, jobs, first, njobs, counter);
  }
  return hipGetLastError();
}

template <int S>
hipError_t launch_s(const DegridArgs& a, int64_t max_items, int lds_bytes, int n_cu,
                    hipStream_t s) {
  if (lds_bytes > 0) {
    int64_t b = (max_items + 15) / 16;
    if (b > n_cu) b = n_cu;
    if (b < 1) b = 1;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&degrid_fp32_kernel<S, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    hipLaunchKernelGGL((degrid_fp32_kernel<S, true>), dim3((unsigned)b), dim3(1024), lds_bytes, s,
                       a);
  } else {
    // persistent: about as many workgroups as can be resident (waves pull items)
    int64_t b = (max_items + 3) / 4;
    if (b > 4 * (int64_t)n_cu) b = 4 * (int64_t)n_cu;
    if (b < 1) b = 1;
    hipLaunchKernelGGL((degrid_fp32_kernel<S, false>), dim3((unsigned)b), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_degrid_fp32_batched(int S, const DegridArgs* jobs, const uint32_t* first,
                                      int njobs, uint32_t* counter, int lds_bytes, int n_cu,
                                      hipStream_t s) {
  switch (S) {
    case 1: return launch_batched_s<1>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    case 3: return launch_batched_s<3>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    case 5: return launch_batched_s<5>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    case 7: return launch_batched_s<7>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    case 9: return launch_batched_s<9>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    case 11: return launch_batched_s<11>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    case 13: return launch_batched_s<13>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    case 15: return launch_batched_s<15>(jobs, first, njobs, counter, lds_bytes, n_cu, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_degrid_fp32(int S, const DegridArgs& a, int64_t max_items, int lds_bytes,
                              int n_cu, hipStream_t s) {
  switch (S) {
    case 1: return launch_s<1>(a, max_items, lds_bytes, n_cu, s);
    case 3: return launch_s<3>(a, max_items, lds_bytes, n_cu, s);
    case 5: return launch_s<5>(a, max_items, lds_bytes, n_cu, s);
    case 7: return launch_s<7>(a, max_items, lds_bytes, n_cu, s);
    case 9: return launch_s<9>(a, max_items, lds_bytes, n_cu, s);
    case 11: return launch_s<11>(a, max_items, lds_bytes, n_cu, s);
    case 13: return launch_s<13>(a, max_items, lds_bytes, n_cu, s);
    case 15: return launch_s<15>(a, max_items, lds_bytes, n_cu, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sepw
