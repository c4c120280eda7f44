// Precision form: gridding and degridding with FP16 or BF16 MFMA operands and
// FP32 accumulation.
//
// Same tile products as the FP32 path (grid.hip, degrid.hip; Section 5's
// separable update as a rank-K product over the visibilities of a tile), but
// with v_mfma_f32_16x16x16{f16,bf16}: K = 16 visibilities (gridding) or all 16
// region columns (degridding) per instruction.  Operands are scaled so that
// they use the 16-bit range well:
//   * per-plane table scale s_k = max |Re, Im| of the plane's table; the
//     16-bit tables hold T / s_k;
//   * gridding: A = Tv / s_k^v (16-bit table), B = W V (s_k^v Tu) / s formed in
//     FP32 from the u-table pre-multiplied by s_k^v, with s a power of two at
//     least max |Re, Im| (W V) times max_k s_k^u s_k^v over the visibilities
//     gridded into the tile so far (a per-tile scale: it restarts with each
//     tile); when s grows the FP32 accumulator is rescaled by the exact power
//     of two s_old / s_new, and the tile's region sums are multiplied by s
//     when they are added into the per-wave LDS ring of grid columns (ring.h),
//     which reaches the grid with atomics 16 columns at a time;
//   * degridding: A = R / s_R with s_R a power of two at least max |Re, Im|
//     over the tile's region, B = conj(Tu / s_k^u) (16-bit table); the FP32
//     epilogue uses the v-table pre-multiplied by s_k^u and multiplies by s_R.
// All tables are zero-padded so that the tap for region index x is base + x.
// Work items are walked in chunks of at most 16 slots of one tile (walk.h);
// slots past the tile's end in the last chunk carry zero weight (gridding) or
// are not written (degridding).  Slot records (table bases and row-bin
// position) run two chunks ahead of the arithmetic; W V, table rows and grid
// regions one chunk ahead, in two alternating register buffers.
// Layout of v_mfma_f32_16x16x16: lane l supplies A[l % 16][4 (l / 16) + m] and
// B[4 (l / 16) + m][l % 16] for m = 0..3; accumulator register r of lane l is
// D[4 (l / 16) + r][l % 16].
#include "ring.h"
#include "walk.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <bool BF16>
struct Lp;

template <>
struct Lp<false> {
  typedef f16x4 vec;
  __device__ static void set(vec& v, int m, float x) { v[m] = (_Float16)x; }
  __device__ static void set_bits(vec& v, int m, uint16_t b) { v[m] = __builtin_bit_cast(_Float16, b); }
  __device__ static f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Lp<true> {
  typedef i16x4 vec;
  __device__ static void set(vec& v, int m, float x) { v[m] = (short)bf16_rne(x); }
  __device__ static void set_bits(vec& v, int m, uint16_t b) { v[m] = (short)b; }
  __device__ static f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

__device__ inline float wave_max(float x) {
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

__device__ inline ChunkPos first_chunk(const TileWalk& tw, int c0, int s_end) {
  ChunkPos p;
  p.c0 = c0;
  p.pe = min(tw.padded_end(), s_end);
  p.re = min(tw.real_end(), s_end);
  p.tx = tw.tx;
  p.ok = true;
  return p;
}

// ---------------------------------------------------------------- gridding

// Operands of one chunk for lane group grp: slots c0 + 4 grp + m.
struct GridBuf {
  float2 y[4];     // W V (0 past the chunk's tile)
  uint32_t tv[4];  // 16-bit v-table taps (re | im << 16) of the lane's row
  float2 tu[4];    // FP32 u-table taps of the lane's column
};

// Slot records and W V of the item's slots, one slot per lane, in batches of
// 64 from the item's first slot: batch A (the one holding the chunk being
// fetched), A + 1 (a chunk can reach into it) and the records of A + 2.
// ds_bpermute hands each lane the slots its group supplies, so every record
// and W V is loaded once instead of once per column lane.
struct Batches {
  SlotRec r0, r1, r2;
  float2 y0, y1;
  int a;           // batch index of r0
};

__device__ inline int bperm_i(int addr, int v) { return __builtin_amdgcn_ds_bpermute(addr, v); }
__device__ inline float bperm_f(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// Add the tile's region sums times s (column x0 + col, rows 4 grp + r) into the ring.
__device__ inline void ring_add_scaled(float* ring, const f32x4& re, const f32x4& im, float s,
                                       int x0, int col, int grp) {
  const int slot = (x0 + col) & (kRing - 1);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float2* p = reinterpret_cast<float2*>(ring) + (4 * grp + r) * kRingPitch + slot;
    float2 v = *p;
    v.x += s * re[r];
    v.y += s * im[r];
    *p = v;
  }
}

template <int S, bool BF16>
__device__ __forceinline__ void grid_lp_item(const GridArgsLp& a, float* ring, float bound, int it,
                                             int lane, int col, int grp) {
  typedef Lp<BF16> L;
  typedef typename L::vec vec;
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int N = a.N, checker = a.checker;
  const uint32_t* __restrict__ lp_v = a.lp_v + col;
  const float2* __restrict__ pad_us = a.pad_us + col;
  const SlotRec* __restrict__ krec = a.krec;
  const float2* __restrict__ yrow = a.yrow;
  float* g = reinterpret_cast<float*>(a.grid);
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  const int s0 = uniform(item.y), last = s_end - 1;
  const int by = ty * C;
  TileWalk tw;
  tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), lane);
  ChunkPos cur = first_chunk(tw, s0, s_end);
  ChunkPos n1 = next_chunk(cur, tw, s_end, lane);

  Batches bt;
  bt.a = 0;
  bt.r0 = krec[min(s0 + lane, last)];
  bt.r1 = krec[min(s0 + 64 + lane, last)];
  bt.r2 = krec[min(s0 + 128 + lane, last)];
  bt.y0 = yrow[rec_pos(bt.r0)];
  bt.y1 = yrow[rec_pos(bt.r1)];

  // operands of chunk p into Bf (batches advance monotonically with p)
  auto fetch = [&](const ChunkPos& p, GridBuf& Bf) {
    const int bl = (p.c0 - s0) >> 6;
    while (bl > bt.a) {
      bt.r0 = bt.r1;
      bt.y0 = bt.y1;
      bt.r1 = bt.r2;
      bt.y1 = yrow[rec_pos(bt.r1)];
      bt.a += 1;
      bt.r2 = krec[min(s0 + 64 * (bt.a + 2) + lane, last)];
    }
    const bool straddle = ((min(p.c0 + 15, p.pe - 1) - s0) >> 6) > bt.a;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int s = p.c0 + 4 * grp + m;
      const int addr = ((s - s0) & 63) << 2;
      int kx = bperm_i(addr, bt.r0.x), ky = bperm_i(addr, bt.r0.y);
      float yr = bperm_f(addr, bt.y0.x), yi = bperm_f(addr, bt.y0.y);
      if (straddle) {
        const int kx1 = bperm_i(addr, bt.r1.x), ky1 = bperm_i(addr, bt.r1.y);
        const float yr1 = bperm_f(addr, bt.y1.x), yi1 = bperm_f(addr, bt.y1.y);
        if (((s - s0) >> 6) > bt.a) {
          kx = kx1;
          ky = ky1;
          yr = yr1;
          yi = yi1;
        }
      }
      const bool in = s < p.pe;   // slots past the chunk's tile carry no weight
      Bf.y[m] = in ? make_float2(yr, yi) : make_float2(0.f, 0.f);
      Bf.tv[m] = lp_v[ky];
      Bf.tu[m] = pad_us[kx];
    }
  };

  int tx = cur.tx;
  int fx = tx * C - H;   // first grid column held by the ring
  f32x4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
  // the accumulator holds (true sum) / scale, scale = 2^es (0 = not yet set);
  // inv = 1 / scale, kept beside it so that no chunk divides
  float scale = 0.f, inv = 0.f;
  int es = 0;

  // One pipeline step: chunk cur from X while the operands of n1 go into Y.
  auto step = [&](GridBuf& X, GridBuf& Y) -> bool {
    fetch(n1, Y);
    if (cur.tx != tx) {
      // the finished tile's region goes into the ring; ring columns no later
      // tile of the item can reach go to the grid
      ring_add_scaled(ring, acc_re, acc_im, scale, tx * C - H, col, grp);
      const int x0 = cur.tx * C - H;
      if (x0 >= fx + kRing) {
        ring_flush16(ring, fx, g, by - H, N, checker, lane);
        ring_flush16(ring, fx + 16, g, by - H, N, checker, lane);
        fx = x0;
      } else if (x0 + 16 > fx + kRing) {
        ring_flush16(ring, fx, g, by - H, N, checker, lane);
        fx += 16;
      }
      acc_re = f32x4{0.f, 0.f, 0.f, 0.f};
      acc_im = f32x4{0.f, 0.f, 0.f, 0.f};
      scale = 0.f;
      inv = 0.f;
      tx = cur.tx;
    }
    // lane's visibilities: slots c0 + 4 grp + m (the K slice it supplies)
    float bre[4], bim[4], mx = 0.f;
    vec a_re, a_im, a_nim;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float2 y = X.y[m];
      bre[m] = y.x * X.tu[m].x - y.y * X.tu[m].y;   // row product (u-table times s_k^v)
      bim[m] = y.x * X.tu[m].y + y.y * X.tu[m].x;
      mx = fmaxf(mx, fmaxf(fabsf(y.x), fabsf(y.y)));
      L::set_bits(a_re, m, (uint16_t)(X.tv[m] & 0xFFFFu));
      L::set_bits(a_im, m, (uint16_t)(X.tv[m] >> 16));
      L::set_bits(a_nim, m, (uint16_t)((X.tv[m] >> 16) ^ 0x8000u));
    }
    // the 16 lanes of a group hold the same four visibilities: the maximum
    // over the chunk needs only the exchanges between groups
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = __int_as_float(uniform(__float_as_int(fmaxf(mx, __shfl_xor(mx, 32, 64))))) * bound;
    if (mx > 0.f) {
      // smallest power of two 2^e >= mx (e kept within +-100, so that 2^-e is finite)
      int e;
      const float fm = frexpf(mx, &e);   // mx = fm 2^e, fm in [0.5, 1)
      e = uniform(min(max(fm == 0.5f ? e - 1 : e, -100), 100));
      if (scale == 0.f || e > es) {
        if (scale != 0.f) {
          const float f = ldexpf(1.f, es - e);   // exact power of two
          acc_re *= f;
          acc_im *= f;
        }
        es = e;
        scale = ldexpf(1.f, e);
        inv = ldexpf(1.f, -e);
      }
    }
    vec b_re, b_im;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      L::set(b_re, m, bre[m] * inv);
      L::set(b_im, m, bim[m] * inv);
    }
    acc_re = L::mfma(a_re, b_re, acc_re);
    acc_im = L::mfma(a_re, b_im, acc_im);
    acc_re = L::mfma(a_nim, b_im, acc_re);
    acc_im = L::mfma(a_im, b_re, acc_im);
    if (!n1.ok) return false;
    cur = n1;
    n1 = next_chunk(n1, tw, s_end, lane);
    return true;
  };

  GridBuf A, B;
  fetch(cur, A);
  while (step(A, B) && step(B, A)) {
  }
  ring_add_scaled(ring, acc_re, acc_im, scale, tx * C - H, col, grp);
  ring_flush16(ring, fx, g, by - H, N, checker, lane);
  ring_flush16(ring, fx + 16, g, by - H, N, checker, lane);
}

template <int S, bool BF16>
__global__ __launch_bounds__(64 * kWaves) void grid_lp_kernel(GridArgsLp a) {
  __shared__ float rings[kWaves * kRingFloats];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float* ring = rings + wave * kRingFloats;
  for (int i = lane; i < kRingFloats; i += 64) ring[i] = 0.f;
  const float bound = *a.lp_bound;
  int stride;
  const int n_items = (int)*a.nitems;
  for (int it = uniform(wave_items(kWaves, &stride)); it < n_items; it += stride)
    grid_lp_item<S, BF16>(a, ring, bound, it, lane, lane & 15, lane >> 4);
}

// ---------------------------------------------------------------- degridding

// Region operand of the tile at column tx: lane (col, grp) holds
// R[y = col][x = 4 grp + m].  The loads are issued at clamped (always valid)
// addresses with no branch; the checkerboard sign, and 0 outside the grid, are
// applied when the region is converted to the 16-bit operand, so no wait is
// forced at the load.
template <int S>
__device__ inline void load_region_lp(const float2* __restrict__ grid, int N, int tx, int gy,
                                      int grp, float2 (&r)[4]) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int64_t row = (int64_t)min(max(gy, 0), N - 1) * N;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int gx = tx * C - H + 4 * grp + m;
    r[m] = grid[row + min(max(gx, 0), N - 1)];
  }
}

struct DegridBuf {
  SlotRec k;       // record of the lane's slot, two chunks ahead
  uint32_t tu[4];  // 16-bit u-table taps x = 4 grp + m
  float2 tv[4];    // FP32 v-table taps y = 4 grp + m (times s_k^u)
  float2 reg[4];   // raw grid region of the chunk's tile
  bool fresh;      // region loaded for this chunk, not yet converted
};

template <int S, bool BF16>
__device__ __forceinline__ void degrid_lp_item(const DegridArgsLp& a, const float2* vs_tab, int it,
                                               int lane, int col, int grp) {
  typedef Lp<BF16> L;
  typedef typename L::vec vec;
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int N = a.N, checker = a.checker;
  const uint32_t* __restrict__ lp_u = a.lp_u + 4 * grp;      // taps x = 4 grp + m
  const float2* __restrict__ pad_vs = vs_tab + 4 * grp;      // taps y = 4 grp + m
  const SlotRec* __restrict__ krec = a.krec;
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  const int gy = ty * C - H + col;
  const bool row_ok = gy >= 0 && gy < N;
  TileWalk tw;
  tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), lane);
  ChunkPos cur = first_chunk(tw, uniform(item.y), s_end);
  ChunkPos n1 = next_chunk(cur, tw, s_end, lane);
  ChunkPos n2 = next_chunk(n1, tw, s_end, lane);
  float sr = 1.f;
  vec a_re, a_im;

  auto taps = [&](DegridBuf& B) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      B.tu[m] = lp_u[B.k.x + m];
      B.tv[m] = pad_vs[B.k.y + m];
    }
  };
  // One pipeline step: chunk cur from X while the record of n2 goes into X.k
  // and the taps (and on a tile change the region) of n1 into Y.
  auto step = [&](DegridBuf& X, DegridBuf& Y) -> bool {
    const SlotRec kc = X.k;
    X.k = krec[min(n2.c0 + col, n2.pe - 1)];
    taps(Y);
    if (X.fresh) {
      // A operand: R (-1)^(x + y) / s_R with s_R a power of two covering the region
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int gx = cur.tx * C - H + 4 * grp + m;
        float f = (checker && ((gx + gy) & 1)) ? -1.f : 1.f;
        if (!row_ok || gx < 0 || gx >= N) f = 0.f;
        X.reg[m] = make_float2(X.reg[m].x * f, X.reg[m].y * f);
      }
      float mx = 0.f;
#pragma unroll
      for (int m = 0; m < 4; ++m) mx = fmaxf(mx, fmaxf(fabsf(X.reg[m].x), fabsf(X.reg[m].y)));
      mx = wave_max(mx);
      // s_R: the smallest power of two 2^e >= mx (1 for an empty region;
      // e within +-100, so that 2^-e is finite)
      int e = 0;
      if (mx > 0.f) {
        const float fm = frexpf(mx, &e);
        e = min(max(fm == 0.5f ? e - 1 : e, -100), 100);
      }
      sr = ldexpf(1.f, e);
      const float inv = ldexpf(1.f, -e);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        L::set(a_re, m, X.reg[m].x * inv);
        L::set(a_im, m, X.reg[m].y * inv);
      }
    }
    Y.fresh = n1.ok && n1.tx != cur.tx;
    if (Y.fresh) load_region_lp<S>(a.grid, N, n1.tx, gy, grp, Y.reg);
    vec b_re, b_im, b_nim;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      L::set_bits(b_re, m, (uint16_t)(X.tu[m] & 0xFFFFu));
      L::set_bits(b_im, m, (uint16_t)(X.tu[m] >> 16));
      L::set_bits(b_nim, m, (uint16_t)((X.tu[m] >> 16) ^ 0x8000u));
    }
    // Z = R conj(Tu): re = Rre Tre + Rim Tim, im = Rim Tre - Rre Tim
    f32x4 z_re = {0.f, 0.f, 0.f, 0.f}, z_im = {0.f, 0.f, 0.f, 0.f};
    z_re = L::mfma(a_re, b_re, z_re);
    z_im = L::mfma(a_im, b_re, z_im);
    z_re = L::mfma(a_im, b_im, z_re);
    z_im = L::mfma(a_re, b_nim, z_im);
    float p_re = 0.f, p_im = 0.f;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      p_re += X.tv[rr].x * z_re[rr] + X.tv[rr].y * z_im[rr];
      p_im += X.tv[rr].x * z_im[rr] - X.tv[rr].y * z_re[rr];
    }
    p_re += __shfl_xor(p_re, 16, 64);
    p_im += __shfl_xor(p_im, 16, 64);
    p_re += __shfl_xor(p_re, 32, 64);
    p_im += __shfl_xor(p_im, 32, 64);
    if (grp == 0 && cur.c0 + col < cur.re) a.yrow[rec_pos(kc)] = make_float2(p_re * sr, p_im * sr);
    if (!n1.ok) return false;
    cur = n1;
    n1 = n2;
    n2 = next_chunk(n2, tw, s_end, lane);
    return true;
  };

  DegridBuf A, B;
  A.k = krec[min(cur.c0 + col, cur.pe - 1)];
  taps(A);
  load_region_lp<S>(a.grid, N, cur.tx, gy, grp, A.reg);
  A.fresh = true;
  B.k = krec[min(n1.c0 + col, n1.pe - 1)];
  B.fresh = false;
  while (step(A, B) && step(B, A)) {
  }
}

// FP32 v-table staged in LDS (LDS = true: one 16-wave workgroup per CU, work
// items from the per-XCD lists, as in the FP32 path) or read through the caches.
template <int S, bool BF16, bool LDS>
__global__ __launch_bounds__(LDS ? 1024 : 64 * kWaves) void degrid_lp_kernel(DegridArgsLp a) {
  extern __shared__ float2 vs_lds[];
  const int lane = threadIdx.x & 63;
  if constexpr (LDS) {
    for (int i = threadIdx.x; i < a.tab_len; i += blockDim.x) vs_lds[i] = a.pad_vs[i];
    __syncthreads();
    for_items(a.lists, a.r8, a.qctr, lane, [&](int it) {
      degrid_lp_item<S, BF16>(a, vs_lds, it, lane, lane & 15, lane >> 4);
    });
  } else {
    int stride;
    const int n_items = (int)*a.nitems;
    for (int it = uniform(wave_items(kWaves, &stride)); it < n_items; it += stride)
      degrid_lp_item<S, BF16>(a, a.pad_vs, it, lane, lane & 15, lane >> 4);
  }
}

int blocks_for(int64_t max_items) {
  int64_t b = (max_items + kWaves - 1) / kWaves;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

template <int S, bool BF16>
void launch_grid_s(const GridArgsLp& a, int64_t max_items, hipStream_t s) {
  const int blocks = blocks_for(max_items);
  hipLaunchKernelGGL((grid_lp_kernel<S, BF16>), dim3(blocks), dim3(64 * kWaves), 0, s, a);
}

template <int S, bool BF16>
void launch_degrid_s(const DegridArgsLp& a, int64_t max_items, int lds_bytes, int n_cu,
                     hipStream_t s) {
  if (lds_bytes > 0) {
    int64_t b = (max_items + 15) / 16;
    if (b > n_cu) b = n_cu;
    if (b < 1) b = 1;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&degrid_lp_kernel<S, BF16, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    hipLaunchKernelGGL((degrid_lp_kernel<S, BF16, true>), dim3((unsigned)b), dim3(1024), lds_bytes,
                       s, a);
  } else {
    const int blocks = blocks_for(max_items);
    hipLaunchKernelGGL((degrid_lp_kernel<S, BF16, false>), dim3(blocks), dim3(64 * kWaves), 0, s,
                       a);
  }
}

}  // namespace

#define SEPW_LP_CASES(F, A, B, ...)                                                \
  switch (S) {                                                                     \
    case 1: F<1, B>(A, max_items, __VA_ARGS__); break;                             \
    case 3: F<3, B>(A, max_items, __VA_ARGS__); break;                             \
    case 5: F<5, B>(A, max_items, __VA_ARGS__); break;                             \
    case 7: F<7, B>(A, max_items, __VA_ARGS__); break;                             \
    case 9: F<9, B>(A, max_items, __VA_ARGS__); break;                             \
    case 11: F<11, B>(A, max_items, __VA_ARGS__); break;                           \
    case 13: F<13, B>(A, max_items, __VA_ARGS__); break;                           \
    case 15: F<15, B>(A, max_items, __VA_ARGS__); break;                           \
    default: return hipErrorInvalidValue;                                          \
  }

hipError_t launch_grid_lp(int S, bool bf16, const GridArgsLp& a, int64_t max_items,
                          hipStream_t s) {
  if (bf16) {
    SEPW_LP_CASES(launch_grid_s, a, true, s)
  } else {
    SEPW_LP_CASES(launch_grid_s, a, false, s)
  }
  return hipGetLastError();
}

hipError_t launch_degrid_lp(int S, bool bf16, const DegridArgsLp& a, int64_t max_items,
                            int lds_bytes, int n_cu, hipStream_t s) {
  if (bf16) {
    SEPW_LP_CASES(launch_degrid_s, a, true, lds_bytes, n_cu, s)
  } else {
    SEPW_LP_CASES(launch_degrid_s, a, false, lds_bytes, n_cu, s)
  }
  return hipGetLastError();
}

#undef SEPW_LP_CASES

}  // namespace sepw
