// Precision form: gridding and degridding with FP16 or BF16 MFMA operands and
// FP32 accumulation.
//
// Same tile products as the FP32 path (grid.hip, degrid.hip: Section 5's
// separable update as a rank-K product over the visibilities of a tile), on
// v_mfma_f32_16x16x32_{f16,bf16}.  The real and imaginary parts of a complex
// operand sit side by side along K (k = 2 j + p holds part p of element j), so
// one instruction forms 16 complex products and sums their real parts, and a
// second one their imaginary parts:
//     Re sum_j a_j b_j = sum_j (Re a_j, Im a_j) . (Re b_j, -Im b_j),
//     Im sum_j a_j b_j = sum_j (Re a_j, Im a_j) . (Im b_j,  Re b_j),
// with no combining arithmetic after the products (conjugates flip signs in
// the second factor).
//
// Operand ranges and precision.
//   * FP16: powers of two chosen once per call keep the operands inside the
//     FP16 range: gridding multiplies W V by 2^(13 - e) with 2^e above
//     max |Re, Im| of W V over the call (the movement pass that places W V
//     records that maximum), degridding multiplies the grid by 2^(9 - e) with
//     2^e above max |Re, Im| of the grid (a reduction pass).  Table taps are
//     at most max |c1| <= 1 and are used unscaled; the FP32 sums are scaled
//     back by the exact inverse power of two.
//   * BF16 has FP32's exponent range and no scales, but only 8 significant
//     bits, so every operand is split into a high and a low part,
//     x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in
//     FP32), and each product takes three instructions,
//     hi hi + hi lo + lo hi; the dropped lo lo term is below 2^-16 relative.
//
// Gridding (tables in LDS, ring in registers, as the FP32 LDS kernel in
// grid.hip).  A chunk is up to 16 slots of one tile; lane (c = l % 16,
// g = l / 16) supplies A[c][k] and B[k][c] for the chunk's visibilities
// j = 4 g + m (m = 0..3):
//     A = (Re Tv_j, Im Tv_j) at region row c,
//     B = the row product y_j Tu_j at the lane's region column (c - x0) & 15,
//         as (Re, -Im) for the real sum and (-Im, -Re) for minus the
//         imaginary sum.
// Slots of a chunk past its tile's end carry y = 0.  Slot records and W V are
// loaded one slot per lane, 64 slots at a time and up to three batches ahead,
// and ds_bpermute hands each lane the four records its group supplies.
//
// Degridding (16-bit tables in LDS).  V_i = sum_y conj(Tv_i[y]) Z[y][i] with
// Z = R conj(Tu)^T the region times the u-taps:
//     stage 1: Z[y][i] = sum_x R[y][x] conj(Tu_i[x]):
//         A1 = (Re R, Im R) and (Im R, -Re R) at row c, columns 4 g + m;
//         B1 = (Re Tu_i, Im Tu_i) of visibility i = c at columns 4 g + m;
//     stage 2: W[i'][i] = sum_y conj(Tv_i'[y]) Z[y][i], of which V_i = W[i][i]:
//         A2 = (Re Tv_i', Im Tv_i') of visibility i' = c at rows 4 g + m;
//         B2 = (Re Z, Im Z) and (Im Z, -Re Z): lane (c, g) holds exactly the
//         rows 4 g + r of Z's column c that it must supply.
// Lane (c, g) holds W[4 g + r][c], so the diagonal W[c][c] sits in lane
// (c, c / 4), register c % 4.  With the grid from the centred FFT the region
// carries (-1)^(x+y) itself (applied with the scale when it is converted),
// so the tables are the plain ones.  FP16 takes A1 from an operand grid
// converted once per call (scale, sign and rounding as the per-region
// conversion, a zero border instead of bounds checks), BF16 its high and
// low parts from two such planes.
//
// Layout of v_mfma_f32_16x16x32: lane l supplies A[l % 16][8 (l / 16) + i]
// and B[8 (l / 16) + i][l % 16], i = 0..7, two 16-bit values per dword (low
// half first); accumulator register r of lane l is D[4 (l / 16) + r][l % 16].
// (The K order within the instruction does not change the sum, so only the
// pairing of A's and B's K positions, identical by construction, matters.)
#include "ring.h"
#include "walk.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kLdsWaves = 16;   // waves per workgroup of the LDS-table launches
// BF16 gridding holds hi and lo operand parts: with 12 waves per CU it gets
// 168 registers and no spills (16 waves: 128 registers, 11 spilled, 12 %
// slower at array scale)
constexpr int lds_waves_grid(bool bf16) { return bf16 ? 12 : kLdsWaves; }
constexpr int kWaves = 4;       // waves per workgroup when the tables stay in memory

template <bool BF16>
struct Lp;

template <>
struct Lp<false> {
  __device__ static uint32_t pack(float a, float b) {
    const f16x2 v = {(_Float16)a, (_Float16)b};   // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
  }
  __device__ static f32x4 mfma(const u32x4& a, const u32x4& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  }
};

template <>
struct Lp<true> {
  __device__ static uint32_t pack(float a, float b) {
    const bf16x2 v = {(__bf16)a, (__bf16)b};   // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
  }
  // the BF16 value in the low / high half of a packed dword, as FP32
  __device__ static float low(uint32_t u) { return __uint_as_float(u << 16); }
  __device__ static float high(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }
  __device__ static f32x4 mfma(const u32x4& a, const u32x4& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
};

// One MFMA operand: eight 16-bit values; l is the low part (BF16 only).
struct Opnd {
  u32x4 h, l;
};

// dword m of o = (a, b)
template <bool BF16>
__device__ __forceinline__ void set_one(Opnd& o, int m, float a, float b) {
  typedef Lp<BF16> L;
  const uint32_t h = L::pack(a, b);
  o.h[m] = h;
  if constexpr (BF16) o.l[m] = L::pack(a - L::low(h), b - L::high(h));
}

// dword m of o1 = (a, b) and of o2 = (b, -a)
template <bool BF16>
__device__ __forceinline__ void set_pair(Opnd& o1, Opnd& o2, int m, float a, float b) {
  typedef Lp<BF16> L;
  const uint32_t h = L::pack(a, b);
  o1.h[m] = h;
  o2.h[m] = L::pack(b, -a);   // bf16(-a) = -bf16(a): the same split
  if constexpr (BF16) {
    const float ra = a - L::low(h), rb = b - L::high(h);
    o1.l[m] = L::pack(ra, rb);
    o2.l[m] = L::pack(rb, -ra);
  }
}

// c + a b (BF16: hi hi + hi lo + lo hi)
template <bool BF16>
__device__ __forceinline__ f32x4 mma(const Opnd& a, const Opnd& b, f32x4 c) {
  typedef Lp<BF16> L;
  if constexpr (BF16) {
    c = L::mfma(a.l, b.h, c);
    c = L::mfma(a.h, b.l, c);
  }
  return L::mfma(a.h, b.h, c);
}

// Exponent e of the smallest power of two above m = max |Re, Im| over the
// finite parts (bits of a non-negative float), clamped to [-100, 100]; 0 when
// m is 0 (any scale then serves: the operands are all 0).
__device__ inline int exp_above(uint32_t bits) {
  const float m = __uint_as_float(bits);
  if (!(m > 0.f) || !(m <= 3.0e38f)) return 0;
  int e;
  (void)frexpf(m, &e);   // m = f 2^e, f in [0.5, 1): m < 2^e
  return min(max(e, -100), 100);
}

__device__ inline float bperm_f(int addr, float v) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// ---------------------------------------------------------------- gridding

// Chunk of at most 16 slots of one tile, as the fetch side walks them.
struct GChunk {
  int c0;       // first slot
  int pe;       // end of the tile's slots inside the item (padded to 4)
  int x0;       // first grid column of the tile's region
  bool first;   // first chunk of its tile
  bool ok;      // false past the item's end
};

template <int S>
__device__ inline GChunk next_gchunk(const GChunk& p, TileWalk& fw, int s_end, int lane) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  GChunk n = p;
  n.first = false;
  if (!p.ok) return n;
  if (p.c0 + 16 < p.pe) {
    n.c0 = p.c0 + 16;
    return n;
  }
  if (p.pe >= s_end || !fw.next(lane)) {
    n.ok = false;
    return n;
  }
  n.c0 = fw.first_slot();
  n.pe = min(fw.padded_end(), s_end);
  n.x0 = fw.tx * C - H;
  n.first = true;
  return n;
}

// Records and W V of the item's slots, one slot per lane, in batches of 64
// from the item's first slot: records of batches a .. a + 3, W V of a .. a + 2
// (W V of a batch is loaded when its records have had a batch's time to
// arrive, and is used a batch later).
struct GBatch {
  SlotRec ra, rb, rc, rd;
  float2 ya, yb, yc;
  int a;
};

// Record and W V of the lane's four slots of one chunk (moved by ds_bpermute).
struct GKeys {
  int kx[4], ky[4];
  float2 y[4];
};

// Taps of one chunk, with its position (its W V stays in the keys it came with).
struct GOps {
  float2 tu[4], tv[4];
  int x0;
  bool first;
};

struct GCtx {
  const SlotRec* krec;
  const float2* yrow;
  const char* tu;   // padded FP32 tables (LDS or memory), byte addressing
  const char* tv;
  float* grid;
  int N, checker, s0, last, y0, lane, col, grp, col8;
  float ys;         // FP16: scale of W V
};

// W V times the FP16 scale (applied when a batch moves up, a batch after its
// load was issued)
template <bool BF16>
__device__ __forceinline__ float2 yscaled(const GCtx& c, float2 y) {
  if constexpr (BF16) return y;
  return make_float2(y.x * c.ys, y.y * c.ys);
}

template <bool BF16>
__device__ __forceinline__ void gbatch_next(const GCtx& c, GBatch& bt) {
  bt.ra = bt.rb;
  bt.rb = bt.rc;
  bt.rc = bt.rd;
  bt.ya = bt.yb;
  bt.yb = yscaled<BF16>(c, bt.yc);
  bt.yc = c.yrow[rec_pos(bt.rc)];
  bt.a += 1;
  bt.rd = load_rec(c.krec + min(c.s0 + 64 * (bt.a + 3) + c.lane, c.last));
}

// Move the records and W V (scaled) of chunk k's slots c0 + 4 grp + m to this lane.
template <bool BF16>
__device__ __forceinline__ void gkeys(const GCtx& c, const GChunk& k, GBatch& bt, GKeys& K) {
  const int r = k.c0 - c.s0;
  while ((r >> 6) > bt.a) gbatch_next<BF16>(c, bt);
  const int off = r & 63;   // the chunk is window [off, off + 16) of batches a, a + 1
  int sx = bt.ra.x, sy = bt.ra.y;
  float yr = bt.ya.x, yi = bt.ya.y;
  if (off > 48) {
    // the chunk reaches into batch a + 1: lanes below off hold its slots
    const bool nb = c.lane < off;
    sx = nb ? bt.rb.x : sx;
    sy = nb ? bt.rb.y : sy;
    yr = nb ? bt.yb.x : yr;
    yi = nb ? bt.yb.y : yi;
  }
  // slots past the tile's end carry no weight
  const bool keep = ((c.lane - off) & 63) < k.pe - k.c0;
  yr = keep ? yr : 0.f;
  yi = keep ? yi : 0.f;
  const int base = ((off + 4 * c.grp) & 63) << 2;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int addr = base + 4 * m;
    K.kx[m] = __builtin_amdgcn_ds_bpermute(addr, sx);
    K.ky[m] = __builtin_amdgcn_ds_bpermute(addr, sy);
    K.y[m] = make_float2(bperm_f(addr, yr), bperm_f(addr, yi));
  }
}

__device__ __forceinline__ void gtaps(const GCtx& c, const GKeys& K, const GChunk& k, GOps& X) {
  const char* tu = c.tu + (((c.col - k.x0) & 15) << 3);   // lane's region column in this tile
  const char* tv = c.tv + c.col8;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    X.tu[m] = *reinterpret_cast<const float2*>(tu + (K.kx[m] << 3));
    X.tv[m] = *reinterpret_cast<const float2*>(tv + (K.ky[m] << 3));
  }
  X.x0 = k.x0;
  X.first = k.first;
}

template <int S, bool BF16>
__device__ __forceinline__ void grid_lp_item(const GridArgsLp& a, const GCtx& c0, int it) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  GCtx c = c0;
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  c.s0 = uniform(item.y);
  c.last = s_end - 1;
  c.y0 = ty * C - H;
  TileWalk fw;
  fw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), c.lane);
  GChunk f;
  f.c0 = c.s0;
  f.pe = min(fw.padded_end(), s_end);
  f.x0 = fw.tx * C - H;
  f.first = true;
  f.ok = true;

  GBatch bt;
  bt.a = 0;
  bt.ra = load_rec(c.krec + min(c.s0 + c.lane, c.last));
  bt.rb = load_rec(c.krec + min(c.s0 + 64 + c.lane, c.last));
  bt.rc = load_rec(c.krec + min(c.s0 + 128 + c.lane, c.last));
  bt.rd = load_rec(c.krec + min(c.s0 + 192 + c.lane, c.last));
  bt.ya = yscaled<BF16>(c, c.yrow[rec_pos(bt.ra)]);
  bt.yb = yscaled<BF16>(c, c.yrow[rec_pos(bt.rb)]);
  bt.yc = c.yrow[rec_pos(bt.rc)];

  RegRing rg;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc_re = zero, acc_ni = zero;   // acc_ni: minus the imaginary sums
  rg.lo_re = zero;
  rg.lo_im = zero;
  rg.hi_re = zero;
  rg.hi_im = zero;
  rg.blk = f.x0 >> 4;
  int x0 = f.x0;
  const float back = 1.f / c.ys;   // exact: c.ys is a power of two

  // chunk in X (W V in K): operands, then the two products; a new tile first
  // banks the finished region and makes the ring hold the new one
  auto process = [&](const GOps& X, const GKeys& K) {
    Opnd A, Bre, Bni;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      set_one<BF16>(A, m, X.tv[m].x, X.tv[m].y);
      const float yx = K.y[m].x, yy = K.y[m].y;
      const float br = yx * X.tu[m].x - yy * X.tu[m].y;   // row product y Tu
      const float bi = yx * X.tu[m].y + yy * X.tu[m].x;
      set_pair<BF16>(Bre, Bni, m, br, -bi);   // (br, -bi) and (-bi, -br)
    }
    if (X.first) {
      f32x4 im;
#pragma unroll
      for (int r = 0; r < 4; ++r) im[r] = -acc_ni[r];
      reg_ring_add(rg, acc_re, im, x0, c.col);
      x0 = X.x0;
      reg_ring_advance(rg, x0, c.grid, c.N, c.checker, c.y0, c.col, c.grp, back);
      acc_re = zero;
      acc_ni = zero;
    }
    acc_re = mma<BF16>(A, Bre, acc_re);
    acc_ni = mma<BF16>(A, Bni, acc_ni);
  };

  // Ping-pong: X holds chunk n (its W V in Kx), Kn the records of chunk
  // n + 1 (= f).  A half-step runs chunk n, reads the taps of n + 1 into Xn
  // and moves the records of n + 2 into Kx (free once chunk n has run).
  auto half = [&](const GOps& X, GKeys& Kx, GOps& Xn, const GKeys& Kn) -> bool {
    process(X, Kx);
    if (!f.ok) return false;
    gtaps(c, Kn, f, Xn);
    f = next_gchunk<S>(f, fw, s_end, c.lane);
    if (f.ok) gkeys<BF16>(c, f, bt, Kx);
    return true;
  };
  GKeys KA, KB;
  GOps XA, XB;
  gkeys<BF16>(c, f, bt, KA);
  gtaps(c, KA, f, XA);
  f = next_gchunk<S>(f, fw, s_end, c.lane);
  if (f.ok) gkeys<BF16>(c, f, bt, KB);
  while (half(XA, KA, XB, KB) && half(XB, KB, XA, KA)) {
  }
  f32x4 im;
#pragma unroll
  for (int r = 0; r < 4; ++r) im[r] = -acc_ni[r];
  reg_ring_add(rg, acc_re, im, x0, c.col);
  reg_ring_shift(rg, c.grid, c.N, c.checker, c.y0, c.col, c.grp, back);
  reg_ring_shift(rg, c.grid, c.N, c.checker, c.y0, c.col, c.grp, back);
}

template <int S, bool BF16, bool LDS>
__global__ __launch_bounds__(64 * (LDS ? lds_waves_grid(BF16) : kWaves)) void grid_lp_kernel(GridArgsLp a) {
  extern __shared__ float2 smem[];
  const int lane = threadIdx.x & 63;
  GCtx c;
  const char* tu = reinterpret_cast<const char*>(a.tab_u);
  const char* tv = reinterpret_cast<const char*>(a.tab_v);
  if constexpr (LDS) {
    const int n = a.tab_len;
    const bool two = a.tab_v != a.tab_u;
    for (int i = threadIdx.x; i < n; i += blockDim.x) smem[i] = a.tab_u[i];
    if (two)
      for (int i = threadIdx.x; i < n; i += blockDim.x) smem[n + i] = a.tab_v[i];
    __syncthreads();
    tu = reinterpret_cast<const char*>(smem);
    tv = reinterpret_cast<const char*>(two ? smem + n : smem);
  }
  c.krec = a.krec;
  c.yrow = a.yrow;
  c.tu = tu;
  c.tv = tv;
  c.grid = reinterpret_cast<float*>(a.grid);
  c.N = a.N;
  c.checker = a.checker;
  c.lane = lane;
  c.col = lane & 15;
  c.grp = lane >> 4;
  c.col8 = c.col << 3;
  c.ys = BF16 ? 1.f : ldexpf(1.f, 13 - exp_above(*a.vmax));
  for_blocks8(a.qctr, (uint32_t)uniform((int)*a.nitems), lane,
              [&](uint32_t it) { grid_lp_item<S, BF16>(a, c, (int)it); });
}

// ---------------------------------------------------------------- degridding

// Degridding pipeline.  The kernel is bound by the texture-address unit,
// which takes about 40 cycles per 64-lane vector-memory instruction whatever
// its width (measured with the TA counters), so the pipeline keeps those
// instructions few: slot records arrive 64 at a time in one coalesced 12-byte
// load per lane and ds_bpermute hands each lane its chunk's record; a tile's
// region takes two 16-byte loads per lane; and the results of four chunks are
// moved by ds_bpermute into one 64-lane store.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
constexpr uint32_t kOob = 0x80000000u;   // byte offset past every buffer resource used here

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0,
                                           (int)(bytes < 0x7FFFFFFF ? bytes : 0x7FFFFFFF),
                                           0x00020000);
}

// One chunk's operands: the record (u base, v base, row-bin position) of slot
// c0 + col and the 16-bit taps 4 grp + m of that visibility (u for stage 1,
// v for stage 2; BF16 high and low parts).
struct DOps {
  u32x3 rec;
  u32x4 tu_h, tu_l, tv_h, tv_l;
};

struct DCtx {
  __amdgpu_buffer_rsrc_t krs;   // tile slot records
  __amdgpu_buffer_rsrc_t yrs;   // results (row-bin order)
  const uint32_t* tu;   // 16-bit padded tables (LDS or memory); BF16 low parts at + tab_len
  const uint32_t* tv;
  int tab_len;
  int col, grp, lane;
  int s0, last;
  float back;           // 1 / gs
};

// Records of the item's slots, one slot per lane, in batches of 64 from the
// item's first slot: batches a, a + 1 (arrived) and a + 2 (in flight).
struct DBatch {
  u32x3 ra, rb, rc;
  int a;
};

__device__ __forceinline__ u32x3 batch_load(const DCtx& c, int j) {
  return __builtin_amdgcn_raw_buffer_load_b96(c.krs, min(c.s0 + 64 * j + c.lane, c.last) * 12, 0, 0);
}

// Record of slot c0 + col of chunk k, moved from the batches by ds_bpermute.
__device__ __forceinline__ u32x3 dkey(const DCtx& c, const ChunkPos& k, DBatch& bt) {
  const int r = k.c0 - c.s0;
  while ((r >> 6) > bt.a) {
    bt.ra = bt.rb;
    bt.rb = bt.rc;
    bt.a += 1;
    bt.rc = batch_load(c, bt.a + 2);
  }
  const int off = r & 63;   // the chunk is window [off, off + 16) of batches a, a + 1
  u32x3 src = bt.ra;
  if (off > 48) {
    // the chunk reaches into batch a + 1: lanes below off hold its slots
    const bool nb = c.lane < off;
#pragma unroll
    for (int i = 0; i < 3; ++i) src[i] = nb ? bt.rb[i] : src[i];
  }
  const int addr = ((off + c.col) & 63) << 2;
  u32x3 k3;
#pragma unroll
  for (int i = 0; i < 3; ++i) k3[i] = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)src[i]);
  return k3;
}

template <bool BF16>
__device__ __forceinline__ void dtaps(const DCtx& c, DOps& B) {
  const uint32_t* pu = c.tu + B.rec[0] + 4 * c.grp;
  const uint32_t* pv = c.tv + B.rec[1] + 4 * c.grp;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    B.tu_h[m] = pu[m];
    B.tv_h[m] = pv[m];
    if constexpr (BF16) {
      B.tu_l[m] = pu[c.tab_len + m];
      B.tv_l[m] = pv[c.tab_len + m];
    }
  }
}

// Pipeline of a work item: chunk n runs while the taps of n + 1 are read
// (its record moved one step earlier) and the record of n + 2 is moved from
// the batches.  The region of a tile is loaded when its first chunk becomes
// n + 1 and converted to MFMA operands when that chunk becomes n, so one raw
// region is in flight.  (A two-entry queue of raw regions, loaded two chunks
// ahead, made the compiler address its entries through a pointer chosen at
// run time, which put the queue in scratch memory: 5 GB of scratch writes
// per call at array scale and a third more time.)
template <int S, bool BF16>
__device__ __forceinline__ void degrid_lp_item(const DegridArgsLp& a, const DCtx& c0, int it) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  DCtx c = c0;
  const int N = a.N;
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  c.s0 = uniform(item.y);
  c.last = s_end - 1;
  const int y0 = ty * C - H;   // first grid row of the item's regions
  const int sel = c.col & 3;                 // register of the lane's diagonal element
  const bool diag = c.grp == (c.col >> 2);   // the lane that holds W[col][col]
  // lane holding V[col] of a chunk, for gathering four chunks' results
  const int vsrc = (c.col + 16 * (c.col >> 2)) << 2;
  TileWalk tw;
  tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), c.lane);
  ChunkPos cur;
  cur.c0 = c.s0;
  cur.pe = min(tw.padded_end(), s_end);
  cur.re = min(tw.real_end(), s_end);
  cur.tx = tw.tx;
  cur.ok = true;
  ChunkPos n1 = next_chunk(cur, tw, s_end, c.lane);
  ChunkPos n2 = next_chunk(n1, tw, s_end, c.lane);

  DBatch bt;
  bt.a = 0;
  bt.ra = batch_load(c, 0);
  bt.rb = batch_load(c, 1);
  bt.rc = batch_load(c, 2);

  // region operands of the current tile: (Re R, Im R) and (Im R, -Re R)
  Opnd ra, rb;
  // The region comes from the operand grid (a.g16: scaled, signed, rounded,
  // a zero border around the grid): one in-bounds 16-byte load per lane (two
  // for BF16: high parts, then low parts one plane further), and (Im, -Re)
  // a half swap and a sign flip of each pair
  const int pitch = a.N + 2 * kG16Border;
  const int64_t plane = (int64_t)pitch * pitch;
  const uint32_t* g16row = a.g16 + (int64_t)(y0 + kG16Border) * pitch;
  const __amdgpu_buffer_rsrc_t g16h = rsrc(g16row, (int64_t)16 * pitch * 4);
  const __amdgpu_buffer_rsrc_t g16l = BF16 ? rsrc(g16row + plane, (int64_t)16 * pitch * 4) : g16h;
  auto load16 = [&](u32x4& gh, u32x4& gl, int tx) {
    const uint32_t off = (uint32_t)(c.col * pitch + tx * C - H + 4 * c.grp + kG16Border) * 4u;
    gh = __builtin_amdgcn_raw_buffer_load_b128(g16h, off, 0, 0);
    if constexpr (BF16) gl = __builtin_amdgcn_raw_buffer_load_b128(g16l, off, 0, 0);
  };
  auto swapneg = [](uint32_t v) { return ((v >> 16) | (v << 16)) ^ 0x80000000u; };
  auto take16 = [&](const u32x4& gh, const u32x4& gl) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ra.h[m] = gh[m];
      rb.h[m] = swapneg(gh[m]);
      if constexpr (BF16) {
        ra.l[m] = gl[m];
        rb.l[m] = swapneg(gl[m]);
      }
    }
  };
  // region of the next tile, loaded one chunk ahead
  u32x4 qh, ql;
  auto load_next = [&](int tx) { load16(qh, ql, tx); };
  auto use_next = [&](int) { take16(qh, ql); };

  // results of up to four chunks: lanes 16 j + col hold V[col] of chunk j of
  // the group, stored with one instruction (offset kOob: nothing to store)
  u32x2 res;
  res[0] = 0u;
  res[1] = 0u;
  uint32_t roff = kOob;
  int rj = 0;
  auto flush = [&]() {
    __builtin_amdgcn_raw_buffer_store_b64(res, c.yrs, roff, 0, 0);
    roff = kOob;
    rj = 0;
  };

  auto step = [&](DOps& X, DOps& Y, u32x3& K) -> bool {
    // taps of n1 (record moved last step), then the record of n2
    Y.rec = K;
    dtaps<BF16>(c, Y);
    K = dkey(c, n2, bt);
    // stage 1: Z = R conj(Tu)^T
    Opnd bu;
    bu.h = X.tu_h;
    bu.l = X.tu_l;
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    const f32x4 zr = mma<BF16>(ra, bu, z);
    const f32x4 zi = mma<BF16>(rb, bu, z);
    // stage 2: W = conj(Tv) Z, V = diag(W)
    Opnd b2a, b2b, av;
#pragma unroll
    for (int r = 0; r < 4; ++r) set_pair<BF16>(b2a, b2b, r, zr[r], zi[r]);
    av.h = X.tv_h;
    av.l = X.tv_l;
    const f32x4 wr = mma<BF16>(av, b2a, z);
    const f32x4 wi = mma<BF16>(av, b2b, z);
    float vr = sel == 0 ? wr[0] : (sel == 1 ? wr[1] : (sel == 2 ? wr[2] : wr[3]));
    float vi = sel == 0 ? wi[0] : (sel == 1 ? wi[1] : (sel == 2 ? wi[2] : wi[3]));
    if constexpr (!BF16) {
      vr *= c.back;
      vi *= c.back;
    }
    (void)diag;
    // gather V[col] into lanes 16 rj + col
    const uint32_t gr = (uint32_t)__builtin_amdgcn_ds_bpermute(vsrc, (int)__float_as_uint(vr));
    const uint32_t gi = (uint32_t)__builtin_amdgcn_ds_bpermute(vsrc, (int)__float_as_uint(vi));
    if (c.grp == rj) {
      res[0] = gr;
      res[1] = gi;
      roff = cur.c0 + c.col < cur.re ? (X.rec[2] & 0x7FFFFFFFu) * 8u : kOob;
    }
    if (++rj == 4) flush();
    if (!n1.ok) return false;
    const bool fresh = n1.tx != cur.tx;
    cur = n1;
    n1 = n2;
    n2 = next_chunk(n2, tw, s_end, c.lane);
    if (fresh) use_next(cur.tx);
    if (n1.ok && n1.tx != cur.tx) load_next(n1.tx);
    return true;
  };

  // the first tile's region is taken at once; later ones are loaded one chunk ahead
  load_next(cur.tx);
  use_next(cur.tx);
  if (n1.ok && n1.tx != cur.tx) load_next(n1.tx);
  DOps A, B;
  A.rec = dkey(c, cur, bt);
  dtaps<BF16>(c, A);
  u32x3 K = dkey(c, n1, bt);
  while (step(A, B, K) && step(B, A, K)) {
  }
  if (rj > 0) flush();
}

template <int S, bool BF16, bool LDS>
__global__ __launch_bounds__(64 * (LDS ? kLdsWaves : kWaves)) void degrid_lp_kernel(DegridArgsLp a) {
  extern __shared__ uint32_t tsm[];
  const int lane = threadIdx.x & 63;
  const int nt = BF16 ? 2 * a.tab_len : a.tab_len;   // dwords of one table (both parts)
  DCtx c;
  c.krs = rsrc(a.krec, a.nslots * (int64_t)sizeof(SlotRec));
  c.yrs = rsrc(a.yrow, a.ycap * (int64_t)sizeof(float2));
  c.tu = a.lp_u;
  c.tv = a.lp_v;
  if constexpr (LDS) {
    const bool two = a.lp_v != a.lp_u;
    for (int i = threadIdx.x; i < nt; i += blockDim.x) tsm[i] = a.lp_u[i];
    if (two)
      for (int i = threadIdx.x; i < nt; i += blockDim.x) tsm[nt + i] = a.lp_v[i];
    __syncthreads();
    c.tu = tsm;
    c.tv = two ? tsm + nt : tsm;
  }
  c.tab_len = a.tab_len;
  c.lane = lane;
  c.col = lane & 15;
  c.grp = lane >> 4;
  const int e = BF16 ? 0 : exp_above(*a.gmax);
  c.back = ldexpf(1.f, e - 9);
  for_items(a.lists, a.r8, a.qctr, lane, [&](int it) { degrid_lp_item<S, BF16>(a, c, it); });
}

template <int S, bool BF16>
void launch_grid_s(const GridArgsLp& a, int lds_bytes, int n_cu, hipStream_t s) {
  if (lds_bytes > 0) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&grid_lp_kernel<S, BF16, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    hipLaunchKernelGGL((grid_lp_kernel<S, BF16, true>), dim3((unsigned)n_cu),
                       dim3(64 * lds_waves_grid(BF16)), lds_bytes, s, a);
  } else {
    hipLaunchKernelGGL((grid_lp_kernel<S, BF16, false>), dim3((unsigned)(4 * n_cu)),
                       dim3(64 * kWaves), 0, s, a);
  }
}

template <int S, bool BF16>
void launch_degrid_s(const DegridArgsLp& a, int lds_bytes, int n_cu, hipStream_t s) {
  if (lds_bytes > 0) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&degrid_lp_kernel<S, BF16, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    hipLaunchKernelGGL((degrid_lp_kernel<S, BF16, true>), dim3((unsigned)n_cu),
                       dim3(64 * kLdsWaves), lds_bytes, s, a);
  } else {
    hipLaunchKernelGGL((degrid_lp_kernel<S, BF16, false>), dim3((unsigned)(4 * n_cu)),
                       dim3(64 * kWaves), 0, s, a);
  }
}

// max |Re, Im| over n complex values, as float bits, into *out (atomic
// maximum: *out must hold 0, or a smaller maximum, at launch)
__global__ __launch_bounds__(256) void absmax_kernel(const float2* __restrict__ g, int64_t n,
                                                     uint32_t* __restrict__ out) {
  __shared__ float sh[4];
  float mx = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    mx = finite_absmax(mx, g[i]);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    if (mx > 0.f) atomicMax(out, __float_as_uint(mx));
  }
}

// 16-bit degridding operands of a whole grid (see launch_lp_grid): the same
// products, rounding and (BF16) high / low split as the kernel's own
// conversion of a region.
template <bool BF16>
__global__ __launch_bounds__(256) void lp_grid_kernel(const float2* __restrict__ g, int N,
                                                      const uint32_t* __restrict__ gmax,
                                                      int checker, uint32_t* __restrict__ out) {
  typedef Lp<BF16> L;
  const float gs = BF16 ? 1.f : ldexpf(1.f, 9 - exp_above(*gmax));
  const int64_t pitch = N + 2 * kG16Border;
  const int64_t n = (int64_t)N * N;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t y = i / N, x = i - y * N;
    const float f = (checker && ((x + y) & 1)) ? -gs : gs;
    const float2 v = g[i];
    const float a = v.x * f, b = v.y * f;
    const int64_t o = (y + kG16Border) * pitch + x + kG16Border;
    const uint32_t h = L::pack(a, b);
    out[o] = h;
    if constexpr (BF16) out[o + pitch * pitch] = L::pack(a - L::low(h), b - L::high(h));
  }
}

}  // namespace

#define SEPW_LP_CASES(F, B, ...)                                \
  switch (S) {                                                  \
    case 1: F<1, B>(__VA_ARGS__); break;                        \
    case 3: F<3, B>(__VA_ARGS__); break;                        \
    case 5: F<5, B>(__VA_ARGS__); break;                        \
    case 7: F<7, B>(__VA_ARGS__); break;                        \
    case 9: F<9, B>(__VA_ARGS__); break;                        \
    case 11: F<11, B>(__VA_ARGS__); break;                      \
    case 13: F<13, B>(__VA_ARGS__); break;                      \
    case 15: F<15, B>(__VA_ARGS__); break;                      \
    default: return hipErrorInvalidValue;                       \
  }

hipError_t launch_grid_lp(int S, bool bf16, const GridArgsLp& a, int lds_bytes, int n_cu,
                          hipStream_t s) {
  if (bf16) {
    SEPW_LP_CASES(launch_grid_s, true, a, lds_bytes, n_cu, s)
  } else {
    SEPW_LP_CASES(launch_grid_s, false, a, lds_bytes, n_cu, s)
  }
  return hipGetLastError();
}

hipError_t launch_degrid_lp(int S, bool bf16, const DegridArgsLp& a, int lds_bytes, int n_cu,
                            hipStream_t s) {
  if (bf16) {
    SEPW_LP_CASES(launch_degrid_s, true, a, lds_bytes, n_cu, s)
  } else {
    SEPW_LP_CASES(launch_degrid_s, false, a, lds_bytes, n_cu, s)
  }
  return hipGetLastError();
}

#undef SEPW_LP_CASES

hipError_t launch_lp_grid(const float2* g, int N, bool bf16, const uint32_t* gmax, int checker,
                          uint32_t* out, hipStream_t s) {
  int64_t b = ((int64_t)N * N + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  if (bf16)
    hipLaunchKernelGGL(lp_grid_kernel<true>, dim3((unsigned)b), dim3(256), 0, s, g, N, gmax,
                       checker, out);
  else
    hipLaunchKernelGGL(lp_grid_kernel<false>, dim3((unsigned)b), dim3(256), 0, s, g, N, gmax,
                       checker, out);
  return hipGetLastError();
}

hipError_t launch_absmax(const float2* g, int64_t n, uint32_t* out, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)b), dim3(256), 0, s, g, n, out);
  return hipGetLastError();
}

}  // namespace sepw
