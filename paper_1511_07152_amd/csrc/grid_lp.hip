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
// so the tables are the plain ones.
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

// Exponent e of the smallest power of two above m = max |Re, Im| (bits of a
// non-negative float), clamped to [-100, 100]; 0 when m is 0 or not finite
// (any scale then serves: the operands are all 0, or the sums are not finite
// anyway).
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

// Taps and W V of one chunk, with its position.
struct GOps {
  float2 tu[4], tv[4], y[4];
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

__device__ __forceinline__ void gbatch_next(const GCtx& c, GBatch& bt) {
  bt.ra = bt.rb;
  bt.rb = bt.rc;
  bt.rc = bt.rd;
  bt.ya = bt.yb;
  bt.yb = bt.yc;
  bt.yc = c.yrow[rec_pos(bt.rc)];
  bt.a += 1;
  bt.rd = load_rec(c.krec + min(c.s0 + 64 * (bt.a + 3) + c.lane, c.last));
}

// Move the records and W V of chunk k's slots c0 + 4 grp + m to this lane.
__device__ __forceinline__ void gkeys(const GCtx& c, const GChunk& k, GBatch& bt, GKeys& K) {
  const int r = k.c0 - c.s0;
  while ((r >> 6) > bt.a) gbatch_next(c, bt);
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
  const int rc8 = ((c.col - k.x0) & 15) << 3;   // lane's region column in this tile
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    X.tu[m] = *reinterpret_cast<const float2*>(c.tu + (K.kx[m] << 3) + rc8);
    X.tv[m] = *reinterpret_cast<const float2*>(c.tv + (K.ky[m] << 3) + c.col8);
    X.y[m] = K.y[m];
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
  bt.ya = c.yrow[rec_pos(bt.ra)];
  bt.yb = c.yrow[rec_pos(bt.rb)];
  bt.yc = c.yrow[rec_pos(bt.rc)];

  RegRing rg;
  f32x4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_ni = acc_re;   // acc_ni: minus the imaginary sums
  rg.lo_re = acc_re;
  rg.lo_im = acc_re;
  rg.hi_re = acc_re;
  rg.hi_im = acc_re;
  rg.blk = f.x0 >> 4;
  int x0 = f.x0;
  const float back = 1.f / c.ys;   // exact: c.ys is a power of two

  // chunk in X: operands, then the two products (a new tile first banks the
  // finished region and makes the ring hold the new one)
  auto process = [&](const GOps& X) {
    Opnd A, Bre, Bni;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      set_one<BF16>(A, m, X.tv[m].x, X.tv[m].y);
      float yx = X.y[m].x, yy = X.y[m].y;
      if constexpr (!BF16) {
        yx *= c.ys;
        yy *= c.ys;
      }
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
      const f32x4 z = {0.f, 0.f, 0.f, 0.f};
      acc_re = mma<BF16>(A, Bre, z);
      acc_ni = mma<BF16>(A, Bni, z);
    } else {
      acc_re = mma<BF16>(A, Bre, acc_re);
      acc_ni = mma<BF16>(A, Bni, acc_ni);
    }
  };

  // X holds chunk n (taps read), K the records of chunk n + 1 (= f)
  GKeys K;
  GOps X;
  gkeys(c, f, bt, K);
  gtaps(c, K, f, X);
  f = next_gchunk<S>(f, fw, s_end, c.lane);
  if (f.ok) gkeys(c, f, bt, K);
  while (true) {
    process(X);
    if (!f.ok) break;
    gtaps(c, K, f, X);
    f = next_gchunk<S>(f, fw, s_end, c.lane);
    if (f.ok) gkeys(c, f, bt, K);
  }
  f32x4 im;
#pragma unroll
  for (int r = 0; r < 4; ++r) im[r] = -acc_ni[r];
  reg_ring_add(rg, acc_re, im, x0, c.col);
  reg_ring_shift(rg, c.grid, c.N, c.checker, c.y0, c.col, c.grp, back);
  reg_ring_shift(rg, c.grid, c.N, c.checker, c.y0, c.col, c.grp, back);
}

template <int S, bool BF16, bool LDS>
__global__ __launch_bounds__(64 * (LDS ? kLdsWaves : kWaves)) void grid_lp_kernel(GridArgsLp a) {
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
  const int n_items = uniform((int)*a.nitems);
  while (true) {
    int it = 0;
    if (lane == 0) it = (int)atomicAdd(a.qctr, 1u);
    it = uniform(__shfl(it, 0, 64));
    if (it >= n_items) break;
    grid_lp_item<S, BF16>(a, c, it);
  }
}

// ---------------------------------------------------------------- degridding

// One chunk's operands: the record of slot c0 + col (loaded two chunks
// ahead), the 16-bit taps 4 grp + m of that visibility (u for stage 1, v for
// stage 2; BF16 high and low parts), and on a tile change the raw region
// values R[y0 + col][x0 + 4 grp + m].
struct DOps {
  SlotRec k;
  u32x4 tu_h, tu_l, tv_h, tv_l;
  float2 reg[4];
  bool fresh;
};

struct DCtx {
  const uint32_t* tu;   // 16-bit padded tables (LDS or memory); BF16 low parts at + tab_len
  const uint32_t* tv;
  int tab_len;
  int s_end, y0, gy, col, grp, lane;
  float gs;             // FP16: scale of the region
  float back;           // 1 / gs
};

template <bool BF16>
__device__ __forceinline__ void dtaps(const DCtx& c, DOps& B) {
  const uint32_t* pu = c.tu + B.k.x + 4 * c.grp;
  const uint32_t* pv = c.tv + B.k.y + 4 * c.grp;
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

// Region values of the tile at column tx for this lane's row (clamped, always
// valid addresses; rows and columns outside the grid get factor 0 when the
// region is converted).
template <int S>
__device__ inline void dregion(const float2* __restrict__ grid, int N, int tx, int gy, int grp,
                               float2 (&r)[4]) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int64_t row = (int64_t)min(max(gy, 0), N - 1) * N;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int gx = tx * C - H + 4 * grp + m;
    r[m] = grid[row + min(max(gx, 0), N - 1)];
  }
}

template <int S, bool BF16>
__device__ __forceinline__ void degrid_lp_item(const DegridArgsLp& a, const DCtx& c0, int it) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  DCtx c = c0;
  const int N = a.N;
  const int4 item = a.items[it];
  const int ty = uniform(item.x), s_end = uniform(item.z);
  c.s_end = s_end;
  c.y0 = ty * C - H;
  c.gy = c.y0 + c.col;
  const bool row_ok = c.gy >= 0 && c.gy < N;
  const int sel = c.col & 3;                 // register of the lane's diagonal element
  const bool diag = c.grp == (c.col >> 2);   // the lane that holds W[col][col]
  TileWalk tw;
  tw.start(a.tdesc + (int64_t)ty * a.ntx, a.ntx, uniform(item.w), c.lane);
  ChunkPos cur;
  cur.c0 = uniform(item.y);
  cur.pe = min(tw.padded_end(), s_end);
  cur.re = min(tw.real_end(), s_end);
  cur.tx = tw.tx;
  cur.ok = true;
  ChunkPos n1 = next_chunk(cur, tw, s_end, c.lane);
  ChunkPos n2 = next_chunk(n1, tw, s_end, c.lane);
  Opnd ra, rb;   // region operands of the current tile: (Re R, Im R) and (Im R, -Re R)

  // One pipeline step: chunk cur from X while the record of n2 goes into X.k
  // and the taps (and on a tile change the region) of n1 into Y.
  auto step = [&](DOps& X, DOps& Y) -> bool {
    const SlotRec kc = X.k;
    X.k = load_rec(a.krec + min(n2.c0 + c.col, n2.pe - 1));
    dtaps<BF16>(c, Y);
    if (X.fresh) {
      // region operands: R (-1)^(x+y) times the scale, 0 outside the grid
      const int gx0 = cur.tx * C - H + 4 * c.grp;
      float f = BF16 ? 1.f : c.gs;
      if (a.checker && ((gx0 + c.gy) & 1)) f = -f;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int gx = gx0 + m;
        const float fm = (row_ok && gx >= 0 && gx < N) ? f : 0.f;
        set_pair<BF16>(ra, rb, m, X.reg[m].x * fm, X.reg[m].y * fm);
        if (a.checker) f = -f;
      }
    }
    Y.fresh = n1.ok && n1.tx != cur.tx;
    if (Y.fresh) dregion<S>(a.grid, N, n1.tx, c.gy, c.grp, Y.reg);
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
    if (diag && cur.c0 + c.col < cur.re) a.yrow[rec_pos(kc)] = make_float2(vr, vi);
    if (!n1.ok) return false;
    cur = n1;
    n1 = n2;
    n2 = next_chunk(n2, tw, s_end, c.lane);
    return true;
  };

  DOps A, B;
  A.k = load_rec(a.krec + min(cur.c0 + c.col, cur.pe - 1));
  dtaps<BF16>(c, A);
  dregion<S>(a.grid, N, cur.tx, c.gy, c.grp, A.reg);
  A.fresh = true;
  B.k = load_rec(a.krec + min(n1.c0 + c.col, n1.pe - 1));
  B.fresh = false;
  while (step(A, B) && step(B, A)) {
  }
}

template <int S, bool BF16, bool LDS>
__global__ __launch_bounds__(64 * (LDS ? kLdsWaves : kWaves)) void degrid_lp_kernel(DegridArgsLp a) {
  extern __shared__ uint32_t tsm[];
  const int lane = threadIdx.x & 63;
  const int nt = BF16 ? 2 * a.tab_len : a.tab_len;   // dwords of one table (both parts)
  DCtx c;
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
  c.gs = ldexpf(1.f, 9 - e);
  c.back = ldexpf(1.f, e - 9);
  for_items(a.lists, a.r8, a.qctr, lane, [&](int it) { degrid_lp_item<S, BF16>(a, c, it); });
}

template <int S, bool BF16>
void launch_grid_s(const GridArgsLp& a, int lds_bytes, int n_cu, hipStream_t s) {
  if (lds_bytes > 0) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&grid_lp_kernel<S, BF16, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    hipLaunchKernelGGL((grid_lp_kernel<S, BF16, true>), dim3((unsigned)n_cu),
                       dim3(64 * kLdsWaves), lds_bytes, s, a);
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
    const float2 v = g[i];
    mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
    if (mx > 0.f) atomicMax(out, __float_as_uint(mx));
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

hipError_t launch_absmax(const float2* g, int64_t n, uint32_t* out, hipStream_t s) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)b), dim3(256), 0, s, g, n, out);
  return hipGetLastError();
}

}  // namespace sepw
