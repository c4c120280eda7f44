// Visibility quantisation, w-plane assignment and counting sort into grid tiles.
//
// u, v, w are in wavelengths (Section 2).  Grid cell j is centred at
// u_j = (j - N/2)/fov; the GCF tables are oversampled by O (Section 2), so each
// visibility is rounded to the nearest 1/O cell:
//   x = u fov + N/2,  t = x O,  q = floor(t + 1/2),
//   cell = floor((q + O/2) / O),  f = q - cell O in [-O/2, O/2),  fi = f + O/2
// and assigned plane k = clamp(floor((w - w_lo) inv_dw), 0, P - 1).  Each FP64
// operation is an explicitly rounded IEEE operation in this order (no
// contraction), so the integer results are reproducible bit for bit.
// Footprints that would leave the grid are dropped (not wrapped).  In facet
// mode (Section 4.1) the coordinates are first shifted, u' = u - w l0/n0,
// v' = v - w m0/n0, and the visibility phase is rotated by
// exp(+2 pi i (u l0 + v m0 + w (n0 - 1))).
//
// Tiles are c x c blocks of cells (c = 17 - S, so that a tile's S x S
// footprints fit in a 16 x 16 region), numbered row-major.  Sorting is a
// two-level counting sort.  Level 1 (by row bin = tile row >> rshift): the
// quantiser writes the histogram of each chunk of kChunk visibilities; a scan
// down the chunks of every bin (chunk groups, then chunks inside a group) gives
// each chunk one contiguous run per non-empty bin, in chunk order, with no
// global atomics; each chunk then places its visibilities with LDS atomics.
// Level 2 (by tile inside the row bin): one workgroup per row bin counts,
// scans and places its visibilities entirely in LDS.  Each row bin owns a
// reserved range of tile slots; inside it the tiles follow each other in
// row-major order, each padded to a multiple of 4 slots (the MFMA group size)
// with zero-weight padding, and tdesc[tile] = (first slot, first slot + count).
// Membership of a visibility in its tile is exact; the order inside a tile is
// not specified.
#include <algorithm>

#include "internal.h"

namespace sepw {

namespace {

constexpr int kThreads = 256;

inline dim3 grid_for(int64_t n, int64_t per_block = kThreads) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return dim3((unsigned)b);
}

struct AxisBin {
  int64_t cell;
  int fi;
  bool ok;
};

__device__ inline AxisBin axis_bin(double u, const QuantGeom& g) {
  AxisBin r;
  double x = __dadd_rn(__dmul_rn(u, g.fov), g.half_n);
  double t = __dmul_rn(x, g.over);
  double q = floor(__dadd_rn(t, 0.5));
  r.ok = isfinite(q) && fabs(q) < 1099511627776.0;  // 2^40
  int64_t qi = r.ok ? (int64_t)q : 0;
  // O is a power of two: floor((q + O/2) / O) is an arithmetic shift, and
  // f + O/2 = q - cell O + O/2 the low bits of q + O/2
  r.cell = (qi + g.O / 2) >> g.lo;
  r.fi = (int)((qi + g.O / 2) & (int64_t)(g.O - 1));
  return r;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t val, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void zero_c64_kernel(float2* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_float2(0.f, 0.f);
}

// ---------------------------------------------------------------- scan
constexpr int kScanItems = 16;
constexpr int kScanBlock = kThreads * kScanItems;   // elements per block

__device__ inline uint32_t block_exclusive(uint32_t v, uint32_t* sh, uint32_t* total) {
  // inclusive wave scan by shuffles, then a scan of the wave totals in LDS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int i = 0; i < kThreads / 64; ++i) {
    if (i < wave) before += sh[i];
    all += sh[i];
  }
  *total = all;
  return before + x - v;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* in, int64_t n,
                                                                uint32_t* partial) {
  __shared__ uint32_t sh[kThreads / 64];
  int64_t base = (int64_t)blockIdx.x * kScanBlock;
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)j * kThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive(s, sh, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void scan_partials_kernel(uint32_t* partial, int64_t nb) {
  __shared__ uint32_t sh[kThreads / 64];
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += kThreads) {
    int64_t i = base + threadIdx.x;
    uint32_t v = i < nb ? partial[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_exclusive(v, sh, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void scan_apply_kernel(const uint32_t* in, int64_t n,
                                                               const uint32_t* partial,
                                                               uint32_t* out) {
  __shared__ uint32_t sh[kThreads / 64];
  // each thread owns kScanItems consecutive elements
  int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  uint32_t vals[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    vals[j] = i < n ? in[i] : 0u;
    s += vals[j];
  }
  uint32_t tot;
  uint32_t run = partial[blockIdx.x] + block_exclusive(s, sh, &tot);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += vals[j];
  }
}


// ---------------------------------------------------------------- facets, items, export
// Facet phase rotation in caller order (Section 4.1), applied to W V on its way
// into tile order and undone on the way back.
__global__ void rotation_kernel(Coords src, int64_t nvis, QuantGeom g, float2* __restrict__ rot) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvis;
       i += (int64_t)gridDim.x * blockDim.x) {
    double uu, vv, ww;
    coords_at(src, i, uu, vv, ww);
    // phase in cycles, reduced to [-1/2, 1/2] before the FP64 sincos
    double cyc = uu * g.l0 + vv * g.m0 + ww * (g.n0 - 1.0);
    double frac = cyc - rint(cyc);
    double s, c;
    sincospi(2.0 * frac, &s, &c);
    rot[i] = make_float2((float)c, (float)s);
  }
}

__device__ inline uint32_t round4(uint32_t n) { return (n + 3u) & ~3u; }

// slot range of row of tiles r: [first slot of its first tile, padded end of its last)
__device__ inline uint2 row_slots(const uint2* __restrict__ tdesc, int ntx, int64_t r) {
  const uint2 a = tdesc[r * ntx], b = tdesc[(r + 1) * ntx - 1];
  return make_uint2(a.x, b.x + round4(b.y - b.x));
}

// Rows of tiles go to 8 work lists by r % 8; list entries are indexed
// (r % 8) r8 + r / 8, so one scan gives every row's first item in list order.
__device__ inline int64_t list_index(int64_t r, int r8) { return (r % 8) * r8 + r / 8; }

__global__ void item_counts_kernel(const uint2* __restrict__ tdesc, int ntx, int nty, int r8,
                                   uint32_t item_slots, uint32_t* __restrict__ nit) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= 8 * (int64_t)r8;
       j += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c = 0;
    const int64_t r = (j % r8) * 8 + j / r8;   // row with list_index(r) == j
    if (j < 8 * (int64_t)r8 && r < nty) {
      const uint2 rs = row_slots(tdesc, ntx, r);
      c = (rs.y - rs.x + item_slots - 1) / item_slots;
    }
    nit[j] = c;
  }
}

// Item k of row r covers slots [a + k M, min(a + (k + 1) M, e)) of the row's
// range [a, e) (M = item_slots, a multiple of 4); the tile holding its first
// slot writes it.
__global__ void items_kernel(const uint2* __restrict__ tdesc, const uint32_t* __restrict__ itoff,
                             int ntx, int nty, int r8, uint32_t item_slots,
                             int4* __restrict__ items) {
  const int64_t nt = (int64_t)ntx * nty;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint2 d = tdesc[t];
    if (d.y == d.x) continue;
    const int64_t r = t / ntx;
    const uint32_t ps = d.x, pe = d.x + round4(d.y - d.x);
    const uint2 rs = row_slots(tdesc, ntx, r);
    const uint32_t o = itoff[list_index(r, r8)];
    uint32_t k = (ps - rs.x + item_slots - 1) / item_slots;
    for (uint32_t b = rs.x + k * item_slots; b < pe; b += item_slots, ++k) {
      const uint32_t e = rs.y - b > item_slots ? b + item_slots : rs.y;
      items[o + k] = make_int4((int)r, (int)b, (int)e, (int)(t - r * ntx));
    }
  }
}

template <class Args>
__global__ void job_prefix_kernel(const Args* __restrict__ jobs, int njobs,
                                  uint32_t* __restrict__ first, uint32_t* __restrict__ counter) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t acc = 0;
  first[0] = 0;
  for (int j = 0; j < njobs; ++j) {
    acc += *jobs[j].nitems;
    first[j + 1] = acc;
  }
  for (int q = 0; q < 8; ++q) counter[q * kCtrStride] = 0u;
}

__global__ void dropped_kernel(const uint32_t* __restrict__ kept, int64_t nvis,
                               int64_t* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = nvis - (int64_t)*kept;
}

__global__ void bins_export_kernel(const uint2* __restrict__ rrec, const uint32_t* __restrict__ place,
                                   const uint32_t* __restrict__ delta, int nbins, int64_t nvis,
                                   int tile_c, int ntx, int32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvis;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t* o = out + 7 * i;
    const uint32_t pl = place[i];
    if (pl == kDropped) {
      o[0] = o[1] = o[2] = o[3] = o[4] = 0;
      o[5] = -1;
      o[6] = 1;
      continue;
    }
    const uint32_t d =
        delta[(i / kL1Chunk) * nbins + (pl >> kPlaceShift)] + (pl & kPlaceMask);
    const uint2 r = rrec[d];
    const int cu = r.x & 0xFFFF, cv = r.x >> 16;
    o[0] = cu;
    o[1] = r.y & 0xFF;
    o[2] = cv;
    o[3] = (r.y >> 8) & 0xFF;
    o[4] = r.y >> 16;
    o[5] = (cv / tile_c) * ntx + cu / tile_c;
    o[6] = 0;
  }
}

// ---------------------------------------------------------------- two-level sort
constexpr int kL1Threads = 1024;
constexpr int kChunk = kL1Chunk;         // visibilities per block in the level-1 passes
constexpr int kLdsChannels = 1024;      // channel scales held in LDS (more: divided per visibility)
static_assert(kChunk % kL1Threads == 0, "level-1 chunk must be a multiple of the block size");

constexpr int kBinsPer = kMaxRowBins / kL1Threads;   // row bins owned by each thread

// Exclusive scan across one 1024-thread workgroup: `sum` is this thread's
// total (thread t owns bins t kBinsPer .. t kBinsPer + kBinsPer - 1); returns
// the sum over the threads before it and sets *total to the workgroup's sum.
__device__ inline uint32_t block_scan_owned(uint32_t sum, uint32_t* wsum, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint32_t run = x - sum, tot = 0;
#pragma unroll
  for (int w = 0; w < kL1Threads / 64; ++w) {
    const uint32_t ws = wsum[w];
    if (w < wave) run += ws;
    tot += ws;
  }
  __syncthreads();   // wsum is reused by the next scan
  *total = tot;
  return run;
}

__global__ __launch_bounds__(kL1Threads) void quantise_rows_kernel(
    Coords src, int64_t nvis, QuantGeom g, int rshift, int nbins, uint32_t* __restrict__ rbin,
    uint2* __restrict__ qrec, uint32_t* __restrict__ chist) {
  __shared__ uint32_t hist[kMaxRowBins];
  __shared__ double cscale[kLdsChannels];
  for (int b = threadIdx.x; b < nbins; b += kL1Threads) hist[b] = 0u;
  // channel-shared rows: the channel scales f / c once per workgroup, and
  // (row, channel) of this thread's visibilities advanced without divisions
  const bool rows = src.uvw != nullptr;
  const bool lds_scale = rows && src.nchan <= kLdsChannels;
  if (lds_scale)
    for (int c = threadIdx.x; c < (int)src.nchan; c += kL1Threads)
      cscale[c] = __ddiv_rn(src.freq[c], kLightSpeed);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  int64_t row = 0, ch = 0, drow = 0, dch = 0;
  if (rows) {
    const int64_t i0 = base + threadIdx.x;
    row = i0 / src.nchan;
    ch = i0 - row * src.nchan;
    drow = kL1Threads / src.nchan;
    dch = kL1Threads - drow * src.nchan;
  }
  for (int m = 0; m < kChunk / kL1Threads; ++m) {
    const int64_t i = base + (int64_t)m * kL1Threads + threadIdx.x;
    if (i >= nvis) break;
    double uu, vv, ww;
    if (rows) {
      const double sc = lds_scale ? cscale[ch] : __ddiv_rn(src.freq[ch], kLightSpeed);
      uu = __dmul_rn(src.uvw[3 * row], sc);
      vv = __dmul_rn(src.uvw[3 * row + 1], sc);
      ww = __dmul_rn(src.uvw[3 * row + 2], sc);
      row += drow;
      ch += dch;
      if (ch >= src.nchan) {
        ch -= src.nchan;
        row += 1;
      }
    } else {
      uu = src.u[i];
      vv = src.v[i];
      ww = src.w[i];
    }
    if (g.facet) {
      uu = __dsub_rn(uu, __ddiv_rn(__dmul_rn(ww, g.l0), g.n0));
      vv = __dsub_rn(vv, __ddiv_rn(__dmul_rn(ww, g.m0), g.n0));
    }
    AxisBin bu = axis_bin(uu, g), bv = axis_bin(vv, g);
    double kt = floor(__dmul_rn(__dsub_rn(ww, g.w_lo), g.inv_dw));
    bool okw = isfinite(kt);
    int k = 0;
    if (okw) k = kt < 0.0 ? 0 : (kt > (double)(g.P - 1) ? g.P - 1 : (int)kt);
    const int h = g.S / 2;
    bool on = bu.ok && bv.ok && okw && bu.cell - h >= 0 && bu.cell + h <= g.N - 1 &&
              bv.cell - h >= 0 && bv.cell + h <= g.N - 1;
    if (on) {
      int cu = (int)bu.cell, cv = (int)bv.cell;
      const uint32_t ty = (uint32_t)(cv / g.tile_c);
      rbin[i] = ty >> rshift;
      qrec[i] = pack_rec(cu, bu.fi, cv, bv.fi, k);
      atomicAdd(&hist[ty >> rshift], 1u);
    } else {
      rbin[i] = kDropped;
      qrec[i] = make_uint2(0u, 0u);
    }
  }
  __syncthreads();
  uint32_t* hrow = chist + (int64_t)blockIdx.x * nbins;
  for (int b = threadIdx.x; b < nbins; b += kL1Threads) hrow[b] = hist[b];
}

// gsum[b][g] = visibilities of row bin b in the chunks of group g
__global__ void group_sums_kernel(const uint32_t* __restrict__ chist, int64_t nch, int nbins,
                                  int ngroups, uint32_t* __restrict__ gsum) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (b >= nbins) return;
  const int64_t c0 = (int64_t)g * kGroupChunks;
  const int64_t c1 = min(c0 + (int64_t)kGroupChunks, nch);
  uint32_t sum = 0;
  for (int64_t c = c0; c < c1; ++c) sum += chist[c * nbins + b];
  gsum[(int64_t)b * ngroups + g] = sum;
}

// One workgroup per row bin: exclusive scan of gsum[b][.] in place, total to
// rowcount[b] (and rowcount[nbins] = 0, so that the scan of rowcount ends with
// the kept count).
__global__ __launch_bounds__(256) void group_scan_kernel(uint32_t* __restrict__ gsum, int ngroups,
                                                         int nbins, uint32_t* __restrict__ rowcount) {
  __shared__ uint32_t wsum[4];
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* p = gsum + (int64_t)b * ngroups;
  uint32_t carry = 0;
  for (int g0 = 0; g0 < ngroups; g0 += 256) {
    const int g = g0 + (int)threadIdx.x;
    const uint32_t v = g < ngroups ? p[g] : 0u;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t run = carry + x - v, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t ws = wsum[w];
      if (w < wave) run += ws;
      tot += ws;
    }
    __syncthreads();
    if (g < ngroups) p[g] = run;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    rowcount[b] = carry;
    if (b == 0) rowcount[nbins] = 0u;
  }
}

// One workgroup per chunk group: walks its chunks in order carrying, per row
// bin, the row-bin position where the next chunk's run starts (rowoff + the
// group's prefix), and writes delta[c][b] = that position minus the run's
// start inside chunk c's bin-ordered staging, plus the chunk's kept count.
__global__ __launch_bounds__(kL1Threads) void chunk_deltas_kernel(
    const uint32_t* __restrict__ chist, const uint32_t* __restrict__ gpre,
    const uint32_t* __restrict__ rowoff, int64_t nch, int nbins, int ngroups,
    uint32_t* __restrict__ delta, uint32_t* __restrict__ ckept) {
  __shared__ uint32_t wsum[kL1Threads / 64];
  const int g = blockIdx.x;
  const int t0 = threadIdx.x * kBinsPer;
  uint32_t carry[kBinsPer];
#pragma unroll
  for (int j = 0; j < kBinsPer; ++j) {
    const int b = t0 + j;
    carry[j] = b < nbins ? rowoff[b] + gpre[(int64_t)b * ngroups + g] : 0u;
  }
  const int64_t c0 = (int64_t)g * kGroupChunks;
  const int64_t c1 = min(c0 + (int64_t)kGroupChunks, nch);
  for (int64_t c = c0; c < c1; ++c) {
    const uint32_t* row = chist + c * nbins;
    uint32_t v[kBinsPer], sum = 0;
#pragma unroll
    for (int j = 0; j < kBinsPer; ++j) {
      v[j] = t0 + j < nbins ? row[t0 + j] : 0u;
      sum += v[j];
    }
    uint32_t total;
    uint32_t run = block_scan_owned(sum, wsum, &total);
    uint32_t* d = delta + c * nbins;
#pragma unroll
    for (int j = 0; j < kBinsPer; ++j) {
      if (t0 + j < nbins) d[t0 + j] = carry[j] - run;
      run += v[j];
      carry[j] += v[j];
    }
    if (threadIdx.x == 0) ckept[c] = total;
  }
}

// Slots reserved for row bin b: its visibilities plus room to pad every
// non-empty tile to a multiple of 4, rounded to 4.
__global__ void pad_sizes_kernel(const uint32_t* __restrict__ rowcount, int nbins, int rshift,
                                 int ntx, int nty, uint32_t* __restrict__ rowpad) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nbins; b += gridDim.x * blockDim.x) {
    uint32_t p = 0;
    if (b < nbins) {
      const uint32_t c = rowcount[b];
      const int64_t r0 = (int64_t)b << rshift;
      const int64_t r1 = min(((int64_t)b + 1) << rshift, (int64_t)nty);
      const int64_t tiles = (r1 - r0) * ntx;
      p = round4(c + 3u * (uint32_t)min((int64_t)c, tiles));
    }
    rowpad[b] = p;
  }
}

// Level-1 placement of one chunk: the scan of its histogram gives the start of
// each bin's run in the chunk's staging; visibilities are laid out in LDS in
// bin order (LDS atomics), each gets its placement word, and each run is copied
// to the row-bin array as one contiguous piece (delta gives its position).
__global__ __launch_bounds__(kL1Threads) void row_scatter_kernel(
    const uint32_t* __restrict__ rbin, const uint2* __restrict__ qrec, int64_t nvis, int nbins,
    const uint32_t* __restrict__ chist, const uint32_t* __restrict__ delta,
    uint2* __restrict__ rrec, uint32_t* __restrict__ place) {
  __shared__ uint32_t cur[kMaxRowBins];   // placement cursors in the staging
  __shared__ uint32_t dl[kMaxRowBins];    // the chunk's row of delta
  __shared__ uint32_t wsum[kL1Threads / 64];
  __shared__ uint2 stage[kChunk];
  __shared__ uint16_t binof[kChunk];   // row bin of each staged record
  const int64_t chunk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t first = chunk * kChunk;
  const int t0 = threadIdx.x * kBinsPer;
  uint32_t v[kBinsPer], sum = 0;
#pragma unroll
  for (int j = 0; j < kBinsPer; ++j) {
    v[j] = t0 + j < nbins ? chist[chunk * nbins + t0 + j] : 0u;
    sum += v[j];
  }
  uint32_t kept;
  uint32_t run = block_scan_owned(sum, wsum, &kept);
#pragma unroll
  for (int j = 0; j < kBinsPer; ++j) {
    if (t0 + j < nbins) {
      cur[t0 + j] = run;
      dl[t0 + j] = delta[chunk * nbins + t0 + j];
    }
    run += v[j];
  }
  __syncthreads();
  // all loads of the thread first, then the LDS placement; the caller-order
  // streams carry the non-temporal hint, leaving the L2 to the row-bin runs
  // (1.69 -> 1.67 ms for the sort at array scale)
  constexpr int kPer = kChunk / kL1Threads;
  uint32_t kk[kPer];
  uint2 qr[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int64_t i = first + (int64_t)m * kL1Threads + threadIdx.x;
    kk[m] = i < nvis ? __builtin_nontemporal_load(rbin + i) : kDropped;
    const uint64_t w =
        i < nvis ? __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(qrec) + i) : 0ull;
    qr[m] = make_uint2((uint32_t)w, (uint32_t)(w >> 32));
  }
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    const int64_t i = first + (int64_t)m * kL1Threads + threadIdx.x;
    if (i >= nvis) break;
    if (kk[m] == kDropped) {
      __builtin_nontemporal_store(kDropped, place + i);
      continue;
    }
    const uint32_t b = kk[m];
    const uint32_t idx = atomicAdd(&cur[b], 1u);
    stage[idx] = qr[m];
    binof[idx] = (uint16_t)b;
    __builtin_nontemporal_store((b << kPlaceShift) | idx, place + i);
  }
  __syncthreads();
  // copy out: consecutive lanes take consecutive staged records (runs stay contiguous)
  for (uint32_t k = threadIdx.x; k < kept; k += kL1Threads) rrec[dl[binof[k]] + k] = stage[k];
}

constexpr int kSortThreads = 1024;

// perm = the row bins by decreasing count (one workgroup, bitonic sort in LDS),
// so that the level-2 workgroups start with the largest bins and the small
// ones fill in at the end.
__global__ __launch_bounds__(kSortThreads) void bin_order_kernel(const uint32_t* __restrict__ rowcount,
                                                                 int nbins, uint32_t* __restrict__ perm) {
  __shared__ uint32_t key[kMaxRowBins];
  __shared__ uint16_t val[kMaxRowBins];
  int n = 1;
  while (n < nbins) n <<= 1;
  for (int i = threadIdx.x; i < n; i += kSortThreads) {
    key[i] = i < nbins ? rowcount[i] + 1u : 0u;   // padding sorts last
    val[i] = (uint16_t)i;
  }
  __syncthreads();
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += kSortThreads) {
        const int p = i ^ j;
        if (p > i) {
          const bool desc = (i & k) == 0;
          const uint32_t a = key[i], b = key[p];
          if (desc ? a < b : a > b) {
            key[i] = b;
            key[p] = a;
            const uint16_t t = val[i];
            val[i] = val[p];
            val[p] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < nbins; i += kSortThreads) perm[i] = val[i];
}

// Level 2: one workgroup per row bin.  Tiles are laid out row-major inside the
// bin's reserved slot range, each padded to a multiple of 4 slots, and
// described by tdesc[tile] = (first slot, first slot + count).  A slot holds
// the padded-table bases of its visibility and the visibility's row-bin
// position (where the data movement keeps W V); padding slots have table base
// 0 and point at zero_row, whose W V stays 0.
// The bin's tile histogram is built in LDS (eight record loads in flight per
// thread), scanned into tile starts, and the records are then placed in
// chunks: a counting sort of each chunk in LDS orders it by destination, so
// that each tile's share of the chunk is written as one contiguous run.
// Dynamic LDS: cursor and chunk count per tile (2 nloc words), then the
// chunk's staged records and their destinations (16 bytes per record).
constexpr int kSortLoads = 8;

template <int C>
__device__ inline int local_tile(uint2 r, int row0, int ntx) {
  const int cu = (int)(r.x & 0xFFFFu), cv = (int)(r.x >> 16);
  return (cv / C - row0) * ntx + cu / C;
}

// Exclusive scan of a[0, n) in place (each thread owns a run of consecutive
// entries, f applied to each entry first); returns the total.
template <class F>
__device__ inline uint32_t block_scan_tiles(uint32_t* a, int n, uint32_t* wsum, F f) {
  const int per = (n + kSortThreads - 1) / kSortThreads;
  const int t0 = threadIdx.x * per, t1 = min(t0 + per, n);
  uint32_t sum = 0;
  for (int t = t0; t < t1; ++t) sum += f(a[t]);
  uint32_t total;
  uint32_t run = block_scan_owned(sum, wsum, &total);
  for (int t = t0; t < t1; ++t) {
    const uint32_t v = f(a[t]);
    a[t] = run;
    run += v;
  }
  return total;
}

// C = tile edge (a template argument, so that the divisions are shifts and multiplications)
template <int C>
__global__ __launch_bounds__(kSortThreads) void row_sort_kernel(
    const uint32_t* __restrict__ rowoff, const uint32_t* __restrict__ prowoff,
    const uint2* __restrict__ rrec, const uint32_t* __restrict__ perm, int rshift, int ntx,
    int nty, int O, int S, uint32_t zero_row, int chunk, uint2* __restrict__ tdesc,
    SlotRec* __restrict__ krec) {
  extern __shared__ uint32_t lds[];
  __shared__ uint32_t wsum[kSortThreads / 64];
  const int L = padded_len(S);
  const int b = (int)perm[blockIdx.x];
  const int row0 = b << rshift;
  const int row1 = min((b + 1) << rshift, nty);
  const int64_t tile0 = (int64_t)row0 * ntx;
  const int nloc = (row1 - row0) * ntx;
  uint32_t* cnt = lds;                 // tile counts, then the next free slot of each tile
  uint32_t* lc = lds + nloc;           // the chunk's count, then start, per tile
  SlotRec* stage = reinterpret_cast<SlotRec*>(lds + 2 * nloc);
  uint32_t* dst = reinterpret_cast<uint32_t*>(stage + chunk);
  const uint32_t s0 = rowoff[b], s1 = rowoff[b + 1];
  const uint32_t pbase = prowoff[b];
  for (int t = threadIdx.x; t < nloc; t += kSortThreads) {
    cnt[t] = 0u;
    lc[t] = 0u;
  }
  __syncthreads();
  for (uint32_t e0 = s0; e0 < s1; e0 += kSortLoads * kSortThreads) {
    uint2 r[kSortLoads];
#pragma unroll
    for (int j = 0; j < kSortLoads; ++j) {
      const uint32_t e = e0 + j * kSortThreads + threadIdx.x;
      r[j] = e < s1 ? rrec[e] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < kSortLoads; ++j)
      if (e0 + j * kSortThreads + threadIdx.x < s1)
        atomicAdd(&cnt[local_tile<C>(r[j], row0, ntx)], 1u);
  }
  __syncthreads();
  // tile starts (padded counts scanned), descriptors and padding records
  {
    const int per = (nloc + kSortThreads - 1) / kSortThreads;
    const int t0 = threadIdx.x * per, t1 = min(t0 + per, nloc);
    uint32_t sum = 0;
    for (int t = t0; t < t1; ++t) sum += round4(cnt[t]);
    uint32_t total;
    uint32_t run = block_scan_owned(sum, wsum, &total);
    for (int t = t0; t < t1; ++t) {
      const uint32_t c = cnt[t];
      const uint32_t p = pbase + run;
      tdesc[tile0 + t] = make_uint2(p, p + c);
      for (uint32_t j = c; j < round4(c); ++j) krec[p + j] = SlotRec{0, 0, (int)zero_row};
      cnt[t] = p;
      run += round4(c);
    }
  }
  __syncthreads();
  constexpr int kMaxPer = 4;   // records per thread and chunk (chunk <= 4096)
  // records of the next chunk are loaded while the current one is placed
  uint2 rn[kMaxPer];
#pragma unroll
  for (int j = 0; j < kMaxPer; ++j) {
    const uint32_t e = s0 + j * kSortThreads + threadIdx.x;
    rn[j] = (j * kSortThreads + (int)threadIdx.x < chunk && e < s1) ? rrec[e] : make_uint2(0u, 0u);
  }
  for (uint32_t c0 = s0; c0 < s1; c0 += chunk) {
    const int n = (int)min((uint32_t)chunk, s1 - c0);
    uint2 r[kMaxPer];
    int tl[kMaxPer];
    uint32_t rk[kMaxPer];
#pragma unroll
    for (int j = 0; j < kMaxPer; ++j) r[j] = rn[j];
    const uint32_t c1 = c0 + chunk;
#pragma unroll
    for (int j = 0; j < kMaxPer; ++j) {
      const uint32_t e = c1 + j * kSortThreads + threadIdx.x;
      if (j * kSortThreads + (int)threadIdx.x < chunk && e < s1) rn[j] = rrec[e];
    }
#pragma unroll
    for (int j = 0; j < kMaxPer; ++j) {
      if (j * kSortThreads + (int)threadIdx.x < n) {
        tl[j] = local_tile<C>(r[j], row0, ntx);
        rk[j] = atomicAdd(&lc[tl[j]], 1u);
      }
    }
    __syncthreads();
    block_scan_tiles(lc, nloc, wsum, [](uint32_t v) { return v; });
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kMaxPer; ++j) {
      if (j * kSortThreads + (int)threadIdx.x < n) {
        const int cu = (int)(r[j].x & 0xFFFFu), cv = (int)(r[j].x >> 16);
        // padded-table bases: tap of region column x is at base + x
        const int k = (int)(r[j].y >> 16);
        const int ox = cu % C, oy = cv % C;
        const int row_u = k * O + (int)(r[j].y & 0xFFu);
        const int row_v = k * O + (int)((r[j].y >> 8) & 0xFFu);
        const uint32_t q = lc[tl[j]] + rk[j];
        stage[q] = SlotRec{row_u * L + C - 1 - ox, row_v * L + C - 1 - oy,
                           (int)((c0 + j * kSortThreads + threadIdx.x) |
                                 ((uint32_t)((cu + cv) & 1) << 31))};
        dst[q] = cnt[tl[j]] + rk[j];
      }
    }
    __syncthreads();
    // runs of consecutive staged records go to consecutive slots
    for (int q = threadIdx.x; q < n; q += kSortThreads) krec[dst[q]] = stage[q];
    for (int t = threadIdx.x; t < nloc; t += kSortThreads) {
      const uint32_t next = t + 1 < nloc ? lc[t + 1] : (uint32_t)n;
      cnt[t] += next - lc[t];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nloc; t += kSortThreads) lc[t] = 0u;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- moving data
// Streams read or written once (placement words, weights, the caller-order
// results) carry the non-temporal hint, which leaves the L2 to the row-bin
// runs, whose partial cache lines merge there (measured: 0.99 -> 0.95 ms for
// both directions at array scale).  Stores into the row-bin array stay
// ordinary: made non-temporal in degridding, they took 3.2 -> 4.1 ms.
typedef float f32x2 __attribute__((ext_vector_type(2)));
// Caller order <-> row-bin order through the level-1 placement.  A workgroup
// handles the same chunk of kChunk caller positions as the level-1 placement:
// the placement words put the chunk's visibilities into LDS in bin order, and
// each bin's run moves to or from the row-bin array as one contiguous piece
// (position = delta[chunk][bin] + staged position), while the caller side
// stays coalesced.  The gridding kernels read W V, and the degridding kernels
// write their results, at the row-bin positions held in the tile slots.
constexpr int kPerThread = kChunk / kL1Threads;

struct MoveLds {
  uint32_t dl[kMaxRowBins];   // the chunk's row of delta
  float2 stage[kChunk];
  uint16_t binof[kChunk];
  float wmax[kL1Threads / 64];
};

__device__ inline void load_deltas(const uint32_t* __restrict__ delta, int64_t chunk, int nbins,
                                   uint32_t* dl) {
  const uint32_t* row = delta + chunk * nbins;
  for (int b = threadIdx.x; b < nbins; b += kL1Threads) dl[b] = row[b];
}

// yrow[row-bin position of i] = V[i] W[i] rot[i] for chunk `chunk` of one job
__device__ inline void to_rows_chunk(const MoveArgs& a, int64_t chunk, MoveLds& L) {
  const int64_t first = chunk * kChunk;
  load_deltas(a.delta, chunk, a.nbins, L.dl);
  uint32_t pl[kPerThread];
  float2 y[kPerThread];
  float wt[kPerThread];
  float2 ro[kPerThread];
  // all loads of the thread first, then the LDS stores
#pragma unroll
  for (int m = 0; m < kPerThread; ++m) {
    const int64_t i = first + (int64_t)m * kL1Threads + threadIdx.x;
    const bool in = i < a.nvis;
    pl[m] = in ? __builtin_nontemporal_load(a.place + i) : kDropped;
    y[m] = in ? a.vis[i] : make_float2(0.f, 0.f);
    wt[m] = (in && a.weight) ? __builtin_nontemporal_load(a.weight + i) : 1.f;
    ro[m] = (in && a.rot) ? a.rot[i] : make_float2(1.f, 0.f);
  }
  float mx = 0.f;   // max |Re, Im| over the finite parts of the placed values
#pragma unroll
  for (int m = 0; m < kPerThread; ++m) {
    if (pl[m] == kDropped) continue;
    float2 v = make_float2(y[m].x * wt[m], y[m].y * wt[m]);
    if (a.rot) v = make_float2(v.x * ro[m].x - v.y * ro[m].y, v.x * ro[m].y + v.y * ro[m].x);
    const uint32_t k = pl[m] & kPlaceMask;
    L.stage[k] = v;
    L.binof[k] = (uint16_t)(pl[m] >> kPlaceShift);
    mx = finite_absmax(mx, v);
  }
  __syncthreads();
  const uint32_t kept = a.ckept[chunk];
  for (uint32_t k = threadIdx.x; k < kept; k += kL1Threads)
    a.yrow[L.dl[L.binof[k]] + k] = L.stage[k];
  if (a.vmax) {
    // one atomic maximum per workgroup (non-negative floats order as their bits)
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) L.wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < kL1Threads / 64; ++w) mx = fmaxf(mx, L.wmax[w]);
      if (mx > 0.f) atomicMax(a.vmax, __float_as_uint(mx));
    }
  }
}

__global__ __launch_bounds__(kL1Threads) void to_rows_kernel(MoveArgs a) {
  __shared__ MoveLds L;
  to_rows_chunk(a, xcd_block(blockIdx.x, gridDim.x), L);
}

// Many jobs in one launch: block b works on chunk b - first[j] of the job j
// with first[j] <= b < first[j + 1].
__global__ __launch_bounds__(kL1Threads) void to_rows_batched_kernel(
    const MoveArgs* __restrict__ jobs, const uint32_t* __restrict__ first, int njobs) {
  __shared__ MoveLds L;
  const uint32_t b = (uint32_t)xcd_block(blockIdx.x, gridDim.x);
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid; else hi = mid - 1;
  }
  to_rows_chunk(jobs[lo], (int64_t)(b - first[lo]), L);
}

// out[i] = yrow[row-bin position of i] conj(rot[i]), 0 for dropped visibilities
__global__ __launch_bounds__(kL1Threads) void from_rows_kernel(
    const float2* __restrict__ yrow, const uint32_t* __restrict__ place,
    const uint32_t* __restrict__ delta, const uint32_t* __restrict__ ckept,
    const float2* __restrict__ rot, int64_t nvis, int nbins, float2* __restrict__ out) {
  __shared__ MoveLds L;
  const int64_t chunk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t first = chunk * kChunk;
  load_deltas(delta, chunk, nbins, L.dl);
  uint32_t pl[kPerThread];
#pragma unroll
  for (int m = 0; m < kPerThread; ++m) {
    const int64_t i = first + (int64_t)m * kL1Threads + threadIdx.x;
    pl[m] = i < nvis ? __builtin_nontemporal_load(place + i) : kDropped;
  }
#pragma unroll
  for (int m = 0; m < kPerThread; ++m)
    if (pl[m] != kDropped) L.binof[pl[m] & kPlaceMask] = (uint16_t)(pl[m] >> kPlaceShift);
  __syncthreads();
  // read in: consecutive lanes take consecutive records of the runs
  const uint32_t kept = ckept[chunk];
  for (uint32_t k = threadIdx.x; k < kept; k += kL1Threads)
    L.stage[k] = yrow[L.dl[L.binof[k]] + k];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kPerThread; ++m) {
    const int64_t i = first + (int64_t)m * kL1Threads + threadIdx.x;
    if (i >= nvis) break;
    float2 y = make_float2(0.f, 0.f);
    if (pl[m] != kDropped) {
      y = L.stage[pl[m] & kPlaceMask];
      if (rot) {
        const float2 ro = rot[i];
        y = make_float2(y.x * ro.x + y.y * ro.y, y.y * ro.x - y.x * ro.y);
      }
    }
    f32x2 t;
    t[0] = y.x;
    t[1] = y.y;
    __builtin_nontemporal_store(t, reinterpret_cast<f32x2*>(out + i));
  }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, grid_for(n), dim3(kThreads), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_zero_c64(float2* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_c64_kernel, grid_for(n), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

int64_t scan_tmp_size(int64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp,
                       hipStream_t s) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb < 1) return hipSuccess;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kThreads), 0, s, tmp, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

hipError_t launch_quantise_rows(const Coords& src, int64_t nvis, QuantGeom g, int rshift, int nbins,
                                uint32_t* rbin, uint2* qrec, uint32_t* chist, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  const int64_t nb = (nvis + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(quantise_rows_kernel, dim3((unsigned)nb), dim3(kL1Threads), 0, s, src, nvis, g,
                     rshift, nbins, rbin, qrec, chist);
  return hipGetLastError();
}

hipError_t launch_level1_counts(const uint32_t* chist, int64_t nvis, int nbins, uint32_t* gsum,
                                uint32_t* rowcount, hipStream_t s) {
  const int64_t nch = (nvis + kChunk - 1) / kChunk;
  const int ngroups = (int)((nch + kGroupChunks - 1) / kGroupChunks);
  if (ngroups == 0) return launch_fill_u32(rowcount, 0u, nbins + 1, s);
  hipLaunchKernelGGL(group_sums_kernel, dim3((unsigned)((nbins + 255) / 256), (unsigned)ngroups),
                     dim3(256), 0, s, chist, nch, nbins, ngroups, gsum);
  hipLaunchKernelGGL(group_scan_kernel, dim3((unsigned)nbins), dim3(256), 0, s, gsum, ngroups, nbins,
                     rowcount);
  return hipGetLastError();
}

hipError_t launch_chunk_deltas(const uint32_t* chist, const uint32_t* gsum,
                               const uint32_t* rowoff, int64_t nvis, int nbins, uint32_t* delta,
                               uint32_t* ckept, hipStream_t s) {
  const int64_t nch = (nvis + kChunk - 1) / kChunk;
  const int ngroups = (int)((nch + kGroupChunks - 1) / kGroupChunks);
  if (ngroups == 0) return hipSuccess;
  hipLaunchKernelGGL(chunk_deltas_kernel, dim3((unsigned)ngroups), dim3(kL1Threads), 0, s, chist,
                     gsum, rowoff, nch, nbins, ngroups, delta, ckept);
  return hipGetLastError();
}

hipError_t launch_pad_sizes(const uint32_t* rowcount, int nbins, int rshift, int ntx, int nty,
                            uint32_t* rowpad, hipStream_t s) {
  hipLaunchKernelGGL(pad_sizes_kernel, grid_for(nbins + 1), dim3(kThreads), 0, s, rowcount, nbins,
                     rshift, ntx, nty, rowpad);
  return hipGetLastError();
}

hipError_t launch_row_scatter(const uint32_t* rbin, const uint2* qrec, int64_t nvis, int nbins,
                              const uint32_t* chist, const uint32_t* delta, uint2* rrec,
                              uint32_t* place, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  const int64_t nb = (nvis + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(row_scatter_kernel, dim3((unsigned)nb), dim3(kL1Threads), 0, s, rbin, qrec, nvis,
                     nbins, chist, delta, rrec, place);
  return hipGetLastError();
}

hipError_t launch_row_sort(const uint32_t* rowcount, const uint32_t* rowoff,
                           const uint32_t* prowoff, const uint2* rrec, int rshift, int nbins,
                           int ntx, int nty, int tile_c, int O, int S, uint32_t zero_row,
                           uint32_t* perm, uint2* tdesc, SlotRec* krec, hipStream_t s) {
  // chunk length: two workgroups per CU when the tile arrays leave room, else one
  const int64_t nloc = (int64_t)ntx << rshift;
  constexpr int64_t kLds = 163840, kStatic = 256;
  int64_t chunk = (kLds / 2 - kStatic - 8 * nloc) / 16;
  if (chunk < 1024) chunk = (kLds - kStatic - 8 * nloc) / 16;
  chunk = std::min<int64_t>(chunk, 4096) & ~63LL;
  if (chunk < 64) return hipErrorInvalidValue;
  const int lds = (int)(8 * nloc + 16 * chunk);
  hipLaunchKernelGGL(bin_order_kernel, dim3(1), dim3(kSortThreads), 0, s, rowcount, nbins, perm);
  auto run = [&](auto kern) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipLaunchKernelGGL(kern, dim3(nbins), dim3(kSortThreads), lds, s, rowoff, prowoff, rrec, perm,
                       rshift, ntx, nty, O, S, zero_row, (int)chunk, tdesc, krec);
    return hipGetLastError();
  };
  switch (tile_c) {
    case 2: return run(&row_sort_kernel<2>);
    case 4: return run(&row_sort_kernel<4>);
    case 6: return run(&row_sort_kernel<6>);
    case 8: return run(&row_sort_kernel<8>);
    case 10: return run(&row_sort_kernel<10>);
    case 12: return run(&row_sort_kernel<12>);
    case 14: return run(&row_sort_kernel<14>);
    case 16: return run(&row_sort_kernel<16>);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dropped(const uint32_t* kept, int64_t nvis, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(dropped_kernel, dim3(1), dim3(64), 0, s, kept, nvis, out);
  return hipGetLastError();
}

hipError_t launch_vis_to_rows(const MoveArgs& a, hipStream_t s) {
  if (a.nvis == 0) return hipSuccess;
  const int64_t nb = (a.nvis + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(to_rows_kernel, dim3((unsigned)nb), dim3(kL1Threads), 0, s, a);
  return hipGetLastError();
}

int64_t move_blocks(int64_t nvis) { return (nvis + kChunk - 1) / kChunk; }

hipError_t launch_vis_to_rows_batched(const MoveArgs* jobs, const uint32_t* first, int njobs,
                                      int64_t total_blocks, hipStream_t s) {
  if (total_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(to_rows_batched_kernel, dim3((unsigned)total_blocks), dim3(kL1Threads), 0, s,
                     jobs, first, njobs);
  return hipGetLastError();
}

hipError_t launch_vis_from_rows(const float2* yrow, const float2* rot, const uint32_t* place,
                                const uint32_t* delta, const uint32_t* ckept, int64_t nvis,
                                int nbins, float2* out, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  const int64_t nb = (nvis + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(from_rows_kernel, dim3((unsigned)nb), dim3(kL1Threads), 0, s, yrow, place, delta,
                     ckept, rot, nvis, nbins, out);
  return hipGetLastError();
}

hipError_t launch_rotation(const Coords& src, int64_t nvis, QuantGeom g, float2* rot,
                           hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(rotation_kernel, grid_for(nvis), dim3(kThreads), 0, s, src, nvis, g, rot);
  return hipGetLastError();
}

hipError_t launch_item_counts(const uint2* tdesc, int ntx, int nty, int r8, int item_slots,
                              uint32_t* nit, hipStream_t s) {
  hipLaunchKernelGGL(item_counts_kernel, grid_for(8 * (int64_t)r8 + 1), dim3(kThreads), 0, s, tdesc,
                     ntx, nty, r8, (uint32_t)item_slots, nit);
  return hipGetLastError();
}

hipError_t launch_items(const uint2* tdesc, const uint32_t* itoff, int ntx, int nty, int r8,
                        int item_slots, int4* items, hipStream_t s) {
  hipLaunchKernelGGL(items_kernel, grid_for((int64_t)ntx * nty), dim3(kThreads), 0, s, tdesc,
                     itoff, ntx, nty, r8, (uint32_t)item_slots, items);
  return hipGetLastError();
}

hipError_t launch_job_prefix(const GridArgs* jobs, int njobs, uint32_t* first, uint32_t* counter,
                             hipStream_t s) {
  hipLaunchKernelGGL(job_prefix_kernel<GridArgs>, dim3(1), dim3(64), 0, s, jobs, njobs, first,
                     counter);
  return hipGetLastError();
}

hipError_t launch_job_prefix(const DegridArgs* jobs, int njobs, uint32_t* first, uint32_t* counter,
                             hipStream_t s) {
  hipLaunchKernelGGL(job_prefix_kernel<DegridArgs>, dim3(1), dim3(64), 0, s, jobs, njobs, first,
                     counter);
  return hipGetLastError();
}

hipError_t launch_bins_export(const uint2* rrec, const uint32_t* place, const uint32_t* delta,
                              int nbins, int64_t nvis, int tile_c, int ntx, int32_t* out,
                              hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(bins_export_kernel, grid_for(nvis), dim3(kThreads), 0, s, rrec, place, delta,
                     nbins, nvis, tile_c, ntx, out);
  return hipGetLastError();
}

}  // namespace sepw
