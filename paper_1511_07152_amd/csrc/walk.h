// Wave-uniform walk over the tiles and slot chunks of one work item.
//
// A work item is a contiguous range of tile slots [first, end) of one row of
// tiles.  The slots of a row are laid out tile by tile (row-major tile order),
// each tile padded to a multiple of 4 slots, and tdesc[tile] = (first slot,
// first slot + count) describes every tile, empty ones included (first == end).
// The walk keeps 64 descriptors of the row in registers (lane t holds tile
// base + t) and steps through the non-empty ones with a ballot mask, so moving
// to the next tile costs no memory round trip except once per 64 tiles.
#pragma once

#include "internal.h"

namespace sepw {

__device__ inline int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline int round4i(int n) { return (n + 3) & ~3; }

// Slot record load marked non-temporal: records are read once per launch, and
// the hint keeps them from displacing grid, W V and result lines in the L2
// (measured: gridding 2.72 -> 2.67 ms, degridding 3.23 -> 3.21 ms at array
// scale).
__device__ inline SlotRec load_rec(const SlotRec* p) {
  const int* q = reinterpret_cast<const int*>(p);
  return SlotRec{__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1),
                 __builtin_nontemporal_load(q + 2)};
}

struct TileWalk {
  const uint2* row;   // descriptors of the row of tiles
  int ntx;            // tiles in the row
  int base;           // tile column held by lane 0
  uint2 d;            // this lane's descriptor (tile base + lane)
  uint64_t live;      // non-empty tiles of the batch not yet visited (bit = lane)
  int tx;             // current tile column

  __device__ void load(int b, int lane) {
    base = b;
    d = (b + lane < ntx) ? row[b + lane] : make_uint2(0u, 0u);
    live = __ballot(d.y > d.x);
  }
  // start at tile column t, which must be non-empty
  __device__ void start(const uint2* r, int n, int t, int lane) {
    row = r;
    ntx = n;
    load(t, lane);
    live &= ~1ull;
    tx = t;
  }
  __device__ int first_slot() const {
    return uniform(__builtin_amdgcn_readlane((int)d.x, tx - base));
  }
  __device__ int real_end() const {
    return uniform(__builtin_amdgcn_readlane((int)d.y, tx - base));
  }
  __device__ int padded_end() const {
    const int f = first_slot();
    return f + round4i(real_end() - f);
  }
  // Move to the next non-empty tile of the row.  Returns false (and leaves the
  // walk unchanged) if the row has none; the batch reloads are bounded by the
  // row length, so the loop always ends.
  __device__ bool next(int lane) {
    while (live == 0ull) {
      if (base + 64 >= ntx) return false;
      load(base + 64, lane);
    }
    const int l = __builtin_ctzll(live);
    live &= live - 1ull;
    tx = base + l;
    return true;
  }
};

// Grid-stride assignment of work items to the waves of a launch: returns this
// wave's first item and sets the stride between its items.  (Renumbering the
// workgroups per XCD, as the movement passes do, was measured slower here.)
__device__ inline int wave_items(int waves_per_block, int* stride) {
  *stride = gridDim.x * waves_per_block;
  return blockIdx.x * waves_per_block + (int)(threadIdx.x >> 6);
}

// Work items are kept in 8 lists, list q holding the items of the rows of
// tiles r with r % 8 == q (rows interleaved, so the lists carry similar work),
// list q = items [lists[q r8], lists[(q + 1) r8]).  A wave pulls items from the
// list of the XCD it runs on (hardware register XCC_ID; each XCD has its own
// L2, and all items of a row then write that row's row-bin data through one
// L2) with one atomic counter per list, and once that list is empty from the
// other lists in turn, so every item is taken exactly once whatever XCD a
// workgroup lands on.  The counters must be zero at launch; launches use only
// as many workgroups as can be resident, so that few waves find the lists
// empty.
__device__ inline int xcd_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7;   // hwreg(XCC_ID, 0, 4)
}

// Claiming work.  Atomics on one cache line are serialised where they are
// performed (measured about 11 ns apart at array scale): with the eight list
// counters in one line, claims queued for tens of microseconds each and set
// the kernels' pace.  The counters therefore sit kCtrStride dwords apart,
// each in a cache line of its own.  A claim may take kClaim consecutive items;
// one is best here (measured: claims of 2 or 4 items put more rows of tiles in
// flight per L2 and made gridding and degridding slower).
constexpr int kClaim = 1;

// Items [0, n) from one counter (zero at launch), kClaim per claim.
template <class F>
__device__ inline void for_counter(uint32_t* __restrict__ ctr, uint32_t n, int lane, F&& body) {
  while (true) {
    int g = 0;
    if (lane == 0) g = (int)atomicAdd(ctr, (uint32_t)kClaim);
    const uint32_t g0 = (uint32_t)uniform(__shfl(g, 0, 64));
    if (g0 >= n) break;
    const uint32_t e = min(g0 + (uint32_t)kClaim, n);
    for (uint32_t i = g0; i < e; ++i) body(i);
  }
}

// Items [0, n) in eight contiguous blocks, block q claimed through counter q
// (kCtrStride dwords apart, all zero at launch): a wave takes the block of
// its XCD first, then the others in turn, so the claims of a launch spread
// over eight cache lines and each XCD works on consecutive items while its
// block lasts.  Every item is taken exactly once.
template <class F>
__device__ inline void for_blocks8(uint32_t* __restrict__ ctr, uint32_t n, int lane, F&& body) {
  const int x = uniform(xcd_id());
  const uint32_t per = (n + 7) / 8;
  for (int l = 0; l < 8; ++l) {
    const int q = (x + l) & 7;
    uint32_t* c = ctr + q * kCtrStride;
    const uint32_t lo = min((uint32_t)q * per, n), hi = min(lo + per, n);
    // a plain read first: blocks that are already used up cost no atomic
    if (lo + __atomic_load_n(c, __ATOMIC_RELAXED) >= hi) continue;
    while (true) {
      uint32_t k = 0;
      if (lane == 0) k = atomicAdd(c, (uint32_t)kClaim);
      k = (uint32_t)uniform((int)__shfl((int)k, 0, 64));
      if (lo + k >= hi) break;
      const uint32_t e = min(lo + k + (uint32_t)kClaim, hi);
      for (uint32_t i = lo + k; i < e; ++i) body(i);
    }
  }
}

template <class F>
__device__ inline void for_items(const uint32_t* __restrict__ lists, int r8,
                                 uint32_t* __restrict__ ctr, int lane, F&& body) {
  const int x = uniform(xcd_id());
  for (int l = 0; l < 8; ++l) {
    const int q = (x + l) & 7;
    uint32_t* c = ctr + q * kCtrStride;
    const int lo = uniform((int)lists[q * r8]), hi = uniform((int)lists[(q + 1) * r8]);
    // a plain read first: lists that are already used up cost no atomic
    if (lo + (int)__atomic_load_n(c, __ATOMIC_RELAXED) >= hi) continue;
    while (true) {
      int n = 0;
      if (lane == 0) n = (int)atomicAdd(c, (uint32_t)kClaim);
      n = uniform(__shfl(n, 0, 64));
      if (lo + n >= hi) break;
      const int e = min(lo + n + kClaim, hi);
      for (int i = lo + n; i < e; ++i) body(i);
    }
  }
}

// Slot records of a work item, one slot per lane, in batches of 64 from the
// item's first slot s0: batches a and a + 1 have arrived, a + 2 is in flight.
// A batch is one coalesced 12-byte load per lane (one vector-memory
// instruction for 64 records, instead of one per chunk; the texture-address
// unit, which spends about the same time on any 64-lane instruction, bounds
// the degridding kernels).  rec_key() hands each lane the record of slot
// c0 + col of a chunk [c0, c0 + 16) with ds_bpermute.
typedef int i32x3u __attribute__((ext_vector_type(3), aligned(4)));

struct RecBatch {
  SlotRec ra, rb, rc;
  int a;
};

__device__ inline SlotRec rec_batch_load(const SlotRec* krec, int s0, int last, int j, int lane) {
  const i32x3u v = __builtin_nontemporal_load(
      reinterpret_cast<const i32x3u*>(krec + min(s0 + 64 * j + lane, last)));
  return SlotRec{v[0], v[1], v[2]};
}

__device__ inline void rec_batch_start(RecBatch& bt, const SlotRec* krec, int s0, int last,
                                       int lane) {
  bt.a = 0;
  bt.ra = rec_batch_load(krec, s0, last, 0, lane);
  bt.rb = rec_batch_load(krec, s0, last, 1, lane);
  bt.rc = rec_batch_load(krec, s0, last, 2, lane);
}

// Record of slot c0 + col (c0 >= s0, non-decreasing from call to call).
__device__ inline SlotRec rec_key(RecBatch& bt, const SlotRec* krec, int s0, int last, int c0,
                                  int col, int lane) {
  const int r = c0 - s0;
  while ((r >> 6) > bt.a) {
    bt.ra = bt.rb;
    bt.rb = bt.rc;
    bt.a += 1;
    bt.rc = rec_batch_load(krec, s0, last, bt.a + 2, lane);
  }
  const int off = r & 63;   // the chunk is window [off, off + 16) of batches a, a + 1
  SlotRec src = bt.ra;
  if (off > 48) {
    // the chunk reaches into batch a + 1: lanes below off hold its slots
    const bool nb = lane < off;
    src.x = nb ? bt.rb.x : src.x;
    src.y = nb ? bt.rb.y : src.y;
    src.z = nb ? bt.rb.z : src.z;
  }
  const int addr = ((off + col) & 63) << 2;
  return SlotRec{__builtin_amdgcn_ds_bpermute(addr, src.x), __builtin_amdgcn_ds_bpermute(addr, src.y),
                 __builtin_amdgcn_ds_bpermute(addr, src.z)};
}

// Position of one chunk of at most 16 slots inside one tile of a work item.
struct ChunkPos {
  int c0;    // first slot
  int pe;    // end of the tile's slots inside the item (padded, multiple of 4)
  int re;    // end of the tile's real visibilities inside the item
  int tx;    // tile column
  bool ok;   // false past the end of the item (position then repeats the last chunk)
};

// Chunk following p: the next 16 slots of the same tile, else the first chunk
// of the next non-empty tile.
__device__ inline ChunkPos next_chunk(const ChunkPos& p, TileWalk& tw, int s_end, int lane) {
  ChunkPos n = p;
  if (!p.ok) return n;
  if (p.c0 + 16 < p.pe) {
    n.c0 = p.c0 + 16;
    return n;
  }
  if (p.pe >= s_end || !tw.next(lane)) {
    n.ok = false;
    return n;
  }
  n.c0 = tw.first_slot();
  n.pe = min(tw.padded_end(), s_end);
  n.re = min(tw.real_end(), s_end);
  n.tx = tw.tx;
  return n;
}

}  // namespace sepw
