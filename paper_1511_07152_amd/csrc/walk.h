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
// wave's first item and sets the stride between its items.  (Giving each XCD
// a contiguous band of rows of tiles instead was measured slower.)
__device__ inline int wave_items(int waves_per_block, int* stride) {
  *stride = gridDim.x * waves_per_block;
  return blockIdx.x * waves_per_block + (int)(threadIdx.x >> 6);
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
