// Internal types and launchers of the separable W-projection library.
// Not part of the ABI; see include/sepw.h for the public contract.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>
#include <stdint.h>

#include <vector>

#include "sepw.h"

namespace sepw {

constexpr uint32_t kDropped = 0xFFFFFFFFu;
constexpr int kRegion = 16;        // MFMA tile region edge (cells): core + S - 1
constexpr int kMaxSupport = 15;    // S <= kRegion - 1 on the tiled MFMA path
constexpr int kMaxCorrRank = 8;    // separable terms of a factored correction table
constexpr int kG16Border = 16;     // zero border (cells) of the FP16 degridding operand grid
// Supports 15 < S <= kMaxWideSupport take the per-visibility path (wide.hip):
// plans keep the quantiser and the level-1 row bins with tiles of
// kWideRegion + 1 - S cells, but no tile slots or work lists.
constexpr int kWideRegion = 32;
constexpr int kMaxWideSupport = 31;
__host__ __device__ inline bool wide_support(int S) { return S > kMaxSupport; }
constexpr int kItemMaxVis = 1024;  // default slots per gridding work item (a slice of a tile row)
constexpr int kDegridItemSlots = 224;  // default slots per degridding work item
constexpr int kItemMinSlots = 64;  // range of the tunable item length
constexpr int kItemMaxSlots = 8192;
constexpr int kMaxRowBins = 4096;  // level-1 sort bins (rows of tiles, possibly grouped)
constexpr int kL1Chunk = 10240;    // visibilities per workgroup in the level-1 passes
constexpr int kMaxSlices = 4096;   // w-slices of the W-stacking hybrid
constexpr int kDensityBins = 16384; // fine w bins of the density-adapted slice edges
constexpr int kGroupChunks = 8;    // level-1 chunks per group of the run-offset scan
// placement word of a kept visibility: row bin << kPlaceShift | its position in
// its chunk's bin-ordered staging (kDropped for dropped visibilities)
constexpr int kPlaceShift = 14;
constexpr uint32_t kPlaceMask = (1u << kPlaceShift) - 1u;
static_assert(kL1Chunk <= (1 << kPlaceShift), "chunk positions must fit the placement word");
static_assert(((uint64_t)kMaxRowBins << kPlaceShift) < 0xFFFFFFFFull,
              "placement words must stay below kDropped");
constexpr int kTargetRowBins = 2048;
constexpr int kCorrMaxD = 64;      // correction table: max tap offset |d| (1/O_c cells) + 1
constexpr int kCtrStride = 64;     // dwords between the 8 work-list counters (own cache lines)

// Padded tables: row length L = 32 - S holds the S taps of a table row at
// offsets c - 1 .. c - 2 + S (c = 17 - S is the tile size) and zeros around
// them, so that tap index col - ox for col in [0, 16) and ox in [0, c) is
// always a valid, predicate-free offset: padded[row][c - 1 + col - ox].
__host__ __device__ inline int padded_len(int S) { return 32 - S; }

// Running maximum of |Re| and |Im| over finite parts only, for the FP16
// form's per-call power-of-two scale: a NaN or Inf value does not set the
// scale (it stays non-finite in the products it enters).
__device__ inline float finite_absmax(float mx, float2 v) {
  const float a = fabsf(v.x), b = fabsf(v.y);
  if (a <= 3.4028235e38f) mx = fmaxf(mx, a);
  if (b <= 3.4028235e38f) mx = fmaxf(mx, b);
  return mx;
}
constexpr int kMaxRowTiles = 16384; // tiles per level-1 bin (level-2 sort in LDS)

// Geometry shared by the binning kernels; all FP64 values are used exactly as
// stored (no recomputation on the device), so host and device agree bit for bit.
struct QuantGeom {
  double fov;        // multiply u by this ...
  double half_n;     // ... then add N/2
  double over;       // oversampling factor O as a double (exact)
  double w_lo;
  double inv_dw;     // P / (w_hi - w_lo), computed once on the host
  int32_t N, S, O, P;
  int32_t lo;        // log2 O
  int32_t tile_c, ntx;
  int32_t facet;
  double l0, m0, n0; // facet centre and n0 = sqrt(1 - l0^2 - m0^2)
};

struct Kernels {
  sepw_kernel_params prm;
  int N, S, O, P;
  double fov, w_lo, w_hi, inv_dw;
  double a_u, b_u, a_v, b_v;
  bool facet;
  double l0, m0, n0;
  double taper_width;
  float2* tab_u = nullptr;     // [P][O][S] complex64
  float2* tab_v = nullptr;     // == tab_u when both axes share coefficients
  double* c1 = nullptr;        // taper at the N pixel positions
  float2* pad_u = nullptr;     // [P][O][L] zero-padded u / v tables
  float2* pad_v = nullptr;
  float2* pad_su = nullptr;    // the same with tap s times (-1)^s (degridding from the FFT)
  float2* pad_sv = nullptr;
  // precision form (FP16 / BF16): 16-bit padded tables for degridding
  // (gridding uses the FP32 padded tables)
  uint32_t* lp_u = nullptr;
  uint32_t* lp_v = nullptr;
  // 16-bit degridding: the grid as MFMA operands, (N + 2 kG16Border)^2 16-bit
  // (Re, Im) pairs with a zero border (BF16: high parts, then low parts)
  uint32_t* g16 = nullptr;
  float2* scratch = nullptr;   // N*N complex64 work grid (degridding, real-output gridding)
  int tab_len = 0;             // entries of one padded table (P O L)
  int lds_bytes = 0;           // > 0: the FP32 kernels stage the tables in LDS
  int lds_bytes_lp = 0;        // > 0: the 16-bit degridding kernels stage their tables in LDS
  int n_cu = 0;                // compute units of the device
  hipfftHandle fft = 0;
  bool fft_ok = false;
  bool borrowed = false;       // fft and scratch belong to another kernels object
  uint64_t generation = 0;     // bumped when the tables are regenerated
  // correction table F_w - F~_w (0 support = none): [P][Oc][Oc][Sc][Sc] complex64,
  // taps (sv, su) with su fastest; corr_tmp = FP64 work space of its generation
  int corr_S = 0, corr_O = 0, corr_nkb = 0;
  float2* corr = nullptr;
  double* corr_tmp = nullptr;
  // the same correction as corr_rank separable terms (FP32 kernels; -1: the
  // correction passes walk the table itself): padded u / v tables of term r,
  // plain and with tap signs (-1)^s, and the LDS bytes of one term's pair
  bool corr_terms = true;      // factor the table when it is (re)generated
  int corr_rank = -1;
  float2* ck_u[kMaxCorrRank] = {};
  float2* ck_v[kMaxCorrRank] = {};
  float2* ck_su[kMaxCorrRank] = {};
  float2* ck_sv[kMaxCorrRank] = {};
  int ck_lds = 0;
  int lds_max = 0;             // LDS bytes one workgroup may use
};

// Tile slot record: padded-table bases of the visibility's u and v taps (tap
// of region column x at base + x) and the row-bin position of its W V.  Twelve
// bytes, loaded as three dwords.  Bit 31 of z holds the parity of
// cell_u + cell_v (the sign (-1)^(cu+cv) that, with the tap signs (-1)^(s+t)
// of the signed tables, makes up the grid-side checkerboard (-1)^(x+y) of the
// centred FFT); rec_pos() is the row-bin position alone.
struct SlotRec {
  int x, y, z;
};
constexpr uint32_t kRecSign = 0x80000000u;
__host__ __device__ inline int rec_pos(const SlotRec& r) { return r.z & 0x7FFFFFFF; }

// Work items of at most `slots` tile slots of one row of tiles, in 8 lists by
// row % 8 (list q = items [itoff[q r8], itoff[(q + 1) r8])).
struct WorkList {
  int slots = kItemMaxVis;     // slots per item (multiple of 4)
  int64_t max_items = 0;       // capacity of items (for the shortest length used so far)
  uint32_t* nit = nullptr;     // [8 r8 + 1] items per row, row r at (r % 8) r8 + r / 8
  uint32_t* itoff = nullptr;   // [8 r8 + 1] exclusive scan of nit
  int4* items = nullptr;       // [max_items] (tile row, first slot, end slot, tile column)
};

struct BatchScratch;   // job tables of the batched launches (api.cpp)

struct Plan {
  Kernels* K = nullptr;
  uint64_t generation = 0;      // K->generation the bins were made for
  int64_t nvis = 0;
  int64_t capacity = 0;         // visibilities the buffers were sized for
  int64_t pcap = 0;             // tile slots the slot-order buffers were sized for
  int tile_c = 0, ntx = 0, nty = 0;
  int64_t ntiles = 0;
  int rshift = 0, nbins = 0;    // level-1 sort: row bin = tile row >> rshift
  uint32_t* rbin = nullptr;     // [nvis] row bin or kDropped (caller order)
  uint2* qrec = nullptr;        // [nvis] packed bins (caller order)
  uint32_t* chist = nullptr;    // [chunks][nbins] level-1 histogram of each chunk
  uint32_t* gsum = nullptr;     // [nbins][groups] per-group sums, then their exclusive scan
  uint32_t* rowcount = nullptr; // [nbins + 1] level-1 histogram
  uint32_t* rowoff = nullptr;   // [nbins + 1] its exclusive scan; rowoff[nbins] = kept count
  uint32_t* delta = nullptr;    // [chunks][nbins] row-bin position of a chunk's run minus
                                // the run's start in the chunk's staging
  uint32_t* ckept = nullptr;    // [chunks] kept visibilities per chunk
  uint32_t* rowpad = nullptr;   // [nbins + 1] tile slots reserved per row bin
  uint32_t* prowoff = nullptr;  // [nbins + 1] exclusive scan of rowpad
  uint32_t* binperm = nullptr;  // [nbins] row bins by decreasing count (level-2 order)
  uint2* rrec = nullptr;        // [nvis] records sorted by row bin
  uint32_t* place = nullptr;    // [nvis] placement word per caller index (or kDropped)
  float2* yrow = nullptr;       // [capacity + 1] row-bin-order W V (grid) or results (degrid);
                                // yrow[capacity] stays 0 (the padding slots point there)
  SlotRec* krec = nullptr;         // [pcap] per tile slot: padded-table bases (u, v) relative to
                                // the tile and the row-bin position of its W V
  uint2* tdesc = nullptr;       // [ntiles] (first slot, first slot + count) per tile
  float2* rot = nullptr;        // [nvis] facet phase rotation, caller order
  int r8 = 0;                   // rows of tiles per work list: ceil(nty / 8)
  uint32_t* qctr = nullptr;     // [8 kCtrStride] work-list counters of a launch, kCtrStride apart
  uint32_t* lp_max = nullptr;   // [2] FP16 scales of the current call: max |Re, Im| of W V
                                // (gridding) and of the grid (degridding), as float bits
  WorkList gl;                  // gridding work items
  WorkList dl;                  // degridding work items (shorter: fewer rows of results in flight)
  uint32_t* scan_tmp = nullptr; // block partials for the scans
  int64_t scan_tmp_len = 0;
  // batched calls led by this plan (plans[0]) keep their job tables here
  BatchScratch* batch = nullptr;
  int blocks_per_cu = 8;        // persistent batched launch width (set by the autotuner)
};

// Workgroups of a launch are dispatched to the 8 XCDs in turn (workgroup b on
// XCD b % 8).  xcd_block(b, nb) renumbers them so that each XCD takes one
// contiguous range of [0, nb): neighbouring chunks, whose runs in the row-bin
// array are adjacent, then meet in one L2 and their partial cache lines merge.
// A bijection of [0, nb) whatever the actual placement.
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b & 7, j = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + j;
}

// packed record: x = cell_u | cell_v << 16 ; y = fi_u | fi_v << 8 | plane << 16
__host__ __device__ inline uint2 pack_rec(int cu, int fu, int cv, int fv, int k) {
  return make_uint2((uint32_t)cu | ((uint32_t)cv << 16),
                    (uint32_t)fu | ((uint32_t)fv << 8) | ((uint32_t)k << 16));
}

// ---- correction table as separable terms (corr_factor.cpp) ----
// Factors C [P][Oc][Oc][Sc][Sc] (FP32) into at most max_rank separable terms
// per plane with every residual entry within tol_rel of C's largest entry and
// writes the terms' u and v tables ([rank][P][O][S] complex64, zero rows for
// planes of lower rank; *shared: the terms are symmetric and tv equals tu).
// Returns the rank (0 for an all-zero table), or -1 when max_rank terms do
// not reach the tolerance.
int factor_corr_table(const float2* C, int P, int O, int S, int Oc, int Sc, int max_rank,
                      double tol_rel, std::vector<float2>* tu, std::vector<float2>* tv,
                      bool* shared);

// ---- host-side PSWF (pswf.cpp) ----
// Legendre coefficients d_j (degree 2j, normalised Legendre basis) of psi_0(c, x)
// and psi_0(c, 0) from the same series.  Returns the number of coefficients.
int pswf_coefficients(double c, double* d, int max_terms, double* psi_at_0);

// Visibility coordinates in wavelengths, caller order: either three arrays
// (u[i], v[i], w[i]) or, channel-shared, rows of metres uvw[row][3] with
// visibility i = row * nchan + ch at u = u_m * (freq[ch] / c) (one IEEE
// division, then one IEEE multiplication per coordinate).
constexpr double kLightSpeed = 299792458.0;   // m/s
struct Coords {
  const double* u = nullptr;
  const double* v = nullptr;
  const double* w = nullptr;
  const double* uvw = nullptr;    // channel-shared rows (metres), or null
  const double* freq = nullptr;   // [nchan] Hz
  int64_t nchan = 1;
};

__device__ inline void coords_at(const Coords& c, int64_t i, double& u, double& v, double& w) {
  if (c.uvw) {
    const int64_t row = i / c.nchan;
    const double s = __ddiv_rn(c.freq[i - row * c.nchan], kLightSpeed);
    u = __dmul_rn(c.uvw[3 * row], s);
    v = __dmul_rn(c.uvw[3 * row + 1], s);
    w = __dmul_rn(c.uvw[3 * row + 2], s);
  } else {
    u = c.u[i];
    v = c.v[i];
    w = c.w[i];
  }
}

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_taper(const double* d_coef, int ncoef, double norm, int N, double* c1, hipStream_t s);
hipError_t launch_ones(double* c1, int N, hipStream_t s);
hipError_t launch_tables(const double* c1, int N, double fov, int P, int O, int S,
                         double w_lo, double w_hi, double a, double b, float2* out, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_zero_c64(float2* p, int64_t n, hipStream_t s);
// two-level counting sort by tile (rows of tiles, then tiles within a row bin);
// chist[chunk][bin] = level-1 histogram of each chunk of kL1Chunk visibilities
hipError_t launch_quantise_rows(const Coords& src, int64_t nvis, QuantGeom g, int rshift, int nbins,
                                uint32_t* rbin, uint2* qrec, uint32_t* chist, hipStream_t s);
// rowcount[bin] = kept visibilities per row bin (rowcount[nbins] = 0); gsum =
// [nbins][groups] exclusive scan over the chunk groups of each bin
hipError_t launch_level1_counts(const uint32_t* chist, int64_t nvis, int nbins, uint32_t* gsum,
                                uint32_t* rowcount, hipStream_t s);
// delta[chunk][bin] and ckept[chunk] from the histograms, group scan and rowoff
hipError_t launch_chunk_deltas(const uint32_t* chist, const uint32_t* gsum,
                               const uint32_t* rowoff, int64_t nvis, int nbins, uint32_t* delta,
                               uint32_t* ckept, hipStream_t s);
// rowpad[b] = slots reserved for row bin b (count + padding room, multiple of 4)
hipError_t launch_pad_sizes(const uint32_t* rowcount, int nbins, int rshift, int ntx, int nty,
                            uint32_t* rowpad, hipStream_t s);
// level-1 placement: records in row-bin order, placement word per visibility
hipError_t launch_row_scatter(const uint32_t* rbin, const uint2* qrec, int64_t nvis, int nbins,
                              const uint32_t* chist, const uint32_t* delta, uint2* rrec,
                              uint32_t* place, hipStream_t s);
// zero_row: row-bin position the padding slots point to (a W V that stays 0);
// perm: [nbins] scratch for the order in which the row bins are sorted
hipError_t launch_row_sort(const uint32_t* rowcount, const uint32_t* rowoff,
                           const uint32_t* prowoff, const uint2* rrec, int rshift, int nbins,
                           int ntx, int nty, int tile_c, int O, int S, uint32_t zero_row,
                           uint32_t* perm, uint2* tdesc, SlotRec* krec, hipStream_t s);
// caller-order W V (times the facet rotation) -> row-bin order
struct MoveArgs {
  const float2* vis;
  const float* weight;      // may be null (all 1)
  const float2* rot;        // may be null
  const uint32_t* place;
  const uint32_t* delta;
  const uint32_t* ckept;
  float2* yrow;
  int64_t nvis;
  int nbins;
  uint32_t* vmax;           // may be null: atomic maximum of max |Re, Im| of the placed
                            // W V (float bits), for the FP16 gridding scale
};
hipError_t launch_vis_to_rows(const MoveArgs& a, hipStream_t s);
// workgroups of the movement pass for nvis visibilities
int64_t move_blocks(int64_t nvis);
// all jobs in one launch: first[j] = first workgroup of job j (device, njobs + 1 entries)
hipError_t launch_vis_to_rows_batched(const MoveArgs* jobs, const uint32_t* first, int njobs,
                                      int64_t total_blocks, hipStream_t s);
// row-bin-order results -> caller order, rotation undone (dropped visibilities get 0)
hipError_t launch_vis_from_rows(const float2* yrow, const float2* rot, const uint32_t* place,
                                const uint32_t* delta, const uint32_t* ckept, int64_t nvis,
                                int nbins, float2* out, hipStream_t s);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s);
int64_t scan_tmp_size(int64_t n);
hipError_t launch_rotation(const Coords& src, int64_t nvis, QuantGeom g, float2* rot,
                           hipStream_t s);
// work items: slices of <= item_slots slots of each row of tiles
// per-row item counts in list order (nit[(r % 8) r8 + r / 8]) and the items in that order
hipError_t launch_item_counts(const uint2* tdesc, int ntx, int nty, int r8, int item_slots,
                              uint32_t* nit, hipStream_t s);
hipError_t launch_items(const uint2* tdesc, const uint32_t* itoff, int ntx, int nty, int r8,
                        int item_slots, int4* items, hipStream_t s);
// W-stacking hybrid (wstack.hip): slice partition, movement and image phase
// edges: null for uniform slices (w_lo, inv_ds), else ns + 1 increasing edges
hipError_t launch_slice_count(const double* w, int64_t nvis, double w_lo, double inv_ds, int ns,
                              const double* edges, uint32_t* count, hipStream_t s);
hipError_t launch_slice_scatter(const double* u, const double* v, const double* w, int64_t nvis,
                                double w_lo, double inv_ds, int ns, const double* edges,
                                const double* centre, uint32_t* cursor, uint32_t* order,
                                double* us, double* vs, double* ws, hipStream_t s);
// counts[b] += finite w in bin b of nfine (<= kDensityBins) uniform bins of [w_lo, w_hi]
hipError_t launch_w_hist(const double* w, int64_t nvis, double w_lo, double inv, int nfine,
                         uint32_t* counts, hipStream_t s);
hipError_t launch_slice_gather(const float2* vis, const float* weight, const uint32_t* order,
                               int64_t nvis, float2* out, hipStream_t s);
hipError_t launch_slice_return(const float2* in, const uint32_t* order, int64_t nvis, float2* out,
                               hipStream_t s);
// out (+)= in exp(sign 2 pi i w_s (n - 1)) over the N x N pixels, times the
// image correction (-1)^(p+q) n^npow / (c1[p] c1[q]) when c1 is not null
hipError_t launch_slice_phase(const float2* in, float2* out, int N, double fov, double w_s,
                              int sign, bool accumulate, const double* c1, int npow,
                              hipStream_t s);

// W snapshots (wsnap.hip): plane fit and residual w, reprojection and its transpose
hipError_t launch_snap_fit(const double* u, const double* v, const double* w, const int64_t* range,
                           const int* snap, const int* first, int nblocks, int ns, double* part,
                           double2* d0, double* wr, unsigned long long* maxbits, hipStream_t s);
hipError_t launch_snap_reproject(const float2* in, float2* out, int N, double fov, double du,
                                 double dv, bool accumulate, hipStream_t s);
// out = the transposed reprojection of X n^npow (written in full), then,
// when c1 is not null, times the image correction before the FFT,
// (-1)^(p+q) / (c1[p] c1[q])
hipError_t launch_snap_reproject_adjoint(const float2* X, float2* out, int N, double fov, double du,
                                         double dv, int npow, const double* c1, hipStream_t s);
hipError_t launch_snap_npow(float2* out, int N, double fov, int npow, hipStream_t s);

// *out = nvis - *kept, one thread
hipError_t launch_dropped(const uint32_t* kept, int64_t nvis, int64_t* out, hipStream_t s);
hipError_t launch_bins_export(const uint2* rrec, const uint32_t* place, const uint32_t* delta,
                              int nbins, int64_t nvis, int tile_c, int ntx, int32_t* out,
                              hipStream_t s);

// Arguments shared by the gridding and degridding kernels.  Work item it =
// items[it] = (tile row, first slot, end slot, tile column of the first slot);
// the slots of a row of tiles are contiguous, tile by tile, each tile padded
// to a multiple of 4 slots.
struct GridArgs {
  const int4* items;
  const uint32_t* nitems;   // device count of items
  const uint32_t* lists;    // work lists (itoff of the plan), r8 rows per list
  int r8;
  uint32_t* qctr;           // list counters, zero at launch
  const uint2* tdesc;       // per tile (first slot, first slot + count)
  const SlotRec* krec;      // per slot (u base, v base, row-bin position)
  const float2* yrow;       // W V in row-bin order
  const float2* tab_u;      // padded tables
  const float2* tab_v;
  int tab_len;              // entries of one padded table (P O L)
  int N, ntx;
  int checker;              // apply (-1)^(x+y) for the centred FFT
  float2* grid;
};

struct DegridArgs {
  const int4* items;
  const uint32_t* nitems;
  const uint32_t* lists;    // work lists (itoff of the plan), r8 rows per list
  int r8;
  uint32_t* qctr;           // list counters, zero at launch
  const uint2* tdesc;
  const SlotRec* krec;
  const float2* grid;
  const float2* tab_u;      // padded tables; with checker, the signed tables (tap s times (-1)^s)
  const float2* tab_v;
  int tab_len;
  int N, ntx;
  int checker;              // the grid comes from the centred FFT: results times (-1)^(cu+cv)
  float2* yrow;             // results in row-bin order (padding slots are not written)
  int accum = 0;            // add the results to yrow instead of storing them
};

// Precision form (FP16 / BF16).  Gridding reads the FP32 padded tables;
// degridding reads 16-bit padded tables holding the taps as (Re, Im) pairs
// (FP16, or for BF16 the high parts followed by the low parts at + tab_len).
struct GridArgsLp {
  const int4* items;
  const uint32_t* nitems;
  const uint2* tdesc;
  const SlotRec* krec;
  const float2* yrow;
  const float2* tab_u;      // FP32 padded tables
  const float2* tab_v;
  int tab_len;
  const uint32_t* vmax;     // FP16: bits of max |Re, Im| of W V over the call
  uint32_t* qctr;           // item counter, zero at launch
  int N, ntx;
  int checker;
  float2* grid;
};

struct DegridArgsLp {
  const int4* items;
  const uint32_t* lists;    // work lists (itoff of the plan), r8 rows per list
  int r8;
  uint32_t* qctr;           // list counters, zero at launch
  const uint2* tdesc;
  const SlotRec* krec;
  const float2* grid;       // the FP32 grid (the kernel reads g16, made from it)
  const uint32_t* lp_u;     // 16-bit padded tables
  const uint32_t* lp_v;
  int tab_len;
  const uint32_t* gmax;     // FP16: bits of max |Re, Im| of the grid
  int N, ntx;
  int checker;              // the grid comes from the centred FFT: region times (-1)^(x+y)
  float2* yrow;
  int64_t nslots;           // tile slots of krec
  int64_t ycap;             // entries of yrow
  const uint32_t* g16 = nullptr;   // the grid as operands (launch_lp_grid)
};

hipError_t launch_grid_fp32(int S, const GridArgs& a, int64_t max_items, hipStream_t s);
// tables staged in LDS (lds_bytes of them), one 16-wave workgroup per CU; the
// work-list counters (a.qctr) must be zero at launch
hipError_t launch_grid_fp32_lds(int S, const GridArgs& a, int lds_bytes, int n_cu,
                                hipStream_t s);
// persistent launch over the items of njobs jobs; first[njobs + 1] = prefix of
// per-job item counts (device), counter = 8 zeroed counters kCtrStride apart
hipError_t launch_grid_fp32_batched(int S, const GridArgs* jobs, const uint32_t* first, int njobs,
                                    uint32_t* counter, int blocks, hipStream_t s);
// first[j + 1] = first[j] + *jobs[j].nitems, first[0] = 0; the 8 counters
// (kCtrStride apart) = 0
hipError_t launch_job_prefix(const GridArgs* jobs, int njobs, uint32_t* first, uint32_t* counter,
                             hipStream_t s);
hipError_t launch_job_prefix(const DegridArgs* jobs, int njobs, uint32_t* first, uint32_t* counter,
                             hipStream_t s);
// lds_bytes > 0: the FP32 tables (gridding) or the 16-bit tables (degridding)
// are staged in LDS by one 16-wave workgroup per CU; else 4 workgroups of 4
// waves per CU read them through the caches.  Counters must be zero at launch.
hipError_t launch_grid_lp(int S, bool bf16, const GridArgsLp& a, int lds_bytes, int n_cu,
                          hipStream_t s);
hipError_t launch_degrid_lp(int S, bool bf16, const DegridArgsLp& a, int lds_bytes, int n_cu,
                            hipStream_t s);
// atomic maximum of max |Re, Im| over n complex values into *out (float bits)
hipError_t launch_absmax(const float2* g, int64_t n, uint32_t* out, hipStream_t s);
// 16-bit degridding operands of an N x N grid: cell (x, y) times (FP16) the
// call's scale 2^(9 - e) (e from *gmax as in the degridding kernel) and,
// with checker, (-1)^(x + y), rounded to a 16-bit (Re, Im) pair at
// (x + B, y + B) of out (pitch N + 2B, B = kG16Border; the border is left as
// it is: zero); BF16 writes the low parts one plane ((N + 2B)^2) further
hipError_t launch_lp_grid(const float2* g, int N, bool bf16, const uint32_t* gmax, int checker,
                          uint32_t* out, hipStream_t s);
// zero-padded FP32 tables: out[k][fi][c - 1 + s] = tab[k][fi][s] * (scale ? scale[k] : 1),
// times (-1)^s when alternate
hipError_t launch_pad_table(const float2* tab, const float* scale, int P, int O, int S, float2* out,
                            hipStream_t s, bool alternate = false);
// 16-bit padded tables (rows of L = 32 - S taps as in the FP32 padded tables):
// FP16 (Re, Im) pairs, or BF16 high parts then low parts at + tab_len
hipError_t launch_lp_table(const float2* tab, int P, int O, int S, int bf16, int tab_len,
                           uint32_t* out, hipStream_t s);
// lds_bytes > 0: stage both padded tables (2 tab_len entries, or one table when
// tab_u == tab_v) in LDS, with workgroups that own a whole CU
hipError_t launch_degrid_fp32(int S, const DegridArgs& a, int64_t max_items, int lds_bytes,
                              int n_cu, hipStream_t s);
// persistent launch over the items of njobs jobs that share one set of tables
// (jobs[0]'s, staged in LDS when lds_bytes > 0); first[njobs + 1] = prefix of
// per-job item counts (device), counter = zeroed device word
hipError_t launch_degrid_fp32_batched(int S, const DegridArgs* jobs, const uint32_t* first,
                                      int njobs, uint32_t* counter, int lds_bytes, int n_cu,
                                      hipStream_t s);

// Per-visibility gridding and degridding for supports above the MFMA region
// (wide.hip).  Inputs in caller order: packed bins and row bins of the plan
// (kDropped: off the grid), raw tables [P][O][S].
struct WideArgs {
  const uint2* qrec;        // (cell_u | cell_v << 16, fi_u | fi_v << 8 | k << 16)
  const uint32_t* rbin;     // kDropped for dropped visibilities
  const float2* tab_u;
  const float2* tab_v;
  const float2* rot;        // facet rotation or null
  int64_t nvis;
  int N, S, O;
  int checker;              // grid side of the centred FFT: (-1)^(x+y)
};
// grid += W V rot Tu Tv over each footprint (atomics)
hipError_t launch_grid_wide(const WideArgs& a, const float2* vis, const float* weight,
                            float2* grid, hipStream_t s);
// out[i] = conj(rot) sum conj(Tv) conj(Tu) grid over the footprint, 0 when dropped
hipError_t launch_degrid_wide(const WideArgs& a, const float2* grid, float2* out, hipStream_t s);

// out[q][p] = in[q][p] (-1)^(p+q) n(l0 + l_p, m0 + m_q)^npow / (c1[p] c1[q])
// real model image in (prediction) / real part of the image out (adjoint)
hipError_t launch_correct_real_in(const float* in, float2* out, const double* c1, int N, double fov,
                                  double l0, double m0, int npow, hipStream_t s);
hipError_t launch_correct_real_out(const float2* in, float* out, const double* c1, int N,
                                   double fov, double l0, double m0, int npow, hipStream_t s);
hipError_t launch_correct(const float2* in, float2* out, const double* c1, int N, double fov,
                          double l0, double m0, int npow, hipStream_t s);

// ---- correction table F_w - F~_w (corr_tables.hip, corr_apply.hip) ----
// largest tap offset |d| in 1/Oc cells of an Sc-tap table
int corr_dmax(int Sc, int Oc);
// FP64 work space of the generation for nkb planes per batch
int64_t corr_tmp_doubles(int N, int Sc, int Oc, int nkb);
// out[k][fu][fv][sv][su] for all P planes (symmetric taper c1 required)
hipError_t launch_corr_tables(const double* c1, int N, double fov, int P, double w_lo, double w_hi,
                              double a_u, double b_u, double a_v, double b_v, int Sc, int Oc,
                              int nkb, double* tmp, float2* out, hipStream_t s);

struct CorrGeom {
  int O, lo;        // oversampling of the separable tables and log2 O
  int Oc, lr;       // correction oversampling and log2(O / Oc)
  int Sc, hc, T2;   // correction support, Sc / 2, Sc^2
  int win;          // edge of the window holding a tile's correction footprints (<= 16)
};

// Correction passes over a plan's work items: gridding adds into grid (which
// already holds the separable gridding), degridding adds into yrow (which
// already holds the separable results).
struct CorrArgs {
  const int4* items;
  const uint32_t* nitems;
  const uint2* tdesc;
  const SlotRec* krec;
  float2* yrow;             // W V (gridding) or results (degridding), row-bin order
  const float2* tab;        // correction table
  CorrGeom g;
  int N, ntx;
  int checker;              // (-1)^(x+y) on grid values, as the separable kernels
  float2* grid;             // gridding: output grid; degridding: input grid
};
hipError_t launch_corr_grid(int S, const CorrArgs& a, int64_t max_items, hipStream_t s);
hipError_t launch_corr_degrid(int S, const CorrArgs& a, int64_t max_items, hipStream_t s);

}  // namespace sepw
