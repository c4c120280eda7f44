// Internal types and launchers of the separable W-projection library.
// Not part of the ABI; see include/sepw.h for the public contract.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>
#include <stdint.h>

#include "sepw.h"

namespace sepw {

constexpr uint32_t kDropped = 0xFFFFFFFFu;
constexpr int kRegion = 16;        // MFMA tile region edge (cells): core + S - 1
constexpr int kMaxSupport = 15;    // S <= kRegion - 1
constexpr int kItemMaxVis = 512;   // visibilities per work item (heavy tiles split)

// Geometry shared by the binning kernels; all FP64 values are used exactly as
// stored (no recomputation on the device), so host and device agree bit for bit.
struct QuantGeom {
  double fov;        // multiply u by this ...
  double half_n;     // ... then add N/2
  double over;       // oversampling factor O as a double (exact)
  double w_lo;
  double inv_dw;     // P / (w_hi - w_lo), computed once on the host
  int32_t N, S, O, P;
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
  float2* scratch = nullptr;   // N*N complex64 work grid for degridding
  hipfftHandle fft = 0;
  bool fft_ok = false;
  uint64_t generation = 0;     // bumped when the tables are regenerated
};

struct Plan {
  Kernels* K = nullptr;
  uint64_t generation = 0;      // K->generation the bins were made for
  int64_t nvis = 0;
  int64_t capacity = 0;         // visibilities the buffers were sized for
  int tile_c = 0, ntx = 0, nty = 0;
  int64_t ntiles = 0;
  int64_t max_items = 0;
  uint32_t* key = nullptr;      // [nvis] tile id or kDropped (caller order)
  uint2* qrec = nullptr;        // [nvis] packed bins (caller order)
  uint32_t* counts = nullptr;   // [ntiles + 1]
  uint32_t* off = nullptr;      // [ntiles + 1] exclusive scan of counts
  uint32_t* cursor = nullptr;   // [ntiles]
  uint2* rec = nullptr;         // [nvis] packed bins, binned order
  int32_t* perm = nullptr;      // [nvis] caller index, binned order
  float2* rot = nullptr;        // [nvis] facet phase rotation, binned order
  float2* ybin = nullptr;       // [nvis] W V (rotated), binned order
  uint32_t* nit = nullptr;      // [ntiles + 1] work items per tile
  uint32_t* itoff = nullptr;    // [ntiles + 1] exclusive scan of nit
  int4* items = nullptr;        // [max_items] (tile, first vis, count, 0)
  uint32_t* scan_tmp = nullptr; // block partials for the scans
  int64_t scan_tmp_len = 0;
};

// packed record: x = cell_u | cell_v << 16 ; y = fi_u | fi_v << 8 | plane << 16
__host__ __device__ inline uint2 pack_rec(int cu, int fu, int cv, int fv, int k) {
  return make_uint2((uint32_t)cu | ((uint32_t)cv << 16),
                    (uint32_t)fu | ((uint32_t)fv << 8) | ((uint32_t)k << 16));
}

// ---- host-side PSWF (pswf.cpp) ----
// Legendre coefficients d_j (degree 2j, normalised Legendre basis) of psi_0(c, x)
// and psi_0(c, 0) from the same series.  Returns the number of coefficients.
int pswf_coefficients(double c, double* d, int max_terms, double* psi_at_0);

// ---- launchers (return hipError_t of the launch) ----
hipError_t launch_taper(const double* d_coef, int ncoef, double norm, int N, double* c1, hipStream_t s);
hipError_t launch_ones(double* c1, int N, hipStream_t s);
hipError_t launch_tables(const double* c1, int N, double fov, int P, int O, int S,
                         double w_lo, double w_hi, double a, double b, float2* out, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_zero_c64(float2* p, int64_t n, hipStream_t s);
hipError_t launch_quantise(const double* u, const double* v, const double* w, int64_t nvis,
                           QuantGeom g, uint32_t* key, uint2* qrec, uint32_t* counts, hipStream_t s);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s);
int64_t scan_tmp_size(int64_t n);
hipError_t launch_scatter(const uint32_t* key, const uint2* qrec, int64_t nvis, uint32_t* cursor,
                          uint2* rec, int32_t* perm, hipStream_t s);
hipError_t launch_rotation(const double* u, const double* v, const double* w, const int32_t* perm,
                           const uint32_t* nkept, int64_t nvis, QuantGeom g, float2* rot, hipStream_t s);
hipError_t launch_item_counts(const uint32_t* off, int64_t ntiles, uint32_t* nit, hipStream_t s);
hipError_t launch_items(const uint32_t* off, const uint32_t* itoff, int64_t ntiles, int4* items,
                        hipStream_t s);
hipError_t launch_bins_export(const uint2* rec, const int32_t* perm, const uint32_t* nkept,
                              int64_t nvis, int tile_c, int ntx, int32_t* out, hipStream_t s);
hipError_t launch_gather(const int32_t* perm, const float2* vis, const float* weight,
                         const float2* rot, const uint32_t* nkept, int64_t nvis, float2* ybin,
                         hipStream_t s);

hipError_t launch_grid_fp32(int S, const int4* items, const uint32_t* nitems, const uint2* rec,
                            const float2* ybin, const float2* tab_u, const float2* tab_v, int O,
                            int N, int tile_c, int ntx, int checker, float2* grid, hipStream_t s,
                            int64_t max_items);
hipError_t launch_degrid_fp32(int S, const int4* items, const uint32_t* nitems, const uint2* rec,
                              const int32_t* perm, const float2* rot, const float2* grid,
                              const float2* tab_u, const float2* tab_v, int O, int N, int tile_c,
                              int ntx, int checker, float2* vis_out, hipStream_t s,
                              int64_t max_items);

// out[q][p] = in[q][p] (-1)^(p+q) n(l0 + l_p, m0 + m_q)^npow / (c1[p] c1[q])
hipError_t launch_correct(const float2* in, float2* out, const double* c1, int N, double fov,
                          double l0, double m0, int npow, hipStream_t s);

}  // namespace sepw
