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
// footprints fit in a 16 x 16 region).  Sorting is a counting sort: global
// histogram by atomics, exclusive scan, atomic-cursor scatter.  Membership of a
// visibility in its bin is exact; the order inside a bin is not specified.
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

__device__ inline int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
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
  r.cell = floor_div(qi + g.O / 2, g.O);
  r.fi = (int)(qi - r.cell * g.O) + g.O / 2;
  return r;
}

__global__ void quantise_kernel(const double* __restrict__ u, const double* __restrict__ v,
                                const double* __restrict__ w, int64_t nvis, QuantGeom g,
                                uint32_t* __restrict__ key, uint2* __restrict__ qrec,
                                uint32_t* __restrict__ counts) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvis;
       i += (int64_t)gridDim.x * blockDim.x) {
    double uu = u[i], vv = v[i], ww = w[i];
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
      uint32_t tile = (uint32_t)(cv / g.tile_c) * (uint32_t)g.ntx + (uint32_t)(cu / g.tile_c);
      key[i] = tile;
      qrec[i] = pack_rec(cu, bu.fi, cv, bv.fi, k);
      atomicAdd(&counts[tile], 1u);
    } else {
      key[i] = kDropped;
      qrec[i] = make_uint2(0u, 0u);
    }
  }
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

// ---------------------------------------------------------------- scatter etc.
__global__ void scatter_kernel(const uint32_t* __restrict__ key, const uint2* __restrict__ qrec,
                               int64_t nvis, uint32_t* __restrict__ cursor,
                               uint2* __restrict__ rec, int32_t* __restrict__ perm) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvis;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t kk = key[i];
    if (kk == kDropped) continue;
    uint32_t pos = atomicAdd(&cursor[kk], 1u);
    rec[pos] = qrec[i];
    perm[pos] = (int32_t)i;
  }
}

__global__ void rotation_kernel(const double* __restrict__ u, const double* __restrict__ v,
                                const double* __restrict__ w, const int32_t* __restrict__ perm,
                                const uint32_t* __restrict__ nkept, QuantGeom g,
                                float2* __restrict__ rot) {
  const int64_t n = *nkept;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = perm[j];
    // phase in cycles, reduced to [-1/2, 1/2] before the FP64 sincos
    double cyc = u[i] * g.l0 + v[i] * g.m0 + w[i] * (g.n0 - 1.0);
    double frac = cyc - rint(cyc);
    double s, c;
    sincospi(2.0 * frac, &s, &c);
    rot[j] = make_float2((float)c, (float)s);
  }
}

__global__ void item_counts_kernel(const uint32_t* __restrict__ off, int64_t ntiles,
                                   uint32_t* __restrict__ nit) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t <= ntiles;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c = t < ntiles ? off[t + 1] - off[t] : 0u;
    nit[t] = (c + kItemMaxVis - 1) / kItemMaxVis;
  }
}

__global__ void items_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ itoff,
                             int64_t ntiles, int4* __restrict__ items) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint32_t first = off[t], cnt = off[t + 1] - first;
    uint32_t o = itoff[t];
    for (uint32_t m = 0; m * kItemMaxVis < cnt; ++m) {
      uint32_t c = cnt - m * kItemMaxVis;
      items[o + m] = make_int4((int)t, (int)(first + m * kItemMaxVis),
                               (int)(c < (uint32_t)kItemMaxVis ? c : kItemMaxVis), 0);
    }
  }
}

__global__ void bins_dropped_kernel(int64_t nvis, int32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nvis;
       i += (int64_t)gridDim.x * blockDim.x) {
    int32_t* o = out + 7 * i;
    o[0] = o[1] = o[2] = o[3] = o[4] = 0;
    o[5] = -1;
    o[6] = 1;
  }
}

__global__ void bins_export_kernel(const uint2* __restrict__ rec, const int32_t* __restrict__ perm,
                                   const uint32_t* __restrict__ nkept, int tile_c, int ntx,
                                   int32_t* __restrict__ out) {
  const int64_t n = *nkept;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    uint2 r = rec[j];
    int cu = r.x & 0xFFFF, cv = r.x >> 16;
    int32_t* o = out + 7 * (int64_t)perm[j];
    o[0] = cu;
    o[1] = r.y & 0xFF;
    o[2] = cv;
    o[3] = (r.y >> 8) & 0xFF;
    o[4] = r.y >> 16;
    o[5] = (cv / tile_c) * ntx + cu / tile_c;
    o[6] = 0;
  }
}

__global__ void gather_kernel(const int32_t* __restrict__ perm, const float2* __restrict__ vis,
                              const float* __restrict__ weight, const float2* __restrict__ rot,
                              const uint32_t* __restrict__ nkept, float2* __restrict__ ybin) {
  const int64_t n = *nkept;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = perm[j];
    float2 y = vis[i];
    if (weight) {
      float wt = weight[i];
      y.x *= wt;
      y.y *= wt;
    }
    if (rot) {
      float2 r = rot[j];
      y = make_float2(y.x * r.x - y.y * r.y, y.x * r.y + y.y * r.x);
    }
    ybin[j] = y;
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

hipError_t launch_quantise(const double* u, const double* v, const double* w, int64_t nvis,
                           QuantGeom g, uint32_t* key, uint2* qrec, uint32_t* counts,
                           hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(quantise_kernel, grid_for(nvis), dim3(kThreads), 0, s, u, v, w, nvis, g,
                     key, qrec, counts);
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

hipError_t launch_scatter(const uint32_t* key, const uint2* qrec, int64_t nvis, uint32_t* cursor,
                          uint2* rec, int32_t* perm, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, grid_for(nvis), dim3(kThreads), 0, s, key, qrec, nvis,
                     cursor, rec, perm);
  return hipGetLastError();
}

hipError_t launch_rotation(const double* u, const double* v, const double* w, const int32_t* perm,
                           const uint32_t* nkept, int64_t nvis, QuantGeom g, float2* rot,
                           hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(rotation_kernel, grid_for(nvis), dim3(kThreads), 0, s, u, v, w, perm, nkept,
                     g, rot);
  return hipGetLastError();
}

hipError_t launch_item_counts(const uint32_t* off, int64_t ntiles, uint32_t* nit, hipStream_t s) {
  hipLaunchKernelGGL(item_counts_kernel, grid_for(ntiles + 1), dim3(kThreads), 0, s, off, ntiles,
                     nit);
  return hipGetLastError();
}

hipError_t launch_items(const uint32_t* off, const uint32_t* itoff, int64_t ntiles, int4* items,
                        hipStream_t s) {
  hipLaunchKernelGGL(items_kernel, grid_for(ntiles), dim3(kThreads), 0, s, off, itoff, ntiles,
                     items);
  return hipGetLastError();
}

hipError_t launch_bins_export(const uint2* rec, const int32_t* perm, const uint32_t* nkept,
                              int64_t nvis, int tile_c, int ntx, int32_t* out, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(bins_dropped_kernel, grid_for(nvis), dim3(kThreads), 0, s, nvis, out);
  hipLaunchKernelGGL(bins_export_kernel, grid_for(nvis), dim3(kThreads), 0, s, rec, perm, nkept,
                     tile_c, ntx, out);
  return hipGetLastError();
}

hipError_t launch_gather(const int32_t* perm, const float2* vis, const float* weight,
                         const float2* rot, const uint32_t* nkept, int64_t nvis, float2* ybin,
                         hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, grid_for(nvis), dim3(kThreads), 0, s, perm, vis, weight, rot,
                     nkept, ybin);
  return hipGetLastError();
}

}  // namespace sepw
