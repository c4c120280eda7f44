// W-stacking hybrid (Section 4.3): the visibilities are partitioned into
// w-slices; each slice is imaged with the separable W-projection path
// on its residual w - w_s, and its image is corrected by the exact phase of
// the slice centre, exp(2 pi i w_s (n - 1)), before the slice images are
// summed (prediction: the model is multiplied by exp(-2 pi i w_s (n - 1))
// before each slice is degridded).
//
// Slice s = clamp(floor((w - w_lo) inv_ds), 0, n_s - 1) with inv_ds =
// n_s / (w_hi - w_lo) computed once on the host, each FP64 operation an
// explicitly rounded IEEE operation in this order (so that the partition is
// reproducible bit for bit); centres w_s = w_lo + (s + 1/2)(w_hi - w_lo)/n_s
// come from the host.  Non-uniform slices (Section 4.3 suggests narrow
// slices where w is dense) come as increasing edges e_0 < ... < e_ns: slice
// s holds e_s <= w < e_{s+1} (w below e_0 in slice 0, at or above e_ns in the
// last), found by binary search, with centre (e_s + e_{s+1}) / 2 from the
// host.  Non-finite w goes to slice 0 with a non-finite
// residual, which the plane quantiser then drops.  n - 1 is evaluated as
// -(l^2 + m^2) / (1 + n), equal to it and free of the cancellation near the
// centre; the phase is reduced to [-1/2, 1/2] cycles before the FP64 sincos.
#include "internal.h"

namespace sepw {

namespace {

constexpr int kThreads = 256;

inline dim3 grid_for(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return dim3((unsigned)b);
}

__device__ inline int slice_of(double w, double w_lo, double inv_ds, int ns,
                               const double* __restrict__ edges) {
  if (edges) {
    if (!isfinite(w)) return 0;
    int lo = 0, hi = ns;   // edges[lo] <= w < edges[hi], the outer edges open
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (w >= edges[mid]) lo = mid;
      else hi = mid;
    }
    return lo;
  }
  const double t = floor(__dmul_rn(__dsub_rn(w, w_lo), inv_ds));
  if (!isfinite(t)) return 0;
  return t < 0.0 ? 0 : (t > (double)(ns - 1) ? ns - 1 : (int)t);
}

// Visibilities per slice (counts must be zero on entry; ns <= kMaxSlices).
__global__ __launch_bounds__(kThreads) void slice_count_kernel(const double* __restrict__ w,
                                                               int64_t nvis, double w_lo,
                                                               double inv_ds, int ns,
                                                               const double* __restrict__ edges,
                                                               uint32_t* __restrict__ count) {
  __shared__ uint32_t hist[kMaxSlices];
  for (int s = threadIdx.x; s < ns; s += kThreads) hist[s] = 0u;
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < nvis;
       i += (int64_t)gridDim.x * kThreads)
    atomicAdd(&hist[slice_of(w[i], w_lo, inv_ds, ns, edges)], 1u);
  __syncthreads();
  for (int s = threadIdx.x; s < ns; s += kThreads)
    if (hist[s]) atomicAdd(&count[s], hist[s]);
}

// Slice order: order[j] = caller index of slice-ordered position j; the
// coordinates in slice order with w replaced by its residual.  cursor starts
// at the slice offsets.  Each workgroup counts its chunk per slice in LDS,
// reserves each slice's run with one global atomic, then places its
// visibilities with LDS atomics (one global atomic per visibility on a few
// slice cursors serialised on those cursors).
constexpr int kScatterChunk = 16 * kThreads;
__global__ __launch_bounds__(kThreads) void slice_scatter_kernel(
    const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
    int64_t nvis, double w_lo, double inv_ds, int ns, const double* __restrict__ edges,
    const double* __restrict__ centre, uint32_t* __restrict__ cursor, uint32_t* __restrict__ order, double* __restrict__ us,
    double* __restrict__ vs, double* __restrict__ ws) {
  __shared__ uint32_t cnt[kMaxSlices];
  const int64_t i0 = (int64_t)blockIdx.x * kScatterChunk;
  const int64_t i1 = min(i0 + (int64_t)kScatterChunk, nvis);
  for (int s = threadIdx.x; s < ns; s += kThreads) cnt[s] = 0u;
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads)
    atomicAdd(&cnt[slice_of(w[i], w_lo, inv_ds, ns, edges)], 1u);
  __syncthreads();
  for (int s = threadIdx.x; s < ns; s += kThreads)
    if (cnt[s]) cnt[s] = atomicAdd(&cursor[s], cnt[s]);   // this chunk's first position
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double wi = w[i];
    const int s = slice_of(wi, w_lo, inv_ds, ns, edges);
    const uint32_t j = atomicAdd(&cnt[s], 1u);
    order[j] = (uint32_t)i;
    us[j] = u[i];
    vs[j] = v[i];
    ws[j] = __dsub_rn(wi, centre[s]);
  }
}

// out[j] = vis[order[j]] weight[order[j]]
__global__ void slice_gather_kernel(const float2* __restrict__ vis, const float* __restrict__ weight,
                                    const uint32_t* __restrict__ order, int64_t nvis,
                                    float2* __restrict__ out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nvis;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = order[j];
    float2 y = vis[i];
    if (weight) {
      const float wt = weight[i];
      y = make_float2(y.x * wt, y.y * wt);
    }
    out[j] = y;
  }
}

// out[order[j]] = in[j]
__global__ void slice_return_kernel(const float2* __restrict__ in, const uint32_t* __restrict__ order,
                                    int64_t nvis, float2* __restrict__ out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nvis;
       j += (int64_t)gridDim.x * blockDim.x)
    out[order[j]] = in[j];
}

// out = in exp(sign 2 pi i w_s (n - 1)) (accumulate: out += ...)
// With c1, the pass also applies the image correction of the separable path
// (the centred transform's (-1)^(p+q), n^npow and 1 / (c1[p] c1[q])), formed
// in FP64 with the phase.
__global__ void slice_phase_kernel(const float2* __restrict__ in, float2* __restrict__ out, int N,
                                   double fov, double w_s, int sign, int accumulate,
                                   const double* __restrict__ c1, int npow) {
  const int64_t total = (int64_t)N * N;
  const double step = fov / (double)N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t ui = (uint32_t)i;   // N <= 32768: pixel indices fit 32 bits
    const int q = (int)(ui / (uint32_t)N), p = (int)(ui - (uint32_t)q * (uint32_t)N);
    const double l = (double)(p - N / 2) * step;
    const double m = (double)(q - N / 2) * step;
    const double r2 = l * l + m * m;
    const double n = sqrt(1.0 - r2);
    const double cyc = w_s * (-r2 / (1.0 + n));
    const double frac = cyc - rint(cyc);
    double sn, cs;
    sincospi(2.0 * (double)sign * frac, &sn, &cs);
    if (c1) {
      double f = 1.0 / (c1[p] * c1[q]);
      if (npow != 0) f = npow > 0 ? f * n : f / n;
      if ((p + q) & 1) f = -f;
      sn *= f;
      cs *= f;
    }
    const float2 a = in[i];
    const float re = (float)(a.x * cs - a.y * sn), im = (float)(a.x * sn + a.y * cs);
    if (accumulate) {
      const float2 o = out[i];
      out[i] = make_float2(o.x + re, o.y + im);
    } else {
      out[i] = make_float2(re, im);
    }
  }
}

// Counts of the finite w in nfine uniform bins of [w_lo, w_hi] (bin index
// floor((w - w_lo) inv) clamped, each FP64 operation rounded as written; a
// non-finite index counts in bin 0).  counts must be zero on entry.
__global__ __launch_bounds__(kThreads) void w_hist_kernel(const double* __restrict__ w,
                                                          int64_t nvis, double w_lo, double inv,
                                                          int nfine,
                                                          uint32_t* __restrict__ counts) {
  __shared__ uint32_t hist[kDensityBins];
  for (int b = threadIdx.x; b < nfine; b += kThreads) hist[b] = 0u;
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < nvis;
       i += (int64_t)gridDim.x * kThreads) {
    const double x = w[i];
    if (!isfinite(x)) continue;
    const double t = floor(__dmul_rn(__dsub_rn(x, w_lo), inv));
    const int b = !isfinite(t) ? 0 : (t < 0.0 ? 0 : (t > (double)(nfine - 1) ? nfine - 1 : (int)t));
    atomicAdd(&hist[b], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nfine; b += kThreads)
    if (hist[b]) atomicAdd(&counts[b], hist[b]);
}

}  // namespace

hipError_t launch_w_hist(const double* w, int64_t nvis, double w_lo, double inv, int nfine,
                         uint32_t* counts, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  int64_t b = (nvis + kThreads - 1) / kThreads;
  if (b > 2048) b = 2048;   // per-workgroup LDS histograms: few workgroups, many visibilities each
  hipLaunchKernelGGL(w_hist_kernel, dim3((unsigned)b), dim3(kThreads), 0, s, w, nvis, w_lo, inv,
                     nfine, counts);
  return hipGetLastError();
}

hipError_t launch_slice_count(const double* w, int64_t nvis, double w_lo, double inv_ds, int ns,
                              const double* edges, uint32_t* count, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(slice_count_kernel, grid_for(nvis), dim3(kThreads), 0, s, w, nvis, w_lo, inv_ds,
                     ns, edges, count);
  return hipGetLastError();
}

hipError_t launch_slice_scatter(const double* u, const double* v, const double* w, int64_t nvis,
                                double w_lo, double inv_ds, int ns, const double* edges,
                                const double* centre, uint32_t* cursor, uint32_t* order,
                                double* us, double* vs, double* ws, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  const int64_t nb = (nvis + kScatterChunk - 1) / kScatterChunk;
  hipLaunchKernelGGL(slice_scatter_kernel, dim3((unsigned)nb), dim3(kThreads), 0, s, u, v, w, nvis,
                     w_lo, inv_ds, ns, edges, centre, cursor, order, us, vs, ws);
  return hipGetLastError();
}

hipError_t launch_slice_gather(const float2* vis, const float* weight, const uint32_t* order,
                               int64_t nvis, float2* out, hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(slice_gather_kernel, grid_for(nvis), dim3(kThreads), 0, s, vis, weight, order,
                     nvis, out);
  return hipGetLastError();
}

hipError_t launch_slice_return(const float2* in, const uint32_t* order, int64_t nvis, float2* out,
                               hipStream_t s) {
  if (nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(slice_return_kernel, grid_for(nvis), dim3(kThreads), 0, s, in, order, nvis, out);
  return hipGetLastError();
}

hipError_t launch_slice_phase(const float2* in, float2* out, int N, double fov, double w_s,
                              int sign, bool accumulate, const double* c1, int npow,
                              hipStream_t s) {
  hipLaunchKernelGGL(slice_phase_kernel, grid_for((int64_t)N * N), dim3(kThreads), 0, s, in, out, N,
                     fov, w_s, sign, accumulate ? 1 : 0, c1, npow);
  return hipGetLastError();
}

}  // namespace sepw
