// Gridding and degridding for supports above the 16-cell MFMA region
// (15 < S <= 31), one visibility per wave.
//
// Same arithmetic as the tiled path (Section 2's gridding and prediction
// sums with Section 3's separable GCF: cell (cu - S/2 + s, cv - S/2 + t) of
// visibility i takes y_i Tu_i[s] Tv_i[t], and degridding sums conj(Tv_i[t])
// conj(Tu_i[s]) R over the same footprint), on the vector unit: the lanes of
// a wave take the S^2 taps of one visibility in turn.  Gridding adds each
// tap with FP32 atomics (footprints of different visibilities overlap);
// degridding reduces the lanes' partial sums.  Visibilities come in the
// caller's order with their packed bins from the quantiser (kDropped: off
// the grid, skipped; degridding writes 0 for them), so this path needs no
// tile slots.  Kept footprints lie inside the grid (the quantiser drops the
// others), and the raw tables [P][O][S] hold the taps.
#include "internal.h"

namespace sepw {

namespace {

constexpr int kThreads = 256;

__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ __launch_bounds__(kThreads) void grid_wide_kernel(WideArgs a,
                                                             const float2* __restrict__ vis,
                                                             const float* __restrict__ weight,
                                                             float* __restrict__ grid) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (kThreads / 64);
  const int S = a.S, h = S / 2, SS = S * S;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); i < a.nvis;
       i += nw) {
    if (a.rbin[i] == kDropped) continue;
    const uint2 q = a.qrec[i];
    const int cu = (int)(q.x & 0xFFFFu), cv = (int)(q.x >> 16);
    const int fu = (int)(q.y & 0xFFu), fv = (int)((q.y >> 8) & 0xFFu), k = (int)(q.y >> 16);
    float2 y = vis[i];
    const float wt = weight ? weight[i] : 1.f;
    y = make_float2(y.x * wt, y.y * wt);
    if (a.rot) y = cmul(y, a.rot[i]);
    const float2* tu = a.tab_u + ((int64_t)k * a.O + fu) * S;
    const float2* tv = a.tab_v + ((int64_t)k * a.O + fv) * S;
    for (int t = lane; t < SS; t += 64) {
      const int ty = t / S, tx = t - ty * S;
      const float2 g = cmul(cmul(y, tu[tx]), tv[ty]);
      const int gx = cu - h + tx, gy = cv - h + ty;
      const float sg = (a.checker && ((gx + gy) & 1)) ? -1.f : 1.f;
      float* p = grid + 2 * ((int64_t)gy * a.N + gx);
      unsafeAtomicAdd(p, sg * g.x);
      unsafeAtomicAdd(p + 1, sg * g.y);
    }
  }
}

__global__ __launch_bounds__(kThreads) void degrid_wide_kernel(WideArgs a,
                                                               const float2* __restrict__ grid,
                                                               float2* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (kThreads / 64);
  const int S = a.S, h = S / 2, SS = S * S;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); i < a.nvis;
       i += nw) {
    if (a.rbin[i] == kDropped) {
      if (lane == 0) out[i] = make_float2(0.f, 0.f);
      continue;
    }
    const uint2 q = a.qrec[i];
    const int cu = (int)(q.x & 0xFFFFu), cv = (int)(q.x >> 16);
    const int fu = (int)(q.y & 0xFFu), fv = (int)((q.y >> 8) & 0xFFu), k = (int)(q.y >> 16);
    const float2* tu = a.tab_u + ((int64_t)k * a.O + fu) * S;
    const float2* tv = a.tab_v + ((int64_t)k * a.O + fv) * S;
    float re = 0.f, im = 0.f;
    for (int t = lane; t < SS; t += 64) {
      const int ty = t / S, tx = t - ty * S;
      const int gx = cu - h + tx, gy = cv - h + ty;
      float2 g = grid[(int64_t)gy * a.N + gx];
      if (a.checker && ((gx + gy) & 1)) g = make_float2(-g.x, -g.y);
      // conj(Tv) conj(Tu) g = conj(Tu Tv) g
      const float2 uv = cmul(tu[tx], tv[ty]);
      re += uv.x * g.x + uv.y * g.y;
      im += uv.x * g.y - uv.y * g.x;
    }
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o, 64);
      im += __shfl_xor(im, o, 64);
    }
    if (lane == 0) {
      float2 v = make_float2(re, im);
      if (a.rot) {
        const float2 r = a.rot[i];
        v = make_float2(v.x * r.x + v.y * r.y, v.y * r.x - v.x * r.y);   // v conj(rot)
      }
      out[i] = v;
    }
  }
}

int blocks_for(int64_t nvis) {
  int64_t b = (nvis + kThreads / 64 - 1) / (kThreads / 64);
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

hipError_t launch_grid_wide(const WideArgs& a, const float2* vis, const float* weight,
                            float2* grid, hipStream_t s) {
  if (a.nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(grid_wide_kernel, dim3(blocks_for(a.nvis)), dim3(kThreads), 0, s, a, vis,
                     weight, reinterpret_cast<float*>(grid));
  return hipGetLastError();
}

hipError_t launch_degrid_wide(const WideArgs& a, const float2* grid, float2* out, hipStream_t s) {
  if (a.nvis == 0) return hipSuccess;
  hipLaunchKernelGGL(degrid_wide_kernel, dim3(blocks_for(a.nvis)), dim3(kThreads), 0, s, a, grid,
                     out);
  return hipGetLastError();
}

}  // namespace sepw
