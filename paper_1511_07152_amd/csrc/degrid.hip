// Degridding on the matrix cores (FP32 MFMA).
//
// Degridding is the adjoint of gridding (Section 2, prediction equation;
// Section 6, prediction for major cycles):
//     V_i = sum_y conj(Tv_i[y - oy_i]) sum_x conj(Tu_i[x - ox_i]) R[y][x]
// over the 16 x 16 grid region R of the visibility's tile.  The inner sums for
// 16 visibilities at once are the dense product Z = R * conj(A_u)^T (M = 16 rows,
// N = 16 visibilities, K = 16 columns), four steps of v_mfma_f32_16x16x4f32 per
// real/imaginary combination; the outer sum is an S-term dot product per
// visibility done on the vector unit from the accumulator layout, reduced
// across the four 16-lane groups.  The region is loaded once per work item and
// stays in registers; the output is written to the caller's order through the
// plan's permutation.  If the grid came from the FFT, the checkerboard
// (-1)^(x+y) of the centred transform is applied on load.
// Lane layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 (l / 16) + r][l % 16].
#include "internal.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

template <int S>
__global__ __launch_bounds__(64 * kWaves) void degrid_fp32_kernel(
    const int4* __restrict__ items, const uint32_t* __restrict__ nitems,
    const uint2* __restrict__ rec, const int32_t* __restrict__ perm,
    const float2* __restrict__ rot, const float2* __restrict__ grid,
    const float2* __restrict__ tab_u, const float2* __restrict__ tab_v, int O, int N, int ntx,
    int checker, float2* __restrict__ vis_out) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int n_items = (int)*nitems;
  const int stride = gridDim.x * kWaves;

  for (int it = blockIdx.x * kWaves + (threadIdx.x >> 6); it < n_items; it += stride) {
    const int4 item = items[it];
    const int ty = item.x / ntx, tx = item.x - ty * ntx;
    const int bx = tx * C, by = ty * C;
    // A operand for step q: R[y = col][x = 4 q + grp]
    float r_re[4], r_im[4];
    const int gy = by - H + col;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gx = bx - H + 4 * q + grp;
      float2 val = make_float2(0.f, 0.f);
      if (gx >= 0 && gx < N && gy >= 0 && gy < N) {
        val = grid[(int64_t)gy * N + gx];
        if (checker && ((gx + gy) & 1)) val = make_float2(-val.x, -val.y);
      }
      r_re[q] = val.x;
      r_im[q] = val.y;
    }
    for (int v0 = 0; v0 < item.z; v0 += 16) {
      const int v = v0 + col;             // this lane's visibility (column of Z)
      const bool valid = v < item.z;
      const int j = item.y + v;
      uint2 r = make_uint2(0u, 0u);
      if (valid) r = rec[j];
      const int ox = (int)(r.x & 0xFFFFu) - bx;
      const int oy = (int)(r.x >> 16) - by;
      const int row = (int)((r.y >> 16) * (uint32_t)O);
      const float2* tu_row = tab_u + (row + (int)(r.y & 0xFFu)) * S;
      const float2* tv_row = tab_v + (row + (int)((r.y >> 8) & 0xFFu)) * S;
      f32x4 z_re = {0.f, 0.f, 0.f, 0.f}, z_im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int s = 4 * q + grp - ox;
        float2 tu = make_float2(0.f, 0.f);
        if (valid && (unsigned)s < (unsigned)S) tu = tu_row[s];
        z_re = __builtin_amdgcn_mfma_f32_16x16x4f32(r_re[q], tu.x, z_re, 0, 0, 0);
        z_re = __builtin_amdgcn_mfma_f32_16x16x4f32(r_im[q], tu.y, z_re, 0, 0, 0);
        z_im = __builtin_amdgcn_mfma_f32_16x16x4f32(r_im[q], tu.x, z_im, 0, 0, 0);
        z_im = __builtin_amdgcn_mfma_f32_16x16x4f32(r_re[q], -tu.y, z_im, 0, 0, 0);
      }
      float p_re = 0.f, p_im = 0.f;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int t = 4 * grp + rr - oy;
        if (valid && (unsigned)t < (unsigned)S) {
          const float2 tv = tv_row[t];
          p_re += tv.x * z_re[rr] + tv.y * z_im[rr];
          p_im += tv.x * z_im[rr] - tv.y * z_re[rr];
        }
      }
      p_re += __shfl_xor(p_re, 16, 64);
      p_im += __shfl_xor(p_im, 16, 64);
      p_re += __shfl_xor(p_re, 32, 64);
      p_im += __shfl_xor(p_im, 32, 64);
      if (grp == 0 && valid) {
        float2 out = make_float2(p_re, p_im);
        if (rot) {  // undo the facet phase rotation: multiply by conj(rot)
          const float2 ro = rot[j];
          out = make_float2(p_re * ro.x + p_im * ro.y, p_im * ro.x - p_re * ro.y);
        }
        vis_out[perm[j]] = out;
      }
    }
  }
}

template <int S>
hipError_t launch_s(const int4* items, const uint32_t* nitems, const uint2* rec,
                    const int32_t* perm, const float2* rot, const float2* grid, const float2* tu,
                    const float2* tv, int O, int N, int ntx, int checker, float2* vis_out,
                    int blocks, hipStream_t s) {
  hipLaunchKernelGGL(degrid_fp32_kernel<S>, dim3(blocks), dim3(64 * kWaves), 0, s, items, nitems,
                     rec, perm, rot, grid, tu, tv, O, N, ntx, checker, vis_out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_degrid_fp32(int S, const int4* items, const uint32_t* nitems, const uint2* rec,
                              const int32_t* perm, const float2* rot, const float2* grid,
                              const float2* tab_u, const float2* tab_v, int O, int N, int tile_c,
                              int ntx, int checker, float2* vis_out, hipStream_t s,
                              int64_t max_items) {
  (void)tile_c;
  int64_t b = (max_items + kWaves - 1) / kWaves;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  const int blocks = (int)b;
#define SEPW_DG(SS) \
  case SS: return launch_s<SS>(items, nitems, rec, perm, rot, grid, tab_u, tab_v, O, N, ntx, checker, vis_out, blocks, s);
  switch (S) {
    SEPW_DG(1) SEPW_DG(3) SEPW_DG(5) SEPW_DG(7) SEPW_DG(9) SEPW_DG(11) SEPW_DG(13) SEPW_DG(15)
    default: return hipErrorInvalidValue;
  }
#undef SEPW_DG
}

}  // namespace sepw
