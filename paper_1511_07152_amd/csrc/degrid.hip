// Degridding on the matrix cores (FP32 MFMA).
//
// Degridding is the adjoint of gridding (Section 2, prediction equation;
// Section 6, prediction for major cycles):
//     V_i = sum_y conj(Tv_i[y - oy_i]) sum_x conj(Tu_i[x - ox_i]) R[y][x]
// over the 16 x 16 grid region R of the visibility's tile.  The inner sums for
// 16 visibilities at once are the dense product Z = R conj(A_u)^T (M = 16 rows,
// N = 16 visibilities, K = 16 columns): four steps of v_mfma_f32_16x16x4f32 per
// real/imaginary combination.  The outer sum is an S-term dot product per
// visibility on the vector unit from the accumulator layout, reduced across the
// four 16-lane groups.
//
// Work item: a slice of <= kItemMaxVis binned visibilities from one row of
// tiles; the region of each tile is read once per tile (consecutive tiles of a
// row share 16 - c of their 16 columns, so the reloads hit the caches).  If the
// grid came from the FFT, the checkerboard (-1)^(x+y) of the centred transform
// is applied on load.  Results are written in binned order (streaming); the
// plan's placement maps move them to the caller's order afterwards.  The facet
// rotation is undone here.
// Lane layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 (l / 16) + r][l % 16].
#include "internal.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

__device__ inline int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

template <int S>
__global__ __launch_bounds__(64 * kWaves) void degrid_fp32_kernel(
    const int4* __restrict__ items, const uint32_t* __restrict__ nitems,
    const uint32_t* __restrict__ off, const uint2* __restrict__ rec,
    const int2* __restrict__ krec, const float2* __restrict__ rot,
    const float2* __restrict__ grid, const float2* __restrict__ tab_u,
    const float2* __restrict__ tab_v, int N, int ntx, int checker, float2* __restrict__ vbin) {
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int n_items = (int)*nitems;
  const int stride = gridDim.x * kWaves;

  for (int it = uniform(blockIdx.x * kWaves + (threadIdx.x >> 6)); it < n_items; it += stride) {
    const int4 item = items[it];
    const int ty = uniform(item.x), je = uniform(item.z);
    int j = uniform(item.y);
    const int by = ty * C;
    const int gy = by - H + col;          // grid row of this lane's A operand
    const bool row_ok = gy >= 0 && gy < N;
    while (j < je) {
      const int tx = uniform((int)(rec[j].x & 0xFFFFu) / C);
      const int bx = tx * C;
      const int tend = min(uniform((int)off[ty * ntx + tx + 1]), je);
      // A operand for step q: R[y = col][x = 4 q + grp]
      float r_re[4], r_im[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gx = bx - H + 4 * q + grp;
        float2 val = make_float2(0.f, 0.f);
        if (row_ok && gx >= 0 && gx < N) {
          val = grid[(int64_t)gy * N + gx];
          if (checker && ((gx + gy) & 1)) val = make_float2(-val.x, -val.y);
        }
        r_re[q] = val.x;
        r_im[q] = val.y;
      }
      // 32 visibilities per iteration (two MFMA column blocks); lane (col, grp)
      // handles visibility v0 + 16 m + col.  Taps come from the padded tables at
      // base + region index, so no per-tap predicate is needed.
      for (int v0 = j; v0 < tend; v0 += 32) {
        int2 kr[2];
        float2 tu[2][4], tv[2][4];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int v = v0 + 16 * m + col;
          kr[m] = v < tend ? krec[v] : make_int2(0, 0);
        }
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            tu[m][q] = tab_u[kr[m].x + 4 * q + grp];
            tv[m][q] = tab_v[kr[m].y + 4 * grp + q];
          }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          if (v0 + 16 * m >= tend) break;   // uniform
          const int v = v0 + 16 * m + col;
          f32x4 z_re = {0.f, 0.f, 0.f, 0.f}, z_im = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            z_re = __builtin_amdgcn_mfma_f32_16x16x4f32(r_re[q], tu[m][q].x, z_re, 0, 0, 0);
            z_im = __builtin_amdgcn_mfma_f32_16x16x4f32(r_im[q], tu[m][q].x, z_im, 0, 0, 0);
            z_re = __builtin_amdgcn_mfma_f32_16x16x4f32(r_im[q], tu[m][q].y, z_re, 0, 0, 0);
            z_im = __builtin_amdgcn_mfma_f32_16x16x4f32(r_re[q], -tu[m][q].y, z_im, 0, 0, 0);
          }
          // V = sum_y conj(Tv[y]) Z[y] over this lane's rows y = 4 grp + rr
          float p_re = 0.f, p_im = 0.f;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            p_re += tv[m][rr].x * z_re[rr] + tv[m][rr].y * z_im[rr];
            p_im += tv[m][rr].x * z_im[rr] - tv[m][rr].y * z_re[rr];
          }
          p_re += __shfl_xor(p_re, 16, 64);
          p_im += __shfl_xor(p_im, 16, 64);
          p_re += __shfl_xor(p_re, 32, 64);
          p_im += __shfl_xor(p_im, 32, 64);
          if (grp == 0 && v < tend) {
            float2 out = make_float2(p_re, p_im);
            if (rot) {  // undo the facet phase rotation: multiply by conj(rot)
              const float2 ro = rot[v];
              out = make_float2(p_re * ro.x + p_im * ro.y, p_im * ro.x - p_re * ro.y);
            }
            vbin[v] = out;
          }
        }
      }
      j = tend;
    }
  }
}

template <int S>
hipError_t launch_s(const DegridArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(degrid_fp32_kernel<S>, dim3(blocks), dim3(64 * kWaves), 0, s, a.items,
                     a.nitems, a.off, a.rec, a.krec, a.rot, a.grid, a.tab_u, a.tab_v, a.N, a.ntx,
                     a.checker, a.vbin);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_degrid_fp32(int S, const DegridArgs& a, int64_t max_items, hipStream_t s) {
  int64_t b = (max_items + kWaves - 1) / kWaves;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  const int blocks = (int)b;
  switch (S) {
    case 1: return launch_s<1>(a, blocks, s);
    case 3: return launch_s<3>(a, blocks, s);
    case 5: return launch_s<5>(a, blocks, s);
    case 7: return launch_s<7>(a, blocks, s);
    case 9: return launch_s<9>(a, blocks, s);
    case 11: return launch_s<11>(a, blocks, s);
    case 13: return launch_s<13>(a, blocks, s);
    case 15: return launch_s<15>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sepw
