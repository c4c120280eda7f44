// Gridding on the matrix cores (FP32 MFMA).
//
// Section 5: with the separable GCF the update of cell (x, y) by visibility i
// is y_i Tu_i[x] Tv_i[y] (y_i = W_i V_i), and the partial product y_i Tu_i is
// formed once and reused for every row.  Over all visibilities binned into one
// c x c tile this is a complex rank-K update of the tile's 16 x 16 region,
//     R += A_v^T diag(y) A_u,   A_u[i][x] = Tu_i[x - ox_i],  A_v[i][y] = Tv_i[y - oy_i],
// which is exactly an MFMA product with K = visibilities: the B operand carries
// the row product y_i Tu_i (the paper's reuse), the A operand the v-row Tv_i.
// c = 17 - S makes the region exactly 16 cells (c = 2 at S = 15, where 225 of
// the 256 MACs are useful).  Complex arithmetic is four real MFMAs
// (v_mfma_f32_16x16x4f32, K = 4 visibilities per instruction).
//
// One wavefront per work item (a tile, or a <= 512-visibility slice of a heavy
// tile); the region lives in the MFMA accumulators and is added to the grid
// with hardware FP32 atomics (regions of neighbouring tiles overlap by S - 1).
// Lane layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 (l / 16) + r][l % 16].
#include "internal.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

template <int S>
__global__ __launch_bounds__(64 * kWaves) void grid_fp32_kernel(
    const int4* __restrict__ items, const uint32_t* __restrict__ nitems,
    const uint2* __restrict__ rec, const float2* __restrict__ ybin,
    const float2* __restrict__ tab_u, const float2* __restrict__ tab_v, int O, int N, int ntx,
    int checker, float2* __restrict__ grid) {
  constexpr int C = kRegion + 1 - S;   // tile core
  constexpr int H = S / 2;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int n_items = (int)*nitems;
  const int stride = gridDim.x * kWaves;
  float* g = reinterpret_cast<float*>(grid);

  for (int it = blockIdx.x * kWaves + (threadIdx.x >> 6); it < n_items; it += stride) {
    const int4 item = items[it];
    const int ty = item.x / ntx, tx = item.x - ty * ntx;
    const int bx = tx * C, by = ty * C;
    f32x4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
    for (int v0 = 0; v0 < item.z; v0 += 4) {
      const int v = v0 + grp;             // this lane's visibility within the group of 4
      float a_re = 0.f, a_im = 0.f, b_re = 0.f, b_im = 0.f;
      if (v < item.z) {
        const int j = item.y + v;
        const uint2 r = rec[j];
        const float2 y = ybin[j];
        const int row = (int)((r.y >> 16) * (uint32_t)O);
        const int s = col - ((int)(r.x & 0xFFFFu) - bx);   // tap for region column col
        const int t = col - ((int)(r.x >> 16) - by);       // tap for region row col
        if ((unsigned)t < (unsigned)S) {
          const float2 tv = tab_v[(row + (int)((r.y >> 8) & 0xFFu)) * S + t];
          a_re = tv.x;
          a_im = tv.y;
        }
        if ((unsigned)s < (unsigned)S) {
          const float2 tu = tab_u[(row + (int)(r.y & 0xFFu)) * S + s];
          b_re = y.x * tu.x - y.y * tu.y;   // row product W V Tu
          b_im = y.x * tu.y + y.y * tu.x;
        }
      }
      acc_re = __builtin_amdgcn_mfma_f32_16x16x4f32(a_re, b_re, acc_re, 0, 0, 0);
      acc_re = __builtin_amdgcn_mfma_f32_16x16x4f32(-a_im, b_im, acc_re, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f32_16x16x4f32(a_re, b_im, acc_im, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f32_16x16x4f32(a_im, b_re, acc_im, 0, 0, 0);
    }
    const int gx = bx - H + col;
    if (gx >= 0 && gx < N) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gy = by - H + 4 * grp + r;
        if (gy >= 0 && gy < N) {
          const float sg = (checker && ((gx + gy) & 1)) ? -1.f : 1.f;
          const int64_t idx = 2 * ((int64_t)gy * N + gx);
          unsafeAtomicAdd(g + idx, sg * acc_re[r]);
          unsafeAtomicAdd(g + idx + 1, sg * acc_im[r]);
        }
      }
    }
  }
}

template <int S>
hipError_t launch_s(const int4* items, const uint32_t* nitems, const uint2* rec,
                    const float2* ybin, const float2* tu, const float2* tv, int O, int N, int ntx,
                    int checker, float2* grid, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(grid_fp32_kernel<S>, dim3(blocks), dim3(64 * kWaves), 0, s, items, nitems,
                     rec, ybin, tu, tv, O, N, ntx, checker, grid);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_fp32(int S, const int4* items, const uint32_t* nitems, const uint2* rec,
                            const float2* ybin, const float2* tab_u, const float2* tab_v, int O,
                            int N, int tile_c, int ntx, int checker, float2* grid, hipStream_t s,
                            int64_t max_items) {
  (void)tile_c;
  int64_t b = (max_items + kWaves - 1) / kWaves;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  const int blocks = (int)b;
  switch (S) {
    case 1: return launch_s<1>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    case 3: return launch_s<3>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    case 5: return launch_s<5>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    case 7: return launch_s<7>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    case 9: return launch_s<9>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    case 11: return launch_s<11>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    case 13: return launch_s<13>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    case 15: return launch_s<15>(items, nitems, rec, ybin, tab_u, tab_v, O, N, ntx, checker, grid, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sepw
