// Gridding on the matrix cores (FP32 MFMA).
//
// Section 5: with the separable GCF the update of cell (x, y) by visibility i
// is y_i Tu_i[x] Tv_i[y] (y_i = W_i V_i), and the partial product y_i Tu_i is
// formed once and reused for every row.  Over the visibilities binned into one
// c x c tile this is a complex rank-K update of the tile's 16 x 16 region,
//     R += A_v^T diag(y) A_u,   A_u[i][x] = Tu_i[x - ox_i],  A_v[i][y] = Tv_i[y - oy_i],
// an MFMA product with K = visibilities: the B operand carries the row product
// y_i Tu_i (the paper's reuse), the A operand the v-row Tv_i.  c = 17 - S makes
// the region exactly 16 cells (c = 2 at S = 15: 225 of 256 MACs useful).
// Complex arithmetic is four real v_mfma_f32_16x16x4f32 per 4 visibilities.
//
// Work item: a slice of <= kItemMaxVis binned visibilities from one row of
// tiles (tiles are sorted row-major, so a slice walks left to right).  The
// region accumulator slides with the tile: moving right by d tiles flushes the
// d*c columns that leave the region (hardware FP32 atomics; regions of
// neighbouring tiles overlap by S - 1) and shifts the rest across lanes.  W V
// arrives already in binned order (moved there by the plan's placement maps),
// so every operand load is a streaming read; the facet rotation is applied
// here.
// Lane layout of v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 (l / 16) + r][l % 16],
// so region column x = l % 16 and region row y = 4 (l / 16) + r.
#include "internal.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

__device__ inline int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// value of lane (lane + sh) within the same 16-lane row, 0 past the row end
__device__ inline float shift_cols(float v, int lane, int col, int sh) {
  float r = __int_as_float(__builtin_amdgcn_ds_bpermute((lane + sh) << 2, __float_as_int(v)));
  return col + sh < 16 ? r : 0.f;
}

// Add columns [0, ncols) of the region whose top-left cell is (gx0, gy0).
__device__ inline void flush_cols(float* g, const f32x4& re, const f32x4& im, int col, int grp,
                                  int gx0, int gy0, int ncols, int N, int checker) {
  if (col >= ncols) return;
  const int gx = gx0 + col;
  if (gx < 0 || gx >= N) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gy = gy0 + 4 * grp + r;
    if (gy >= 0 && gy < N) {
      const float sg = (checker && ((gx + gy) & 1)) ? -1.f : 1.f;
      const int64_t idx = 2 * ((int64_t)gy * N + gx);
      unsafeAtomicAdd(g + idx, sg * re[r]);
      unsafeAtomicAdd(g + idx + 1, sg * im[r]);
    }
  }
}

// One work item (a slice of one row of tiles) of one gridding job.
template <int S>
__device__ inline void grid_item(const GridArgs& a, int it, int lane, int col, int grp) {
  constexpr int C = kRegion + 1 - S;   // tile core
  constexpr int H = S / 2;
  const int N = a.N, ntx = a.ntx, checker = a.checker;
  const int2* __restrict__ krec = a.krec;
  const float2* __restrict__ ybin = a.ybin;
  const float2* __restrict__ rot = a.rot;
  const float2* __restrict__ tab_u = a.tab_u;
  const float2* __restrict__ tab_v = a.tab_v;
  float* g = reinterpret_cast<float*>(a.grid);
  const int4 item = a.items[it];
  const int ty = uniform(item.x), je = uniform(item.z);
  int j = uniform(item.y);
  const int by = ty * C;
  int tx = uniform((int)(a.rec[j].x & 0xFFFFu) / C);
  f32x4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
  while (true) {
    const int bx = tx * C;
    const int tend = min(uniform((int)a.off[ty * ntx + tx + 1]), je);
    // 16 visibilities per iteration, four MFMA groups; lane (col, grp) supplies
    // region row/column col of visibility v0 + 4 m + grp.  The padded tables
    // make tap col of a visibility simply base + col.
    for (int v0 = j; v0 < tend; v0 += 16) {
      int2 kr[4];
      float2 yv[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int v = v0 + 4 * m + grp;
        kr[m] = make_int2(0, 0);
        yv[m] = make_float2(0.f, 0.f);   // padding visibilities carry zero weight
        if (v < tend) {
          kr[m] = krec[v];
          yv[m] = ybin[v];
          if (rot) {
            const float2 ro = rot[v];
            yv[m] = make_float2(yv[m].x * ro.x - yv[m].y * ro.y, yv[m].x * ro.y + yv[m].y * ro.x);
          }
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const float2 tv = tab_v[kr[m].y + col];
        const float2 tu = tab_u[kr[m].x + col];
        const float b_re = yv[m].x * tu.x - yv[m].y * tu.y;   // row product W V Tu
        const float b_im = yv[m].x * tu.y + yv[m].y * tu.x;
        if (v0 + 4 * m < tend) {   // uniform: skip all-padding groups
          acc_re = __builtin_amdgcn_mfma_f32_16x16x4f32(tv.x, b_re, acc_re, 0, 0, 0);
          acc_im = __builtin_amdgcn_mfma_f32_16x16x4f32(tv.x, b_im, acc_im, 0, 0, 0);
          acc_re = __builtin_amdgcn_mfma_f32_16x16x4f32(-tv.y, b_im, acc_re, 0, 0, 0);
          acc_im = __builtin_amdgcn_mfma_f32_16x16x4f32(tv.y, b_re, acc_im, 0, 0, 0);
        }
      }
    }
    j = tend;
    if (j >= je) break;
    // slide the region to the next non-empty tile of the row
    const int txn = uniform((int)(a.rec[j].x & 0xFFFFu) / C);
    const int sh = (txn - tx) * C;
    if (sh >= 16) {
      flush_cols(g, acc_re, acc_im, col, grp, bx - H, by - H, 16, N, checker);
      acc_re = f32x4{0.f, 0.f, 0.f, 0.f};
      acc_im = f32x4{0.f, 0.f, 0.f, 0.f};
    } else {
      flush_cols(g, acc_re, acc_im, col, grp, bx - H, by - H, sh, N, checker);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc_re[r] = shift_cols(acc_re[r], lane, col, sh);
        acc_im[r] = shift_cols(acc_im[r], lane, col, sh);
      }
    }
    tx = txn;
  }
  flush_cols(g, acc_re, acc_im, col, grp, tx * C - H, by - H, 16, N, checker);
}

template <int S>
__global__ __launch_bounds__(64 * kWaves) void grid_fp32_kernel(GridArgs a) {
  const int lane = threadIdx.x & 63;
  const int n_items = (int)*a.nitems;
  const int stride = gridDim.x * kWaves;
  for (int it = uniform(blockIdx.x * kWaves + (threadIdx.x >> 6)); it < n_items; it += stride)
    grid_item<S>(a, it, lane, lane & 15, lane >> 4);
}

// Persistent launch over the work items of many jobs (facets, snapshots):
// waves take (job, item) pairs from one atomic counter over the concatenated
// item lists (jobs ordered by decreasing size on the host), so uneven jobs
// share the GPU without a launch per job.
template <int S>
__global__ __launch_bounds__(64 * kWaves) void grid_fp32_batched_kernel(
    const GridArgs* __restrict__ jobs, const uint32_t* __restrict__ first, int njobs,
    uint32_t* __restrict__ counter) {
  const int lane = threadIdx.x & 63;
  const uint32_t total = first[njobs];
  while (true) {
    uint32_t gi = 0;
    if (lane == 0) gi = atomicAdd(counter, 1u);
    gi = (uint32_t)uniform((int)__shfl(gi, 0, 64));
    if (gi >= total) break;
    int lo = 0, hi = njobs - 1;   // last job with first[job] <= gi
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (first[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    const int job = uniform(lo);
    grid_item<S>(jobs[job], (int)(gi - first[job]), lane, lane & 15, lane >> 4);
  }
}

template <int S>
hipError_t launch_s(const GridArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(grid_fp32_kernel<S>, dim3(blocks), dim3(64 * kWaves), 0, s, a);
  return hipGetLastError();
}

template <int S>
hipError_t launch_batched_s(const GridArgs* jobs, const uint32_t* first, int njobs,
                            uint32_t* counter, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(grid_fp32_batched_kernel<S>, dim3(blocks), dim3(64 * kWaves), 0, s, jobs,
                     first, njobs, counter);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_grid_fp32_batched(int S, const GridArgs* jobs, const uint32_t* first, int njobs,
                                    uint32_t* counter, int blocks, hipStream_t s) {
  switch (S) {
    case 1: return launch_batched_s<1>(jobs, first, njobs, counter, blocks, s);
    case 3: return launch_batched_s<3>(jobs, first, njobs, counter, blocks, s);
    case 5: return launch_batched_s<5>(jobs, first, njobs, counter, blocks, s);
    case 7: return launch_batched_s<7>(jobs, first, njobs, counter, blocks, s);
    case 9: return launch_batched_s<9>(jobs, first, njobs, counter, blocks, s);
    case 11: return launch_batched_s<11>(jobs, first, njobs, counter, blocks, s);
    case 13: return launch_batched_s<13>(jobs, first, njobs, counter, blocks, s);
    case 15: return launch_batched_s<15>(jobs, first, njobs, counter, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_grid_fp32(int S, const GridArgs& a, int64_t max_items, hipStream_t s) {
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
