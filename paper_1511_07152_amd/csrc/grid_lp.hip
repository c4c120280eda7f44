// Precision form: gridding and degridding with FP16 or BF16 MFMA operands and
// FP32 accumulation.
//
// Same tile products as the FP32 path (grid.hip, degrid.hip; Section 5's
// separable update as a rank-K product over the visibilities of a tile), but
// with v_mfma_f32_16x16x16{f16,bf16}: K = 16 visibilities (gridding) or all 16
// region columns (degridding) per instruction.  Operands are scaled so that
// they use the 16-bit range well:
//   * per-plane table scale s_k = max |Re, Im| of the plane's table; the
//     16-bit tables hold T / s_k;
//   * gridding: A = Tv / s_k^v (16-bit table), B = W V (s_k^v Tu) / s formed in
//     FP32 from the u-table pre-multiplied by s_k^v, with s a power of two at
//     least max |Re, Im| (W V) times max_k s_k^u s_k^v over the visibilities
//     gridded into the region so far (it only grows while the region slides,
//     and restarts when the region is flushed whole); when s grows the FP32
//     accumulator is rescaled by the exact power of two s_old / s_new, and
//     flushes multiply by s;
//   * degridding: A = R / s_R with s_R a power of two at least max |Re, Im|
//     over the tile's region, B = conj(Tu / s_k^u) (16-bit table); the FP32
//     epilogue uses the v-table pre-multiplied by s_k^u and multiplies by s_R.
// All tables are zero-padded so that the tap for region index x is base + x.
// Layout of v_mfma_f32_16x16x16: lane l supplies A[l % 16][4 (l / 16) + m] and
// B[4 (l / 16) + m][l % 16] for m = 0..3; accumulator register r of lane l is
// D[4 (l / 16) + r][l % 16].
#include "internal.h"

namespace sepw {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

__device__ inline int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ inline uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <bool BF16>
struct Lp;

template <>
struct Lp<false> {
  typedef f16x4 vec;
  __device__ static void set(vec& v, int m, float x) { v[m] = (_Float16)x; }
  __device__ static void set_bits(vec& v, int m, uint16_t b) { v[m] = __builtin_bit_cast(_Float16, b); }
  __device__ static f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Lp<true> {
  typedef i16x4 vec;
  __device__ static void set(vec& v, int m, float x) { v[m] = (short)bf16_rne(x); }
  __device__ static void set_bits(vec& v, int m, uint16_t b) { v[m] = (short)b; }
  __device__ static f32x4 mfma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

__device__ inline float wave_max(float x) {
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

// smallest power of two >= x (x > 0)
__device__ inline float pow2_ceil(float x) {
  int e;
  float f = frexpf(x, &e);   // x = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, f == 0.5f ? e - 1 : e);
}

__device__ inline float shift_cols(float v, int lane, int col, int sh) {
  float r = __int_as_float(__builtin_amdgcn_ds_bpermute((lane + sh) << 2, __float_as_int(v)));
  return col + sh < 16 ? r : 0.f;
}

__device__ inline void flush_cols(float* g, const f32x4& re, const f32x4& im, float scale,
                                  int col, int grp, int gx0, int gy0, int ncols, int N,
                                  int checker) {
  if (col >= ncols) return;
  const int gx = gx0 + col;
  if (gx < 0 || gx >= N) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gy = gy0 + 4 * grp + r;
    if (gy >= 0 && gy < N) {
      const float sg = (checker && ((gx + gy) & 1)) ? -scale : scale;
      const int64_t idx = 2 * ((int64_t)gy * N + gx);
      unsafeAtomicAdd(g + idx, sg * re[r]);
      unsafeAtomicAdd(g + idx + 1, sg * im[r]);
    }
  }
}

template <int S, bool BF16>
__global__ __launch_bounds__(64 * kWaves) void grid_lp_kernel(
    const int4* __restrict__ items, const uint32_t* __restrict__ nitems,
    const uint32_t* __restrict__ off, const uint2* __restrict__ rec,
    const int2* __restrict__ krec, const float2* __restrict__ ybin,
    const float2* __restrict__ rot, const float2* __restrict__ pad_us,
    const uint32_t* __restrict__ lp_v, const float* __restrict__ lp_bound, int N, int ntx,
    int checker, float2* __restrict__ grid) {
  typedef Lp<BF16> L;
  typedef typename L::vec vec;
  constexpr int C = kRegion + 1 - S;
  constexpr int H = S / 2;
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  const int n_items = (int)*nitems;
  const int stride = gridDim.x * kWaves;
  const float bound = *lp_bound;
  float* g = reinterpret_cast<float*>(grid);

  for (int it = uniform(blockIdx.x * kWaves + (threadIdx.x >> 6)); it < n_items; it += stride) {
    const int4 item = items[it];
    const int ty = uniform(item.x), je = uniform(item.z);
    int j = uniform(item.y);
    const int by = ty * C;
    int tx = uniform((int)(rec[j].x & 0xFFFFu) / C);
    f32x4 acc_re = {0.f, 0.f, 0.f, 0.f}, acc_im = {0.f, 0.f, 0.f, 0.f};
    float scale = 0.f;   // accumulator holds (true sum) / scale; 0 = not yet set
    while (true) {
      const int bx = tx * C;
      const int tend = min(uniform((int)off[ty * ntx + tx + 1]), je);
      for (int v0 = j; v0 < tend; v0 += 16) {
        // lane's visibilities: v0 + 4 grp + m, m = 0..3 (the K slice it supplies)
        float bre[4], bim[4], mx = 0.f;
        vec a_re, a_im, a_nim;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int v = v0 + 4 * grp + m;
          int2 kr = make_int2(0, 0);
          float2 y = make_float2(0.f, 0.f);
          if (v < tend) {
            kr = krec[v];
            y = ybin[v];
            if (rot) {
              const float2 ro = rot[v];
              y = make_float2(y.x * ro.x - y.y * ro.y, y.x * ro.y + y.y * ro.x);
            }
          }
          const uint32_t tv = lp_v[kr.y + col];
          const float2 tu = pad_us[kr.x + col];
          bre[m] = y.x * tu.x - y.y * tu.y;   // row product (u-table times s_k^v)
          bim[m] = y.x * tu.y + y.y * tu.x;
          mx = fmaxf(mx, fmaxf(fabsf(y.x), fabsf(y.y)));
          L::set_bits(a_re, m, (uint16_t)(tv & 0xFFFFu));
          L::set_bits(a_im, m, (uint16_t)(tv >> 16));
          L::set_bits(a_nim, m, (uint16_t)((tv >> 16) ^ 0x8000u));
        }
        mx = wave_max(mx) * bound;
        if (mx > 0.f) {
          const float sn = pow2_ceil(mx);
          if (scale == 0.f) {
            scale = sn;                     // accumulator is still zero
          } else if (sn > scale) {
            const float f = scale / sn;     // exact: both are powers of two
            acc_re *= f;
            acc_im *= f;
            scale = sn;
          }
        }
        const float inv = scale > 0.f ? 1.f / scale : 0.f;
        vec b_re, b_im;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          L::set(b_re, m, bre[m] * inv);
          L::set(b_im, m, bim[m] * inv);
        }
        acc_re = L::mfma(a_re, b_re, acc_re);
        acc_im = L::mfma(a_re, b_im, acc_im);
        acc_re = L::mfma(a_nim, b_im, acc_re);
        acc_im = L::mfma(a_im, b_re, acc_im);
      }
      j = tend;
      if (j >= je) break;
      const int txn = uniform((int)(rec[j].x & 0xFFFFu) / C);
      const int sh = (txn - tx) * C;
      if (sh >= 16) {
        flush_cols(g, acc_re, acc_im, scale, col, grp, bx - H, by - H, 16, N, checker);
        acc_re = f32x4{0.f, 0.f, 0.f, 0.f};
        acc_im = f32x4{0.f, 0.f, 0.f, 0.f};
        scale = 0.f;
      } else {
        flush_cols(g, acc_re, acc_im, scale, col, grp, bx - H, by - H, sh, N, checker);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc_re[r] = shift_cols(acc_re[r], lane, col, sh);
          acc_im[r] = shift_cols(acc_im[r], lane, col, sh);
        }
      }
      tx = txn;
    }
    flush_cols(g, acc_re, acc_im, scale, col, grp, tx * C - H, by - H, 16, N, checker);
  }
}

template <int S, bool BF16>
__global__ __launch_bounds__(64 * kWaves) void degrid_lp_kernel(
    const int4* __restrict__ items, const uint32_t* __restrict__ nitems,
    const uint32_t* __restrict__ off, const uint2* __restrict__ rec,
    const int2* __restrict__ krec, const float2* __restrict__ rot,
    const float2* __restrict__ grid, const uint32_t* __restrict__ lp_u,
    const float2* __restrict__ pad_vs, int N, int ntx, int checker,
    float2* __restrict__ vbin) {
  typedef Lp<BF16> L;
  typedef typename L::vec vec;
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
    const int gy = by - H + col;
    const bool row_ok = gy >= 0 && gy < N;
    while (j < je) {
      const int tx = uniform((int)(rec[j].x & 0xFFFFu) / C);
      const int bx = tx * C;
      const int tend = min(uniform((int)off[ty * ntx + tx + 1]), je);
      // A operand: R[y = col][x = 4 grp + m], scaled by a power of two
      float rre[4], rim[4], mx = 0.f;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int gx = bx - H + 4 * grp + m;
        float2 val = make_float2(0.f, 0.f);
        if (row_ok && gx >= 0 && gx < N) {
          val = grid[(int64_t)gy * N + gx];
          if (checker && ((gx + gy) & 1)) val = make_float2(-val.x, -val.y);
        }
        rre[m] = val.x;
        rim[m] = val.y;
        mx = fmaxf(mx, fmaxf(fabsf(val.x), fabsf(val.y)));
      }
      mx = wave_max(mx);
      const float sr = mx > 0.f ? pow2_ceil(mx) : 1.f;
      const float inv = 1.f / sr;
      vec a_re, a_im;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        L::set(a_re, m, rre[m] * inv);
        L::set(a_im, m, rim[m] * inv);
      }
      for (int v0 = j; v0 < tend; v0 += 16) {
        const int v = v0 + col;   // this lane's visibility (column of Z)
        const bool valid = v < tend;
        const int2 kr = valid ? krec[v] : make_int2(0, 0);
        vec b_re, b_im, b_nim;
        float2 tv[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const uint32_t tu = lp_u[kr.x + 4 * grp + m];
          tv[m] = pad_vs[kr.y + 4 * grp + m];
          L::set_bits(b_re, m, (uint16_t)(tu & 0xFFFFu));
          L::set_bits(b_im, m, (uint16_t)(tu >> 16));
          L::set_bits(b_nim, m, (uint16_t)((tu >> 16) ^ 0x8000u));
        }
        // Z = R conj(Tu): re = Rre Tre + Rim Tim, im = Rim Tre - Rre Tim
        f32x4 z_re = {0.f, 0.f, 0.f, 0.f}, z_im = {0.f, 0.f, 0.f, 0.f};
        z_re = L::mfma(a_re, b_re, z_re);
        z_im = L::mfma(a_im, b_re, z_im);
        z_re = L::mfma(a_im, b_im, z_re);
        z_im = L::mfma(a_re, b_nim, z_im);
        float p_re = 0.f, p_im = 0.f;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          p_re += tv[rr].x * z_re[rr] + tv[rr].y * z_im[rr];
          p_im += tv[rr].x * z_im[rr] - tv[rr].y * z_re[rr];
        }
        p_re += __shfl_xor(p_re, 16, 64);
        p_im += __shfl_xor(p_im, 16, 64);
        p_re += __shfl_xor(p_re, 32, 64);
        p_im += __shfl_xor(p_im, 32, 64);
        if (grp == 0 && valid) {
          float2 out = make_float2(p_re * sr, p_im * sr);
          if (rot) {
            const float2 ro = rot[v];
            out = make_float2(out.x * ro.x + out.y * ro.y, out.y * ro.x - out.x * ro.y);
          }
          vbin[v] = out;
        }
      }
      j = tend;
    }
  }
}

template <int S, bool BF16>
void launch_grid_s(const GridArgsLp& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((grid_lp_kernel<S, BF16>), dim3(blocks), dim3(64 * kWaves), 0, s, a.items,
                     a.nitems, a.off, a.rec, a.krec, a.ybin, a.rot, a.pad_us, a.lp_v, a.lp_bound,
                     a.N, a.ntx, a.checker, a.grid);
}

template <int S, bool BF16>
void launch_degrid_s(const DegridArgsLp& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((degrid_lp_kernel<S, BF16>), dim3(blocks), dim3(64 * kWaves), 0, s, a.items,
                     a.nitems, a.off, a.rec, a.krec, a.rot, a.grid, a.lp_u, a.pad_vs, a.N, a.ntx,
                     a.checker, a.vbin);
}

int blocks_for(int64_t max_items) {
  int64_t b = (max_items + kWaves - 1) / kWaves;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

#define SEPW_LP_CASES(F, A, B, ST)                                                    \
  switch (S) {                                                                     \
    case 1: F<1, B>(A, blocks, ST); break;                                          \
    case 3: F<3, B>(A, blocks, ST); break;                                          \
    case 5: F<5, B>(A, blocks, ST); break;                                          \
    case 7: F<7, B>(A, blocks, ST); break;                                          \
    case 9: F<9, B>(A, blocks, ST); break;                                          \
    case 11: F<11, B>(A, blocks, ST); break;                                        \
    case 13: F<13, B>(A, blocks, ST); break;                                        \
    case 15: F<15, B>(A, blocks, ST); break;                                        \
    default: return hipErrorInvalidValue;                                          \
  }

hipError_t launch_grid_lp(int S, bool bf16, const GridArgsLp& a, int64_t max_items,
                          hipStream_t s) {
  const int blocks = blocks_for(max_items);
  if (bf16) {
    SEPW_LP_CASES(launch_grid_s, a, true, s)
  } else {
    SEPW_LP_CASES(launch_grid_s, a, false, s)
  }
  return hipGetLastError();
}

hipError_t launch_degrid_lp(int S, bool bf16, const DegridArgsLp& a, int64_t max_items,
                            hipStream_t s) {
  const int blocks = blocks_for(max_items);
  if (bf16) {
    SEPW_LP_CASES(launch_degrid_s, a, true, s)
  } else {
    SEPW_LP_CASES(launch_degrid_s, a, false, s)
  }
  return hipGetLastError();
}

#undef SEPW_LP_CASES

}  // namespace sepw
