// W snapshots (Section 4.2): for each snapshot a plane w ~ u d_u + v d_v is
// fitted, the snapshot is imaged with the separable path on the residual
// w' = w - (d_u u + d_v v), and its image, which is the sky in the warped
// coordinate l^s = l + d0 (n(l) - 1), is reprojected: output pixel l takes the
// snapshot image at l^s.  Prediction is the adjoint.
//
// Plane fit (least squares through the origin over the visibilities with
// finite u, v, w): sums Suu, Suv, Svv, Suw, Svw per block of a snapshot, then
// per snapshot in block order (deterministic), d_u = (Suw Svv - Svw Suv) / det,
// d_v = (Svw Suu - Suw Suv) / det with det = Suu Svv - Suv^2, and d0 = 0 unless
// det > 1e-12 Suu Svv.  The residual is formed with explicitly rounded FP64
// operations in that order; its largest magnitude sets the residual w range.
// Reprojection samples the snapshot image at the fractional pixel
// x = l^s N / fov + N/2 (y alike) by separable cubic convolution (Keys,
// a = -1/2) over the 4 x 4 nearest pixels (pixels off the image count 0);
// its transpose sends each pixel back with the same weights (a gather when the
// warp is close to the identity, FP32 atomics otherwise).
#include <algorithm>
#include <cmath>

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

// Block b covers visibilities [range[2b], range[2b + 1]) of one snapshot;
// part[5b + j] = its sums (Suu, Suv, Svv, Suw, Svw).
__global__ __launch_bounds__(kThreads) void snap_sums_kernel(const double* __restrict__ u,
                                                             const double* __restrict__ v,
                                                             const double* __restrict__ w,
                                                             const int64_t* __restrict__ range,
                                                             double* __restrict__ part) {
  __shared__ double red[5][kThreads / 64];
  const int64_t i0 = range[2 * blockIdx.x], i1 = range[2 * blockIdx.x + 1];
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double uu = u[i], vv = v[i], ww = w[i];
    if (!isfinite(uu) || !isfinite(vv) || !isfinite(ww)) continue;
    s[0] += uu * uu;
    s[1] += uu * vv;
    s[2] += vv * vv;
    s[3] += uu * ww;
    s[4] += vv * ww;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double x = s[j];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) red[j][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double t = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) t += red[threadIdx.x][k];
    part[5 * (int64_t)blockIdx.x + threadIdx.x] = t;
  }
}

// d0[s] from the block sums of snapshot s (blocks first[s] .. first[s + 1]).
__global__ void snap_solve_kernel(const double* __restrict__ part, const int* __restrict__ first,
                                  int ns, double2* __restrict__ d0) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = first[s]; b < first[s + 1]; ++b)
    for (int j = 0; j < 5; ++j) t[j] += part[5 * (int64_t)b + j];
  const double suu = t[0], suv = t[1], svv = t[2], suw = t[3], svw = t[4];
  const double det = __dsub_rn(__dmul_rn(suu, svv), __dmul_rn(suv, suv));
  if (!(det > 1e-12 * suu * svv)) {
    d0[s] = make_double2(0.0, 0.0);
    return;
  }
  d0[s] = make_double2(__ddiv_rn(__dsub_rn(__dmul_rn(suw, svv), __dmul_rn(svw, suv)), det),
                       __ddiv_rn(__dsub_rn(__dmul_rn(svw, suu), __dmul_rn(suw, suv)), det));
}

// wr = w - (d_u u + d_v v) per visibility; *maxbits = bits of max |wr| over
// finite values (non-negative doubles order like their bit patterns).
__global__ __launch_bounds__(kThreads) void snap_residual_kernel(
    const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
    const int64_t* __restrict__ range, const int* __restrict__ snap, const double2* __restrict__ d0,
    double* __restrict__ wr, unsigned long long* __restrict__ maxbits) {
  __shared__ double red[kThreads / 64];
  const int64_t i0 = range[2 * blockIdx.x], i1 = range[2 * blockIdx.x + 1];
  const double2 d = d0[snap[blockIdx.x]];
  double m = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
    const double r = __dsub_rn(w[i], __dadd_rn(__dmul_rn(d.x, u[i]), __dmul_rn(d.y, v[i])));
    wr[i] = r;
    if (isfinite(r)) m = fmax(m, fabs(r));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kThreads / 64; ++k) m = fmax(m, red[k]);
    atomicMax(maxbits, (unsigned long long)__double_as_longlong(m));
  }
}

// Keys' cubic convolution kernel (a = -1/2) at distance t, in FP32: the
// weights are FP32 anyway, and t, at most 2 pixels, is formed in FP64 first.
__device__ inline float keys(float t) {
  t = fabsf(t);
  if (t <= 1.f) return (1.5f * t - 2.5f) * t * t + 1.f;
  if (t < 2.f) return ((-0.5f * t + 2.5f) * t - 4.f) * t + 2.f;
  return 0.f;
}

struct Taps {
  int i0;          // first tap pixel
  float wt[4];     // weights (0 for taps off the image)
};

__device__ inline Taps taps(double x, int N) {
  Taps t;
  const double x0 = floor(x);
  const double f = x - x0;
  t.i0 = (int)x0 - 1;
  const float wd[4] = {keys((float)(1.0 + f)), keys((float)f), keys((float)(1.0 - f)),
                        keys((float)(2.0 - f))};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int i = t.i0 + k;
    t.wt[k] = (i >= 0 && i < N) ? wd[k] : 0.f;
  }
  return t;
}

// Fractional pixel coordinates of l^s, m^s for output pixel (p, q), and n:
// x = l^s N / fov + N/2 = p + d_u (n - 1) N / fov (y alike).  step and pix do
// not depend on the pixel (the compiler hoists them out of pixel loops), so a
// sample point costs one square root and one division.
__device__ inline void sample_point(int p, int q, int N, double fov, double du, double dv,
                                    double& x, double& y, double& n) {
  const double step = fov / (double)N, pix = (double)N / fov;
  const double l = (double)(p - N / 2) * step, m = (double)(q - N / 2) * step;
  const double r2 = l * l + m * m;
  n = sqrt(1.0 - r2);
  const double nm1 = -r2 / (1.0 + n);
  x = (double)p + du * nm1 * pix;
  y = (double)q + dv * nm1 * pix;
}

// out (+)= the snapshot image sampled at l^s
__global__ void snap_reproject_kernel(const float2* __restrict__ in, float2* __restrict__ out, int N,
                                      double fov, double du, double dv, int accumulate) {
  const int64_t total = (int64_t)N * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t ue = (uint32_t)e;   // N <= 32768: pixel indices fit 32 bits
    const int q = (int)(ue / (uint32_t)N), p = (int)(ue - (uint32_t)q * (uint32_t)N);
    double x, y, n;
    sample_point(p, q, N, fov, du, dv, x, y, n);
    float sr = 0.f, si = 0.f;
    if (fabs(x) < 4.0 * N && fabs(y) < 4.0 * N) {
      const Taps tx = taps(x, N), ty = taps(y, N);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (ty.wt[j] == 0.f) continue;
        const float2* row = in + (int64_t)(ty.i0 + j) * N;
        float rr = 0.f, ri = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (tx.wt[i] == 0.f) continue;
          const float2 g = row[tx.i0 + i];
          rr += tx.wt[i] * g.x;
          ri += tx.wt[i] * g.y;
        }
        sr += ty.wt[j] * rr;
        si += ty.wt[j] * ri;
      }
    }
    if (accumulate) {
      const float2 o = out[e];
      out[e] = make_float2(o.x + sr, o.y + si);
    } else {
      out[e] = make_float2(sr, si);
    }
  }
}

// out += transpose of the reprojection applied to X n^npow (out zeroed first)
__global__ void snap_reproject_adjoint_kernel(const float2* __restrict__ X, float2* __restrict__ out,
                                              int N, double fov, double du, double dv, int npow) {
  const int64_t total = (int64_t)N * N;
  float* o = reinterpret_cast<float*>(out);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t ue = (uint32_t)e;   // N <= 32768: pixel indices fit 32 bits
    const int q = (int)(ue / (uint32_t)N), p = (int)(ue - (uint32_t)q * (uint32_t)N);
    double x, y, n;
    sample_point(p, q, N, fov, du, dv, x, y, n);
    if (!(fabs(x) < 4.0 * N && fabs(y) < 4.0 * N)) continue;
    float2 val = X[e];
    if (npow) {
      const float s = (float)(npow > 0 ? n : 1.0 / n);
      val = make_float2(val.x * s, val.y * s);
    }
    const Taps tx = taps(x, N), ty = taps(y, N);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (ty.wt[j] == 0.f) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float wgt = ty.wt[j] * tx.wt[i];
        if (wgt == 0.f) continue;
        float* c = o + 2 * ((int64_t)(ty.i0 + j) * N + tx.i0 + i);
        atomicAdd(c, wgt * val.x);
        atomicAdd(c + 1, wgt * val.y);
      }
    }
  }
}

// Gather form of the transpose, for warps close to the identity.  Snapshot
// pixel j receives w(x_b - j_x) w(y_b - j_y) X'_b from every output pixel b
// whose sample point (x_b, y_b) = g(b) lies within 2 pixels of j on both axes
// (the same weights as the forward sampling), and is written (not added).  A
// workgroup takes 16 x 16 snapshot pixels: the pre-image p* of the tile centre
// c comes from the fixed-point iteration p <- p + (c - g(p)); the sample
// points and values of the 26 x 26 output pixels from floor(p*) - 12 go to
// LDS.  Each
// pixel then refines its own pre-image by one more iteration from
// p* + (j - c), and scans the 5 x 5 output pixels from ceil(q - 2.32).
// With the warp's Jacobian within eps <= 0.1 of the identity (max-norm):
// |g(b) - g(p_j)| >= (1 - eps) |b - p_j|, so every contributor lies within
// 2 / (1 - eps) < 2.223 of p_j; the start p* + (j - c) is within
// eps |j - c| / (1 - eps) < 0.84 of p_j and the iteration shrinks the error
// by eps, so the refined q is within 0.084 of p_j: every contributor lies in
// [q - 2.307, q + 2.307], whose integers (at most five) are the ones scanned.
// All of them lie in [p* - 10.8, p* + 11.2], inside the box.  The
// launcher checks the bound and otherwise zeroes the output and uses the
// scatter kernel above.
constexpr int kGTile = 16, kGBox = 26, kGScan = 5;

__device__ inline void warp_at(double p, double q, int N, double fov, double du, double dv,
                               double& x, double& y) {
  const double step = fov / (double)N, pix = (double)N / fov;
  const double l = (p - (double)(N / 2)) * step, m = (q - (double)(N / 2)) * step;
  const double r2 = l * l + m * m;
  const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));
  x = p + du * nm1 * pix;
  y = q + dv * nm1 * pix;
}

__global__ __launch_bounds__(kGTile * kGTile) void snap_adjoint_gather_kernel(
    const float2* __restrict__ X, float2* __restrict__ out, int N, double fov, double du, double dv,
    int npow, const double* __restrict__ c1) {
  __shared__ double sx[kGBox * kGBox], sy[kGBox * kGBox];
  __shared__ float2 sv[kGBox * kGBox];
  const int tx0 = blockIdx.x * kGTile, ty0 = blockIdx.y * kGTile;
  const double cx = tx0 + 0.5 * (kGTile - 1), cy = ty0 + 0.5 * (kGTile - 1);
  double px = cx, py = cy;
  for (int it = 0; it < 8; ++it) {
    double x, y;
    warp_at(px, py, N, fov, du, dv, x, y);
    px += cx - x;
    py += cy - y;
  }
  const int ox = (int)floor(px) - 12, oy = (int)floor(py) - 12;   // box origin
  for (int e = threadIdx.x; e < kGBox * kGBox; e += kGTile * kGTile) {
    const int bp = ox + (e % kGBox), bq = oy + (e / kGBox);
    double x = 1e300, y = 1e300;
    float2 val = make_float2(0.f, 0.f);
    if (bp >= 0 && bp < N && bq >= 0 && bq < N) {
      double n;
      sample_point(bp, bq, N, fov, du, dv, x, y, n);
      if (fabs(x) < 4.0 * N && fabs(y) < 4.0 * N) {
        val = X[(int64_t)bq * N + bp];
        if (npow) {
          const float s = (float)(npow > 0 ? n : 1.0 / n);
          val = make_float2(val.x * s, val.y * s);
        }
      } else {
        x = y = 1e300;
      }
    }
    sx[e] = x;
    sy[e] = y;
    sv[e] = val;
  }
  __syncthreads();
  const int jx = tx0 + (threadIdx.x % kGTile), jy = ty0 + (threadIdx.x / kGTile);
  if (jx >= N || jy >= N) return;
  // this pixel's pre-image, from the tile's translation and one iteration
  double qx = px + (jx - cx), qy = py + (jy - cy);
  {
    double x, y;
    warp_at(qx, qy, N, fov, du, dv, x, y);
    qx += jx - x;
    qy += jy - y;
  }
  const int cp = (int)ceil(qx - 2.32) - ox, cq = (int)ceil(qy - 2.32) - oy;
  float ar = 0.f, ai = 0.f;
  for (int b = 0; b < kGScan; ++b) {
    const int qq = cq + b;
    if (qq < 0 || qq >= kGBox) continue;
    for (int a = 0; a < kGScan; ++a) {
      const int pp = cp + a;
      if (pp < 0 || pp >= kGBox) continue;
      const int e = qq * kGBox + pp;
      const double dx = sx[e] - (double)jx, dy = sy[e] - (double)jy;
      if (fabs(dx) < 2.0 && fabs(dy) < 2.0) {
        const float wgt = keys((float)dy) * keys((float)dx);
        ar += wgt * sv[e].x;
        ai += wgt * sv[e].y;
      }
    }
  }
  if (c1) {
    // the snapshot image's correction before its FFT, as the separate pass
    // would apply it: (-1)^(p+q) / (c1[p] c1[q]) in FP64
    double f = 1.0 / (c1[jx] * c1[jy]);
    if ((jx + jy) & 1) f = -f;
    ar = (float)(ar * f);
    ai = (float)(ai * f);
  }
  out[(int64_t)jy * N + jx] = make_float2(ar, ai);
}

// out *= n^npow
__global__ void snap_npow_kernel(float2* __restrict__ out, int N, double fov, int npow) {
  const int64_t total = (int64_t)N * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t ue = (uint32_t)e;   // N <= 32768: pixel indices fit 32 bits
    const int q = (int)(ue / (uint32_t)N), p = (int)(ue - (uint32_t)q * (uint32_t)N);
    double x, y, n;
    sample_point(p, q, N, fov, 0.0, 0.0, x, y, n);
    const float s = (float)(npow > 0 ? n : 1.0 / n);
    const float2 v = out[e];
    out[e] = make_float2(v.x * s, v.y * s);
  }
}

}  // namespace

hipError_t launch_snap_fit(const double* u, const double* v, const double* w, const int64_t* range,
                           const int* snap, const int* first, int nblocks, int ns, double* part,
                           double2* d0, double* wr, unsigned long long* maxbits, hipStream_t s) {
  if (nblocks > 0) {
    hipLaunchKernelGGL(snap_sums_kernel, dim3((unsigned)nblocks), dim3(kThreads), 0, s, u, v, w,
                       range, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(snap_solve_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, part,
                     first, ns, d0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nblocks == 0) return e;
  hipLaunchKernelGGL(snap_residual_kernel, dim3((unsigned)nblocks), dim3(kThreads), 0, s, u, v, w,
                     range, snap, d0, wr, maxbits);
  return hipGetLastError();
}

hipError_t launch_snap_reproject(const float2* in, float2* out, int N, double fov, double du,
                                 double dv, bool accumulate, hipStream_t s) {
  hipLaunchKernelGGL(snap_reproject_kernel, grid_for((int64_t)N * N), dim3(kThreads), 0, s, in, out,
                     N, fov, du, dv, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_snap_reproject_adjoint(const float2* X, float2* out, int N, double fov, double du,
                                         double dv, int npow, const double* c1, hipStream_t s) {
  // bound on the warp's deviation from the identity: max |d| (|l| + |m|) / n
  // over the image, |l|, |m| <= fov / 2
  const double eps = std::max(std::fabs(du), std::fabs(dv)) * fov / std::sqrt(1.0 - 0.5 * fov * fov);
  if (eps <= 0.1) {
    const unsigned nt = (unsigned)((N + kGTile - 1) / kGTile);
    hipLaunchKernelGGL(snap_adjoint_gather_kernel, dim3(nt, nt), dim3(kGTile * kGTile), 0, s, X, out,
                       N, fov, du, dv, npow, c1);
  } else {
    hipError_t e = launch_zero_c64(out, (int64_t)N * N, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(snap_reproject_adjoint_kernel, grid_for((int64_t)N * N), dim3(kThreads), 0, s,
                       X, out, N, fov, du, dv, npow);
    e = hipGetLastError();
    if (e == hipSuccess && c1) e = launch_correct(out, out, c1, N, fov, 0.0, 0.0, 0, s);
    return e;
  }
  return hipGetLastError();
}

hipError_t launch_snap_npow(float2* out, int N, double fov, int npow, hipStream_t s) {
  hipLaunchKernelGGL(snap_npow_kernel, grid_for((int64_t)N * N), dim3(kThreads), 0, s, out, N, fov,
                     npow);
  return hipGetLastError();
}

}  // namespace sepw
