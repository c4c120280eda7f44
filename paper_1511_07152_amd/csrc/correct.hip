// Grid correction around the FFT.
//
// Section 2: the image is F^-1 of the convolved grid divided by c, the inverse
// transform of the anti-aliasing kernel; with Section 3's separable taper
// c(l, m) = c1(l) c1(m).  The dirty-image equation carries a factor n on the
// left (I_D / n), the prediction equation a factor 1/n on the model (I / n).
// The FFT library computes the uncentred transform, so the centred one
// (pixel p at l_p = (p - N/2) fov/N, cell j at u_j = (j - N/2)/fov) also needs
// the checkerboard (-1)^(p+q) on the image side; the grid-side checkerboard
// is folded into the gridding/degridding kernels.
//
//   out[q][p] = in[q][p] (-1)^(p+q) n(l0 + l_p, m0 + m_q)^npow / (c1[p] c1[q])
//
// One pass over the N x N complex64 image (HBM-bound); n and the taper ratio
// are formed in FP64.  For real images the input (prediction from a real
// model) or the output (the real part of an image, for the adjoint of a real
// model's prediction) is float32, read or written by the same pass.
#include "internal.h"

namespace sepw {

namespace {

// in and out may be the same array (in-place correction): each element is
// read once and then written by the same thread, so neither is __restrict__.
// MODE: 0 complex -> complex, 1 real -> complex, 2 complex -> real part.
template <int MODE>
__global__ void correct_kernel(const void* in_, void* out_, const double* __restrict__ c1, int N,
                               double fov, double l0, double m0, int npow) {
  const int64_t total = (int64_t)N * N;
  const double step = fov / (double)N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t ui = (uint32_t)i;   // N <= 32768: pixel indices fit 32 bits
    const int q = (int)(ui / (uint32_t)N), p = (int)(ui - (uint32_t)q * (uint32_t)N);
    double f = 1.0 / (c1[p] * c1[q]);
    if (npow != 0) {
      const double l = l0 + (double)(p - N / 2) * step;
      const double m = m0 + (double)(q - N / 2) * step;
      const double n = sqrt(1.0 - l * l - m * m);
      f = npow > 0 ? f * n : f / n;
    }
    if ((p + q) & 1) f = -f;
    if constexpr (MODE == 1) {
      const float v = static_cast<const float*>(in_)[i];
      static_cast<float2*>(out_)[i] = make_float2((float)(v * f), 0.f);
    } else {
      const float2 v = static_cast<const float2*>(in_)[i];
      if constexpr (MODE == 2)
        static_cast<float*>(out_)[i] = (float)(v.x * f);
      else
        static_cast<float2*>(out_)[i] = make_float2((float)(v.x * f), (float)(v.y * f));
    }
  }
}

}  // namespace

namespace {
dim3 correct_blocks(int N) {
  int64_t total = (int64_t)N * N;
  int64_t b = (total + 255) / 256;
  if (b > 16384) b = 16384;
  return dim3((unsigned)b);
}
}  // namespace

hipError_t launch_correct(const float2* in, float2* out, const double* c1, int N, double fov,
                          double l0, double m0, int npow, hipStream_t s) {
  hipLaunchKernelGGL(correct_kernel<0>, correct_blocks(N), dim3(256), 0, s,
                     static_cast<const void*>(in), static_cast<void*>(out), c1, N, fov, l0, m0, npow);
  return hipGetLastError();
}

hipError_t launch_correct_real_in(const float* in, float2* out, const double* c1, int N, double fov,
                                  double l0, double m0, int npow, hipStream_t s) {
  hipLaunchKernelGGL(correct_kernel<1>, correct_blocks(N), dim3(256), 0, s,
                     static_cast<const void*>(in), static_cast<void*>(out), c1, N, fov, l0, m0, npow);
  return hipGetLastError();
}

hipError_t launch_correct_real_out(const float2* in, float* out, const double* c1, int N,
                                   double fov, double l0, double m0, int npow, hipStream_t s) {
  hipLaunchKernelGGL(correct_kernel<2>, correct_blocks(N), dim3(256), 0, s,
                     static_cast<const void*>(in), static_cast<void*>(out), c1, N, fov, l0, m0, npow);
  return hipGetLastError();
}

}  // namespace sepw
