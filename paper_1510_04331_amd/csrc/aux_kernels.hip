// Small per-frame kernels: rotation parameters and float64 flux sums.

#include <algorithm>

#include "internal.h"

namespace graphic {

namespace {

// Three-shear factors of Sect. 3.4 for every frame: the rotation R(theta) is
// S_x(-tan(theta/2)) S_y(sin theta) S_x(-tan(theta/2)).  R(theta) has period
// 360 degrees, so theta is first brought to [-180, 180] (IEEE remainder,
// exact).  For |theta| > 90 degrees an exact half-turn is then taken out
// (flip = 1) and theta is reduced by 180 degrees toward zero, so that
// tan(theta/2) stays bounded.
__global__ void rotation_params_kernel(const double* __restrict__ theta_deg, double sign, long long T,
                                       int* __restrict__ flip, double* __restrict__ neg_tan_half,
                                       double* __restrict__ sin_theta) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  double th = remainder(sign * theta_deg[i], 360.0);
  int fl = 0;
  if (fabs(th) > 90.0) {
    fl = 1;
    th = th - copysign(180.0, th);
  }
  const double rad = th * (3.14159265358979323846 / 180.0);
  flip[i] = fl;
  neg_tan_half[i] = -tan(0.5 * rad);
  sin_theta[i] = sin(rad);
}

// One block per frame; float64 partial sums combined in a fixed order, so the
// result does not depend on scheduling.
__global__ void __launch_bounds__(256) frame_sums_kernel(const float* __restrict__ frames, long long npix,
                                                         double* __restrict__ flux, int slot) {
  __shared__ double part[256];
  const long long f = blockIdx.x;
  const float* fr = frames + f * npix;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < npix; i += 256) acc += (double)fr[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) flux[2 * f + slot] = part[0];
}

// Compacted list of the half-turned frames of one chunk (any order; each
// listed frame is processed independently).
__global__ void __launch_bounds__(256) flip_list_kernel(const int* __restrict__ flip, long long f0, long long n,
                                                        int* __restrict__ list, int* __restrict__ count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (long long i = threadIdx.x; i < n; i += 256)
    if (flip[f0 + i] != 0) list[atomicAdd(&cnt, 1)] = (int)i;
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

// Values 100 + U(-8, 8) from a counter hash (no state): a sky-like level with
// noise, written with vector stores only.
__global__ void __launch_bounds__(256) fill_noise_kernel(float* __restrict__ p, size_t n, unsigned seed) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    unsigned h = (unsigned)i * 0x9E3779B1u ^ seed ^ (unsigned)(i >> 32) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    p[i] = 100.0f + ((float)(h >> 8) * (1.0f / 16777216.0f) - 0.5f) * 16.0f;
  }
}

// Non-finite scan: *flag becomes 1 if any of the n values is NaN or +-inf
// (exponent bits all set).  Reads float4 / double2 where the base allows;
// the flag is only written by a block that found one.
__global__ void __launch_bounds__(256) clear_flag_kernel(int* __restrict__ flag) {
  if (threadIdx.x == 0) *flag = 0;
}

__global__ void __launch_bounds__(256) nonfinite_f32_kernel(const float* __restrict__ p, size_t n,
                                                            int* __restrict__ flag) {
  int bad = 0;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    bad |= (__float_as_uint(p[i]) & 0x7f800000u) == 0x7f800000u;
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

__global__ void __launch_bounds__(256) nonfinite_f64_kernel(const double* __restrict__ p, size_t n,
                                                            int* __restrict__ flag) {
  int bad = 0;
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    bad |= ((unsigned long long)__double_as_longlong(p[i]) & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_clear_flag(int* flag, hipStream_t s) {
  hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(256), 0, s, flag);
  return hipGetLastError();
}

hipError_t launch_nonfinite_f32(const float* p, size_t n, int* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(nonfinite_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, flag);
  return hipGetLastError();
}

hipError_t launch_nonfinite_f64(const double* p, size_t n, int* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(nonfinite_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, flag);
  return hipGetLastError();
}

hipError_t launch_fill_noise(float* p, size_t n, unsigned seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_noise_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, seed);
  return hipGetLastError();
}

hipError_t launch_flip_list(const int* flip, long long f0, long long n, int* list, int* count, hipStream_t s) {
  hipLaunchKernelGGL(flip_list_kernel, dim3(1), dim3(256), 0, s, flip, f0, n, list, count);
  return hipGetLastError();
}

hipError_t launch_rotation_params(const double* theta_deg, double sign, long long T, int* flip,
                                  double* neg_tan_half, double* sin_theta, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((T + 255) / 256);
  hipLaunchKernelGGL(rotation_params_kernel, dim3(blocks), dim3(256), 0, s, theta_deg, sign, T, flip,
                     neg_tan_half, sin_theta);
  return hipGetLastError();
}

hipError_t launch_frame_sums(const float* frames, long long T, int N, double* flux, int slot,
                             hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(frame_sums_kernel, dim3((unsigned)T), dim3(256), 0, s, frames, (long long)N * N, flux,
                     slot);
  return hipGetLastError();
}

}  // namespace graphic
