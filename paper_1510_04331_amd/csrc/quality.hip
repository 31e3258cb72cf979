// Image-quality test of Sect. 4.1 (gfx950): the root mean square of a - b in
// concentric annuli around (cx, cy), per frame.  The paper applies it to the
// difference between an image and its double-shifted (there and back) or
// double-rotated copy; the shifts and rotations are the library's own passes.
//
// Pixel (x, y) (x the column) belongs to annulus k when
// (k w)^2 <= d^2 < ((k + 1) w)^2 with d^2 = (x - cx)^2 + (y - cy)^2, all in
// float64 without contraction, so membership never depends on a rounded
// square root: the first guess floor(sqrt(d^2) / w) is corrected against the
// exact squared bounds.
//
// A block takes kRows rows of one frame, accumulates squared differences and
// pixel counts per annulus in LDS (float64 / uint32 atomics), then adds its
// non-empty annuli to rms[t][k] (float64 atomics) and, for frame 0, to
// counts[k]; a last kernel turns the sums into sqrt(sum / count), NaN for an
// empty annulus.  The float64 sums take the atomics' order, so results agree
// with a sequential sum to rounding, not bit for bit.

#include <algorithm>

#include "internal.h"

namespace graphic {

namespace {

constexpr int kRows = 16;          // rows of a frame per block
constexpr int kThreads = 256;

__global__ void ring_zero_kernel(double* rms, long long n, long long* counts, int n_rings) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) rms[i] = 0.0;
  if (i < n_rings) counts[i] = 0;
}

__device__ __forceinline__ int ring_of(double d2, double w) {
#pragma clang fp contract(off)
  int k = (int)floor(sqrt(d2) / w);
  if (k > 0 && d2 < ((double)k * w) * ((double)k * w)) --k;
  if (d2 >= ((double)(k + 1) * w) * ((double)(k + 1) * w)) ++k;
  return k;
}

__global__ void __launch_bounds__(kThreads) ring_sum_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                           int N, double cx, double cy, double w, int n_rings,
                                                           double* rms, long long* counts) {
#pragma clang fp contract(off)
  extern __shared__ double s_sum[];                     // [n_rings] sums, then [n_rings] uint32 counts
  unsigned* s_cnt = reinterpret_cast<unsigned*>(s_sum + n_rings);
  for (int k = threadIdx.x; k < n_rings; k += kThreads) {
    s_sum[k] = 0.0;
    s_cnt[k] = 0u;
  }
  __syncthreads();
  const long long t = blockIdx.y;
  const int y0 = blockIdx.x * kRows;
  const int rows = min(kRows, N - y0);
  const size_t frame = (size_t)t * N * N;
  for (int i = threadIdx.x; i < rows * N; i += kThreads) {
    const int y = y0 + i / N, x = i % N;
    const double dx = (double)x - cx, dy = (double)y - cy;
    const double d2 = dx * dx + dy * dy;
    const int k = ring_of(d2, w);
    if (k < n_rings) {
      const size_t at = frame + (size_t)y * N + x;
      const double v = b ? (double)a[at] - (double)b[at] : (double)a[at];
      atomicAdd(&s_sum[k], v * v);
      if (t == 0) atomicAdd(&s_cnt[k], 1u);           // every frame has frame 0's annuli
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_rings; k += kThreads) {
    if (s_sum[k] != 0.0) atomicAdd(&rms[t * n_rings + k], s_sum[k]);
    if (t == 0 && s_cnt[k] != 0u)
      atomicAdd(reinterpret_cast<unsigned long long*>(&counts[k]), (unsigned long long)s_cnt[k]);
  }
}

__global__ void ring_finish_kernel(double* rms, long long n, int n_rings, const long long* counts) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long c = counts[i % n_rings];
  rms[i] = c > 0 ? sqrt(rms[i] / (double)c) : __longlong_as_double(0x7ff8000000000000LL);
}

}  // namespace

static size_t annular_rms_lds_bytes(int n_rings) { return (size_t)n_rings * (sizeof(double) + sizeof(unsigned)); }

hipError_t launch_annular_rms(const float* a, const float* b, long long T, int N, double cx, double cy, double width,
                              int n_rings, double* rms, long long* counts, hipStream_t s) {
  if (T <= 0 || N <= 0 || n_rings <= 0 || n_rings > kMaxRings || T > 65535) return hipErrorInvalidValue;
  const long long n = T * n_rings;
  const unsigned zb = (unsigned)((std::max<long long>(n, n_rings) + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(ring_zero_kernel, dim3(zb), dim3(kThreads), 0, s, rms, n, counts, n_rings);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = annular_rms_lds_bytes(n_rings);
  if ((e = set_dynamic_lds(ring_sum_kernel, lds)) != hipSuccess) return e;
  hipLaunchKernelGGL(ring_sum_kernel, dim3((unsigned)((N + kRows - 1) / kRows), (unsigned)T), dim3(kThreads), lds, s,
                     a, b, N, cx, cy, width, n_rings, rms, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(ring_finish_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, rms, n,
                     n_rings, counts);
  return hipGetLastError();
}

}  // namespace graphic
