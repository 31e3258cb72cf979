// Image pre-processing (Sect. 3.2, 3.2.1 and 3.2.2): star masks, nearest-sky
// subtraction, the bad pixel map of one frame (median and standard deviation
// of its finite pixels) and the neighbour repair of bad pixels.
//
// The frame median is an exact radix select over totalOrder keys: four 8-bit
// digits, each a histogram kept per block (no global atomics) and merged in a
// fixed order by one block, so the result does not depend on scheduling.
// Sums (mean, standard deviation) are float64 in two passes with per-block
// partials merged in a fixed order.

#include <cmath>

#include "internal.h"

namespace graphic {

namespace {

constexpr int kPreBlocks = 256;          // blocks of the frame reductions
constexpr int kPreThreads = 256;

__device__ __forceinline__ unsigned pkey(float v) {
  const unsigned b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float pval(unsigned k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__global__ void mask_disk_kernel(float* __restrict__ cube, long long T, int n, const double* __restrict__ xs,
                                 const double* __restrict__ ys, double r2) {
  const long long npix = (long long)n * n;
  const long long f = blockIdx.y;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (long long)gridDim.x * blockDim.x) {
    const double dx = (double)(i % n) - xs[f], dy = (double)(i / n) - ys[f];
    if (dx * dx + dy * dy <= r2) cube[f * npix + i] = __int_as_float(0x7FC00000);
  }
}

__global__ void subtract_nearest_kernel(float* __restrict__ cube, long long T, int n,
                                        const double* __restrict__ times, const float* __restrict__ skies,
                                        const double* __restrict__ sky_times, int S) {
  const long long npix = (long long)n * n;
  const long long f = blockIdx.y;
  const double t = times[f];
  int best = 0;
  double bd = fabs(sky_times[0] - t);
  for (int s = 1; s < S; ++s) {
    const double d = fabs(sky_times[s] - t);
    if (d < bd) {
      bd = d;
      best = s;
    }
  }
  const float* sky = skies + (size_t)best * npix;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (long long)gridDim.x * blockDim.x)
    cube[f * npix + i] = cube[f * npix + i] - sky[i];
}

// ---- frame statistics ----
// state: [0] prefix, [1] rank, [2] count in the chosen bin, [3] finite count,
//        [4] smallest key above lo (reduced), [5] digit position
struct FrameSel {
  unsigned prefix, rank, inbin, count, above, pad;
  double mean, sigma, median;
};

// Pass over the frame: per-block partial count and sum of finite values.
__global__ void __launch_bounds__(kPreThreads) stat_sum_kernel(const float* __restrict__ v, long long npix,
                                                               double* __restrict__ part /* [blocks][2] */) {
  __shared__ double s[2][kPreThreads];
  double c = 0.0, m = 0.0;
  for (long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x; i < npix; i += (long long)gridDim.x * kPreThreads)
    if (isfinite(v[i])) {
      c += 1.0;
      m += (double)v[i];
    }
  s[0][threadIdx.x] = c;
  s[1][threadIdx.x] = m;
  __syncthreads();
  for (int w = kPreThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s[0][0];
    part[2 * blockIdx.x + 1] = s[1][0];
  }
}

// Per-block partial sum of squared deviations from the mean.
__global__ void __launch_bounds__(kPreThreads) stat_dev_kernel(const float* __restrict__ v, long long npix,
                                                               const FrameSel* __restrict__ st,
                                                               double* __restrict__ part) {
  __shared__ double s[kPreThreads];
  const double mean = st->mean;
  double q = 0.0;
  for (long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x; i < npix; i += (long long)gridDim.x * kPreThreads)
    if (isfinite(v[i])) {
      const double d = (double)v[i] - mean;
      q += d * d;
    }
  s[threadIdx.x] = q;
  __syncthreads();
  for (int w = kPreThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// One block: merges partials in block order.  mode 0: count and mean, and the
// select's start; mode 1: sigma.
__global__ void __launch_bounds__(kPreThreads) stat_merge_kernel(const double* __restrict__ part, int nblocks,
                                                                 int mode, FrameSel* __restrict__ st) {
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    double c = 0.0, m = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      c += part[2 * b];
      m += part[2 * b + 1];
    }
    st->count = (unsigned)c;
    st->mean = c > 0.0 ? m / c : 0.0;
    st->prefix = 0u;
    st->rank = st->count == 0u ? 0u : (st->count - 1u) / 2u;
    st->above = 0xFFFFFFFFu;
  } else {
    double q = 0.0;
    for (int b = 0; b < nblocks; ++b) q += part[b];
    st->sigma = st->count > 0u ? sqrt(q / (double)st->count) : 0.0;
  }
}

// Per-block histogram of digit `d` of the finite keys that carry the prefix.
__global__ void __launch_bounds__(kPreThreads) sel_hist_kernel(const float* __restrict__ v, long long npix, int d,
                                                               const FrameSel* __restrict__ st,
                                                               unsigned* __restrict__ hist /* [blocks][256] */) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned mask = d == 3 ? 0u : (0xFFFFFFFFu << (8 * (d + 1)));
  const unsigned prefix = st->prefix;
  for (long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x; i < npix; i += (long long)gridDim.x * kPreThreads) {
    const float x = v[i];
    if (!isfinite(x)) continue;
    const unsigned k = pkey(x);
    if ((k & mask) == prefix) atomicAdd(&h[(k >> (8 * d)) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[blockIdx.x * 256 + threadIdx.x] = h[threadIdx.x];
}

// One block: merges the block histograms (fixed order) and picks the bin of
// the current rank.
__global__ void __launch_bounds__(256) sel_pick_kernel(const unsigned* __restrict__ hist, int nblocks, int d,
                                                       FrameSel* __restrict__ st) {
  __shared__ unsigned c[256];
  unsigned x = 0u;
  for (int b = 0; b < nblocks; ++b) x += hist[b * 256 + threadIdx.x];
  c[threadIdx.x] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned k = st->rank;
    unsigned below = 0u;
    int bin = 255;
    for (int i = 0; i < 256; ++i) {
      if (below + c[i] > k) {
        bin = i;
        break;
      }
      below += c[i];
    }
    st->prefix |= (unsigned)bin << (8 * d);
    st->rank = k - below;
    st->inbin = c[bin];
  }
}

// Per-block smallest finite key above lo.
__global__ void __launch_bounds__(kPreThreads) sel_above_kernel(const float* __restrict__ v, long long npix,
                                                                const FrameSel* __restrict__ st,
                                                                unsigned* __restrict__ part) {
  __shared__ unsigned s[kPreThreads];
  const unsigned lo = st->prefix;
  unsigned m = 0xFFFFFFFFu;
  for (long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x; i < npix; i += (long long)gridDim.x * kPreThreads) {
    const float x = v[i];
    if (!isfinite(x)) continue;
    const unsigned k = pkey(x);
    if (k > lo && k < m) m = k;
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = kPreThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = min(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// One block: the median from lo, its run length and the smallest key above.
__global__ void sel_finish_kernel(const unsigned* __restrict__ part, int nblocks, FrameSel* __restrict__ st) {
  if (threadIdx.x != 0) return;
  unsigned m = 0xFFFFFFFFu;
  for (int b = 0; b < nblocks; ++b) m = min(m, part[b]);
  const unsigned K = st->count;
  const unsigned k_lo = K == 0u ? 0u : (K - 1u) / 2u;
  const unsigned step = K / 2u - k_lo;
  const float lo = pval(st->prefix);
  const float hi = (st->rank + step < st->inbin) ? lo : pval(m);
  st->median = K == 0u ? (double)__int_as_float(0x7FC00000) : (double)((lo + hi) * 0.5f);
}

__global__ void flag_kernel(const float* __restrict__ v, long long npix, const FrameSel* __restrict__ st,
                            double c_sigma, unsigned char* __restrict__ map) {
  const double med = st->median, lim = c_sigma * st->sigma;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (long long)gridDim.x * blockDim.x) {
    const float x = v[i];
    map[i] = (!isfinite(x) || fabs((double)x - med) > lim) ? 1 : 0;
  }
}

// ---- bad pixel repair ----
__global__ void apply_map_kernel(float* __restrict__ cube, long long T, int n, const unsigned char* __restrict__ map) {
  const long long npix = (long long)n * n;
  const long long f = blockIdx.y;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (long long)gridDim.x * blockDim.x)
    if (map[i]) cube[f * npix + i] = __int_as_float(0x7FC00000);
}

// One repair pass (reads src, writes every pixel of dst): a NaN pixel takes
// the float32 median of its non-NaN 8-neighbours, when it has any.  flags[0]
// collects "a NaN is left", flags[1] "a pixel changed".
__global__ void repair_pass_kernel(const float* __restrict__ src, float* __restrict__ dst, long long T, int n,
                                   int* __restrict__ flags) {
  const long long npix = (long long)n * n;
  const long long f = blockIdx.y;
  const float* s = src + f * npix;
  bool left = false, changed = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npix; i += (long long)gridDim.x * blockDim.x) {
    float x = s[i];
    if (isnan(x)) {
      const int r = (int)(i / n), c = (int)(i % n);
      unsigned k[8];
      int m = 0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if ((dy == 0 && dx == 0) || r + dy < 0 || r + dy >= n || c + dx < 0 || c + dx >= n) continue;
          const float y = s[(long long)(r + dy) * n + (c + dx)];
          if (!isnan(y)) k[m++] = pkey(y);
        }
      if (m > 0) {
        for (int a = 1; a < m; ++a) {         // insertion sort of at most 8 keys
          const unsigned key = k[a];
          int b = a - 1;
          while (b >= 0 && k[b] > key) {
            k[b + 1] = k[b];
            --b;
          }
          k[b + 1] = key;
        }
        x = (pval(k[(m - 1) / 2]) + pval(k[m / 2])) * 0.5f;
        changed = true;
      } else {
        left = true;
      }
    }
    dst[f * npix + i] = x;
  }
  if (left) atomicOr(&flags[0], 1);
  if (changed) atomicOr(&flags[1], 1);
}

dim3 frame_grid(long long npix, long long T) {
  const long long bx = std::min<long long>((npix + 255) / 256, 1024);
  return dim3((unsigned)bx, (unsigned)T);
}

}  // namespace

hipError_t launch_mask_disk(float* cube, long long T, int n, const double* xs, const double* ys, double radius,
                            hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(mask_disk_kernel, frame_grid((long long)n * n, T), dim3(256), 0, s, cube, T, n, xs, ys,
                     radius * radius);
  return hipGetLastError();
}

hipError_t launch_subtract_nearest(float* cube, long long T, int n, const double* times, const float* skies,
                                   const double* sky_times, int S, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(subtract_nearest_kernel, frame_grid((long long)n * n, T), dim3(256), 0, s, cube, T, n, times,
                     skies, sky_times, S);
  return hipGetLastError();
}

size_t frame_stats_ws_bytes() {
  return sizeof(FrameSel) + 256 + (size_t)kPreBlocks * 256 * sizeof(unsigned) + (size_t)kPreBlocks * 2 * sizeof(double);
}

hipError_t launch_badpix_map(const float* frame, int n, double c_sigma, unsigned char* map, double* stats, void* ws,
                             hipStream_t s) {
  const long long npix = (long long)n * n;
  char* w = static_cast<char*>(ws);
  FrameSel* st = reinterpret_cast<FrameSel*>(w);
  unsigned* hist = reinterpret_cast<unsigned*>(w + ((sizeof(FrameSel) + 255) / 256) * 256);
  double* part = reinterpret_cast<double*>(reinterpret_cast<char*>(hist) + (size_t)kPreBlocks * 256 * sizeof(unsigned));
  unsigned* upart = hist;                      // reused for the minima once the select is done
  const dim3 g(kPreBlocks), b(kPreThreads);
  hipLaunchKernelGGL(stat_sum_kernel, g, b, 0, s, frame, npix, part);
  hipLaunchKernelGGL(stat_merge_kernel, dim3(1), b, 0, s, part, kPreBlocks, 0, st);
  hipLaunchKernelGGL(stat_dev_kernel, g, b, 0, s, frame, npix, st, part);
  hipLaunchKernelGGL(stat_merge_kernel, dim3(1), b, 0, s, part, kPreBlocks, 1, st);
  for (int d = 3; d >= 0; --d) {
    hipLaunchKernelGGL(sel_hist_kernel, g, b, 0, s, frame, npix, d, st, hist);
    hipLaunchKernelGGL(sel_pick_kernel, dim3(1), dim3(256), 0, s, hist, kPreBlocks, d, st);
  }
  hipLaunchKernelGGL(sel_above_kernel, g, b, 0, s, frame, npix, st, upart);
  hipLaunchKernelGGL(sel_finish_kernel, dim3(1), dim3(64), 0, s, upart, kPreBlocks, st);
  hipLaunchKernelGGL(flag_kernel, dim3(kPreBlocks), b, 0, s, frame, npix, st, c_sigma, map);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && stats) {
    e = hipMemcpyAsync(stats, &st->median, sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(stats + 1, &st->mean, 2 * sizeof(double), hipMemcpyDeviceToDevice, s);
  }
  return e;
}

hipError_t launch_apply_map(float* cube, long long T, int n, const unsigned char* map, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(apply_map_kernel, frame_grid((long long)n * n, T), dim3(256), 0, s, cube, T, n, map);
  return hipGetLastError();
}

hipError_t launch_repair_pass(const float* src, float* dst, long long T, int n, int* flags, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(repair_pass_kernel, frame_grid((long long)n * n, T), dim3(256), 0, s, src, dst, T, n, flags);
  return hipGetLastError();
}

}  // namespace graphic
