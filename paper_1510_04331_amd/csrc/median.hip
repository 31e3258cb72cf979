// Exact per-pixel median of a float32 stack (gfx950).
//
// The classical ADI reference PSF is the per-pixel median of the recentred
// frames (Sect. 3.3), and the derotated residuals are merged with a per-pixel
// median (Sect. 3.4).  The result is exact: values are ordered by IEEE
// totalOrder through the usual order-preserving uint32 key, lo is the element
// of rank (T-1)/2, hi the element of rank T/2, and the median is
// (lo + hi) * 0.5 in float32.
//
// Layout: a block of 1024 threads owns 16 consecutive pixels and all T values
// of each (16 waves; lanes = 16 pixels x 4 frame groups, so every load reads
// 64 contiguous bytes of one frame).  Thread (pixel, g) keeps the keys of
// frames g, g+64, g+128, ... in registers, so the stack is read from HBM once.
// The rank-(T-1)/2 key is found by a most-significant-digit-first radix select
// with four 8-bit digits; each digit builds a 256-bin histogram per pixel in
// LDS and one wave per pixel scans it.  hi is lo itself when at least T/2+1
// keys are <= lo, otherwise the smallest key above lo.

#include "internal.h"

#ifndef GRAPHIC_MEDIAN_PIX
#define GRAPHIC_MEDIAN_PIX 16
#endif

namespace graphic {

namespace {

constexpr int kGroups = 64;       // frame groups (threads) per pixel
constexpr int kBins = 256;
constexpr int kHistPitch = kBins + 1;   // +1 word: pixels land on distinct banks

__device__ __forceinline__ unsigned key_of(float v) {
  unsigned b = __float_as_uint(v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float val_of(unsigned k) {
  unsigned b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(b);
}

// kPix pixels per block (one wave per pixel for the histogram scans).  With
// resid != nullptr every value is also written back as value - median
// (in place is allowed: each thread rewrites exactly the values it read).
// Inclusive prefix sum over the 64 lanes of a wave with DPP: four row_shr
// steps scan each row of 16 lanes, two row_bcast steps carry across rows.
__device__ __forceinline__ unsigned wave_incl_scan(unsigned x) {
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t frames_rsrc(const float* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes, 0x00020000);
}

template <int VPT, int kPix, bool BUF>
__global__ void __launch_bounds__(kPix * kGroups) median_kernel(const float* __restrict__ stack, long long T,
                                                                long long npix, float* __restrict__ out,
                                                                float* resid) {
  constexpr int kThreads = kPix * kGroups;
  __shared__ unsigned hist[kPix * kHistPitch];
  __shared__ unsigned sel_prefix[kPix], sel_rank[kPix], sel_cnt[kPix], sel_min[kPix];
  __shared__ float sel_med[kPix];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int px = lane % kPix;
  const int g = lane / kPix + (64 / kPix) * wave;   // frame group 0..63
  const long long pix = (long long)blockIdx.x * kPix + px;
  const bool pix_ok = pix < npix;

  // Frames 64 i .. 64 i + 63 form group i; one wave-uniform buffer descriptor
  // per group keeps the per-lane address a single 32-bit offset
  // (g * npix + pix) * 4, and offsets past the group's frames read 0.
  const long long pix0 = (long long)blockIdx.x * kPix;
  const unsigned voff = pix_ok ? (unsigned)(((long long)g * npix + (pix - pix0)) * 4) : 0x80000000u;
  auto group = [&](int i) {
    const long long f0 = (long long)kGroups * i;
    const long long nf = T - f0 < kGroups ? T - f0 : kGroups;
    const long long bytes = nf > 0 ? (nf - 1) * npix * 4 + (npix - pix0) * 4 : 0;
    return frames_rsrc(stack + f0 * npix + pix0, (unsigned)(bytes < 0x7fffffffLL ? bytes : 0x7fffffffLL));
  };
  unsigned key[VPT];
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const long long t = g + (long long)kGroups * i;
    const bool valid = t < T;
    float v;
    if constexpr (BUF) {
      v = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(group(i), (int)voff, 0, 0));
    } else {
      v = (valid && pix_ok) ? stack[t * npix + pix] : 0.0f;   // frames too large for 32-bit offsets
    }
    key[i] = valid ? key_of(v) : 0xFFFFFFFFu;   // padding sorts after every real (non-NaN) value
  }

  const unsigned k_lo = (unsigned)((T - 1) / 2);
  if (tid < kPix) {
    sel_prefix[tid] = 0u;
    sel_rank[tid] = k_lo;
  }

  unsigned prefix = 0u, mask = 0u;
#pragma unroll 1
  for (int d = 3; d >= 0; --d) {
    for (int i = tid; i < kPix * kHistPitch; i += kThreads) hist[i] = 0u;
    __syncthreads();
    prefix = sel_prefix[px];
    const int sh = 8 * d;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      if ((key[i] & mask) == prefix) atomicAdd(&hist[px * kHistPitch + ((key[i] >> sh) & 0xFFu)], 1u);
    }
    __syncthreads();
    // wave w scans the histogram of pixel w: lane l holds bins l, l+64, l+128, l+192
    {
      const int w = wave;
      const unsigned k = sel_rank[w];
      unsigned carry = 0u;
      int found_bin = -1;
      unsigned below = 0u, inbin = 0u;
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        const unsigned x = hist[w * kHistPitch + blk * 64 + lane];
        const unsigned incl = wave_incl_scan(x);
        const unsigned tot = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
        const unsigned long long hit = __ballot(carry + incl > k);
        if (found_bin < 0 && hit != 0ull) {
          const int l0 = __ffsll((long long)hit) - 1;
          found_bin = blk * 64 + l0;
          const unsigned incl0 = (unsigned)__builtin_amdgcn_readlane((int)incl, l0);
          const unsigned x0 = (unsigned)__builtin_amdgcn_readlane((int)x, l0);
          below = carry + incl0 - x0;
          inbin = x0;
        }
        carry += tot;
      }
      if (lane == 0) {
        sel_prefix[w] = sel_prefix[w] | ((unsigned)found_bin << sh);
        sel_rank[w] = k - below;
        sel_cnt[w] = inbin;
        sel_min[w] = 0xFFFFFFFFu;
      }
    }
    mask |= 0xFFu << sh;
    __syncthreads();
  }

  // After the last digit, sel_rank is lo's rank among the keys equal to lo and
  // sel_cnt is how many keys equal lo; rank T/2 still hits lo iff it falls
  // inside that run, otherwise hi is the smallest key above lo.
  const unsigned lo_key = sel_prefix[px];
  unsigned local_min = 0xFFFFFFFFu;
#pragma unroll
  for (int i = 0; i < VPT; ++i)
    if (key[i] > lo_key && key[i] < local_min) local_min = key[i];
  atomicMin(&sel_min[px], local_min);
  __syncthreads();

  if (g == 0) {
    const unsigned step = (unsigned)(T / 2) - k_lo;      // 0 (odd T) or 1
    const float lo = val_of(lo_key);
    const float hi = (sel_rank[px] + step < sel_cnt[px]) ? lo : val_of(sel_min[px]);
    const float med = (lo + hi) * 0.5f;
    sel_med[px] = med;
    if (pix_ok) out[pix] = med;
  }
  if (resid != nullptr) {
    __syncthreads();
    const float med = sel_med[px];
    const float* rbase = resid;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const long long f0 = (long long)kGroups * i;
      if constexpr (BUF) {
        const long long nf = T - f0 < kGroups ? T - f0 : kGroups;
        const long long bytes = nf > 0 ? (nf - 1) * npix * 4 + (npix - pix0) * 4 : 0;
        const __amdgpu_buffer_rsrc_t r =
            frames_rsrc(rbase + f0 * npix + pix0, (unsigned)(bytes < 0x7fffffffLL ? bytes : 0x7fffffffLL));
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(val_of(key[i]) - med), r, (int)voff, 0, 0);
      } else {
        const long long t = g + f0;
        if (pix_ok && t < T) resid[t * npix + pix] = val_of(key[i]) - med;
      }
    }
  }
}

}  // namespace

hipError_t launch_median(const float* stack, long long T, long long npix, float* out, float* resid,
                         hipStream_t s) {
  if (T <= 0 || npix <= 0) return hipSuccess;
  const long long vpt = (T + kGroups - 1) / kGroups;
  constexpr int PIX = GRAPHIC_MEDIAN_PIX;
  const unsigned blocks = (unsigned)((npix + PIX - 1) / PIX);
  // 32-bit buffer offsets cover 64 frames of the stack when 64 * npix * 4 < 2^31
  const bool buf = (long long)kGroups * npix * 4 < 0x7fffffffLL;
#define GRAPHIC_MEDIAN_CASE(V)                                                                            \
  if (vpt <= V) {                                                                                        \
    if (buf)                                                                                             \
      hipLaunchKernelGGL((median_kernel<V, PIX, true>), dim3(blocks), dim3(PIX * kGroups), 0, s, stack, T, \
                         npix, out, resid);                                                              \
    else                                                                                                 \
      hipLaunchKernelGGL((median_kernel<V, PIX, false>), dim3(blocks), dim3(PIX * kGroups), 0, s, stack, T, \
                         npix, out, resid);                                                              \
    return hipGetLastError();                                                                            \
  }
  GRAPHIC_MEDIAN_CASE(1)
  GRAPHIC_MEDIAN_CASE(2)
  GRAPHIC_MEDIAN_CASE(4)
  GRAPHIC_MEDIAN_CASE(8)
  GRAPHIC_MEDIAN_CASE(16)
  GRAPHIC_MEDIAN_CASE(32)
  GRAPHIC_MEDIAN_CASE(64)
#undef GRAPHIC_MEDIAN_CASE
  return hipErrorInvalidValue;   // T > 4096: rejected on the host before launch
}

}  // namespace graphic
