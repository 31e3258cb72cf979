// Exact per-pixel median of a float32 stack (gfx950).
//
// The classical ADI reference PSF is the per-pixel median of the recentred
// frames (Sect. 3.3), and the derotated residuals are merged with a per-pixel
// median (Sect. 3.4).  The result is exact: values are ordered by IEEE
// totalOrder through the usual order-preserving uint32 key, lo is the element
// of rank (T-1)/2, hi the element of rank T/2, and the median is
// (lo + hi) * 0.5 in float32.
//
// Layout: a block owns kPix consecutive pixels (16, or 8 as the tuned
// alternative) and all T values of each (kPix waves; lanes = kPix pixels x
// 64/kPix frame groups, so every load reads 4 kPix contiguous bytes of a
// frame).  Thread (pixel, g) keeps the keys of
// frames g, g+64, g+128, ... in registers, so the stack is read from HBM once.
// The rank-(T-1)/2 key is found by a most-significant-digit-first radix select
// with up to four 8-bit digits; each digit builds a 256-bin histogram per
// pixel in LDS and one wave per pixel scans it.  Every lane of a wave owns a
// private sub-histogram (pixel, lane group), so the atomic adds of one wave
// never collide on an address; keys outside the selected prefix add to a
// spare slot of their lane's sub-histogram instead of branching around.  The select
// stops early once every pixel's selected bin holds a single key.  hi is lo
// itself when at least T/2+1 keys are <= lo, otherwise the smallest key above
// lo.

#include "internal.h"

namespace graphic {

namespace {

constexpr int kGroups = 64;       // frame groups (threads) per pixel
constexpr int kBins = 256;
constexpr int kHistWords = kBins + 1;   // 256 bins + 1 slot for keys outside the prefix (odd: spreads banks)

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
  constexpr int kSub = 64 / kPix;                  // lane groups of one pixel inside a wave
  // one sub-histogram per (pixel, lane group), in dynamic LDS
  extern __shared__ unsigned hist[];
  __shared__ unsigned sel_prefix[kPix], sel_rank[kPix], sel_cnt[kPix], sel_min[kPix], sel_lo[kPix];
  __shared__ float sel_med[kPix];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int px = lane % kPix;
  const int sub = lane / kPix;
  const int g = sub + kSub * wave;                 // frame group 0..63
  // The hardware deals consecutive block ids to the eight XCDs in turn; the
  // remap gives each XCD a contiguous run of pixel tiles, so the two 64-byte
  // halves of a 128-byte line are read by blocks that run side by side on
  // one L2 (and each frame row is read in long runs).
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned tile = (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  const long long pix = (long long)tile * kPix + px;
  const bool pix_ok = pix < npix;
  unsigned* my_hist = hist + (px * kSub + sub) * kHistWords;

  // Frames 64 i .. 64 i + 63 form group i.  One wave-uniform buffer
  // descriptor per group keeps the per-lane address a single 32-bit offset
  // (g * npix + px) * 4: the base advances by 64 frames per group, full groups
  // share one extent, and the last group's extent ends after frame T - 1, so
  // lanes past it (and groups past T) read 0 and their stores are dropped.
  const int Ti = (int)T;                                   // T <= 4096
  const long long pix0 = (long long)tile * kPix;
  const unsigned voff = pix_ok ? (unsigned)(((long long)g * npix + (pix - pix0)) * 4) : 0x80000000u;
  const unsigned extent = (unsigned)(((long long)(kGroups - 1) * npix + kPix) * 4);
  const int last = (Ti - 1) / kGroups;
  const unsigned extent_last =
      (unsigned)((((long long)(Ti - 1) - (long long)kGroups * last) * npix + (npix - pix0)) * 4);
  const unsigned long long gstride = (unsigned long long)kGroups * (unsigned long long)npix * 4ull;
  auto group_ext = [&](int i) { return i < last ? extent : (i == last ? extent_last : 0u); };
  unsigned key[VPT];
  unsigned long long gaddr = reinterpret_cast<unsigned long long>(stack + pix0);   // group i's base, advanced per group
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const bool valid = g + kGroups * i < Ti;
    float v;
    if constexpr (BUF) {
      v = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          frames_rsrc(reinterpret_cast<const float*>(gaddr), group_ext(i)), (int)voff, 0, 0));
      gaddr += gstride;
    } else {
      v = (valid && pix_ok) ? stack[(long long)(g + kGroups * i) * npix + pix] : 0.0f;   // frames too large for 32-bit offsets
    }
    key[i] = valid ? key_of(v) : 0xFFFFFFFFu;   // padding sorts after every real (non-NaN) value
  }

  const unsigned k_lo = (unsigned)((T - 1) / 2);
  if (tid < kPix) {
    sel_prefix[tid] = 0u;
    sel_rank[tid] = k_lo;
    sel_lo[tid] = 0xFFFFFFFFu;
  }

  unsigned mask = 0u;
  bool single = false;                              // every pixel's bin holds one key
#pragma unroll 1
  for (int d = 3; d >= 0; --d) {
    for (int i = tid; i < kPix * kSub * kHistWords; i += kThreads) hist[i] = 0u;
    __syncthreads();
    const unsigned prefix = sel_prefix[px];
    const int sh = 8 * d;
    // (mask = 0 and prefix = 0 for the first digit: every key counts)
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const unsigned bin = ((key[i] & mask) == prefix) ? ((key[i] >> sh) & 0xFFu) : (unsigned)kBins;
      atomicAdd(&my_hist[bin], 1u);
    }
    __syncthreads();
    // wave w scans the histogram of pixel w: lane l holds bins l, l+64, l+128, l+192
    for (int w = wave; w < kPix; w += kThreads / 64) {
      const unsigned k = sel_rank[w];
      unsigned carry = 0u;
      int found_bin = -1;
      unsigned below = 0u, inbin = 0u;
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        const int bin = blk * 64 + lane;
        unsigned x = 0u;
#pragma unroll
        for (int q = 0; q < kSub; ++q) x += hist[(w * kSub + q) * kHistWords + bin];
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
    if (d > 0) {
      unsigned most = 0u;
#pragma unroll
      for (int q = 0; q < kPix; ++q) most = max(most, sel_cnt[q]);
      if (most <= 1u) {                             // block-uniform
        single = true;
        break;
      }
    }
  }

  // lo: the full key is the prefix after four digits; after an early stop it
  // is the one key that carries the selected prefix.
  unsigned lo_key;
  if (single) {
    const unsigned prefix = sel_prefix[px];
#pragma unroll
    for (int i = 0; i < VPT; ++i)
      if ((key[i] & mask) == prefix) atomicMin(&sel_lo[px], key[i]);
    __syncthreads();
    lo_key = sel_lo[px];
  } else {
    lo_key = sel_prefix[px];
  }
  // sel_rank is lo's rank among the keys that carry its prefix and sel_cnt
  // how many keys carry it (after four digits: how many equal lo); rank T/2
  // still hits lo iff it falls inside that run, otherwise hi is the smallest
  // key above lo.
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
    unsigned long long raddr = reinterpret_cast<unsigned long long>(resid + pix0);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const float r = val_of(key[i]) - med;
      if constexpr (BUF) {
        __builtin_amdgcn_raw_buffer_store_b32(
            __float_as_int(r), frames_rsrc(reinterpret_cast<const float*>(raddr), group_ext(i)), (int)voff, 0, 0);
        raddr += gstride;
      } else {
        const int t = g + kGroups * i;
        if (pix_ok && t < Ti) resid[(long long)t * npix + pix] = r;
      }
    }
  }
}

}  // namespace

template <int PIX>
static hipError_t launch_median_pix(const float* stack, long long T, long long npix, float* out, float* resid,
                                    hipStream_t s) {
  const long long vpt = (T + kGroups - 1) / kGroups;
  const unsigned blocks = (unsigned)((npix + PIX - 1) / PIX);
  // 32-bit buffer offsets cover 64 frames of the stack when 64 * npix * 4 < 2^31
  const bool buf = (long long)kGroups * npix * 4 < 0x7fffffffLL;
  const size_t lds = (size_t)PIX * (64 / PIX) * kHistWords * sizeof(unsigned);
#define GRAPHIC_MEDIAN_CASE(V)                                                                              \
  if (vpt <= V) {                                                                                          \
    if (buf) {                                                                                             \
      hipFuncSetAttribute((const void*)median_kernel<V, PIX, true>,                                        \
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                           \
      hipLaunchKernelGGL((median_kernel<V, PIX, true>), dim3(blocks), dim3(PIX * kGroups), lds, s, stack, T, \
                         npix, out, resid);                                                                \
    } else {                                                                                               \
      hipFuncSetAttribute((const void*)median_kernel<V, PIX, false>,                                       \
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                           \
      hipLaunchKernelGGL((median_kernel<V, PIX, false>), dim3(blocks), dim3(PIX * kGroups), lds, s, stack, \
                         T, npix, out, resid);                                                             \
    }                                                                                                      \
    return hipGetLastError();                                                                              \
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

hipError_t launch_median(const float* stack, long long T, long long npix, float* out, float* resid, int variant,
                         hipStream_t s) {
  if (T <= 0 || npix <= 0) return hipSuccess;
  return variant == 1 ? launch_median_pix<8>(stack, T, npix, out, resid, s)
                      : launch_median_pix<16>(stack, T, npix, out, resid, s);
}

}  // namespace graphic
