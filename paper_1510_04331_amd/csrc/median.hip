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
// frames g, g+64, g+128, ... in registers (on a tile-major stack: the VPT
// consecutive frames from g VPT on, VPT being ceil(T/64) rounded up to a
// power of two), so the stack is read from HBM once.
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

// Shared state of one block's select (one slot per pixel of the tile).
template <int kPix>
struct SelShared {
  unsigned prefix[kPix], rank[kPix], cnt[kPix], min[kPix], lo[kPix];
  float med[kPix];
};

// Geometry of a block's pixel tile and its frame groups.
template <int kPix>
struct Tile {
  int tid, lane, wave, px, sub, g;
  long long pix, pix0;
  bool pix_ok;
  unsigned voff, extent, extent_last;
  int last, Ti;
  unsigned long long gstride;

  __device__ Tile(long long T, long long npix) {
    constexpr int kSub = 64 / kPix;
    tid = threadIdx.x;
    lane = tid & 63;
    wave = tid >> 6;
    px = lane % kPix;
    sub = lane / kPix;
    g = sub + kSub * wave;                         // frame group 0..63
    // The hardware deals consecutive block ids to the eight XCDs in turn; the
    // remap gives each XCD a contiguous run of pixel tiles, so the two
    // 64-byte halves of a 128-byte line are read by blocks that run side by
    // side on one L2 (and each frame row is read in long runs).
    const unsigned nb = gridDim.x, b = blockIdx.x;
    const unsigned tile = (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
    pix0 = (long long)tile * kPix;
    pix = pix0 + px;
    pix_ok = pix < npix;
    // Frames 64 i .. 64 i + 63 form group i.  One wave-uniform buffer
    // descriptor per group keeps the per-lane address a single 32-bit offset
    // (g * npix + px) * 4: the base advances by 64 frames per group, full
    // groups share one extent, and the last group's extent ends after frame
    // T - 1, so lanes past it (and groups past T) read 0 and their stores are
    // dropped.
    Ti = (int)T;                                   // T <= 4096
    voff = pix_ok ? (unsigned)(((long long)g * npix + px) * 4) : 0x80000000u;
    extent = (unsigned)(((long long)(kGroups - 1) * npix + kPix) * 4);
    last = (Ti - 1) / kGroups;
    extent_last = (unsigned)((((long long)(Ti - 1) - (long long)kGroups * last) * npix + (npix - pix0)) * 4);
    gstride = (unsigned long long)kGroups * (unsigned long long)npix * 4ull;
  }
  __device__ unsigned group_ext(int i) const { return i < last ? extent : (i == last ? extent_last : 0u); }
};

// Keys of frames g, g + 64, g + 128, ... of this thread's pixel; frames past
// T get the largest key.
template <int VPT, int kPix, bool BUF>
__device__ __forceinline__ void load_keys(const Tile<kPix>& t, const float* __restrict__ stack, long long npix,
                                          unsigned (&key)[VPT]) {
  unsigned long long gaddr = reinterpret_cast<unsigned long long>(stack + t.pix0);   // group i's base
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const bool valid = t.g + kGroups * i < t.Ti;
    float v;
    if constexpr (BUF) {
      v = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(
          frames_rsrc(reinterpret_cast<const float*>(gaddr), t.group_ext(i)), (int)t.voff, 0, 0));
      gaddr += t.gstride;
    } else {
      v = (valid && t.pix_ok) ? stack[(long long)(t.g + kGroups * i) * npix + t.pix] : 0.0f;   // frames too large for 32-bit offsets
    }
    key[i] = valid ? key_of(v) : 0xFFFFFFFFu;   // padding sorts after every real (non-NaN) value
  }
}

// Writes value - med for every frame of this thread (in place is allowed:
// each thread rewrites exactly the values it read).
template <int VPT, int kPix, bool BUF>
__device__ __forceinline__ void store_diff(const Tile<kPix>& t, float* resid, long long npix,
                                           const unsigned (&key)[VPT], const float (&med)[VPT]) {
  unsigned long long raddr = reinterpret_cast<unsigned long long>(resid + t.pix0);
  // fresh copies of the group extents, so that the descriptors are rebuilt
  // here instead of being kept live (64 of them) across the select
  unsigned ext = t.extent, ext_last = t.extent_last;
  int last = t.last;
  asm volatile("" : "+s"(ext), "+s"(ext_last), "+s"(last));
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const float r = val_of(key[i]) - med[i];
    if constexpr (BUF) {
      const unsigned e = i < last ? ext : (i == last ? ext_last : 0u);
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(r), frames_rsrc(reinterpret_cast<const float*>(raddr), e),
                                            (int)t.voff, 0, 0);
      raddr += t.gstride;
    } else {
      const int f = t.g + kGroups * i;
      if (t.pix_ok && f < t.Ti) resid[(long long)f * npix + t.pix] = r;
    }
  }
}

// Exact median of the keys whose bit is set in `bits` (bit i: key[i]); K is
// how many keys of the pixel take part (K >= 1), the same for every pixel, or
// with PPK per pixel in Kp[px] (LDS).  Every thread of the block calls it; on
// return sh.med[px] holds the median of every pixel.
template <int VPT, int kPix, bool PPK = false>
__device__ __forceinline__ void select_median(const Tile<kPix>& t, const unsigned (&key)[VPT],
                                              unsigned long long bits, unsigned K, unsigned* hist,
                                              SelShared<kPix>& sh, const unsigned* Kp = nullptr) {
  constexpr int kThreads = kPix * kGroups;
  constexpr int kSub = 64 / kPix;
  unsigned* my_hist = hist + (t.px * kSub + t.sub) * kHistWords;
  if (t.tid < kPix) {
    const unsigned Kt = PPK ? Kp[t.tid] : K;
    sh.prefix[t.tid] = 0u;
    sh.rank[t.tid] = Kt == 0u ? 0u : (Kt - 1u) / 2u;
    sh.lo[t.tid] = 0xFFFFFFFFu;
  }
  // Without per-pixel key counts the sub-histograms are cleared with
  // unrolled 16-byte stores (hist is 16-byte aligned and holds a whole number
  // of vectors) and the digit loop is unrolled, so that the first digit,
  // whose prefix is empty, takes every key without the prefix test.  With
  // per-pixel counts (a 64-bit participation mask per thread, 1024 threads)
  // either change makes the kernel spill, so that variant keeps the plain
  // loops.
  constexpr int kVec = kPix * kSub * kHistWords / 4;
  static_assert((kPix * kSub * kHistWords) % 4 == 0, "whole 16-byte vectors");
  auto zero_hist = [&]() {
    if constexpr (PPK) {
      for (int i = t.tid; i < kPix * kSub * kHistWords; i += kThreads) hist[i] = 0u;
    } else {
      uint4* h4 = reinterpret_cast<uint4*>(hist);
      const uint4 z = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (int k = 0; k < kVec / kThreads; ++k) h4[t.tid + k * kThreads] = z;
      if (kVec % kThreads != 0 && t.tid < kVec % kThreads) h4[(kVec / kThreads) * kThreads + t.tid] = z;
    }
  };
  unsigned mask = 0u;
  bool single = false;                              // every pixel's bin holds one key
  constexpr int kDigitUnroll = PPK ? 1 : 4;
  // With few keys per thread the histograms are cleared once: after each
  // digit's scan every thread takes its own adds back, which costs VPT
  // atomics instead of a pass over all sub-histograms and a barrier.
  constexpr bool kUnadd = !PPK && VPT <= 8;
  unsigned added[kUnadd ? VPT : 1];
  if constexpr (kUnadd) {
    zero_hist();
    __syncthreads();
  }
#pragma unroll kDigitUnroll
  for (int d = 3; d >= 0; --d) {
    if constexpr (!kUnadd) {
      zero_hist();
      __syncthreads();
    }
    const unsigned prefix = sh.prefix[t.px];
    const int shft = 8 * d;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const bool part = ((bits >> i) & 1ull) != 0ull;
      unsigned bin;
      if constexpr (PPK) {
        // (mask = 0 and prefix = 0 for the first digit)
        const bool in = part && (key[i] & mask) == prefix;
        bin = in ? ((key[i] >> shft) & 0xFFu) : (unsigned)kBins;
      } else if (d == 3) {
        bin = part ? key[i] >> 24 : (unsigned)kBins;               // empty prefix
      } else {
        // the prefix is zero in this digit and below, so (key ^ prefix) >>
        // shft is the digit when the key carries the prefix and at least 256
        // (the spare slot) when it does not
        bin = part ? min((key[i] ^ prefix) >> shft, (unsigned)kBins) : (unsigned)kBins;
      }
      atomicAdd(&my_hist[bin], 1u);
      if constexpr (kUnadd) added[i] = bin;
    }
    __syncthreads();
    // wave w scans the histogram of pixel w: lane l holds bins l, l+64, l+128, l+192
    for (int w = t.wave; w < kPix; w += kThreads / 64) {
      const unsigned k = sh.rank[w];
      unsigned carry = 0u;
      int found_bin = -1;
      unsigned below = 0u, inbin = 0u;
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        const int bin = blk * 64 + t.lane;
        unsigned x = 0u;
#pragma unroll
        for (int q = 0; q < kSub; ++q) x += hist[(w * kSub + q) * kHistWords + bin];
        const unsigned incl = wave_incl_scan(x);
        const unsigned tot = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
        const unsigned long long hit = __ballot(carry + incl > k);
        if (hit != 0ull) {                          // wave-uniform: the later blocks are not needed
          const int l0 = __ffsll((long long)hit) - 1;
          found_bin = blk * 64 + l0;
          const unsigned incl0 = (unsigned)__builtin_amdgcn_readlane((int)incl, l0);
          const unsigned x0 = (unsigned)__builtin_amdgcn_readlane((int)x, l0);
          below = carry + incl0 - x0;
          inbin = x0;
          break;
        }
        carry += tot;
      }
      if (t.lane == 0) {
        sh.prefix[w] = sh.prefix[w] | ((unsigned)found_bin << shft);
        sh.rank[w] = k - below;
        sh.cnt[w] = inbin;
        sh.min[w] = 0xFFFFFFFFu;
      }
    }
    mask |= 0xFFu << shft;
    __syncthreads();
    if (d > 0) {
      unsigned most = 0u;
#pragma unroll
      for (int q = 0; q < kPix; ++q) most = max(most, sh.cnt[q]);
      if (most <= 1u) {                             // block-uniform
        single = true;
        break;
      }
      // every scan of this digit is done (barrier above): restore the zeros
      // for the next digit, whose adds commute with these
      if constexpr (kUnadd) {
#pragma unroll
        for (int i = 0; i < VPT; ++i) atomicSub(&my_hist[added[i]], 1u);
      }
    }
  }

  // lo: the full key is the prefix after four digits; after an early stop it
  // is the one taking-part key that carries the selected prefix.
  unsigned lo_key;
  if (single) {
    const unsigned prefix = sh.prefix[t.px];
    if constexpr (PPK) {
#pragma unroll
      for (int i = 0; i < VPT; ++i)
        if (((bits >> i) & 1ull) != 0ull && (key[i] & mask) == prefix) atomicMin(&sh.lo[t.px], key[i]);
    } else {
      // Every key takes part here.  The keys with the prefix are those whose
      // key ^ prefix has no bit under the mask, and key ^ prefix keeps their
      // order; every other key's key ^ prefix is larger.  So the thread's
      // smallest key ^ prefix is its smallest key with the prefix when it has
      // no bit under the mask, and then one atomic per thread suffices (the
      // variant above keeps one per key: it has no register to spare).
      unsigned vmin = 0xFFFFFFFFu;
#pragma unroll
      for (int i = 0; i < VPT; ++i) vmin = min(vmin, key[i] ^ prefix);
      atomicMin(&sh.lo[t.px], (vmin & mask) == 0u ? (vmin ^ prefix) : 0xFFFFFFFFu);
    }
    __syncthreads();
    lo_key = sh.lo[t.px];
  } else {
    lo_key = sh.prefix[t.px];
  }
  // sh.rank is lo's rank among the keys that carry its prefix and sh.cnt how
  // many keys carry it (after four digits: how many equal lo); rank K/2 still
  // hits lo iff it falls inside that run, otherwise hi is the smallest
  // taking-part key above lo.
  unsigned local_min = 0xFFFFFFFFu;
  if constexpr (PPK) {
#pragma unroll
    for (int i = 0; i < VPT; ++i)
      if (((bits >> i) & 1ull) != 0ull && key[i] > lo_key && key[i] < local_min) local_min = key[i];
  } else if (lo_key != 0xFFFFFFFFu) {
    // key - (lo + 1) wraps for the keys at or below lo, above every value
    // of a key above lo, so the smallest of them gives the smallest key
    // above lo (every key takes part here); the largest key stays "none"
    const unsigned base = lo_key + 1u;
    unsigned dmin = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < VPT; ++i) dmin = min(dmin, key[i] - base);
    local_min = dmin <= 0xFFFFFFFEu - lo_key ? dmin + base : 0xFFFFFFFFu;
  }
  atomicMin(&sh.min[t.px], local_min);
  __syncthreads();
  if (t.g == 0) {
    const unsigned Kx = PPK ? Kp[t.px] : K;
    const unsigned k_lo = Kx == 0u ? 0u : (Kx - 1u) / 2u;
    const unsigned step = Kx / 2 - k_lo;                 // 0 (odd K) or 1
    const float lo = val_of(lo_key);
    const float hi = (sh.rank[t.px] + step < sh.cnt[t.px]) ? lo : val_of(sh.min[t.px]);
    sh.med[t.px] = (lo + hi) * 0.5f;
  }
  __syncthreads();
}

template <int VPT, int kPix, bool BUF>
__global__ void __launch_bounds__(kPix * kGroups) median_kernel(const float* __restrict__ stack, long long T,
                                                                long long npix, float* __restrict__ out,
                                                                float* resid) {
  extern __shared__ __align__(16) unsigned hist[];     // one sub-histogram per (pixel, lane group)
  __shared__ SelShared<kPix> sh;
  const Tile<kPix> t(T, npix);
  unsigned key[VPT];
  load_keys<VPT, kPix, BUF>(t, stack, npix, key);
  select_median<VPT, kPix>(t, key, ~0ull, (unsigned)T, hist, sh);
  const float med = sh.med[t.px];
  if (t.g == 0 && t.pix_ok) out[t.pix] = med;
  if (resid != nullptr) {
    float m[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) m[i] = med;
    store_diff<VPT, kPix, BUF>(t, resid, npix, key, m);
  }
}

// The same on a tile-major stack.  The block's kPix pixels (16, or 8 = one
// half of a 16-pixel run) over all T frames lie in one run of 64 T bytes.
// Thread (px, g) holds the VPT consecutive frames g VPT + i of its pixel, at
// byte ((g VPT + i) * 16 + px0 + px) * 4 of the run (px0: 0, or 8 for the
// second half): its loads and stores differ only by i * 64 bytes, which the
// instructions' immediate offset carries, so one offset register and one
// wave-uniform descriptor (extent 64 T bytes) serve all of them.  Frames past
// T lie beyond the extent: they read 0 and their stores are dropped.  (The
// select does not depend on which frames a thread holds.)  The register budget
// is that of four waves per SIMD, so with kPix = 8 two blocks fit a compute
// unit.
template <int VPT, int kPix>
__global__ void __launch_bounds__(kPix * kGroups) __attribute__((amdgpu_waves_per_eu(4)))
median_tm_kernel(const float* __restrict__ stack, long long T, long long npix, float* __restrict__ out, float* resid) {
  static_assert(kTilePix % kPix == 0, "a tile is a whole run or a part of one");
  extern __shared__ __align__(16) unsigned hist[];
  __shared__ SelShared<kPix> sh;
  const Tile<kPix> t(T, npix);
  const long long run0 = (t.pix0 / kTilePix) * T * kTilePix;         // float index of the run
  const unsigned run_bytes = (unsigned)T * kTilePix * 4u;
  const int f0 = t.g * VPT;                                          // this thread's first frame
  const unsigned voff = (unsigned)(f0 * kTilePix + (int)(t.pix0 % kTilePix) + t.px) * 4u;
  constexpr unsigned kFrameBytes = kTilePix * 4u;
  static_assert((VPT - 1) * kFrameBytes < 4096u, "frame steps fit the 12-bit immediate offset");
  const __amdgpu_buffer_rsrc_t src = frames_rsrc(stack + run0, run_bytes);
  const int n_mine = t.Ti - f0;                                      // frames of this thread below T
  unsigned key[VPT];
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const float v = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(src, (int)(voff + i * kFrameBytes), 0, 0));
    key[i] = i < n_mine ? key_of(v) : 0xFFFFFFFFu;
  }
  select_median<VPT, kPix>(t, key, ~0ull, (unsigned)T, hist, sh);
  const float med = sh.med[t.px];
  if (t.g == 0) out[t.pix] = med;
  if (resid != nullptr) {
    const __amdgpu_buffer_rsrc_t dst = frames_rsrc(resid + run0, run_bytes);
    // a fresh copy of the offset, so that the stores take i * 64 as their
    // immediate offset instead of 64 offsets kept live across the select
    unsigned soff = voff;
    asm volatile("" : "+v"(soff));
#pragma unroll
    for (int i = 0; i < VPT; ++i)
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(val_of(key[i]) - med), dst, (int)(soff + i * kFrameBytes),
                                            0, 0);
  }
}

// Per-frame medians over selected frames: for every frame f, the median of
// the frames whose bit is set in row f of the selection (sel[f][g] bit i:
// frame g + 64 i), written to psf[f] (nullable) and subtracted from frame f
// into resid (nullable; in place allowed).
//
// A block owns PB pixels, one wave each.  The block first reads its pixels'
// whole stack (coalesced over the pixels) into LDS; each wave then sorts its
// pixel's keys once, by a bitonic network over (key, frame) pairs held as
// element e = lane * VPT + r, and keeps the sorted keys and the sorted
// position of every frame in LDS.  A bitmap over sorted positions marks the
// selected frames: from one frame to the next only the frames that enter or
// leave the selection flip their bit, so with sliding selections a frame
// costs O(1) LDS updates.  Each lane counts the marked positions of its own
// VPT-bit stretch, a wave prefix sum locates the lanes holding ranks
// (K - 1) / 2 and K / 2 of the K selected keys, and those lanes find the bit
// within their stretch.  The two keys give the median exactly as the
// radix select does: (lo + hi) * 0.5 in float32.
__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int mask) {
  const int lo = __shfl_xor((int)(unsigned)v, mask);
  const int hi = __shfl_xor((int)(unsigned)(v >> 32), mask);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Index of the j-th set bit (from 0) of m (j < popcount(m)).
__device__ __forceinline__ int nth_set_bit(unsigned m, unsigned j) {
  int r = 0;
#pragma unroll
  for (int step = 16; step >= 1; step >>= 1) {
    const unsigned low = (unsigned)__popc(m & ((1u << step) - 1u));
    if (j >= low) {
      j -= low;
      m >>= step;
      r += step;
    }
  }
  return r;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

//
// Long sequences run in row groups (CH): the block then holds the n_keys
// frames list[0..n_keys) that the group's rows select, sel rows index that
// list (bit i of word g: list entry g + 64 i), the n_rows per-frame medians go
// to psf[0..n_rows) and resid is unused; a row that selects nothing takes
// psf_all, the median of every frame.
template <int VPT, int PB, bool CH>
__global__ void __launch_bounds__(PB * 64)
median_window_kernel(const float* __restrict__ stack, long long npix, const int* __restrict__ list, int n_keys,
                     int n_rows, const unsigned long long* __restrict__ sel, const float* __restrict__ psf_all,
                     float* __restrict__ psf, float* resid) {
  constexpr int TP = 64 * VPT;                          // padded frame count of one pixel
  constexpr int kWords = TP / 32;                       // bitmap words of one pixel
  static_assert(VPT >= 1 && VPT <= 32 && (VPT & (VPT - 1)) == 0, "VPT: power of two up to 32");
  extern __shared__ unsigned s_dyn[];
  unsigned* s_key = s_dyn;                                                       // [PB][TP]
  unsigned short* s_pos = reinterpret_cast<unsigned short*>(s_key + PB * TP);    // [PB][TP]
  unsigned* s_bits = reinterpret_cast<unsigned*>(s_pos + PB * TP);              // [PB][kWords]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int Ti = n_rows;
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned tile = (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  const long long pix0 = (long long)tile * PB;

  // 1. the tile's stack into LDS: thread (px, g) reads frames g + 64 i, so a
  //    wave's load covers PB neighbouring pixels of 64 / PB frames
  {
    const int px = lane % PB, g = lane / PB + (64 / PB) * w;
    const bool ok = pix0 + px < npix;
#pragma unroll 4
    for (int i = 0; i < VPT; ++i) {
      const int f = g + 64 * i;
      const bool in = ok && f < n_keys;
      const long long fr = CH ? (in ? list[f] : 0) : f;
      s_key[px * TP + f] = in ? key_of(stack[fr * npix + pix0 + px]) : 0xFFFFFFFFu;
    }
  }
  __syncthreads();

  // 2. wave w sorts pixel w: (key << 11 | frame), frames past T sort last
  unsigned* key = s_key + w * TP;
  unsigned short* pos = s_pos + w * TP;
  unsigned* bits = s_bits + w * kWords;
  {
    unsigned long long v[VPT];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
      const int e = lane * VPT + r;
      v[r] = ((unsigned long long)key[e] << 11) | (unsigned)e;
    }
#pragma unroll
    for (int k = 2; k <= TP; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        if (j >= VPT) {                                 // partner in lane ^ (j / VPT), same register
          const bool upper = (lane & (j / VPT)) != 0;
          const bool asc = ((lane * VPT) & k) == 0;
#pragma unroll
          for (int r = 0; r < VPT; ++r) {
            const unsigned long long o = shfl_xor_u64(v[r], j / VPT);
            v[r] = (asc != upper) ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
          }
        } else {                                        // partner in this lane
#pragma unroll
          for (int r = 0; r < VPT; ++r) {
            if ((r & j) != 0) continue;
            const bool asc = (((lane * VPT + r) & k) == 0);
            const unsigned long long x = v[r], y = v[r | j];
            const unsigned long long lo = x < y ? x : y, hi = x < y ? y : x;
            v[r] = asc ? lo : hi;
            v[r | j] = asc ? hi : lo;
          }
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
      const int e = lane * VPT + r;
      key[e] = (unsigned)(v[r] >> 11);
      pos[(int)(v[r] & 0x7FFu)] = (unsigned short)e;
    }
    for (int i = lane; i < kWords; i += 64) bits[i] = 0u;
    wave_sync();
  }

  // 3. frame loop: flip the bits of the frames that enter or leave the
  //    selection, count per lane, locate ranks (K - 1) / 2 and K / 2
  const long long pix = pix0 + w;
  const bool pix_ok = pix < npix;
  const int b0 = lane * VPT;
  unsigned long long prev = 0ull;
  unsigned long long cur = sel[lane];
#pragma unroll 1
  for (int f = 0; f < Ti; ++f) {
    const unsigned long long nxt = f + 1 < Ti ? sel[(size_t)(f + 1) * kGroups + lane] : 0ull;
    unsigned long long d = cur ^ prev;
    prev = cur;
    while (d != 0ull) {
      const int i = __ffsll((long long)d) - 1;
      d &= d - 1ull;
      const int p = pos[lane + 64 * i];
      atomicXor(&bits[p >> 5], 1u << (p & 31));
    }
    wave_sync();
    const unsigned word = bits[b0 >> 5];
    const unsigned m = VPT == 32 ? word : (word >> (b0 & 31)) & ((1u << (VPT & 31)) - 1u);
    const unsigned cnt = (unsigned)__popc(m);
    const unsigned incl = wave_incl_scan(cnt);
    const unsigned K = (unsigned)__builtin_amdgcn_readlane((int)incl, 63);
    auto key_of_rank = [&](unsigned k) -> unsigned {
      const int L = __ffsll((long long)__ballot(incl > k)) - 1;
      const int at = b0 + nth_set_bit(m, k - (incl - cnt));
      return key[__builtin_amdgcn_readlane(at, L)];
    };
    float med;
    if (CH && K == 0u) {                                // K is wave-uniform
      med = pix_ok ? psf_all[pix] : 0.0f;
    } else {
      const unsigned klo = K == 0u ? 0u : (K - 1u) / 2u;
      const float lo = val_of(key_of_rank(klo));
      const float hi = K / 2u == klo ? lo : val_of(key_of_rank(K / 2u));
      med = (lo + hi) * 0.5f;
    }
    if (lane == 0 && pix_ok) {
      if (psf != nullptr) psf[(size_t)f * npix + pix] = med;
      if constexpr (!CH) {
        if (resid != nullptr) resid[(size_t)f * npix + pix] = val_of(key[pos[f]]) - med;
      }
    }
    cur = nxt;
    wave_sync();
  }
}

// The same per-frame medians with Q pixels per wave, 64 / Q lanes each.  The
// selection is a property of the frame, not of the pixel, so all Q pixels see
// the same count K and the same ranks: one pass over the changed selection
// bits, one loop and one segmented scan serve Q pixels.  Each lane covers
// Q VPT bitmap bits.  Rank (K - 1) / 2 takes the bit search; rank K / 2, when
// it differs, is the next marked bit after it in the same lane or the lowest
// marked bit of the next lane that has one.  The launcher uses Q = 2: with
// Q = 4 the LDS-bound residency leaves too few waves to hide the loop's LDS
// latency (54 against 40 ms at 1024 x 512^2).
// Inclusive prefix sums over each group of 64 / Q lanes of the wave (Q = 4:
// rows of 16; Q = 2: the row_bcast:15 step joins rows 0-1 and 2-3).
template <int Q>
__device__ __forceinline__ unsigned seg_incl_scan(unsigned x) {
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  if constexpr (Q == 2)
    x += (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  return x;
}

// Index of the j-th set bit (from 0) of a 64-bit m (j < popcount(m)).
__device__ __forceinline__ int nth_set_bit64(unsigned long long m, unsigned j) {
  const unsigned lo = (unsigned)m, lowc = (unsigned)__popc(lo);
  return j < lowc ? nth_set_bit(lo, j) : 32 + nth_set_bit((unsigned)(m >> 32), j - lowc);
}

template <int VPT, int PB, bool CH, int Q>
__global__ void __launch_bounds__(PB * 64 / Q)
median_window_q_kernel(const float* __restrict__ stack, long long npix, const int* __restrict__ list,
                       int n_keys, int n_rows, const unsigned long long* __restrict__ sel,
                       const float* __restrict__ psf_all, float* __restrict__ psf, float* resid) {
  constexpr int TP = 64 * VPT;                          // padded frame count of one pixel
  constexpr int kWords = TP / 32;                       // bitmap words of one pixel
  constexpr int LP = 64 / Q;                            // lanes per pixel
  constexpr int BQ = Q * VPT;                           // bitmap bits per lane
  static_assert(VPT >= 1 && VPT <= 32 && (VPT & (VPT - 1)) == 0, "VPT: power of two up to 32");
  static_assert((Q == 2 || Q == 4) && PB % Q == 0 && BQ <= 64, "Q pixels per wave, at most 64 bits per lane");
  extern __shared__ unsigned s_dyn[];
  unsigned* s_key = s_dyn;                                                       // [PB][TP]
  unsigned short* s_pos = reinterpret_cast<unsigned short*>(s_key + PB * TP);    // [PB][TP]
  unsigned* s_bits = reinterpret_cast<unsigned*>(s_pos + PB * TP);              // [PB][kWords]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int Ti = n_rows;
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned tile = (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  const long long pix0 = (long long)tile * PB;

  // 1. the tile's stack into LDS, coalesced over the pixels
  for (int idx = tid; idx < PB * TP; idx += PB * LP) {
    const int px = idx % PB, f = idx / PB;
    const bool in = pix0 + px < npix && f < n_keys;
    const long long fr = CH ? (in ? list[f] : 0) : f;
    s_key[px * TP + f] = in ? key_of(stack[fr * npix + pix0 + px]) : 0xFFFFFFFFu;
  }
  __syncthreads();

  // 2. wave w sorts pixels Q w ... Q w + Q - 1, one after the other
  for (int q = 0; q < Q; ++q) {
    unsigned* key = s_key + (Q * w + q) * TP;
    unsigned short* pos = s_pos + (Q * w + q) * TP;
    unsigned long long v[VPT];
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
      const int e = lane * VPT + r;
      v[r] = ((unsigned long long)key[e] << 11) | (unsigned)e;
    }
#pragma unroll
    for (int k = 2; k <= TP; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        if (j >= VPT) {
          const bool upper = (lane & (j / VPT)) != 0;
          const bool asc = ((lane * VPT) & k) == 0;
#pragma unroll
          for (int r = 0; r < VPT; ++r) {
            const unsigned long long o = shfl_xor_u64(v[r], j / VPT);
            v[r] = (asc != upper) ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
          }
        } else {
#pragma unroll
          for (int r = 0; r < VPT; ++r) {
            if ((r & j) != 0) continue;
            const bool asc = (((lane * VPT + r) & k) == 0);
            const unsigned long long x = v[r], y = v[r | j];
            const unsigned long long lo = x < y ? x : y, hi = x < y ? y : x;
            v[r] = asc ? lo : hi;
            v[r | j] = asc ? hi : lo;
          }
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < VPT; ++r) {
      const int e = lane * VPT + r;
      key[e] = (unsigned)(v[r] >> 11);
      pos[(int)(v[r] & 0x7FFu)] = (unsigned short)e;
    }
  }
  for (int i = lane; i < Q * kWords; i += 64) s_bits[Q * w * kWords + i] = 0u;
  wave_sync();

  // 3. frame loop: lanes h LP ... h LP + LP - 1 serve pixel Q w + h
  const int h = lane / LP, hl = lane % LP;
  const unsigned short* wpos = s_pos + Q * w * TP;
  unsigned* wbits = s_bits + Q * w * kWords;
  const unsigned* key = s_key + (Q * w + h) * TP;
  const unsigned short* pos = wpos + h * TP;
  const unsigned* bits = wbits + h * kWords;
  const long long pix = pix0 + Q * w + h;
  const bool pix_ok = pix < npix;
  const int b0 = hl * BQ;
  unsigned long long prev = 0ull;
  unsigned long long cur = sel[lane];
#pragma unroll 1
  for (int f = 0; f < Ti; ++f) {
    const unsigned long long nxt = f + 1 < Ti ? sel[(size_t)(f + 1) * kGroups + lane] : 0ull;
    unsigned long long d = cur ^ prev;
    prev = cur;
    while (d != 0ull) {
      const int i = __ffsll((long long)d) - 1;
      d &= d - 1ull;
      int p[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) p[q] = wpos[q * TP + lane + 64 * i];
#pragma unroll
      for (int q = 0; q < Q; ++q) atomicXor(&wbits[q * kWords + (p[q] >> 5)], 1u << (p[q] & 31));
    }
    wave_sync();
    unsigned long long m;
    if constexpr (BQ == 64) {
      m = *reinterpret_cast<const unsigned long long*>(bits + (b0 >> 5));
    } else {
      const unsigned word = bits[b0 >> 5];
      m = BQ == 32 ? word : (word >> (b0 & 31)) & ((1u << (BQ & 31)) - 1u);
    }
    const unsigned cnt = (unsigned)__popcll(m);
    const unsigned incl = seg_incl_scan<Q>(cnt);
    const unsigned K = (unsigned)__builtin_amdgcn_readlane((int)incl, LP - 1);   // the same in every group
    // position held by the first lane of each group with incl > k, from v
    auto pick = [&](unsigned k, int v) -> int {
      const unsigned long long bal = __ballot(incl > k);
      int a = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const unsigned seg = (unsigned)(bal >> (q * LP)) & (unsigned)((1ull << LP) - 1ull);
        const int aq = __builtin_amdgcn_readlane(v, q * LP + __ffs((int)seg) - 1);
        a = h == q ? aq : a;
      }
      return a;
    };
    float med;
    if (CH && K == 0u) {                                // K is wave-uniform
      med = pix_ok ? psf_all[pix] : 0.0f;
    } else {
      const unsigned klo = K == 0u ? 0u : (K - 1u) / 2u;
      const unsigned before = incl - cnt;               // selected positions ahead of this lane's stretch
      const int r_lo = nth_set_bit64(m, klo - before);
      const float lo = val_of(key[pick(klo, b0 + r_lo)]);
      float hi = lo;
      if (K / 2u != klo) {
        // rank klo + 1: the next marked bit after rank klo's in the same
        // lane, else the lowest marked bit of the next lane that has one
        const bool holds_lo = klo >= before && klo < incl;
        const unsigned long long above = m & ~((2ull << r_lo) - 1ull);
        const int r_hi = holds_lo ? __ffsll((long long)above) - 1 : __ffsll((long long)m) - 1;
        hi = val_of(key[pick(klo + 1u, b0 + r_hi)]);
      }
      med = (lo + hi) * 0.5f;
    }
    if (hl == 0 && pix_ok) {
      if (psf != nullptr) psf[(size_t)f * npix + pix] = med;
      if constexpr (!CH) {
        if (resid != nullptr) resid[(size_t)f * npix + pix] = val_of(key[pos[f]]) - med;
      }
    }
    cur = nxt;
    wave_sync();
  }
}

// Per-pixel median ignoring NaN values (the master sky of Sect. 3.2.1: star
// regions are NaN); a pixel with no value left is NaN.
template <int VPT, bool BUF>
__global__ void __launch_bounds__(16 * kGroups) median_nan_kernel(const float* __restrict__ stack, long long T,
                                                                  long long npix, float* __restrict__ out) {
  constexpr int kPix = 16;
  extern __shared__ __align__(16) unsigned hist[];
  __shared__ SelShared<kPix> sh;
  __shared__ unsigned s_K[kPix];
  const Tile<kPix> t(T, npix);
  unsigned key[VPT];
  load_keys<VPT, kPix, BUF>(t, stack, npix, key);      // frames past T get a NaN key
  unsigned long long bits = 0ull;
#pragma unroll
  for (int i = 0; i < VPT; ++i)
    if (!isnan(val_of(key[i]))) bits |= 1ull << i;
  if (t.tid < kPix) s_K[t.tid] = 0u;
  __syncthreads();
  atomicAdd(&s_K[t.px], (unsigned)__popcll(bits));
  __syncthreads();
  select_median<VPT, kPix, true>(t, key, bits, 0u, hist, sh, s_K);
  if (t.g == 0 && t.pix_ok) out[t.pix] = s_K[t.px] == 0u ? __int_as_float(0x7FC00000) : sh.med[t.px];
}

// Frame selection of the per-frame PSF: row f marks the frames k with
// |t_k - t_f| < t_max and |alpha_k - alpha_f| > alpha_min, packed as
// sel[f][g] bit i = frame g + 64 i; a row with no frame falls back to every
// frame.  counts[f] = frames in row f.  One block of 64 threads per row.
__global__ void __launch_bounds__(64) select_frames_kernel(const double* __restrict__ times,
                                                           const double* __restrict__ parang, long long T,
                                                           double t_max, double alpha_min,
                                                           unsigned long long* __restrict__ sel,
                                                           int* __restrict__ counts) {
  const long long f = blockIdx.x;
  const int g = threadIdx.x;
  const double tf = times[f], af = parang[f];
  unsigned long long bits = 0ull, all = 0ull;
  for (int i = 0; i < 64; ++i) {
    const long long k = g + 64LL * i;
    if (k >= T) break;
    all |= 1ull << i;
    if (fabs(times[k] - tf) < t_max && fabs(parang[k] - af) > alpha_min) bits |= 1ull << i;
  }
  int c = __popcll(bits);
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (c == 0) {
    bits = all;
    c = (int)T;
  }
  sel[f * 64 + g] = bits;
  if (g == 0) counts[f] = c;
}

// Row groups of a long sequence.  Block g takes rows g kWinRows ... (one
// block of four waves per group).  The union pass tests every frame k against
// the group's rows with the selection's own comparisons and compacts the
// selected frames in frame order (a wave ballot per 256 frames); the rows pass
// then re-tests each row against the union only.  The union pass costs T x
// kWinRows comparisons per group, which bounds the sequences this serves to a
// few hundred thousand frames.
constexpr int kPlanThreads = 256;

__global__ void __launch_bounds__(256) window_plan_init_kernel(int* __restrict__ need, long long n_groups,
                                                               int* __restrict__ flags) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n_groups) need[i] = -1;
  if (i == 0) *flags = 0;
}

__global__ void __launch_bounds__(kPlanThreads) window_plan_kernel(const double* __restrict__ times,
                                                                   const double* __restrict__ parang, long long T,
                                                                   double t_max, double alpha_min,
                                                                   int* __restrict__ list, int* __restrict__ counts,
                                                                   int* __restrict__ need,
                                                                   unsigned long long* __restrict__ sel,
                                                                   int* __restrict__ flags) {
  constexpr int kWaves = kPlanThreads / 64;
  __shared__ double s_t[kWinRows], s_a[kWinRows];       // the group's rows
  __shared__ double s_lt[kWinKeys], s_la[kWinKeys];     // the union's frames
  __shared__ int s_wc[kWaves];
  __shared__ int s_n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const long long grp = blockIdx.x, f0 = grp * kWinRows;
  const int nr = (int)(T - f0 < kWinRows ? T - f0 : kWinRows);
  if (tid < nr) {
    s_t[tid] = times[f0 + tid];
    s_a[tid] = parang[f0 + tid];
  }
  if (tid == 0) s_n = 0;
  __syncthreads();
  int* glist = list + grp * kWinKeys;
  for (long long k0 = 0; k0 < T; k0 += kPlanThreads) {
    const long long k = k0 + tid;
    double tk = 0.0, ak = 0.0;
    bool in = false;
    if (k < T) {
      tk = times[k];
      ak = parang[k];
      for (int r = 0; r < nr && !in; ++r) in = fabs(tk - s_t[r]) < t_max && fabs(ak - s_a[r]) > alpha_min;
    }
    const unsigned long long b = __ballot(in);
    if (lane == 0) s_wc[w] = __popcll(b);
    __syncthreads();
    int at = s_n + __popcll(b & ((1ull << lane) - 1ull));
    for (int i = 0; i < w; ++i) at += s_wc[i];
    if (in) {
      if (at < kWinKeys) {
        glist[at] = (int)k;
        s_lt[at] = tk;
        s_la[at] = ak;
      }
      atomicMax(&need[k / kWinRows], (int)grp);
    }
    __syncthreads();
    if (tid == 0) {
      int add = 0;
      for (int i = 0; i < kWaves; ++i) add += s_wc[i];
      s_n += add;
    }
    __syncthreads();
  }
  const int n = s_n;
  if (tid == 0) counts[grp] = n;
  if (n > kWinKeys) return;                              // rejected on the host
  // each wave builds rows w, w + kWaves, ...; lane j owns word j of a row
  for (int r = w; r < nr; r += kWaves) {
    const double tf = s_t[r], af = s_a[r];
    unsigned long long bits = 0ull;
    for (int i = 0; i < kWinKeys / 64; ++i) {
      const int e = lane + 64 * i;
      if (e >= n) break;
      if (fabs(s_lt[e] - tf) < t_max && fabs(s_la[e] - af) > alpha_min) bits |= 1ull << i;
    }
    sel[(f0 + r) * 64 + lane] = bits;
    if (__ballot(bits != 0ull) == 0ull && lane == 0) atomicOr(flags, 1);
  }
}

// resid = stack - psf, elementwise (in place allowed: each thread rewrites
// what it reads).
__global__ void __launch_bounds__(256) window_resid_kernel(const float* stack, const float* __restrict__ psf,
                                                           float* resid, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    resid[i] = stack[i] - psf[i];
}

// ---------------------------------------------------------------------------
// Stacks too deep for registers (T > 4096, e.g. a whole night of frames): the
// same exact median, by a radix select that streams the stack from HBM once
// per 8-bit digit instead of reading it once into registers.  A block owns 64
// consecutive pixels (one 256-byte segment of every frame) and keeps one
// 256-bin histogram per pixel in LDS; its four waves take frames w, w + 4,
// w + 8, ... of all 64 pixels.  After the four digits lo, the key of rank
// (T-1)/2, is known exactly, with its rank among the keys equal to it and how
// many there are; when rank T/2 falls past that run (even T), one more pass
// takes the smallest key above lo.  With resid, a last pass writes value -
// median for every frame (in place allowed: each thread rewrites the values
// it reads).
// ---------------------------------------------------------------------------
constexpr int kStreamPix = 64;
constexpr int kStreamWaves = 4;
constexpr int kStreamPitch = 257;       // words per pixel histogram (odd: spreads the banks)
constexpr int kStreamUnroll = 8;        // frames per thread in flight

__global__ void __launch_bounds__(kStreamPix * kStreamWaves)
median_stream_kernel(const float* __restrict__ stack, long long T, long long npix, float* __restrict__ out,
                     float* resid) {
  extern __shared__ unsigned shist[];                  // kStreamPix x kStreamPitch words
  __shared__ unsigned s_prefix[kStreamPix], s_rank[kStreamPix], s_cnt[kStreamPix], s_min[kStreamPix];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long pix = (long long)blockIdx.x * kStreamPix + lane;
  const bool ok = pix < npix;
  const float* col = stack + (ok ? pix : 0);
  if (tid < kStreamPix) {
    s_prefix[tid] = 0u;
    s_rank[tid] = (unsigned)((T - 1) / 2);
    s_min[tid] = 0xFFFFFFFFu;
  }
  unsigned mask = 0u;
  for (int d = 3; d >= 0; --d) {
    for (int i = tid; i < kStreamPix * kStreamPitch; i += kStreamPix * kStreamWaves) shist[i] = 0u;
    __syncthreads();
    const unsigned prefix = s_prefix[lane];
    const int shft = 8 * d;
    unsigned* h = shist + lane * kStreamPitch;
    if (ok) {
      long long t = wave;
      for (; t + (kStreamUnroll - 1) * kStreamWaves < T; t += kStreamUnroll * kStreamWaves) {
        unsigned k[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) k[u] = key_of(col[(t + u * kStreamWaves) * npix]);
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u)
          if ((k[u] & mask) == prefix) atomicAdd(&h[(k[u] >> shft) & 0xFFu], 1u);
      }
      for (; t < T; t += kStreamWaves) {
        const unsigned k = key_of(col[t * npix]);
        if ((k & mask) == prefix) atomicAdd(&h[(k >> shft) & 0xFFu], 1u);
      }
    }
    __syncthreads();
    // wave w scans the histograms of pixels w, w + 4, ...: lane l sums bins
    // 4l .. 4l + 3, a wave prefix sum finds the lane whose bins hold rank r
    for (int q = wave; q < kStreamPix; q += kStreamWaves) {
      const unsigned r = s_rank[q];
      const unsigned* hq = shist + q * kStreamPitch + 4 * lane;
      const unsigned c0 = hq[0], c1 = hq[1], c2 = hq[2], c3 = hq[3];
      const unsigned x = c0 + c1 + c2 + c3;
      const unsigned incl = wave_incl_scan(x);
      const unsigned long long hit = __ballot(incl > r);
      const int l0 = hit ? __ffsll((long long)hit) - 1 : 63;
      if (lane == l0) {
        unsigned acc = incl - x;                       // keys below this lane's bins
        int b = 0;
        unsigned c = c0;
        if (acc + c0 <= r) { acc += c0; b = 1; c = c1;
          if (acc + c1 <= r) { acc += c1; b = 2; c = c2;
            if (acc + c2 <= r) { acc += c2; b = 3; c = c3; } } }
        s_prefix[q] |= (unsigned)(4 * lane + b) << shft;
        s_rank[q] = r - acc;
        s_cnt[q] = c;
      }
    }
    mask |= 0xFFu << shft;
    __syncthreads();
  }
  // s_prefix is lo's key, s_rank its rank among the keys equal to it and
  // s_cnt how many keys equal it: rank T/2 is lo itself iff it stays in that run
  const unsigned lo_key = s_prefix[lane];
  const unsigned stepr = (unsigned)(T / 2 - (T - 1) / 2);        // 0 (odd T) or 1
  const bool need_hi = ok && s_rank[lane] + stepr >= s_cnt[lane];
  if (__syncthreads_or(need_hi)) {                               // block-uniform
    if (need_hi) {
      unsigned m = 0xFFFFFFFFu;
      for (long long t = wave; t < T; t += kStreamWaves) {
        const unsigned k = key_of(col[t * npix]);
        if (k > lo_key) m = min(m, k);
      }
      atomicMin(&s_min[lane], m);
    }
    __syncthreads();
  }
  const float lo = val_of(lo_key);
  const float hi = need_hi ? val_of(s_min[lane]) : lo;
  const float med = (lo + hi) * 0.5f;
  if (wave == 0 && ok) out[pix] = med;
  if (resid != nullptr && ok) {
    float* rc = resid + pix;
    for (long long t = wave; t < T; t += kStreamWaves) rc[t * npix] = col[t * npix] - med;
  }
}

}  // namespace

// Deep stacks: one launch of the streaming select.
static hipError_t launch_median_stream(const float* stack, long long T, long long npix, float* out, float* resid,
                                       hipStream_t s) {
  const size_t lds = (size_t)kStreamPix * kStreamPitch * sizeof(unsigned);
  const long long blocks = (npix + kStreamPix - 1) / kStreamPix;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (hipError_t e = set_dynamic_lds(median_stream_kernel, lds); e != hipSuccess) return e;
  hipLaunchKernelGGL(median_stream_kernel, dim3((unsigned)blocks), dim3(kStreamPix * kStreamWaves), lds, s, stack, T,
                     npix, out, resid);
  return hipGetLastError();
}

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
      if (hipError_t e = set_dynamic_lds(median_kernel<V, PIX, true>, lds); e != hipSuccess) return e;     \
      hipLaunchKernelGGL((median_kernel<V, PIX, true>), dim3(blocks), dim3(PIX * kGroups), lds, s, stack, T, \
                         npix, out, resid);                                                                \
    } else {                                                                                               \
      if (hipError_t e = set_dynamic_lds(median_kernel<V, PIX, false>, lds); e != hipSuccess) return e;    \
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

hipError_t launch_select_frames(const double* times, const double* parang, long long T, double t_max,
                                double alpha_min, unsigned long long* sel, int* counts, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(select_frames_kernel, dim3((unsigned)T), dim3(64), 0, s, times, parang, T, t_max, alpha_min,
                     sel, counts);
  return hipGetLastError();
}

// Up to 1024 keys per pixel two pixels share a wave (1.2x at 1024 frames,
// 1.9x at 256); at 2048 the one-pixel form keeps twice the waves that its
// LDS allows per compute unit and is faster (134 against 164 ms at 2048 x
// 512^2).
template <int V, int PB, bool CH>
static hipError_t launch_window_v(const float* stack, long long npix, const int* list, int n_keys, int n_rows,
                                  const unsigned long long* sel, const float* psf_all, float* psf, float* resid,
                                  hipStream_t s) {
  constexpr int TP = 64 * V;
  const size_t lds = (size_t)PB * TP * (sizeof(unsigned) + sizeof(unsigned short)) + (size_t)PB * (TP / 32) * 4;
  const unsigned blocks = (unsigned)((npix + PB - 1) / PB);
  if constexpr (V <= 16) {
    if (hipError_t e = set_dynamic_lds(median_window_q_kernel<V, PB, CH, 2>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL((median_window_q_kernel<V, PB, CH, 2>), dim3(blocks), dim3(PB * 32), lds, s, stack, npix,
                       list, n_keys, n_rows, sel, psf_all, psf, resid);
  } else {
    if (hipError_t e = set_dynamic_lds(median_window_kernel<V, PB, CH>, lds); e != hipSuccess) return e;
    hipLaunchKernelGGL((median_window_kernel<V, PB, CH>), dim3(blocks), dim3(PB * 64), lds, s, stack, npix, list,
                       n_keys, n_rows, sel, psf_all, psf, resid);
  }
  return hipGetLastError();
}

// Keys per lane from the frames one block holds; pixels per block: at most
// about 50 KB of LDS, so that three blocks share a compute unit and their
// frame loops hide each other's latency.
template <bool CH>
static hipError_t launch_window_any(const float* stack, long long npix, const int* list, int n_keys, int n_rows,
                                    const unsigned long long* sel, const float* psf_all, float* psf, float* resid,
                                    hipStream_t s) {
  const int vpt = (n_keys + kGroups - 1) / kGroups;
#define GRAPHIC_WINDOW_CASE(V, PB)                                                                          \
  if (vpt <= V)                                                                                            \
    return launch_window_v<V, PB, CH>(stack, npix, list, n_keys, n_rows, sel, psf_all, psf, resid, s);
  GRAPHIC_WINDOW_CASE(1, 16)
  GRAPHIC_WINDOW_CASE(2, 16)
  GRAPHIC_WINDOW_CASE(4, 16)
  GRAPHIC_WINDOW_CASE(8, 16)
  GRAPHIC_WINDOW_CASE(16, 8)
  GRAPHIC_WINDOW_CASE(32, 4)
#undef GRAPHIC_WINDOW_CASE
  return hipErrorInvalidValue;   // more than 2048 keys: rejected on the host before launch
}

hipError_t launch_median_window(const float* stack, long long T, long long npix, const unsigned long long* sel,
                                float* psf, float* resid, hipStream_t s) {
  if (T <= 0 || npix <= 0) return hipSuccess;
  if (T > kWinKeys) return hipErrorInvalidValue;
  return launch_window_any<false>(stack, npix, nullptr, (int)T, (int)T, sel, nullptr, psf, resid, s);
}

hipError_t launch_window_plan(const double* times, const double* parang, long long T, double t_max,
                              double alpha_min, int* list, int* counts, int* need, unsigned long long* sel,
                              int* flags, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  const long long groups = (T + kWinRows - 1) / kWinRows;
  hipLaunchKernelGGL(window_plan_init_kernel, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, need, groups,
                     flags);
  hipLaunchKernelGGL(window_plan_kernel, dim3((unsigned)groups), dim3(kPlanThreads), 0, s, times, parang, T, t_max,
                     alpha_min, list, counts, need, sel, flags);
  return hipGetLastError();
}

hipError_t launch_median_window_rows(const float* stack, long long npix, const int* list, int n_keys, int n_rows,
                                     const unsigned long long* sel, const float* psf_all, float* psf,
                                     hipStream_t s) {
  if (n_rows <= 0 || npix <= 0) return hipSuccess;
  if (n_keys < 0 || n_keys > kWinKeys || n_rows > kWinRows) return hipErrorInvalidValue;
  return launch_window_any<true>(stack, npix, list, n_keys, n_rows, sel, psf_all, psf, nullptr, s);
}

hipError_t launch_window_resid(const float* stack, const float* psf, float* resid, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(window_resid_kernel, dim3(blocks), dim3(256), 0, s, stack, psf, resid, n);
  return hipGetLastError();
}

hipError_t launch_median_nan(const float* stack, long long T, long long npix, float* out, hipStream_t s) {
  if (T <= 0 || npix <= 0) return hipSuccess;
  const long long vpt = (T + kGroups - 1) / kGroups;
  const unsigned blocks = (unsigned)((npix + 15) / 16);
  const bool buf = (long long)kGroups * npix * 4 < 0x7fffffffLL;
  const size_t lds = (size_t)16 * 4 * kHistWords * sizeof(unsigned);
#define GRAPHIC_NAN_CASE(V)                                                                                 \
  if (vpt <= V) {                                                                                          \
    if (buf) {                                                                                             \
      if (hipError_t e = set_dynamic_lds(median_nan_kernel<V, true>, lds); e != hipSuccess) return e;      \
      hipLaunchKernelGGL((median_nan_kernel<V, true>), dim3(blocks), dim3(16 * kGroups), lds, s, stack, T, npix, \
                         out);                                                                             \
    } else {                                                                                               \
      if (hipError_t e = set_dynamic_lds(median_nan_kernel<V, false>, lds); e != hipSuccess) return e;     \
      hipLaunchKernelGGL((median_nan_kernel<V, false>), dim3(blocks), dim3(16 * kGroups), lds, s, stack, T,  \
                         npix, out);                                                                       \
    }                                                                                                      \
    return hipGetLastError();                                                                              \
  }
  GRAPHIC_NAN_CASE(1)
  GRAPHIC_NAN_CASE(2)
  GRAPHIC_NAN_CASE(4)
  GRAPHIC_NAN_CASE(8)
  GRAPHIC_NAN_CASE(16)
  GRAPHIC_NAN_CASE(32)
  GRAPHIC_NAN_CASE(64)
#undef GRAPHIC_NAN_CASE
  return hipErrorInvalidValue;
}

template <int PIX>
static hipError_t launch_median_tm_pix(const float* stack, long long T, long long npix, float* out, float* resid,
                                       hipStream_t s) {
  const long long vpt = (T + kGroups - 1) / kGroups;
  const unsigned blocks = (unsigned)(npix / PIX);
  const size_t lds = (size_t)PIX * (64 / PIX) * kHistWords * sizeof(unsigned);
#define GRAPHIC_TM_CASE(V)                                                                                  \
  if (vpt <= V) {                                                                                          \
    if (hipError_t e = set_dynamic_lds(median_tm_kernel<V, PIX>, lds); e != hipSuccess) return e;          \
    hipLaunchKernelGGL((median_tm_kernel<V, PIX>), dim3(blocks), dim3(PIX * kGroups), lds, s, stack, T, npix, \
                       out, resid);                                                                        \
    return hipGetLastError();                                                                              \
  }
  GRAPHIC_TM_CASE(1)
  GRAPHIC_TM_CASE(2)
  GRAPHIC_TM_CASE(4)
  GRAPHIC_TM_CASE(8)
  GRAPHIC_TM_CASE(16)
  GRAPHIC_TM_CASE(32)
  GRAPHIC_TM_CASE(64)
#undef GRAPHIC_TM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_median_tile_major(const float* stack, long long T, long long npix, float* out, float* resid,
                                    int variant, hipStream_t s) {
  if (T <= 0 || npix <= 0) return hipSuccess;
  if (npix % kTilePix != 0 || T > 4096) return hipErrorInvalidValue;
  return variant == 1 ? launch_median_tm_pix<8>(stack, T, npix, out, resid, s)
                      : launch_median_tm_pix<16>(stack, T, npix, out, resid, s);
}

hipError_t launch_median(const float* stack, long long T, long long npix, float* out, float* resid, int variant,
                         hipStream_t s) {
  if (T <= 0 || npix <= 0) return hipSuccess;
  if (T > (long long)kGroups * 64) return launch_median_stream(stack, T, npix, out, resid, s);
  return variant == 1 ? launch_median_pix<8>(stack, T, npix, out, resid, s)
                      : launch_median_pix<16>(stack, T, npix, out, resid, s);
}

}  // namespace graphic
