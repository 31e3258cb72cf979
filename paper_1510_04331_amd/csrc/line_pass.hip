// Line passes: one-dimensional Fourier shifts of zero-padded lines (gfx950).
//
// Every geometric operation of the pipeline is a sequence of passes, each of
// which shifts every line of a frame along one axis by its own amount
// (Sect. 3.3.1: the 2-D shift phasor is separable, so the 2-D shift is a pass
// along y followed by a pass along x; Sect. 3.4: each shear is a pass whose
// shift grows linearly with the line coordinate).
//
// One "job" handles two real lines packed as one complex line z = a + i b':
//   * same-shift pairing (shift passes): b' = b, both lines use shift s;
//   * mirror pairing (shear passes): lines c-d and c+d have opposite shifts;
//     b' is b reversed about the centre of the source support.  Reversal R
//     satisfies R K_s R = K_{-s} for the periodic shift operator K_s (its
//     kernel is even), so one phasor serves both lines and no spectral
//     separation is needed.
// The length-P transform of a support of at most P points is split into its
// even and odd bins (two half-size transforms of M = P/2 points, the first
// radix-2 stage done as a fold), each half-size transform is a four-step
// transform M = Ma x Mb in registers with one LDS transpose, the phasor is
// applied between the forward and inverse transforms, and the last radix-2
// stage is done as an unfold that writes only the requested output window.
//
// The even-bin half of a job runs on Ma lanes and the odd-bin half on the next
// Ma lanes; every lane holds Mb complex values.  LDS exchanges move the real
// parts and then the imaginary parts through one float buffer, which halves
// the LDS footprint per wave.
//
// Memory access: blocks never straddle frames, so every base address is
// wave-uniform and all loads and stores are bounds-checked buffer
// instructions: an offset outside the frame reads 0 (the zero padding) and a
// store outside it is dropped, which keeps the kernel free of branches.
//
// Phasor: bin k of the length-P transform (signed index kt) gets
// exp(-2 pi i kt s / P); the Nyquist bin gets cos(pi s).  The phase kt*s/P is
// formed and reduced modulo one in float64 as kt = (2 k2 + h) + 2 Mb k1' with
// a per-lane factor for (2 k2 + h) and a per-job table over k1', each entry
// evaluated from its own float64-reduced phase.

#include <algorithm>

#include <atomic>

#include "dft_codelets.h"
#include "internal.h"

namespace graphic {

template <int M>
struct Shape {
  static constexpr int lg = __builtin_ctz(M);
  static constexpr int Ma = 1 << (lg / 2);
  static constexpr int Mb = M / Ma;
  static constexpr int JOB = 2 * Ma;
  static constexpr int ROWP = Ma + 1;                  // padded LDS row (floats)
  static constexpr int HALF = Mb * ROWP;               // floats per half-job
  static constexpr int PER_JOB_F = 2 * HALF + 2 * Ma;  // + phasor table (complex)
  static constexpr int PER_JOB_F_DB = 4 * HALF + 2 * Ma;  // double-buffered exchanges
  static_assert(Mb == Ma || Mb == 2 * Ma, "square or 1:2 four-step split");
};

// ---------------------------------------------------------------------------
// exp(-2 pi i * kk * q) * scale with the phase reduced in float64:
// ph = kk*q mod 1 in [-1/2, 1/2], then the nearest quarter turn is taken out
// (so the float32 angle is at most pi/4) and sin/cos come from their Taylor
// series (remainders below 2e-9 on [-pi/4, pi/4]).
// ---------------------------------------------------------------------------
__device__ __forceinline__ cf phase_exp(double kk, double q, float scale) {
  double ph = kk * q;
  ph -= rint(ph);
  const double qt = rint(4.0 * ph);                   // quarter turns, -2..2
  const float a = (float)((ph - 0.25 * qt) * -6.283185307179586476925);
  const float a2 = a * a;
  float sn = fmaf(a2, 2.7557319e-6f, -1.9841270e-4f);
  sn = fmaf(a2, sn, 8.3333333e-3f);
  sn = fmaf(a2, sn, -1.6666667e-1f);
  sn = a * fmaf(a2, sn, 1.0f);
  float cs = fmaf(a2, -2.7557319e-7f, 2.4801587e-5f);
  cs = fmaf(a2, cs, -1.3888889e-3f);
  cs = fmaf(a2, cs, 4.1666667e-2f);
  cs = fmaf(a2, cs, -0.5f);
  cs = fmaf(a2, cs, 1.0f);
  // exp(-i 2 pi (r + qt/4)) = exp(-i 2 pi r) * (-i)^qt
  const int qi = ((int)qt) & 3;
  float re = cs, im = sn;
  if (qi == 1) { re = sn; im = -cs; }
  else if (qi == 2) { re = -cs; im = -sn; }
  else if (qi == 3) { re = -sn; im = cs; }
  return {re * scale, im * scale};
}

// Launch shape of the column passes per half-size M: jobs per block (G),
// occupancy target in waves per SIMD (W, which bounds the register budget)
// and whether the exchanges use separate real / imaginary buffers (DB: fewer
// barriers, twice the LDS).  Measured on MI355X; each can be overridden at
// build time.
#ifndef GRAPHIC_COL_G_256
#define GRAPHIC_COL_G_256 16
#endif
#ifndef GRAPHIC_COL_W_256
#define GRAPHIC_COL_W_256 4
#endif
#ifndef GRAPHIC_COL_DB_256
#define GRAPHIC_COL_DB_256 1
#endif
#ifndef GRAPHIC_COL_G_512
#define GRAPHIC_COL_G_512 8
#endif
#ifndef GRAPHIC_COL_W_512
#define GRAPHIC_COL_W_512 2
#endif
#ifndef GRAPHIC_COL_DB_512
#define GRAPHIC_COL_DB_512 1
#endif
#ifndef GRAPHIC_COL_G_1024
#define GRAPHIC_COL_G_1024 8
#endif
#ifndef GRAPHIC_COL_W_1024
#define GRAPHIC_COL_W_1024 4
#endif
#ifndef GRAPHIC_COL_DB_1024
#define GRAPHIC_COL_DB_1024 0
#endif
#ifndef GRAPHIC_COL_G_2048
#define GRAPHIC_COL_G_2048 8
#endif
#ifndef GRAPHIC_COL_W_2048
#define GRAPHIC_COL_W_2048 2
#endif
#ifndef GRAPHIC_COL_DB_2048
#define GRAPHIC_COL_DB_2048 0
#endif
// Occupancy target (waves per SIMD) of the same-pair row pass at M = 1024
// (canonical window).
#ifndef GRAPHIC_ROW_W_1024
#define GRAPHIC_ROW_W_1024 4
#endif
// Row passes at M = 1024 that read their twiddle factors from LDS
// (persistent blocks of 16 waves) instead of the global tables, by index
// pattern: bit 0 window to window (the shift's row pass), bit 1 window to
// full line (first x-shear), bit 2 full line to window (last x-shear).
#ifndef GRAPHIC_ROW_LDS_TW
#define GRAPHIC_ROW_LDS_TW 6
#endif
#ifndef GRAPHIC_COL_WAVE_LAYOUT
#define GRAPHIC_COL_WAVE_LAYOUT 0
#endif
#ifndef GRAPHIC_COL_STAGED
#define GRAPHIC_COL_STAGED 1
#endif

// Thread layout of a pass.  Row passes, and column passes when
// GRAPHIC_COL_WAVE_LAYOUT is set, keep every job inside one wave (lanes =
// positions of the job), so exchanges need only wave-level ordering.  The
// default column layout puts consecutive jobs (adjacent columns) on
// consecutive lanes, which makes every load and store a contiguous row
// segment, at the price of block-wide barriers.
template <int KIND>
constexpr bool lanes_on_jobs() {
  return KIND == kColPass && !GRAPHIC_COL_WAVE_LAYOUT;
}

template <int M>
constexpr bool col_db() {
  return lanes_on_jobs<kColPass>() &&
         (M == 256 ? GRAPHIC_COL_DB_256 : M == 512 ? GRAPHIC_COL_DB_512 : M == 1024 ? GRAPHIC_COL_DB_1024
          : M == 2048 ? GRAPHIC_COL_DB_2048 : 1);
}

template <int M, int KIND, bool MIR = false, int IO = kIoWinWin>
constexpr int waves_per_eu() {
  if (KIND == kColPass && lanes_on_jobs<KIND>()) {
    if (M == 256) return GRAPHIC_COL_W_256;
    if (M == 512) return GRAPHIC_COL_W_512;
    if (M == 1024) return GRAPHIC_COL_W_1024;
    if (M == 2048) return GRAPHIC_COL_W_2048;
  }
  // rows of M = 1024: the mirror-paired shears fit 4 waves without spilling;
  // the same-pair pass of the canonical window spills one value at 4 and is
  // still faster there (6.89 -> 6.75 ms per 2048 frames of 1024^2); its
  // general index path would spill 8 and keeps 3
  return M <= 256 ? 4 : (M == 1024 ? (MIR ? 4 : (IO == kIoGeneric ? 3 : GRAPHIC_ROW_W_1024)) : 2);
}

typedef int v2i __attribute__((ext_vector_type(2)));

// Cache policy of the frame loads: the x-shears that read their twiddle
// factors from the global tables read their frames with the non-temporal
// hint (each value is read once, and the tables then stay cached: measured
// 0.3-0.6 ms faster per 2048 frames of 1024^2); the y-shear, which writes back
// the lines it reads, and the shift passes were measured slower or unchanged
// with it and keep the default.  With the tables in LDS the first x-shear is
// faster with the default policy (7.35 -> 6.11 ms per 2048 frames of
// 1024^2): the waves that share a 128-byte line of the tile-major stack then
// find it in L2; the last x-shear, which reads whole frame-major lines once,
// keeps the hint (8.0 -> 7.64 ms).
constexpr int kCpolDefault = 0;
constexpr int kCpolNonTemporal = 2;
#ifndef GRAPHIC_PRIO_ALL
#define GRAPHIC_PRIO_ALL 0
#endif

template <int CPOL = kCpolDefault>
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, int soff = 0) {
  return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, soff, CPOL));
}
__device__ __forceinline__ cf buf_ld2(__amdgpu_buffer_rsrc_t r, unsigned off, int soff) {
  const v2i t = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, soff, 0);
  return {__int_as_float(t.x), __int_as_float(t.y)};
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, float v, int soff = 0) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, (int)off, soff, 0);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned bytes) {
  // third dword of the gfx9 buffer descriptor: 32-bit raw data, bounds-checked
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

constexpr unsigned kOOB = 0x80000000u;   // beyond every frame: reads 0, writes dropped

// Products with a factor stored as its offset from one, w = 1 + d (the fold
// table): x w = x + x d in four fused multiply-adds, the same count as a
// plain complex product.  With d = 0 (the even half, whose lanes read the
// table out of bounds and get zero) the result is x exactly.
__device__ __forceinline__ cf cmul_1p(cf x, cf d) {
  return {fmaf(x.x, d.x, fmaf(-x.y, d.y, x.x)), fmaf(x.x, d.y, fmaf(x.y, d.x, x.y))};
}
// x conj(1 + d)
__device__ __forceinline__ cf cmulc_1p(cf x, cf d) {
  return {fmaf(x.x, d.x, fmaf(x.y, d.y, x.x)), fmaf(x.y, d.x, fmaf(-x.x, d.y, x.y))};
}

// LDS floats of a block: exchange buffers (or, for staged column blocks, the
// larger of those and the staging tile of M rows x 2G lines), then the
// per-job phasor tables.
template <int M, int KIND, int G, bool STG>
constexpr int lds_floats() {
  using S = Shape<M>;
  constexpr bool LJ = lanes_on_jobs<KIND>() && !STG;
  constexpr int BUF = G * 2 * S::HALF;
  constexpr int region = (LJ && col_db<M>()) ? 2 * BUF : BUF;
  constexpr int stg = STG ? M * (2 * G + 1) : 0;
  return (region > stg ? region : stg) + 2 * G * S::Ma;
}

// One block of jobs: frame f, jobs [jb*G, jb*G + G) of that frame.
//
// STG (staged column blocks, canonical window geometry only): every wave owns
// one job, as in a row block, so the transform's exchanges need only
// wave-level ordering; the block first copies its 2G source columns (the
// window rows) into an LDS tile with row-contiguous loads, and writes its
// results back through the same tile with row-contiguous stores.
//
// TM (bit 0: source, bit 1: destination) selects tile-major cube arrays: a
// row of the frame is then M / 16 chunks of 16 pixels, cs = 64 T bytes apart,
// and each of the job's two rows gets its own wave-uniform descriptor (row
// passes with M >= 1024 run one job per wave).
template <int M, int KIND, int G, int IO, bool MIR, bool STG = false, int TM = 0, int TWL = 0>
__device__ __forceinline__ void process_block(const LinePass& p, const unsigned f, const unsigned jb,
                                              float* wlds = nullptr, const float2* lfold = nullptr,
                                              const float2* lfwd = nullptr) {
  using S = Shape<M>;
  constexpr int Ma = S::Ma, Mb = S::Mb, JOB = S::JOB;
  // TWL: 0 twiddles from the global tables; 1 fold and forward tables in LDS
  // (one-wave row jobs, each with its own LDS area)
  static_assert(TWL == 0 || (TWL == 1 && Ma == Mb && KIND == kRowPass && G == 1 && JOB == 64 && !STG),
                "LDS twiddles: one-wave row jobs of a square four-step split");
  static_assert(!STG || (KIND == kColPass && IO == kIoWinWin), "staging covers the window-to-window column pass");
  constexpr bool TMS = (TM & 1) != 0, TMD = (TM & 2) != 0;
  static_assert(!TM || (M >= 1024 && (KIND == kColPass || G * JOB == 64)), "tile-major rows: one job per wave");
  static_assert(!TMS || KIND == kRowPass, "tile-major sources are read by row passes");
  static_assert(!TMD || (KIND == kRowPass ? (IO == kIoWinWin || IO == kIoFullWin) : STG),
                "tile-major destinations: window stores of row passes or staged column stores");
  // Column blocks span several waves: their exchanges use separate buffers
  // for real and imaginary parts, so each exchange needs one barrier.  Row
  // blocks are one wave (barriers are free, LDS bounds occupancy): one buffer.
  constexpr bool LJ = lanes_on_jobs<KIND>() && !STG;
  constexpr bool DB = LJ && col_db<M>();
  constexpr int BUF = G * 2 * S::HALF;
  constexpr int SP = 2 * G + 1;                        // staging tile pitch (floats per row)
  extern __shared__ float lds_raw[];
  // TWL == 1: the wave's own exchange area and phasor table (wlds)
  float* lds = TWL == 1 ? wlds : lds_raw;
  float* stg = lds_raw;                                // staging tile (aliases the exchange buffers)
  cf* ptab = reinterpret_cast<cf*>(lds + (lds_floats<M, KIND, G, STG>() - 2 * G * Ma));

  const int tid = TWL == 1 ? (int)(threadIdx.x & 63u) : (int)threadIdx.x;
  int jl, r;
  if constexpr (!LJ) {
    jl = tid / JOB;
    r = tid % JOB;
  } else {
    jl = tid % G;
    r = tid / G;
  }
  const int h = r / Ma;        // 0: even bins, 1: odd bins
  const int n1 = r % Ma;

  // LDS float addressing: (job, half, row k2, column c); the column kernel
  // keeps the job index fastest so that lanes of one wave (consecutive jobs)
  // hit consecutive words.
  auto lidx = [&](int hh, int k2, int c) -> int {
    if constexpr (!LJ)
      return (jl * 2 + hh) * S::HALF + k2 * S::ROWP + c;
    else
      return ((hh * Mb + k2) * S::ROWP + c) * G + jl;
  };
  auto tidx = [&](int k1) -> int {
    if constexpr (!LJ)
      return jl * Ma + k1;
    else
      return k1 * G + jl;
  };
  // exchange ordering: a block barrier when jobs span waves, otherwise only a
  // wave-level ordering point (LDS operations of one wave complete in order)
  auto xsync = [&]() {
    if constexpr (LJ) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  };

  const int j = (int)jb * G + jl;
  const bool job_ok = j < p.n_jobs;

  const int P = p.P;
  const int c = P / 2;
  const int flipf = p.flip != nullptr ? (p.flip[f] != 0) : 0;
  const int line_lo = p.line_lo + (p.flip_lines ? flipf : 0);
  // Line coordinates are periodic (mod P): with P = N a half-turned frame's
  // support wraps, and padded line P is line 0 (shift -c * coef).
  int la, lb2;
  bool b_exists = true;
  if (MIR) {
    la = c - j;                     // j in [0, c]
    lb2 = (c + j) & (P - 1);
    b_exists = (j != 0) && (lb2 != la);
  } else {
    la = line_lo + 2 * j;
    lb2 = la + 1;
  }
  const int ra = (la - line_lo + P) & (P - 1);    // rank of the line inside the line set
  const int rb = (lb2 - line_lo + P) & (P - 1);
  const bool a_ok = job_ok && ra < p.n_lines;
  const bool b_ok = job_ok && b_exists && rb < p.n_lines;
  // frame -> source / destination arrays (and constant shift) of its cube
  // (a null array in the cube entry means the launch's own array, indexed by f)
  const float* src_base = p.src;
  float* dst_base = p.dst;
  const double* sh0 = p.sh0;
  long long fsrc = f, fdst = f, fsh = f;
  long long tmT = 1;
  if (p.n_cubes > 0) {
    int ci = 0;
    for (int q2 = 1; q2 < p.n_cubes; ++q2)
      if ((long long)f >= p.cubes[q2].frame0) ci = q2;
    const long long fl = (long long)f - p.cubes[ci].frame0;
    if (p.cubes[ci].src) { src_base = p.cubes[ci].src; fsrc = fl; }
    if (p.cubes[ci].dst) { dst_base = p.cubes[ci].dst; fdst = fl; }
    if (p.cubes[ci].sh0) { sh0 = p.cubes[ci].sh0; fsh = fl; }
    tmT = p.cubes[ci].tm_T;
  }
  double s = 0.0;
  if (sh0) s += sh0[fsh];
  if (p.sh1) s += p.sh1[f] * (double)(la - c);
  const double q = s / (double)P;

  const int in_off = p.in_off + (p.flip_in_off ? flipf : 0);
  const int L = p.in_len;
  const int R = 2 * in_off + L - 1;
  const bool rev = p.flip_src_reverse && flipf;
  const bool rev_b = MIR ? !rev : rev;
  const int lia = rev ? (p.n_lines - 1 - ra) : ra;
  const int lib = rev ? (p.n_lines - 1 - rb) : rb;

  const __amdgpu_buffer_rsrc_t src = make_rsrc(src_base + (size_t)fsrc * p.src_fs, (unsigned)p.src_fs * 4u);
  const __amdgpu_buffer_rsrc_t dst = make_rsrc(dst_base + (size_t)fdst * p.dst_fs, (unsigned)p.dst_fs * 4u);
  const __amdgpu_buffer_rsrc_t tfold = make_rsrc(p.tw.fold, 2u * M * 8u);
  const __amdgpu_buffer_rsrc_t tfwd = make_rsrc(p.tw.fwd, (unsigned)M * 8u);
  const __amdgpu_buffer_rsrc_t tinv = make_rsrc(p.tw.inv, (unsigned)M * 8u);
  const unsigned ls4 = (unsigned)p.src_ls * 4u;
  const int ps4 = p.src_ps * 4;
  // tile-major arrays: byte offset of row position x from the row's first
  // chunk, and the descriptor of row y of local frame fl (its M / 16 chunks)
  const unsigned cs = (unsigned)(tmT * 64);
  auto tmo = [&](int x) -> unsigned { return (unsigned)(x >> 4) * cs + (unsigned)(x & 15) * 4u; };
  auto tm_row = [&](const float* base, long long fl, int y) {
    const int yu = __builtin_amdgcn_readfirstlane(y);
    return make_rsrc(base + ((long long)yu * (M / kTilePix) * tmT + fl) * kTilePix,
                     (unsigned)(M / kTilePix - 1) * cs + 64u);
  };
  auto off_src = [&](int x) -> unsigned { return TMS ? tmo(x) : (unsigned)(x * ps4); };
  const __amdgpu_buffer_rsrc_t srcA = TMS ? tm_row(src_base, fsrc, a_ok ? lia : 0) : src;
  const __amdgpu_buffer_rsrc_t srcB = TMS ? tm_row(src_base, fsrc, b_ok ? lib : 0) : src;
  const unsigned base_a = a_ok ? (TMS ? 0u : (unsigned)lia * ls4) : kOOB;
  const unsigned base_b = b_ok ? (TMS ? 0u : (unsigned)lib * ls4) : kOOB;
  // the canonical geometries (P = 2N, frame not half-turned) use static
  // index patterns; everything else takes the general path
  constexpr bool fast = IO != kIoGeneric;

  // ---- per-job phasor table over k1 (read after the first exchange) ----
  if (h == 0) {
    const int k1s = n1 < Ma / 2 ? n1 : n1 - Ma;
    ptab[tidx(n1)] = phase_exp((double)(2 * Mb) * (double)k1s, q, 1.0f / (float)P);
  }

  // Waves issue their input loads at raised priority so that every wave's
  // requests are in flight early; measured per pass: it helps the shift
  // passes and the first shear, and slows the y-shear and the last shear.
  constexpr bool kLoadPrio = GRAPHIC_PRIO_ALL || (!(KIND == kColPass && MIR) && IO != kIoFullWin);
  constexpr int kLdPol = (KIND == kRowPass && MIR && (TWL == 0 || IO == kIoFullWin)) ? kCpolNonTemporal : kCpolDefault;
  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(2);

  // ---- load, pack and fold into this half's branch ----
  const float sg = h ? -1.0f : 1.0f;
  const unsigned tw_lane = (unsigned)(h * M + n1) * 8u;
  // twiddle factors of this lane: fold / unfold offsets d = w - 1 (n = n1 +
  // Ma n2 of half h; the even half reads out of bounds, d = 0, and fetches
  // nothing), forward four-step (n1 k2), inverse four-step (the conjugate of
  // the forward factor at (c1, n1) when Ma == Mb, so both read one table);
  // from LDS as TWL selects
  const unsigned tw_fold_lane = h ? tw_lane : kOOB;
  auto tw_fold = [&](int n2) -> cf {
    if constexpr (TWL == 1) {
      const float2 t = lfold[h * M + n1 + Ma * n2];
      return {t.x, t.y};
    }
    else return buf_ld2(tfold, tw_fold_lane, Ma * n2 * 8);
  };
  auto tw_fwd = [&](int k2) -> cf {
    if constexpr (TWL != 0) {
      const float2 t = lfwd[n1 + Ma * k2];
      return {t.x, t.y};
    }
    else return buf_ld2(tfwd, (unsigned)n1 * 8u, k2 * Ma * 8);
  };
  auto tw_inv = [&](int c1, int qq) -> cf {
    if constexpr (TWL != 0) {
      const float2 t = lfwd[n1 + Ma * c1];
      return {t.x, -t.y};
    } else if constexpr (Ma == Mb) {
      const cf t = buf_ld2(tfwd, (unsigned)n1 * 8u, c1 * Ma * 8);
      return {t.x, -t.y};
    } else {
      return buf_ld2(tinv, (unsigned)n1 * 8u, (c1 * Mb + Ma * qq) * 8);
    }
  };
  cf v[Mb];
  // staged blocks: line ranks of the block's 2G lines (slot sl of the tile)
  auto slot_line = [&](int sl, int& rank, bool& ok, bool dst_side) {
    const int jj = MIR ? (int)jb * G + (sl < G ? sl : sl - G) : (int)jb * G + (sl >> 1);
    const bool isb = MIR ? sl >= G : (sl & 1) != 0;
    int l, lbb;
    bool bex = true;
    if (MIR) {
      l = c - jj;
      lbb = (c + jj) & (P - 1);
      bex = (jj != 0) && (lbb != l);
    } else {
      l = line_lo + 2 * jj;
      lbb = l + 1;
    }
    const int line = isb ? lbb : l;
    const int rk = (line - line_lo + P) & (P - 1);
    ok = jj < p.n_jobs && rk < p.n_lines && (!isb || bex);
    rank = dst_side ? ((line - (p.dst_line_lo + (p.flip_lines ? flipf : 0)) + P) & (P - 1)) : rk;
  };
  if constexpr (STG) {
    // tile row u = window position u of every line; slot order keeps each
    // row's global addresses contiguous (mirror pairs: the a lines run
    // downward from the centre, the b lines upward)
    {
      // thread -> fixed slot, rows u0, u0 + JOB/2, ... (2G threads per row)
      const int sl = tid % (2 * G);
      int rk;
      bool ok;
      slot_line(sl, rk, ok, false);
      const unsigned lbase = ok ? (unsigned)rk * ls4 : kOOB;
#pragma unroll 8
      for (int u = tid / (2 * G); u < M; u += JOB / 2)
        stg[u * SP + sl] = buf_ld(src, ok ? lbase + (unsigned)(u * ps4) : kOOB);
    }
    __syncthreads();
    const int sa = MIR ? jl : 2 * jl, sb = MIR ? G + jl : 2 * jl + 1;
#pragma unroll
    for (int n2 = 0; n2 < Mb; ++n2) {
      const int k = (n2 + Mb / 2) % Mb;
      const int ua = n1 + Ma * k;
      const int ub = MIR ? (Ma - 1 - n1) + Ma * (Mb - 1 - k) : ua;
      const float av = stg[ua * SP + sa], bv = stg[ub * SP + sb];
      const float sc = n2 < Mb / 2 ? sg : 1.0f;
      const cf w = tw_fold(n2);
      v[n2] = cmul_1p({sc * av, sc * bv}, w);
    }
    __syncthreads();      // the tile is free: exchanges may overwrite it
  } else if constexpr (fast && (IO == kIoWinWin || IO == kIoWinFull)) {
    // support [M/2, 3M/2): element m = n1 + Ma n2 has exactly one valid
    // candidate, position u = n1 + Ma ((n2 + Mb/2) mod Mb) of the source line
    const unsigned la_lane = base_a + off_src(n1);
    const unsigned lb_lane = base_b + off_src(MIR ? (Ma - 1 - n1) : n1);
#pragma unroll
    for (int n2 = 0; n2 < Mb; ++n2) {
      const int k = (n2 + Mb / 2) % Mb;
      const int sa = (int)off_src(Ma * k);
      const int sb = (int)off_src(MIR ? Ma * (Mb - 1 - k) : Ma * k);
      const float av = buf_ld<kLdPol>(srcA, la_lane, sa), bv = buf_ld<kLdPol>(srcB, lb_lane, sb);
      const float sc = n2 < Mb / 2 ? sg : 1.0f;    // the valid candidate is n = m + M below Mb/2
      const cf w = tw_fold(n2);
      v[n2] = cmul_1p({sc * av, sc * bv}, w);
    }
  } else if constexpr (fast && IO == kIoFullWin) {
    // support [0, P): both candidates n = m and n = m + M are valid
    const unsigned la_lane = base_a + off_src(n1);
    const unsigned lb_lane = base_b + off_src(MIR ? (Ma - 1 - n1) : n1);
#pragma unroll
    for (int n2 = 0; n2 < Mb; ++n2) {
      const int sa0 = (int)off_src(Ma * n2), sa1 = (int)off_src(Ma * n2 + M);
      const int sb0 = (int)off_src(MIR ? Ma * (2 * Mb - 1 - n2) : Ma * n2);
      const int sb1 = (int)off_src(MIR ? Ma * (Mb - 1 - n2) : Ma * n2 + M);
      const float a0 = buf_ld<kLdPol>(srcA, la_lane, sa0), a1 = buf_ld<kLdPol>(srcA, la_lane, sa1);
      const float b0 = buf_ld<kLdPol>(srcB, lb_lane, sb0), b1 = buf_ld<kLdPol>(srcB, lb_lane, sb1);
      const cf w = tw_fold(n2);
      v[n2] = cmul_1p({fmaf(sg, a1, a0), fmaf(sg, b1, b0)}, w);
    }
  } else {
#pragma unroll
    for (int n2 = 0; n2 < Mb; ++n2) {
      const int m = n1 + Ma * n2;
      cf z[2];
#pragma unroll
      for (int cnd = 0; cnd < 2; ++cnd) {
        const int n = m + cnd * M;
        const int u = (n - in_off + P) & (P - 1);
        const bool in = u < L;
        const unsigned pa = (unsigned)(rev ? (L - 1 - u) : u);
        const unsigned pb = (unsigned)(rev_b ? (L - 1 - u) : u);
        const unsigned oa = in ? base_a + off_src((int)pa) : kOOB;
        const unsigned ob = in ? base_b + off_src((int)pb) : kOOB;
        z[cnd] = {buf_ld<kLdPol>(srcA, oa), buf_ld<kLdPol>(srcB, ob)};
      }
      const cf w = tw_fold(n2);
      v[n2] = cmul_1p({fmaf(sg, z[1].x, z[0].x), fmaf(sg, z[1].y, z[0].y)}, w);
    }
  }

  if constexpr (kLoadPrio) __builtin_amdgcn_s_setprio(0);

  // ---- step A: length-Mb transforms over n2, twiddle ----
  Dft<Mb, -1>::run(v);
#pragma unroll
  for (int k2 = 0; k2 < Mb; ++k2) v[k2] = cmul(v[k2], tw_fwd(k2));

  // ---- exchange 1 (real parts, then imaginary parts) ----
  constexpr int NQ = Mb / Ma;
  cf wv[NQ][Ma];
  auto ex1_read = [&](int part) {
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq)
#pragma unroll
      for (int c1 = 0; c1 < Ma; ++c1) {
        const float t = lds[(DB ? part * BUF : 0) + lidx(h, n1 + Ma * qq, c1)];
        if (part) wv[qq][c1].y = t;
        else wv[qq][c1].x = t;
      }
  };
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if (!DB && part) xsync();
#pragma unroll
    for (int k2 = 0; k2 < Mb; ++k2) lds[(DB ? part * BUF : 0) + lidx(h, k2, n1)] = part ? v[k2].y : v[k2].x;
    if constexpr (!DB) {
      xsync();
      ex1_read(part);
    }
  }
  if constexpr (DB) {
    xsync();
    ex1_read(0);
    ex1_read(1);
  }

  // ---- step C: length-Ma transforms over n1, phasor, inverse, twiddle ----
#pragma unroll
  for (int qq = 0; qq < NQ; ++qq) {
    const int k2 = n1 + Ma * qq;
    cf* w = wv[qq];
    Dft<Ma, -1>::run(w);
    const cf tlo = phase_exp((double)(2 * k2 + h), q, 1.0f);
    const bool nyq_lane = (h == 0) && (k2 == 0);
#pragma unroll
    for (int k1 = 0; k1 < Ma; ++k1) {
      cf ph = cmul(tlo, ptab[tidx(k1)]);
      if (k1 == Ma / 2 && nyq_lane) ph.y = 0.f;   // real, symmetric Nyquist term
      w[k1] = cmul(w[k1], ph);
    }
    Dft<Ma, +1>::run(w);
#pragma unroll
    for (int c1 = 0; c1 < Ma; ++c1) w[c1] = cmul(w[c1], tw_inv(c1, qq));
  }

  // ---- exchange 2 ----
  auto ex2_read = [&](int part) {
#pragma unroll
    for (int k2 = 0; k2 < Mb; ++k2) {
      const float t = lds[(DB ? part * BUF : 0) + lidx(h, k2, n1)];
      if (part) v[k2].y = t;
      else v[k2].x = t;
    }
  };
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if (!DB || part == 0) xsync();
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq)
#pragma unroll
      for (int c1 = 0; c1 < Ma; ++c1)
        lds[(DB ? part * BUF : 0) + lidx(h, n1 + Ma * qq, c1)] = part ? wv[qq][c1].y : wv[qq][c1].x;
    if constexpr (!DB) {
      xsync();
      ex2_read(part);
    }
  }
  if constexpr (DB) {
    xsync();
    ex2_read(0);
    ex2_read(1);
  }

  // ---- step A': length-Mb inverse transforms over k2 ----
  Dft<Mb, +1>::run(v);

  // ---- unfold: y[m] = e + W o and y[m + M] = e - W o with W = exp(+2 pi i m/P).
  // The odd half applies W to its own values first; then each half sends its
  // value X (e, or W o) to the other and forms y = sg * X_own + X_other, whose
  // real part is line a and imaginary part line b' at position n = m + h M. ----
#pragma unroll
  for (int n2 = 0; n2 < Mb; ++n2) v[n2] = cmulc_1p(v[n2], tw_fold(n2));

  const int dst_lo = p.dst_line_lo + (p.flip_lines ? flipf : 0);
  const unsigned dls4 = (unsigned)p.dst_ls * 4u;
  const int dps4 = p.dst_ps * 4;
  const int orow_a = (la - dst_lo + P) & (P - 1), orow_b = (lb2 - dst_lo + P) & (P - 1);
  const unsigned obase_a = a_ok ? (TMD ? 0u : (unsigned)orow_a * dls4) : kOOB;
  const unsigned obase_b = b_ok ? (TMD ? 0u : (unsigned)orow_b * dls4) : kOOB;
  auto off_dst = [&](int x) -> unsigned { return TMD ? tmo(x) : (unsigned)(x * dps4); };
  constexpr bool TMDR = TMD && KIND == kRowPass;
  const __amdgpu_buffer_rsrc_t dstA = TMDR ? tm_row(dst_base, fdst, a_ok ? orow_a : 0) : dst;
  const __amdgpu_buffer_rsrc_t dstB = TMDR ? tm_row(dst_base, fdst, b_ok ? orow_b : 0) : dst;
  if constexpr (DB) {
    xsync();
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int n2 = 0; n2 < Mb; ++n2) lds[part * BUF + lidx(h, n2, n1)] = part ? v[n2].y : v[n2].x;
    xsync();
  }
  if constexpr (STG) {
    // half h keeps the window positions of n2 >= Mb/2 (h = 0) or n2 < Mb/2
    // (h = 1): Mb/2 values per part, held until every wave has left its
    // exchange buffers, then written through the tile
    float yv[2][Mb / 2];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      xsync();
#pragma unroll
      for (int n2 = 0; n2 < Mb; ++n2) lds[lidx(h, n2, n1)] = part ? v[n2].y : v[n2].x;
      xsync();
#pragma unroll
      for (int q = 0; q < Mb / 2; ++q) {
        const int n2 = q + (h ? 0 : Mb / 2);
        const float own = h ? (part ? v[q].y : v[q].x) : (part ? v[q + Mb / 2].y : v[q + Mb / 2].x);
        yv[part][q] = fmaf(sg, own, lds[lidx(1 - h, n2, n1)]);
      }
    }
    __syncthreads();
    const int sa = MIR ? jl : 2 * jl, sb = MIR ? G + jl : 2 * jl + 1;
#pragma unroll
    for (int q = 0; q < Mb / 2; ++q) {
      const int n2 = q + (h ? 0 : Mb / 2);
      const int k = (n2 + Mb / 2) % Mb;
      const int ua = n1 + Ma * k;
      const int ub = MIR ? (Ma - 1 - n1) + Ma * (Mb - 1 - k) : ua;
      stg[ua * SP + sa] = yv[0][q];
      stg[ub * SP + sb] = yv[1][q];
    }
    __syncthreads();
    {
      const int sl = tid % (2 * G);
      int rk;
      bool ok;
      slot_line(sl, rk, ok, true);
      if constexpr (TMD) {
        // column rk of a tile-major stack: its rows are M / 16 chunks apart
        float* col = dst_base + ((long long)(rk >> 4) * tmT + fdst) * kTilePix + (rk & 15);
        const long long rstep = (long long)(M / kTilePix) * tmT * kTilePix;
#pragma unroll 8
        for (int u = tid / (2 * G); u < M; u += JOB / 2)
          if (ok) col[u * rstep] = stg[u * SP + sl];
      } else {
        const unsigned lbase = ok ? (unsigned)rk * dls4 : kOOB;
#pragma unroll 8
        for (int u = tid / (2 * G); u < M; u += JOB / 2)
          buf_st(dst, ok ? lbase + (unsigned)(u * dps4) : kOOB, stg[u * SP + sl]);
      }
    }
    return;
  }
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if constexpr (!DB) {
      xsync();
#pragma unroll
      for (int n2 = 0; n2 < Mb; ++n2) lds[lidx(h, n2, n1)] = part ? v[n2].y : v[n2].x;
      xsync();
    }
    const int pb = DB ? part * BUF : 0;
    const unsigned obase = part ? obase_b : obase_a;
    const __amdgpu_buffer_rsrc_t dd = part ? dstB : dstA;
    if constexpr (fast && (IO == kIoWinWin || IO == kIoFullWin)) {
      // window [M/2, 3M/2): half h writes n2 >= Mb/2 (h = 0) or n2 < Mb/2 (h = 1),
      // at window position n1 + Ma ((n2 + Mb/2) mod Mb) (reversed for line b')
      const bool rv = part && MIR;
      const unsigned lane = obase + off_dst(rv ? (Ma - 1 - n1) : n1);
#pragma unroll
      for (int n2 = 0; n2 < Mb; ++n2) {
        const float y = fmaf(sg, part ? v[n2].y : v[n2].x, lds[pb + lidx(1 - h, n2, n1)]);
        const int k = (n2 + Mb / 2) % Mb;
        const bool mine = (n2 >= Mb / 2) == (h == 0);
        buf_st(dd, mine ? lane : kOOB, y, (int)off_dst(rv ? Ma * (Mb - 1 - k) : Ma * k));
      }
    } else if constexpr (fast && IO == kIoWinFull) {
      // all P positions: n = m + h M (reversed, P - 1 - n, for line b')
      const bool rv = part && MIR;
      const unsigned lane =
          obase + (unsigned)((rv ? (Ma - 1 - n1) + (1 - h) * M : n1 + h * M) * dps4);
#pragma unroll
      for (int n2 = 0; n2 < Mb; ++n2) {
        const float y = fmaf(sg, part ? v[n2].y : v[n2].x, lds[pb + lidx(1 - h, n2, n1)]);
        buf_st(dst, lane, y, (rv ? Ma * (Mb - 1 - n2) : Ma * n2) * dps4);
      }
    } else {
#pragma unroll
      for (int n2 = 0; n2 < Mb; ++n2) {
        const float y = fmaf(sg, part ? v[n2].y : v[n2].x, lds[pb + lidx(1 - h, n2, n1)]);
        const int n = n1 + Ma * n2 + h * M;
        const int pos = (part && MIR) ? ((R - n) % P + P) % P : n;
        const int u = pos - p.out_off;
        buf_st(dst, (u >= 0 && u < p.out_len) ? obase + (unsigned)(u * dps4) : kOOB, y);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Half size M = 2048 (P = 4096): one job on two waves.
//
// With the four-step split M = Ma x Mb = 32 x 64 a one-wave job would hold
// Mb = 64 complex values per lane, more than the registers of the two waves a
// SIMD must run to hide latency.  Here wave h of a job holds the even (h = 0)
// or odd (h = 1) bins, and its 64 lanes are (e, n1): e = lane / 32 splits the
// 64-point transforms over n2 / k2 into two 32-point halves, so every lane
// holds 32 values.
//   * forward, decimation in frequency over n2 = j + 32 s: lane e forms
//     (t_0 + (-1)^e t_1) W_64^(j e) from the two folded inputs of s = 0, 1
//     (it loads both), then a 32-point transform gives the bins k2 = 2k + e;
//     the fold twiddle of the odd half and W_64^(j e) are one table factor;
//   * step C as in process_block, one k2 row per lane;
//   * inverse, decimation in time over k2 = 2k + e: 32-point inverse
//     transforms give Y_e[j]; each value is scaled by the conjugate table
//     factor, the two e halves are combined with a lane swap across the 32-lane
//     halves (permlane32_swap), and the two h waves through LDS: with
//     A, B (wave 0) and C, D (wave 1) the scaled values, P0 = A + B,
//     M0 = A - B, P1 = C + D, M1 = C - D, the outputs at m + 1024 q of the
//     padded line (m = n1 + 32 j) are P0 + P1, M0 + i M1, P0 - P1, M0 - i M1
//     for q = 0 .. 3.
// Canonical index patterns only (window or whole line in, window or whole
// line out); half-turned frames and other geometries take process_block.
// ---------------------------------------------------------------------------
constexpr int kSplitM = 2048;
constexpr int kSplitMa = 32, kSplitMb = 64;
constexpr int kSplitRowp = kSplitMa + 1;                 // padded LDS row (floats)
constexpr int kSplitHalf = kSplitMb * kSplitRowp;        // floats of one wave's exchange area
constexpr int kSplitJobF = 2 * kSplitHalf;               // floats of a job's exchange areas

template <int KIND, int G, bool STG>
constexpr int split_lds_floats() {
  constexpr int ex = G * kSplitJobF;
  constexpr int stg = STG ? kSplitM * (2 * G + 1) : 0;
  return (ex > stg ? ex : stg) + G * 2 * 2 * kSplitMa;   // + per-wave phasor tables
}

// e ? b : a for a lane-dependent e, on both parts.
__device__ __forceinline__ cf csel(bool e, cf a, cf b) { return {e ? b.x : a.x, e ? b.y : a.y}; }

template <int KIND, int G, int IO, bool MIR, bool STG>
__device__ __forceinline__ void process_block_split(const LinePass& p, const unsigned f, const unsigned jb) {
  constexpr int M = kSplitM, Ma = kSplitMa, Mb = kSplitMb, ROWP = kSplitRowp;
  constexpr int P = 2 * M;
  constexpr int NT = G * 128;                            // threads of the block
  static_assert(IO == kIoWinWin || IO == kIoWinFull || IO == kIoFullWin, "canonical index patterns");
  static_assert(!STG || (KIND == kColPass && IO == kIoWinWin), "staging covers the window-to-window column pass");
  static_assert(KIND == kColPass ? STG : G == 1, "row passes: one job per block");
  extern __shared__ float lds_raw[];
  const int tid = threadIdx.x;
  const int jl = __builtin_amdgcn_readfirstlane(tid >> 7);          // job of the block
  const int h = __builtin_amdgcn_readfirstlane((tid >> 6) & 1);     // wave of the job: even / odd bins
  const int lane = tid & 63;
  const int e = lane >> 5;                               // half of the 64-point transforms
  const int n1 = lane & 31;
  float* xa = lds_raw + jl * kSplitJobF + h * kSplitHalf;          // this wave's exchange area
  float* xo = lds_raw + jl * kSplitJobF + (1 - h) * kSplitHalf;    // the other wave's
  constexpr int kPtab = split_lds_floats<KIND, G, STG>() - G * 2 * 2 * Ma;
  cf* ptab = reinterpret_cast<cf*>(lds_raw + kPtab) + (jl * 2 + h) * Ma;
  float* stg = lds_raw;
  constexpr int SP = 2 * G + 1;

  const int j = (int)jb * G + jl;
  const bool job_ok = j < p.n_jobs;
  const int c = P / 2;
  const int line_lo = p.line_lo;
  int la, lb2;
  bool b_exists = true;
  if (MIR) {
    la = c - j;
    lb2 = (c + j) & (P - 1);
    b_exists = (j != 0) && (lb2 != la);
  } else {
    la = line_lo + 2 * j;
    lb2 = la + 1;
  }
  const int ra = (la - line_lo + P) & (P - 1);
  const int rb = (lb2 - line_lo + P) & (P - 1);
  const bool a_ok = job_ok && ra < p.n_lines;
  const bool b_ok = job_ok && b_exists && rb < p.n_lines;
  const float* src_base = p.src;
  float* dst_base = p.dst;
  const double* sh0 = p.sh0;
  long long fsrc = f, fdst = f, fsh = f;
  if (p.n_cubes > 0) {
    int ci = 0;
    for (int q2 = 1; q2 < p.n_cubes; ++q2)
      if ((long long)f >= p.cubes[q2].frame0) ci = q2;
    const long long fl = (long long)f - p.cubes[ci].frame0;
    if (p.cubes[ci].src) { src_base = p.cubes[ci].src; fsrc = fl; }
    if (p.cubes[ci].dst) { dst_base = p.cubes[ci].dst; fdst = fl; }
    if (p.cubes[ci].sh0) { sh0 = p.cubes[ci].sh0; fsh = fl; }
  }
  double sft = 0.0;
  if (sh0) sft += sh0[fsh];
  if (p.sh1) sft += p.sh1[f] * (double)(la - c);
  const double q = sft / (double)P;

  const __amdgpu_buffer_rsrc_t src = make_rsrc(src_base + (size_t)fsrc * p.src_fs, (unsigned)p.src_fs * 4u);
  const __amdgpu_buffer_rsrc_t dst = make_rsrc(dst_base + (size_t)fdst * p.dst_fs, (unsigned)p.dst_fs * 4u);
  const __amdgpu_buffer_rsrc_t tsplit = make_rsrc(p.tw.split, 4u * Ma * Ma * 8u);
  const __amdgpu_buffer_rsrc_t tfwd = make_rsrc(p.tw.fwd, (unsigned)M * 8u);
  const __amdgpu_buffer_rsrc_t tinv = make_rsrc(p.tw.inv, (unsigned)M * 8u);
  const unsigned ls4 = (unsigned)p.src_ls * 4u;
  const int ps4 = p.src_ps * 4;
  // per-lane table row of (h, e, n1): entry j at + j * Ma
  const unsigned tw_lane = (unsigned)(((h * 2 + e) * Ma) * Ma + n1) * 8u;

  // per-wave phasor table over k1
  if (e == 0) {
    const int k1s = n1 < Ma / 2 ? n1 : n1 - Ma;
    ptab[n1] = phase_exp((double)(2 * Mb) * (double)k1s, q, 1.0f / (float)P);
  }

  // ---- load and fold: a_e[j] = T[h][e][n1][j] * ((-1)^h z_s0 + (-1)^e (-i)^h z_s1) for a window
  // input (z_s0 at window position m + 1024, z_s1 at m, m = n1 + 32 j), or with
  // z_s = z[m + 1024 s] + (-1)^h z[m + 1024 s + 2048] for a whole-line input ----
  const float sgn_h = h ? -1.0f : 1.0f;
  const float sgn_e = e ? -1.0f : 1.0f;
  // (-1)^e (-i)^h z_s1 as a select: h = 0: sgn_e z; h = 1: sgn_e (z.y, -z.x)
  auto rot = [&](cf z) -> cf { return h ? cf{sgn_e * z.y, -sgn_e * z.x} : cf{sgn_e * z.x, sgn_e * z.y}; };
  cf v[32];
  if constexpr (STG) {
    {
      const int sl = tid % (2 * G);
      int rk = 0;
      bool ok = false;
      {
        const int jj = MIR ? (int)jb * G + (sl < G ? sl : sl - G) : (int)jb * G + (sl >> 1);
        const bool isb = MIR ? sl >= G : (sl & 1) != 0;
        int l, lbb;
        bool bex = true;
        if (MIR) {
          l = c - jj;
          lbb = (c + jj) & (P - 1);
          bex = (jj != 0) && (lbb != l);
        } else {
          l = line_lo + 2 * jj;
          lbb = l + 1;
        }
        const int line = isb ? lbb : l;
        rk = (line - line_lo + P) & (P - 1);
        ok = jj < p.n_jobs && rk < p.n_lines && (!isb || bex);
      }
      const unsigned lbase = ok ? (unsigned)rk * ls4 : kOOB;
#pragma unroll 8
      for (int u = tid / (2 * G); u < M; u += NT / (2 * G))
        stg[u * SP + sl] = buf_ld(src, ok ? lbase + (unsigned)(u * ps4) : kOOB);
    }
    __syncthreads();
    const int sa = MIR ? jl : 2 * jl, sb = MIR ? G + jl : 2 * jl + 1;
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) {
      const int m = n1 + Ma * jj;
      const int ub1 = MIR ? (M - 1 - (m + 1024)) : m + 1024, ub0 = MIR ? (M - 1 - m) : m;
      const cf z0 = {stg[(m + 1024) * SP + sa], stg[ub1 * SP + sb]};
      const cf z1 = {stg[m * SP + sa], stg[ub0 * SP + sb]};
      const cf r = rot(z1);
      const cf w = buf_ld2(tsplit, tw_lane, Ma * jj * 8);
      v[jj] = cmul({fmaf(sgn_h, z0.x, r.x), fmaf(sgn_h, z0.y, r.y)}, w);
    }
    __syncthreads();      // the tile is free: exchanges may overwrite it
  } else {
    constexpr int kLdPol = (KIND == kRowPass && MIR) ? kCpolNonTemporal : kCpolDefault;
    const unsigned base_a = a_ok ? (unsigned)ra * ls4 : kOOB;
    const unsigned base_b = b_ok ? (unsigned)rb * ls4 : kOOB;
    // window input: b' at window position u is b at N - 1 - u; whole line: at P - 1 - u.
    // Positions are n1 + pos with pos <= L - Ma: the lane part goes in the
    // per-lane offset, the rest (never negative) in the uniform one.
    constexpr int L = IO == kIoFullWin ? P : M;
    const unsigned la_lane = base_a + (unsigned)(n1 * ps4);
    const unsigned lb_lane = base_b + (unsigned)((MIR ? (Ma - 1 - n1) : n1) * ps4);
    auto ldz = [&](int pos) -> cf {
      const int ob = MIR ? (L - Ma - pos) : pos;
      return {buf_ld<kLdPol>(src, la_lane, pos * ps4), buf_ld<kLdPol>(src, lb_lane, ob * ps4)};
    };
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) {
      cf z0, z1;
      if constexpr (IO == kIoFullWin) {
        const cf y0 = ldz(Ma * jj), y1 = ldz(Ma * jj + 1024), y2 = ldz(Ma * jj + 2048), y3 = ldz(Ma * jj + 3072);
        z0 = {fmaf(sgn_h, y2.x, y0.x), fmaf(sgn_h, y2.y, y0.y)};
        z1 = {fmaf(sgn_h, y3.x, y1.x), fmaf(sgn_h, y3.y, y1.y)};
        const cf r = rot(z1);
        const cf w = buf_ld2(tsplit, tw_lane, Ma * jj * 8);
        v[jj] = cmul({z0.x + r.x, z0.y + r.y}, w);
      } else {
        z0 = ldz(Ma * jj + 1024);
        z1 = ldz(Ma * jj);
        const cf r = rot(z1);
        const cf w = buf_ld2(tsplit, tw_lane, Ma * jj * 8);
        v[jj] = cmul({fmaf(sgn_h, z0.x, r.x), fmaf(sgn_h, z0.y, r.y)}, w);
      }
    }
  }

  auto wsync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  // ---- 32-point transforms over j: bins k2 = 2k + e; twiddle W_M^(n1 k2) ----
  Dft<32, -1>::run(v);
#pragma unroll
  for (int k = 0; k < 32; ++k)
    v[k] = cmul(v[k], buf_ld2(tfwd, (unsigned)(e * Ma + n1) * 8u, 2 * k * Ma * 8));

  // ---- exchange 1 (this wave's area): lane L takes row k2 = L ----
  cf w[32];
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if (part) wsync();
#pragma unroll
    for (int k = 0; k < 32; ++k) xa[(2 * k + e) * ROWP + n1] = part ? v[k].y : v[k].x;
    wsync();
#pragma unroll
    for (int c1 = 0; c1 < 32; ++c1) {
      const float t = xa[lane * ROWP + c1];
      if (part) w[c1].y = t;
      else w[c1].x = t;
    }
  }

  // ---- step C: 32-point transform over n1, phasor, inverse, twiddle W_M^(-n1 k2) ----
  {
    const int k2 = lane;
    Dft<32, -1>::run(w);
    const cf tlo = phase_exp((double)(2 * k2 + h), q, 1.0f);
    const bool nyq_lane = (h == 0) && (k2 == 0);
#pragma unroll
    for (int k1 = 0; k1 < 32; ++k1) {
      cf ph = cmul(tlo, ptab[k1]);
      if (k1 == Ma / 2 && nyq_lane) ph.y = 0.f;   // real, symmetric Nyquist term
      w[k1] = cmul(w[k1], ph);
    }
    Dft<32, +1>::run(w);
#pragma unroll
    for (int c1 = 0; c1 < 32; ++c1) w[c1] = cmul(w[c1], buf_ld2(tinv, (unsigned)k2 * 8u, c1 * Mb * 8));
  }

  // ---- exchange 2: lane (e, n1) takes k2 = 2k + e of column n1 ----
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    wsync();
#pragma unroll
    for (int c1 = 0; c1 < 32; ++c1) xa[lane * ROWP + c1] = part ? w[c1].y : w[c1].x;
    wsync();
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const float t = xa[(2 * k + e) * ROWP + n1];
      if (part) v[k].y = t;
      else v[k].x = t;
    }
  }

  // ---- 32-point inverse transforms over k: Y_e[j]; scaled by conj(T[h][e][n1][j]) ----
  Dft<32, +1>::run(v);
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) v[jj] = cmulc(v[jj], buf_ld2(tsplit, tw_lane, Ma * jj * 8));

  // ---- combine the e halves: lane (e, n1) gets P = X0 + X1 and M = X0 - X1 at j = 2i + e ----
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const auto rx = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * i].x), __float_as_uint(v[2 * i + 1].x),
                                                     false, false);
    const auto ry = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * i].y), __float_as_uint(v[2 * i + 1].y),
                                                     false, false);
    const cf x0 = {__uint_as_float(rx[0]), __uint_as_float(ry[0])};
    const cf x1 = {__uint_as_float(rx[1]), __uint_as_float(ry[1])};
    v[2 * i] = cadd(x0, x1);         // P
    v[2 * i + 1] = csub(x0, x1);     // M
  }

  // ---- combine the h waves through LDS: wave 0 sends M0 and keeps P0, wave 1
  // sends P1 and keeps i M1; own = P0 or i M1, other = P1 or M0.  Each wave
  // writes its own area (its earlier reads of it come first in program order)
  // and reads the other's after the barrier. ----
  {
    float2* xa2 = reinterpret_cast<float2*>(xa);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const cf s = h ? v[2 * i] : v[2 * i + 1];
      xa2[i * 64 + lane] = make_float2(s.x, s.y);
    }
  }
  __syncthreads();
  cf own[16], oth[16];
  {
    const float2* xo2 = reinterpret_cast<const float2*>(xo);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const float2 t = xo2[i * 64 + lane];
      oth[i] = {t.x, t.y};
      own[i] = h ? cf{-v[2 * i + 1].y, v[2 * i + 1].x} : v[2 * i];
    }
  }
  // outputs X = other + own at m + 1024 h and Y = +-(own - other) at m + 1024 h + 2048
  // (wave 0: X = P0 + P1 at q = 0, Y = P0 - P1 at q = 2; wave 1: X = M0 + i M1 at
  // q = 1, Y = M0 - i M1 at q = 3), m = n1 + 32 j, j = 2i + e
  const float ysg = h ? -1.0f : 1.0f;
  if constexpr (STG) {
    __syncthreads();                 // the exchange areas (aliasing the tile) are read
    const int sa = MIR ? jl : 2 * jl, sb = MIR ? G + jl : 2 * jl + 1;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int m = n1 + Ma * (2 * i + e);
      // window positions: q = 1 (wave 1, X) at m, q = 2 (wave 0, Y) at m + 1024
      const cf y = h ? cadd(oth[i], own[i]) : csub(own[i], oth[i]);
      const int u = h ? m : m + 1024;
      stg[u * SP + sa] = y.x;
      stg[(MIR ? M - 1 - u : u) * SP + sb] = y.y;
    }
    __syncthreads();
    {
      const int sl = tid % (2 * G);
      int rk = 0;
      bool ok = false;
      {
        const int jj = MIR ? (int)jb * G + (sl < G ? sl : sl - G) : (int)jb * G + (sl >> 1);
        const bool isb = MIR ? sl >= G : (sl & 1) != 0;
        int l, lbb;
        bool bex = true;
        if (MIR) {
          l = c - jj;
          lbb = (c + jj) & (P - 1);
          bex = (jj != 0) && (lbb != l);
        } else {
          l = line_lo + 2 * jj;
          lbb = l + 1;
        }
        const int line = isb ? lbb : l;
        const int rkk = (line - line_lo + P) & (P - 1);
        ok = jj < p.n_jobs && rkk < p.n_lines && (!isb || bex);
        rk = (line - p.dst_line_lo + P) & (P - 1);
      }
      const unsigned dls4 = (unsigned)p.dst_ls * 4u;
      const int dps4 = p.dst_ps * 4;
      const unsigned lbase = ok ? (unsigned)rk * dls4 : kOOB;
#pragma unroll 8
      for (int u = tid / (2 * G); u < M; u += NT / (2 * G))
        buf_st(dst, ok ? lbase + (unsigned)(u * dps4) : kOOB, stg[u * SP + sl]);
    }
    return;
  } else {
    const int dst_lo = p.dst_line_lo;
    const unsigned dls4 = (unsigned)p.dst_ls * 4u;
    const int dps4 = p.dst_ps * 4;
    const int orow_a = (la - dst_lo + P) & (P - 1), orow_b = (lb2 - dst_lo + P) & (P - 1);
    const unsigned obase_a = a_ok ? (unsigned)orow_a * dls4 : kOOB;
    const unsigned obase_b = b_ok ? (unsigned)orow_b * dls4 : kOOB;
    // Output positions u = ul + uc: ul = n1 + Ma e per lane, uc = 2 i Ma +
    // 1024 h (+ 2048) uniform, at most UC.  b' is reversed about the end of the
    // output line (length LO): b at LO - 1 - u = (LO - 1 - ul - UC) + (UC - uc).
    constexpr int LO = IO == kIoWinFull ? P : M;
    constexpr int UC = IO == kIoWinFull ? 30 * Ma + 1024 + 2048 : 30 * Ma + 1024;
    const int ul = n1 + Ma * e;
    const unsigned oa_lane = obase_a + (unsigned)(ul * dps4);
    const unsigned ob_lane = obase_b + (unsigned)((MIR ? LO - 1 - UC - ul : ul) * dps4);
    auto st2 = [&](cf y, int uc) {
      buf_st(dst, oa_lane, y.x, uc * dps4);
      buf_st(dst, ob_lane, y.y, (MIR ? UC - uc : uc) * dps4);
    };
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const cf X = cadd(oth[i], own[i]);
      const cf Y = {ysg * (own[i].x - oth[i].x), ysg * (own[i].y - oth[i].y)};
      if constexpr (IO == kIoWinFull) {
        st2(X, 2 * i * Ma + 1024 * h);
        st2(Y, 2 * i * Ma + 1024 * h + 2048);
      } else {
        // window: wave 1 stores X at window position m, wave 0 stores Y at m + 1024
        st2(h ? X : Y, 2 * i * Ma + 1024 * (1 - h));
      }
    }
  }
}

// Occupancy of the two-wave jobs (waves per SIMD), measured on MI355X at
// 256 x 2048^2: 4, except the first x-shear (window in, whole line out),
// which is fastest at 3 (5.1 against 6.5 ms).
template <int IO>
constexpr int split_waves_per_eu() {
  return IO == kIoWinFull ? 3 : 4;
}

template <int KIND, int G, int IO, bool MIR>
__global__ void __launch_bounds__(G * 128)
__attribute__((amdgpu_waves_per_eu(split_waves_per_eu<IO>(), split_waves_per_eu<IO>())))
line_pass_split_kernel(const LinePass p) {
  const unsigned nb = gridDim.x;
  const unsigned b = blockIdx.x;
  const unsigned lb = (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  const unsigned bpf = (unsigned)p.blocks_per_frame;
  const unsigned f = lb / bpf;
  const unsigned jb = lb - f * bpf;
  if (p.flip != nullptr && (p.flip_in_off || p.flip_src_reverse) && p.flip[f] != 0)
    return;   // whole block leaves together, before any barrier
  process_block_split<KIND, G, IO, MIR, KIND == kColPass>(p, f, jb);
}

template <int KIND, int IO>
constexpr bool staged() {
  return GRAPHIC_COL_STAGED && KIND == kColPass && IO == kIoWinWin && lanes_on_jobs<KIND>();
}

// Block slot lb of a pass -> frame f and block jb of that frame (with frame
// groups: frame fastest inside each group of p.frame_group frames).
__device__ __forceinline__ void slot_frame_block(const LinePass& p, unsigned lb, unsigned& f, unsigned& jb) {
  const unsigned bpf = (unsigned)p.blocks_per_frame;
  if (p.frame_group > 1) {
    const unsigned fg = (unsigned)p.frame_group;
    const unsigned grp = lb / (fg * bpf);
    const unsigned rem = lb - grp * (fg * bpf);
    const unsigned f0 = grp * fg;
    const unsigned cnt = min(fg, (unsigned)p.n_frames - f0);
    jb = rem / cnt;
    f = f0 + (rem - jb * cnt);
  } else {
    f = lb / bpf;
    jb = lb - f * bpf;
  }
}

// Canonical-geometry and general kernels over a regular grid.  The hardware
// deals consecutive block ids to the eight XCDs in turn; the remap gives each
// XCD a contiguous range of blocks, so neighbouring lines share its L2.  When
// the pass reads half-turned frames through a different support (first shear
// and column shear of a rotation), those frames are skipped here and handled
// by line_pass_flipped_kernel.
//
// With p.frame_group = g > 1 the blocks of g consecutive frames are
// interleaved (frame fastest, then block of the frame; the last group may
// hold fewer frames), so that blocks running side by side touch the same
// lines of neighbouring frames: in a tile-major stack those are adjacent
// 64-byte pieces of one run.
template <int M, int KIND, int G, int IO, bool MIR, int TM>
__global__ void __launch_bounds__(G * Shape<M>::JOB)
__attribute__((amdgpu_waves_per_eu(waves_per_eu<M, KIND, MIR, IO>(), waves_per_eu<M, KIND, MIR, IO>())))
line_pass_kernel(const LinePass p) {
  const unsigned nb = gridDim.x;
  const unsigned b = blockIdx.x;
  const unsigned lb = (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  unsigned f, jb;
  slot_frame_block(p, lb, f, jb);
  if (IO != kIoGeneric && p.flip != nullptr && (p.flip_in_off || p.flip_src_reverse) && p.flip[f] != 0)
    return;   // whole block leaves together, before any barrier
  process_block<M, KIND, G, IO, MIR, staged<KIND, IO>(), TM>(p, f, jb);
}

// ---------------------------------------------------------------------------
// Row passes at M = 1024 with the twiddle tables in LDS.
//
// Every job of a pass multiplies by the same twiddle factors: the fold /
// unfold factors (2M complex values) and the forward four-step factors (M;
// the inverse ones are their conjugates).  Read from the global tables, each
// one-wave job issues 128 table loads (tens of KiB) through the vector memory
// path, and the transform stalls on their latency between its stages.  With
// the loads removed altogether (wrong results, timing only) the five line
// passes ran 12 of 48 ms faster per 2048 frames of 1024^2.  Here a block of
// kRowLdsWaves waves copies the 24 KiB of tables into LDS once; after that
// single barrier every wave walks its own sequence of slots (slot = frame and
// job, ordered as the blocks of line_pass_kernel) with its own exchange area,
// so the waves of a compute unit drift apart and overlap their loads with
// each other's arithmetic.  Sixteen exchange areas and the tables take the
// whole 160 KiB of LDS: one block per compute unit, four waves per SIMD.
// Slots s of XCD x (block b = x + 8 i) are the contiguous run of that XCD.
// Measured per 2048 frames of 1024^2 (with the default cache policy, see
// kLdPol): first x-shear 8.85 -> 6.1 ms, last x-shear 8.9 -> 8.45 ms; the
// shift's row pass gained nothing and keeps the global tables.  Staged column
// blocks of 16 jobs with the tables in LDS (one block per compute unit) were
// slower (shift_y 7.1 -> 8.6 ms, shear_y 16.2 -> 16.6), and the forward table
// alone in LDS beside the tile of 8 jobs changed nothing.
// ---------------------------------------------------------------------------
constexpr int kRowLdsM = 1024;
constexpr int kRowLdsWaves = 16;
constexpr int row_lds_wave_floats() { return lds_floats<kRowLdsM, kRowPass, 1, false>(); }
constexpr int row_lds_floats() { return kRowLdsWaves * row_lds_wave_floats() + 3 * kRowLdsM * 2; }

template <int IO, bool MIR, int TM>
__global__ void __launch_bounds__(kRowLdsWaves * 64)
line_pass_rows_lds_kernel(const LinePass p) {
  constexpr int M = kRowLdsM;
  extern __shared__ float lds_raw[];
  // 8-byte aligned pairs: one 64-bit LDS read per factor
  float2* lfold = reinterpret_cast<float2*>(lds_raw + kRowLdsWaves * row_lds_wave_floats());
  float2* lfwd = lfold + 2 * M;
  for (int i = threadIdx.x; i < 3 * M; i += kRowLdsWaves * 64) lfold[i] = i < 2 * M ? p.tw.fold[i] : p.tw.fwd[i - 2 * M];
  __syncthreads();
  const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float* wlds = lds_raw + wave * row_lds_wave_floats();
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned lb = (nb & 7u) == 0 ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
  const unsigned long long n_slots = (unsigned long long)p.n_frames * (unsigned)p.blocks_per_frame;
  const unsigned long long stride = (unsigned long long)nb * kRowLdsWaves;
  for (unsigned long long s = (unsigned long long)lb * kRowLdsWaves + wave; s < n_slots; s += stride) {
    unsigned f, jb;
    slot_frame_block(p, (unsigned)s, f, jb);
    if (IO != kIoGeneric && p.flip != nullptr && (p.flip_in_off || p.flip_src_reverse) && p.flip[f] != 0)
      continue;   // half-turned frames take line_pass_flipped_kernel
    process_block<M, kRowPass, 1, IO, MIR, false, TM, 1>(p, f, jb, wlds, lfold, lfwd);
  }
}

// General path for the half-turned frames listed in p.flip_list (count in
// p.flip_count): a fixed grid walks the (frame, block) pairs.
template <int M, int KIND, int G, bool MIR, int TM>
__global__ void __launch_bounds__(G * Shape<M>::JOB, (waves_per_eu<M, KIND, false, kIoGeneric>()))
line_pass_flipped_kernel(const LinePass p) {
  const unsigned bpf = (unsigned)p.blocks_per_frame;
  const unsigned work = (unsigned)(*p.flip_count) * bpf;
  for (unsigned w = blockIdx.x; w < work; w += gridDim.x) {
    const unsigned f = (unsigned)p.flip_list[w / bpf];
    process_block<M, KIND, G, kIoGeneric, MIR, false, TM>(p, f, w % bpf);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Launch
// ---------------------------------------------------------------------------

// Compute units of the current device (persistent launches size their grid
// to it); cached per device.
static int compute_units() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n <= 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

template <int M>
constexpr int col_jobs_per_block() {
  using S = Shape<M>;
  if (!lanes_on_jobs<kColPass>()) return 64 / S::JOB > 0 ? 64 / S::JOB : 1;
  if (M == 256) return GRAPHIC_COL_G_256;
  if (M == 512) return GRAPHIC_COL_G_512;
  if (M == 1024) return GRAPHIC_COL_G_1024;
  if (M == 2048) return GRAPHIC_COL_G_2048;
  constexpr int budget = 140 * 1024;
  int g = 16;
  while (g > 1 && (g * S::PER_JOB_F_DB * 4 > budget || g * S::JOB > 1024)) g /= 2;
  return g;
}

template <int M>
constexpr int row_jobs_per_block() {
  return 64 / Shape<M>::JOB > 0 ? 64 / Shape<M>::JOB : 1;
}

template <int M, int KIND, int G, int IO, bool MIR, int TM = 0>
static hipError_t launch_g(LinePass p, hipStream_t st) {
  using S = Shape<M>;
  static_assert(G * S::JOB <= 1024, "block too large");
  static_assert(lds_floats<M, KIND, G, staged<KIND, IO>()>() * 4 <= 160 * 1024, "LDS per block above 160 KiB");
  p.blocks_per_frame = (p.n_jobs + G - 1) / G;
  const long long blocks = p.n_frames * (long long)p.blocks_per_frame;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool flipped = IO != kIoGeneric && p.flip != nullptr && (p.flip_in_off || p.flip_src_reverse);
  if ((TM & 2) && flipped) return hipErrorInvalidValue;   // the general path stores frame-major only
  hipError_t e;
  if constexpr (KIND == kRowPass && M == kRowLdsM && G == 1 && IO != kIoGeneric &&
                ((GRAPHIC_ROW_LDS_TW >> (IO - 1)) & 1)) {
    constexpr size_t lds = (size_t)row_lds_floats() * sizeof(float);
    static_assert(lds <= 160 * 1024, "LDS per block above 160 KiB");
    if ((e = set_dynamic_lds(line_pass_rows_lds_kernel<IO, MIR, TM>, lds)) != hipSuccess) return e;
    const long long grid = std::min<long long>((blocks + kRowLdsWaves - 1) / kRowLdsWaves, compute_units());
    hipLaunchKernelGGL((line_pass_rows_lds_kernel<IO, MIR, TM>), dim3((unsigned)grid), dim3(kRowLdsWaves * 64), lds,
                       st, p);
  } else {
    constexpr size_t lds = (size_t)lds_floats<M, KIND, G, staged<KIND, IO>()>() * sizeof(float);
    if ((e = set_dynamic_lds(line_pass_kernel<M, KIND, G, IO, MIR, TM>, lds)) != hipSuccess) return e;
    hipLaunchKernelGGL((line_pass_kernel<M, KIND, G, IO, MIR, TM>), dim3((unsigned)blocks), dim3(G * S::JOB), lds,
                       st, p);
  }
  e = hipGetLastError();
  if (e != hipSuccess || !flipped) return e;
  // half-turned frames: general path over the device-side list
  constexpr int TMF = TM & 1;
  const size_t lds_flip = (size_t)lds_floats<M, KIND, G, false>() * sizeof(float);
  if ((e = set_dynamic_lds(line_pass_flipped_kernel<M, KIND, G, MIR, TMF>, lds_flip)) != hipSuccess) return e;
  const long long fb = std::min<long long>(blocks, 2048);
  hipLaunchKernelGGL((line_pass_flipped_kernel<M, KIND, G, MIR, TMF>), dim3((unsigned)fb), dim3(G * S::JOB), lds_flip,
                     st, p);
  return hipGetLastError();
}

// Index pattern of a pass: the canonical window is [M/2, 3M/2) of the padded
// line (P = 2N); "full" is the whole padded line.
static int io_kind(const LinePass& p) {
  const int M = p.P / 2;
  const bool win_in = p.in_off == M / 2 && p.in_len == M;
  const bool full_in = p.in_off == 0 && p.in_len == p.P;
  const bool win_out = p.out_off == M / 2 && p.out_len == M;
  const bool full_out = p.out_off == 0 && p.out_len == p.P;
  if (M < 16) return kIoGeneric;
  if (win_in && win_out) return kIoWinWin;
  if (win_in && full_out) return kIoWinFull;
  if (full_in && win_out && !p.flip) return kIoFullWin;
  return kIoGeneric;
}

// Instantiations that the operations use: the shift passes pair adjacent
// lines, the rotation passes pair mirrored lines.
template <int M, int KIND, int G>
static hipError_t launch_io(const LinePass& p, hipStream_t st) {
  const int io = io_kind(p);
  if (!p.mirror) {
    if (io == kIoWinWin) return launch_g<M, KIND, G, kIoWinWin, false>(p, st);
    return launch_g<M, KIND, G, kIoGeneric, false>(p, st);
  }
  switch (io) {
    case kIoWinWin: return launch_g<M, KIND, G, kIoWinWin, true>(p, st);
    case kIoWinFull:
      if constexpr (KIND == kRowPass) return launch_g<M, KIND, G, kIoWinFull, true>(p, st);
      break;
    case kIoFullWin:
      if constexpr (KIND == kRowPass) return launch_g<M, KIND, G, kIoFullWin, true>(p, st);
      break;
    default: break;
  }
  return launch_g<M, KIND, G, kIoGeneric, true>(p, st);
}

// Alternative tile width (jobs per block) of the staged column pass per M,
// offered to the autotuner as variant 1.
template <int M>
constexpr int col_jobs_alt() {
  return M == 256 ? 8 : M == 512 ? 16 : M == 1024 ? 4 : M == 2048 ? 4 : 0;
}

// Tile-major passes of the ADI reduction (M = 1024, cube launches): the
// shift row pass (in place), the first and last rotation shears (source,
// destination) and the shift column pass (destination).
template <int M>
static hipError_t launch_tile_major(const LinePass& p, int kind, int variant, hipStream_t st) {
  if constexpr (M == 1024) {
    const int tm = (p.src_tm ? 1 : 0) | (p.dst_tm ? 2 : 0);
    const int io = io_kind(p);
    if (p.n_cubes < 1 || (long long)M * 4 * p.cubes[0].tm_T > 0x7fffffffLL) return hipErrorInvalidValue;
    for (int i = 1; i < p.n_cubes; ++i)
      if ((long long)M * 4 * p.cubes[i].tm_T > 0x7fffffffLL) return hipErrorInvalidValue;
    constexpr int GR = row_jobs_per_block<M>();
    if (kind == kRowPass) {
      if (tm == 3 && !p.mirror && io == kIoWinWin) return launch_g<M, kRowPass, GR, kIoWinWin, false, 3>(p, st);
      if (tm == 1 && p.mirror && io == kIoWinFull) return launch_g<M, kRowPass, GR, kIoWinFull, true, 1>(p, st);
      if (tm == 2 && p.mirror && io == kIoFullWin) return launch_g<M, kRowPass, GR, kIoFullWin, true, 2>(p, st);
    } else if (GRAPHIC_COL_STAGED && lanes_on_jobs<kColPass>() && tm == 2 && !p.mirror && io == kIoWinWin) {
      constexpr int GA = col_jobs_alt<M>();
      if (variant == 1 && GA > 0) return launch_g<M, kColPass, (GA > 0 ? GA : 1), kIoWinWin, false, 2>(p, st);
      return launch_g<M, kColPass, col_jobs_per_block<M>(), kIoWinWin, false, 2>(p, st);
    }
  }
  return hipErrorInvalidValue;
}

// Two-wave jobs at M = 2048: G jobs per block.  Row passes: 1.  Staged
// column passes: 4 for the shift's pairing of adjacent columns (two blocks
// per compute unit), 8 for the mirrored pairs of the y-shear (one block, but
// row runs of 32 bytes on each side instead of 16: 10.5 against 12.3 ms at
// 256 x 2048^2); the other width is the tuned alternative.
// Half-turned frames take the general one-wave path.
template <int KIND, int G, int IO, bool MIR>
static hipError_t launch_split(LinePass p, hipStream_t st) {
  constexpr bool STG = KIND == kColPass;
  constexpr size_t lds = (size_t)split_lds_floats<KIND, G, STG>() * sizeof(float);
  static_assert(lds <= 160 * 1024, "LDS per block above 160 KiB");
  p.blocks_per_frame = (p.n_jobs + G - 1) / G;
  const long long blocks = p.n_frames * (long long)p.blocks_per_frame;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipError_t e = set_dynamic_lds(line_pass_split_kernel<KIND, G, IO, MIR>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((line_pass_split_kernel<KIND, G, IO, MIR>), dim3((unsigned)blocks), dim3(G * 128), lds, st, p);
  e = hipGetLastError();
  const bool flipped = p.flip != nullptr && (p.flip_in_off || p.flip_src_reverse);
  if (e != hipSuccess || !flipped) return e;
  // half-turned frames: general path over the device-side list (one-wave jobs)
  constexpr int GF = KIND == kColPass ? col_jobs_per_block<kSplitM>() : row_jobs_per_block<kSplitM>();
  p.blocks_per_frame = (p.n_jobs + GF - 1) / GF;
  const long long fblocks = p.n_frames * (long long)p.blocks_per_frame;
  const size_t lds_flip = (size_t)lds_floats<kSplitM, KIND, GF, false>() * sizeof(float);
  if ((e = set_dynamic_lds(line_pass_flipped_kernel<kSplitM, KIND, GF, MIR, 0>, lds_flip)) != hipSuccess) return e;
  const long long fb = std::min<long long>(fblocks, 2048);
  hipLaunchKernelGGL((line_pass_flipped_kernel<kSplitM, KIND, GF, MIR, 0>), dim3((unsigned)fb),
                     dim3(GF * Shape<kSplitM>::JOB), lds_flip, st, p);
  return hipGetLastError();
}

static hipError_t launch_split_m(const LinePass& p, int kind, int variant, hipStream_t st, bool* done) {
  *done = true;
  const int io = io_kind(p);
  if (kind == kRowPass) {
    if (io == kIoWinWin) return p.mirror ? launch_split<kRowPass, 1, kIoWinWin, true>(p, st)
                                         : launch_split<kRowPass, 1, kIoWinWin, false>(p, st);
    if (io == kIoWinFull && p.mirror) return launch_split<kRowPass, 1, kIoWinFull, true>(p, st);
    if (io == kIoFullWin && p.mirror) return launch_split<kRowPass, 1, kIoFullWin, true>(p, st);
  } else if (io == kIoWinWin) {
    if (p.mirror) return variant == 1 ? launch_split<kColPass, 4, kIoWinWin, true>(p, st)
                                      : launch_split<kColPass, 8, kIoWinWin, true>(p, st);
    return variant == 1 ? launch_split<kColPass, 8, kIoWinWin, false>(p, st)
                        : launch_split<kColPass, 4, kIoWinWin, false>(p, st);
  }
  *done = false;
  return hipSuccess;
}

template <int M>
static hipError_t launch_m(const LinePass& p, int kind, int variant, hipStream_t st) {
  if (p.src_tm || p.dst_tm) return launch_tile_major<M>(p, kind, variant, st);
  if constexpr (M == kSplitM) {
    bool done = false;
    const hipError_t e = launch_split_m(p, kind, variant, st, &done);
    if (done) return e;
  }
  if (kind == kRowPass) return launch_io<M, kRowPass, row_jobs_per_block<M>()>(p, st);
  constexpr int GA = col_jobs_alt<M>();
  if constexpr (GA > 0 && GRAPHIC_COL_STAGED && lanes_on_jobs<kColPass>()) {
    if (variant == 1 && io_kind(p) == kIoWinWin) {
      return p.mirror ? launch_g<M, kColPass, GA, kIoWinWin, true>(p, st)
                      : launch_g<M, kColPass, GA, kIoWinWin, false>(p, st);
    }
  }
  return launch_io<M, kColPass, col_jobs_per_block<M>()>(p, st);
}

hipError_t launch_line_pass(const LinePass& p, int kind, int variant, hipStream_t s) {
  const long long total = p.n_frames * (long long)p.n_jobs;
  if (total <= 0) return hipSuccess;
  switch (p.P / 2) {
    case 8: return launch_m<8>(p, kind, variant, s);
    case 16: return launch_m<16>(p, kind, variant, s);
    case 32: return launch_m<32>(p, kind, variant, s);
    case 64: return launch_m<64>(p, kind, variant, s);
    case 128: return launch_m<128>(p, kind, variant, s);
    case 256: return launch_m<256>(p, kind, variant, s);
    case 512: return launch_m<512>(p, kind, variant, s);
    case 1024: return launch_m<1024>(p, kind, variant, s);
    case 2048: return launch_m<2048>(p, kind, variant, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace graphic
