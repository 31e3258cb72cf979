// C ABI of libgraphic: validation, workspace layout and pass orchestration.
//
// The operations are composed from three kernel families:
//   line passes (line_pass.hip)  -- Fourier shifts of every line of a frame,
//   the exact median (median.hip) and small per-frame kernels (aux_kernels.hip).
//
//   shift  (Sect. 3.3.1):  column pass (dy), row pass (dx), both in place on out.
//   rotate (Sect. 3.4):    x-shear of every window row into a N x P scratch
//                          frame, y-shear of every scratch column (in place),
//                          x-shear of every window row into out.
//   adi    (Sect. 3):      shift -> median PSF (which also rewrites the stack
//                          as residuals S - PSF) -> rotate(residuals, -parang)
//                          -> median.

#include "../../include/graphic.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace graphic;

namespace {

constexpr size_t kAlign = 256;
// Frame counts: up to 4096 frames a pixel's values stay in registers (one
// read of the stack); deeper stacks take the streaming select (one read per
// digit), up to 2^24 frames.  The NaN-ignoring median keeps the register form.
constexpr long long kMaxT_Median = 1LL << 24;
constexpr int kMaxT_RegisterMedian = 4096;
constexpr int kMaxT_NanMedian = 4096;
// Per-frame medians of the selection window: up to kWinKeys frames one block
// holds every value of its pixels; longer sequences run in row groups (each
// group's selections must span at most kWinKeys frames), up to kMaxT_Window
// frames (the plan compares every frame with every row).  With the residuals
// written in place and no PSF cube, each group's PSF waits in a ring of
// kWinRing groups until no later group reads the frames it overwrites.
constexpr long long kMaxT_Window = 1LL << 18;
constexpr int kWinRing = 9;
constexpr size_t kDefaultChunkBytes = size_t(4) << 30;   // rotation scratch per chunk (fewer, fuller launches)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

struct TimingSlot {
  std::string family;
  hipEvent_t start, stop;
};

}  // namespace

struct graphic_ctx_s {
  int device = 0;
  void* tables = nullptr;                 // one device allocation for every M (and the scan flag)
  int* scan_flag = nullptr;               // device int of the non-finite scan, after the tables
  TwiddleTables tw[16] = {};              // indexed by log2(M)
  bool timing = false;
  std::vector<TimingSlot> pending;
  struct Acc {
    std::string family;
    double ms = 0.0;
    long long n = 0;
  };
  std::vector<Acc> acc;
  size_t chunk_bytes = kDefaultChunkBytes;
  bool tile_major = true;                 // workspace stacks of the large canonical sizes are tile-major
  // Block order of the row passes over tile-major stacks: blocks of this many
  // consecutive frames are interleaved.  The x-shears run as persistent
  // blocks whose 16 waves take 16 consecutive slots; with the whole launch as
  // one group (frame fastest throughout) they were fastest: per 2048 frames
  // of 1024^2, 6.15 + 8.22 ms with groups of 32, 5.86 + 7.94 ms with all
  // frames.  The shift's row pass also gains a little (6.89 -> 6.81 ms
  // against groups of 64).
  int frame_group = 4096;                 // the shift's row pass
  int frame_group_shear = 4096;           // the two x-shears
  // tuned launch variants (-1: not tuned, the default variant 0 runs)
  int col_var[16][2];                     // [log2 M][pairing: 0 same, 1 mirror] of the staged column pass
  int med_var[8];                         // [log2 of the median's values per thread]
  int tmm_var[8];                         // the same for the tile-major median
  graphic_ctx_s() {
    for (auto& a : col_var) a[0] = a[1] = -1;
    for (int& v : med_var) v = -1;
    for (int& v : tmm_var) v = -1;
  }
};

namespace {

// ---------------------------------------------------------------------------
// Twiddle tables (float64 on the host, rounded once to float32)
// ---------------------------------------------------------------------------
void host_tables(int M, std::vector<float2>& fwd, std::vector<float2>& inv, std::vector<float2>& fold) {
  const int lg = ilog2(M);
  const int Ma = 1 << (lg / 2), Mb = M / Ma;
  const double two_pi = 6.283185307179586476925286766559;
  fwd.assign(M, float2{0, 0});
  inv.assign(M, float2{0, 0});
  fold.assign(2 * M, float2{0, 0});
  for (int k2 = 0; k2 < Mb; ++k2)
    for (int n1 = 0; n1 < Ma; ++n1) {
      const long e = (long)n1 * k2 % M;
      const double a = two_pi * (double)e / M;
      fwd[k2 * Ma + n1] = float2{(float)std::cos(a), (float)-std::sin(a)};
      inv[n1 * Mb + k2] = float2{(float)std::cos(a), (float)std::sin(a)};
    }
  // fold factors of the odd half, stored as their offset from one:
  // exp(-2 pi i m / 2M) - 1 = (-2 sin^2(a/2), -sin a); the even half (factor
  // one, offset zero) is never read
  for (int m = 0; m < M; ++m) {
    const double a = two_pi * (double)m / (2.0 * M);
    const double sh = std::sin(0.5 * a);
    fold[M + m] = float2{(float)(-2.0 * sh * sh), (float)-std::sin(a)};
  }
}

// Table of the two-wave jobs at M = 2048 (Ma = 32, Mb = 64, P = 4096):
// split[((h*2 + e)*Ma + j)*Ma + n1] = exp(-2 pi i (h (n1 + Ma j) / P + j e / Mb)).
constexpr int kSplitTabM = 2048, kSplitTabMa = 32, kSplitTabMb = 64;
constexpr size_t kSplitTabN = (size_t)4 * kSplitTabMa * kSplitTabMa;

void host_split_table(std::vector<float2>& t) {
  const double two_pi = 6.283185307179586476925286766559;
  const int Ma = kSplitTabMa, Mb = kSplitTabMb, P = 2 * kSplitTabM;
  t.assign(kSplitTabN, float2{0, 0});
  for (int h = 0; h < 2; ++h)
    for (int e = 0; e < 2; ++e)
      for (int j = 0; j < Ma; ++j)
        for (int n1 = 0; n1 < Ma; ++n1) {
          // phase in turns, reduced exactly in integers: h (n1 + Ma j) / P + j e / Mb
          const long num = (long)h * (n1 + Ma * j) + (long)j * e * (P / Mb);
          const double a = two_pi * (double)(num % P) / P;
          t[((h * 2 + e) * Ma + j) * Ma + n1] = float2{(float)std::cos(a), (float)-std::sin(a)};
        }
}

graphic_status build_tables(graphic_ctx ctx) {
  size_t total = 0;
  for (int M = kMinM; M <= kMaxM; M *= 2) total += (size_t)4 * M * sizeof(float2);
  const size_t split_off = total / sizeof(float2);
  total += kSplitTabN * sizeof(float2);
  std::vector<float2> host(total / sizeof(float2));
  {
    std::vector<float2> st;
    host_split_table(st);
    std::memcpy(&host[split_off], st.data(), kSplitTabN * sizeof(float2));
  }
  size_t off = 0;
  std::vector<size_t> offs;
  for (int M = kMinM; M <= kMaxM; M *= 2) {
    std::vector<float2> f, i, fo;
    host_tables(M, f, i, fo);
    offs.push_back(off);
    std::memcpy(&host[off], f.data(), M * sizeof(float2));
    std::memcpy(&host[off + M], i.data(), M * sizeof(float2));
    std::memcpy(&host[off + 2 * M], fo.data(), 2 * M * sizeof(float2));
    off += 4 * M;
  }
  if (hipMalloc(&ctx->tables, total + 256) != hipSuccess) return GRAPHIC_ERR_NOMEM;
  if (hipMemcpy(ctx->tables, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) return GRAPHIC_ERR_HIP;
  ctx->scan_flag = reinterpret_cast<int*>(static_cast<char*>(ctx->tables) + total);
  int idx = 0;
  for (int M = kMinM; M <= kMaxM; M *= 2, ++idx) {
    const float2* base = static_cast<const float2*>(ctx->tables) + offs[idx];
    TwiddleTables& t = ctx->tw[ilog2(M)];
    t.fwd = base;
    t.inv = base + M;
    t.fold = base + 2 * M;
    t.split = M == kSplitTabM ? static_cast<const float2*>(ctx->tables) + split_off : nullptr;
  }
  return GRAPHIC_OK;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }

constexpr uint32_t kAllFlags = GRAPHIC_KEEP_PADDED | GRAPHIC_CHECK_FINITE;

// Geometry checks; `allowed` is the set of geom flags the caller accepts.
graphic_status check_geom(const graphic_geom* g, int* P_out, uint32_t allowed = 0) {
  if (!g) return GRAPHIC_ERR_ARG;
  if ((g->flags & ~allowed) != 0) return GRAPHIC_ERR_ARG;
  if (g->n_frames < 1) return GRAPHIC_ERR_ARG;
  if (g->n < 4 || g->n > 4096 || (g->n % 2) != 0) return GRAPHIC_ERR_ARG;
  int P = g->pad;
  if (P == 0) {
    P = 1;
    while (P < 2 * g->n) P *= 2;
  }
  if (!is_pow2(P) || P < g->n || P < 2 * kMinM || P > 2 * kMaxM) return g->pad ? GRAPHIC_ERR_ARG : GRAPHIC_ERR_UNSUPPORTED;
  *P_out = P;
  return GRAPHIC_OK;
}

// Workspace of the per-frame medians: the selection rows and counts; for row
// groups also the group lists, counts and last readers, the flags, the
// all-frames median and the PSF ring.
struct WindowLayout {
  size_t sel = 0, counts = 0, list = 0, gcount = 0, need = 0, flags = 0, psf_all = 0, ring = 0, total = 0;
};

WindowLayout window_layout(long long T, long long npix) {
  WindowLayout L;
  size_t o = 0;
  L.sel = o;
  o += align_up((size_t)T * 64 * sizeof(unsigned long long));
  L.counts = o;
  o += align_up((size_t)T * sizeof(int));
  if (T > kWinKeys) {
    const size_t groups = (size_t)((T + kWinRows - 1) / kWinRows);
    L.list = o;
    o += align_up(groups * kWinKeys * sizeof(int));
    L.gcount = o;
    o += align_up(groups * sizeof(int));
    L.need = o;
    o += align_up(groups * sizeof(int));
    L.flags = o;
    o += kAlign;
    L.psf_all = o;
    o += align_up((size_t)npix * sizeof(float));
    L.ring = o;
    o += align_up((size_t)kWinRing * kWinRows * (size_t)npix * sizeof(float));
  }
  L.total = o;
  return L;
}

size_t window_ws_bytes(long long T, long long npix) { return window_layout(T, npix).total; }

bool overlap_bad(const void* a, const void* b, size_t bytes) {
  if (a == b) return false;
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

// [a, a + abytes) and [b, b + bbytes) share a byte.
bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bbytes && y < x + abytes;
}

// Input [T][N][N] and output [T][P][P] of a GRAPHIC_KEEP_PADDED call: no
// shared byte, except out == in when P == N.
bool padded_overlap_bad(const void* in, const void* out, long long T, int N, int P) {
  if (P == N) return overlap_bad(in, out, (size_t)T * N * N * sizeof(float));
  return ranges_overlap(in, (size_t)T * N * N * sizeof(float), out, (size_t)T * P * P * sizeof(float));
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------
struct RotLayout {
  size_t params = 0;      // flip (int), -tan(theta/2), sin(theta) per frame
  size_t chunk_frames = 0;
  size_t scratch = 0;     // chunk_frames * N * P floats
  size_t total = 0;
};

RotLayout rot_layout(long long T, int N, int P, size_t chunk_bytes, size_t avail /*0 = choose*/) {
  RotLayout L;
  // flip flags, -tan(theta/2), sin(theta), half-turned frame list, its count
  L.params = align_up((size_t)T * sizeof(int)) + 2 * align_up((size_t)T * sizeof(double)) +
             align_up((size_t)T * sizeof(int)) + kAlign;
  const size_t per_frame = (size_t)N * P * sizeof(float);
  size_t cf = avail ? (avail > L.params ? (avail - L.params) / per_frame : 0)
                    : std::max<size_t>(1, chunk_bytes / per_frame);
  if (cf > (size_t)T) cf = (size_t)T;
  L.chunk_frames = cf;
  L.scratch = align_up(cf * per_frame);
  L.total = L.params + L.scratch;
  return L;
}

size_t shift_ws(long long, int, int) { return 0; }

// ---------------------------------------------------------------------------
// Launch helpers (with optional event timing)
// ---------------------------------------------------------------------------
struct Timer {
  graphic_ctx ctx;
  hipStream_t st;
  const char* fam;
  hipEvent_t a = nullptr, b = nullptr;
  Timer(graphic_ctx c, hipStream_t s, const char* f) : ctx(c), st(s), fam(f) {
    if (ctx->timing) {
      hipEventCreate(&a);
      hipEventCreate(&b);
      hipEventRecord(a, st);
    }
  }
  void done() {
    if (ctx->timing) {
      hipEventRecord(b, st);
      ctx->pending.push_back({fam, a, b});
    }
  }
};

graphic_status hip_ok(hipError_t e) { return e == hipSuccess ? GRAPHIC_OK : GRAPHIC_ERR_HIP; }

int col_variant(graphic_ctx ctx, int P, int mirror) {
  const int v = ctx->col_var[ilog2(P / 2) & 15][mirror ? 1 : 0];
  return v < 0 ? 0 : v;
}

// Tuning class of a frame count: log2 of the median's values per thread
// (0 .. 6 for the register form; 7 for the streaming select, which has no variants).
int median_class(long long T) {
  return T > kMaxT_RegisterMedian ? 7 : ilog2((int)((T + 63) / 64));
}

int median_variant(graphic_ctx ctx, long long T) {
  const int v = ctx->med_var[median_class(T)];
  return v < 0 ? 0 : v;
}

// Tile-major median: 8-pixel tiles (two blocks per compute unit) unless tuned.
int tm_median_variant(graphic_ctx ctx, long long T) {
  const int v = ctx->tmm_var[median_class(T)];
  return v >= 0 ? v : 1;
}

graphic_status run_pass(graphic_ctx ctx, const LinePass& p, int kind, const char* family, hipStream_t st) {
  Timer t(ctx, st, family);
  hipError_t e = launch_line_pass(p, kind, kind == kColPass ? col_variant(ctx, p.P, p.mirror) : 0, st);
  t.done();
  return hip_ok(e);
}

LinePass base_pass(graphic_ctx ctx, int P) {
  LinePass p;
  std::memset(&p, 0, sizeof(p));
  p.P = P;
  p.tw = ctx->tw[ilog2(P / 2)];
  return p;
}

// ---------------------------------------------------------------------------
// Batched passes over one size class (every cube has the same N and P).  A
// single-cube call is a batch of one.
// ---------------------------------------------------------------------------
struct ShiftItem {
  const float* in;
  float* out;
  long long T;
  const double* dx;
  const double* dy;
};

struct RotItem {
  const float* src;
  float* dst;
  long long T;
  const double* theta;
};

// Shift (Sect. 3.3.1): column pass (content moves by dy along y) then row pass
// (dx along x); up to kMaxCubesPerLaunch cubes per launch.
// With tm the outputs are tile-major stacks (the inputs stay frame-major).
graphic_status do_shift_batch(graphic_ctx ctx, int N, int P, const ShiftItem* it, int n, hipStream_t st,
                              bool tm = false) {
  const int o = (P - N) / 2;
  for (int i0 = 0; i0 < n; i0 += kMaxCubesPerLaunch) {
    const int g = std::min(kMaxCubesPerLaunch, n - i0);
    LinePass c = base_pass(ctx, P);
    c.src_fs = c.dst_fs = (long long)N * N;
    c.src_ls = c.dst_ls = 1;
    c.src_ps = c.dst_ps = N;
    c.line_lo = o;
    c.n_lines = N;
    c.in_off = o;
    c.in_len = N;
    c.out_off = o;
    c.out_len = N;
    c.dst_line_lo = o;
    c.mirror = 0;
    c.n_jobs = N / 2;
    c.n_cubes = g;
    long long F = 0;
    for (int k = 0; k < g; ++k) {
      c.cubes[k] = CubeRef{it[i0 + k].in, it[i0 + k].out, it[i0 + k].dy, F, it[i0 + k].T};
      F += it[i0 + k].T;
    }
    c.n_frames = F;
    // the column pass keeps frame-by-frame block order: its frame-major reads
    // of 16-column strips then share 128-byte lines between neighbouring
    // blocks, which matters more than the adjacency of its tile-major stores
    c.dst_tm = tm ? 1 : 0;
    graphic_status s = run_pass(ctx, c, kColPass, "shift_y", st);
    if (s != GRAPHIC_OK) return s;
    LinePass r = c;
    r.src_ls = r.dst_ls = N;
    r.src_ps = r.dst_ps = 1;
    r.src_tm = r.dst_tm = tm ? 1 : 0;
    r.frame_group = tm ? ctx->frame_group : 0;
    for (int k = 0; k < g; ++k)
      r.cubes[k] = CubeRef{it[i0 + k].out, it[i0 + k].out, it[i0 + k].dx, c.cubes[k].frame0, it[i0 + k].T};
    if ((s = run_pass(ctx, r, kRowPass, "shift_x", st)) != GRAPHIC_OK) return s;
  }
  return GRAPHIC_OK;
}

// Three-shear rotation (Sect. 3.4) of every frame of the class, chunked over
// the concatenated frames; a chunk may span cubes (at most
// kMaxCubesPerLaunch of them).  dst may alias src.  With tm, src and dst are
// tile-major stacks.
graphic_status do_rotate_batch(graphic_ctx ctx, int N, int P, const RotItem* it, int n, double sign, void* ws,
                               size_t ws_bytes, hipStream_t st, bool tm = false) {
  long long F = 0;
  // cube start frames (a small batch keeps them on the stack, so that a
  // single-cube rotation makes no allocation at all)
  long long start_small[kMaxCubesPerLaunch + 1];
  std::vector<long long> start_big;
  if (n > kMaxCubesPerLaunch) start_big.assign(n + 1, 0);
  long long* start = n > kMaxCubesPerLaunch ? start_big.data() : start_small;
  for (int i = 0; i < n; ++i) {
    start[i] = F;
    F += it[i].T;
  }
  start[n] = F;
  RotLayout L = rot_layout(F, N, P, ctx->chunk_bytes, ws_bytes);
  if (L.chunk_frames < 1) return GRAPHIC_ERR_WORKSPACE;
  char* w = static_cast<char*>(ws);
  int* flip = reinterpret_cast<int*>(w);
  double* ntan = reinterpret_cast<double*>(w + align_up((size_t)F * sizeof(int)));
  double* sn = reinterpret_cast<double*>(w + align_up((size_t)F * sizeof(int)) + align_up((size_t)F * sizeof(double)));
  int* flip_list = reinterpret_cast<int*>(w + align_up((size_t)F * sizeof(int)) + 2 * align_up((size_t)F * sizeof(double)));
  int* flip_count = reinterpret_cast<int*>(reinterpret_cast<char*>(flip_list) + align_up((size_t)F * sizeof(int)));
  float* scratch = reinterpret_cast<float*>(w + L.params);
  for (int i = 0; i < n; ++i) {
    Timer t(ctx, st, "aux");
    hipError_t e = launch_rotation_params(it[i].theta, sign, it[i].T, flip + start[i], ntan + start[i],
                                          sn + start[i], st);
    t.done();
    if (e != hipSuccess) return GRAPHIC_ERR_HIP;
  }
  const int o = (P - N) / 2;
  int c0 = 0;   // first cube of the current chunk
  for (long long f0 = 0; f0 < F;) {
    while (start[c0 + 1] <= f0) ++c0;
    const int c1 = std::min(n, c0 + kMaxCubesPerLaunch);   // cubes [c0, c1) may take part
    const long long nf = std::min<long long>((long long)L.chunk_frames, start[c1] - f0);
    {
      Timer t(ctx, st, "aux");
      hipError_t e = launch_flip_list(flip, f0, nf, flip_list, flip_count, st);
      t.done();
      if (e != hipSuccess) return GRAPHIC_ERR_HIP;
    }
    int ncub = 0;
    while (c0 + ncub < c1 && start[c0 + ncub] < f0 + nf) ++ncub;
    // x-shear 1: window rows of every cube frame -> all P columns of the scratch frame
    LinePass a = base_pass(ctx, P);
    a.dst = scratch;
    a.src_fs = (long long)N * N;
    a.dst_fs = (long long)N * P;
    a.src_ls = N;
    a.src_ps = 1;
    a.dst_ls = P;
    a.dst_ps = 1;
    a.line_lo = o;
    a.n_lines = N;
    a.in_off = o;
    a.in_len = N;
    a.out_off = 0;
    a.out_len = P;
    a.dst_line_lo = o;
    a.mirror = 1;
    a.n_jobs = N / 2 + 1;
    a.n_frames = nf;
    a.sh1 = ntan + f0;
    a.flip = flip + f0;
    a.flip_list = flip_list;
    a.flip_count = flip_count;
    a.flip_src_reverse = 1;
    a.flip_lines = 1;
    a.flip_in_off = 1;
    a.n_cubes = ncub;
    for (int k = 0; k < ncub; ++k)
      a.cubes[k] = CubeRef{it[c0 + k].src, nullptr, nullptr, start[c0 + k] - f0, it[c0 + k].T};
    a.src_tm = tm ? 1 : 0;
    a.frame_group = tm ? ctx->frame_group_shear : 0;
    graphic_status s = run_pass(ctx, a, kRowPass, "shear_x1", st);
    if (s != GRAPHIC_OK) return s;
    // y-shear: every scratch column, window rows in and out (in place)
    LinePass b = base_pass(ctx, P);
    b.src = scratch;
    b.dst = scratch;
    b.src_fs = b.dst_fs = (long long)N * P;
    b.src_ls = b.dst_ls = 1;
    b.src_ps = b.dst_ps = P;
    b.line_lo = 0;
    b.n_lines = P;
    b.in_off = o;
    b.in_len = N;
    b.out_off = o;
    b.out_len = N;
    b.dst_line_lo = 0;
    b.mirror = 1;
    b.n_jobs = P / 2 + 1;
    b.n_frames = nf;
    b.sh1 = sn + f0;
    b.flip = flip + f0;
    b.flip_list = flip_list;
    b.flip_count = flip_count;
    b.flip_in_off = 1;
    if ((s = run_pass(ctx, b, kColPass, "shear_y", st)) != GRAPHIC_OK) return s;
    // x-shear 2: window rows, all P columns in, window columns out to every cube frame
    LinePass c = base_pass(ctx, P);
    c.src = scratch;
    c.src_fs = (long long)N * P;
    c.dst_fs = (long long)N * N;
    c.src_ls = P;
    c.src_ps = 1;
    c.dst_ls = N;
    c.dst_ps = 1;
    c.line_lo = o;
    c.n_lines = N;
    c.in_off = 0;
    c.in_len = P;
    c.out_off = o;
    c.out_len = N;
    c.dst_line_lo = o;
    c.mirror = 1;
    c.n_jobs = N / 2 + 1;
    c.n_frames = nf;
    c.sh1 = ntan + f0;
    c.n_cubes = ncub;
    for (int k = 0; k < ncub; ++k)
      c.cubes[k] = CubeRef{nullptr, it[c0 + k].dst, nullptr, start[c0 + k] - f0, it[c0 + k].T};
    c.dst_tm = tm ? 1 : 0;
    c.frame_group = tm ? ctx->frame_group_shear : 0;
    if ((s = run_pass(ctx, c, kRowPass, "shear_x2", st)) != GRAPHIC_OK) return s;
    f0 += nf;
  }
  return GRAPHIC_OK;
}

// Whole zero-padded output (GRAPHIC_KEEP_PADDED) of the shift: the column
// pass takes the N window columns to all P rows of the P x P output, then the
// row pass takes every output row's N window columns to all P columns, in
// place (the columns outside the window are never read).  Each job loads its
// two lines before it stores them, and jobs own disjoint lines.
graphic_status do_shift_padded(graphic_ctx ctx, int N, int P, long long T, const float* in, float* out,
                               const double* dx, const double* dy, hipStream_t st) {
  const int o = (P - N) / 2;
  LinePass c = base_pass(ctx, P);
  c.src = in;
  c.dst = out;
  c.src_fs = (long long)N * N;
  c.dst_fs = (long long)P * P;
  c.src_ls = c.dst_ls = 1;
  c.src_ps = N;
  c.dst_ps = P;
  c.line_lo = o;
  c.n_lines = N;
  c.in_off = o;
  c.in_len = N;
  c.out_off = 0;
  c.out_len = P;
  c.dst_line_lo = 0;
  c.n_jobs = N / 2;
  c.n_frames = T;
  c.sh0 = dy;
  graphic_status s = run_pass(ctx, c, kColPass, "shift_y", st);
  if (s != GRAPHIC_OK) return s;
  // A pass reads its support [in_off, in_off + in_len) from positions
  // 0 .. in_len - 1 of the source line: the row pass's source lines start at
  // the window's first column.
  LinePass r = base_pass(ctx, P);
  r.src = out + o;
  r.dst = out;
  r.src_fs = r.dst_fs = (long long)P * P;
  r.src_ls = r.dst_ls = P;
  r.src_ps = r.dst_ps = 1;
  r.line_lo = 0;
  r.n_lines = P;
  r.in_off = o;
  r.in_len = N;
  r.out_off = 0;
  r.out_len = P;
  r.dst_line_lo = 0;
  r.n_jobs = P / 2;
  r.n_frames = T;
  r.sh0 = dx;
  return run_pass(ctx, r, kRowPass, "shift_x", st);
}

// Whole zero-padded output (GRAPHIC_KEEP_PADDED) of the rotation: the first
// x-shear as in do_rotate_batch (window rows to all P columns of the
// scratch), the y-shear from the scratch's window rows to all P rows of the
// P x P output, and the second x-shear over every output row, whole line to
// whole line, in place.
graphic_status do_rotate_padded(graphic_ctx ctx, int N, int P, long long T, const float* in, float* out,
                                const double* theta, void* ws, size_t ws_bytes, hipStream_t st) {
  RotLayout L = rot_layout(T, N, P, ctx->chunk_bytes, ws_bytes);
  if (L.chunk_frames < 1) return GRAPHIC_ERR_WORKSPACE;
  char* w = static_cast<char*>(ws);
  int* flip = reinterpret_cast<int*>(w);
  double* ntan = reinterpret_cast<double*>(w + align_up((size_t)T * sizeof(int)));
  double* sn = reinterpret_cast<double*>(w + align_up((size_t)T * sizeof(int)) + align_up((size_t)T * sizeof(double)));
  int* flip_list = reinterpret_cast<int*>(w + align_up((size_t)T * sizeof(int)) + 2 * align_up((size_t)T * sizeof(double)));
  int* flip_count = reinterpret_cast<int*>(reinterpret_cast<char*>(flip_list) + align_up((size_t)T * sizeof(int)));
  float* scratch = reinterpret_cast<float*>(w + L.params);
  {
    Timer t(ctx, st, "aux");
    hipError_t e = launch_rotation_params(theta, 1.0, T, flip, ntan, sn, st);
    t.done();
    if (e != hipSuccess) return GRAPHIC_ERR_HIP;
  }
  const int o = (P - N) / 2;
  for (long long f0 = 0; f0 < T;) {
    const long long nf = std::min<long long>((long long)L.chunk_frames, T - f0);
    {
      Timer t(ctx, st, "aux");
      hipError_t e = launch_flip_list(flip, f0, nf, flip_list, flip_count, st);
      t.done();
      if (e != hipSuccess) return GRAPHIC_ERR_HIP;
    }
    LinePass a = base_pass(ctx, P);
    a.src = in + (size_t)f0 * N * N;
    a.dst = scratch;
    a.src_fs = (long long)N * N;
    a.dst_fs = (long long)N * P;
    a.src_ls = N;
    a.src_ps = 1;
    a.dst_ls = P;
    a.dst_ps = 1;
    a.line_lo = o;
    a.n_lines = N;
    a.in_off = o;
    a.in_len = N;
    a.out_off = 0;
    a.out_len = P;
    a.dst_line_lo = o;
    a.mirror = 1;
    a.n_jobs = N / 2 + 1;
    a.n_frames = nf;
    a.sh1 = ntan + f0;
    a.flip = flip + f0;
    a.flip_list = flip_list;
    a.flip_count = flip_count;
    a.flip_src_reverse = 1;
    a.flip_lines = 1;
    a.flip_in_off = 1;
    graphic_status s = run_pass(ctx, a, kRowPass, "shear_x1", st);
    if (s != GRAPHIC_OK) return s;
    float* dst = out + (size_t)f0 * P * P;
    LinePass b = base_pass(ctx, P);
    b.src = scratch;
    b.dst = dst;
    b.src_fs = (long long)N * P;
    b.dst_fs = (long long)P * P;
    b.src_ls = b.dst_ls = 1;
    b.src_ps = b.dst_ps = P;
    b.line_lo = 0;
    b.n_lines = P;
    b.in_off = o;
    b.in_len = N;
    b.out_off = 0;
    b.out_len = P;
    b.dst_line_lo = 0;
    b.mirror = 1;
    b.n_jobs = P / 2 + 1;
    b.n_frames = nf;
    b.sh1 = sn + f0;
    b.flip = flip + f0;
    b.flip_list = flip_list;
    b.flip_count = flip_count;
    b.flip_in_off = 1;
    if ((s = run_pass(ctx, b, kColPass, "shear_y", st)) != GRAPHIC_OK) return s;
    LinePass c = base_pass(ctx, P);
    c.src = dst;
    c.dst = dst;
    c.src_fs = c.dst_fs = (long long)P * P;
    c.src_ls = c.dst_ls = P;
    c.src_ps = c.dst_ps = 1;
    c.line_lo = 0;
    c.n_lines = P;
    c.in_off = 0;
    c.in_len = P;
    c.out_off = 0;
    c.out_len = P;
    c.dst_line_lo = 0;
    c.mirror = 1;
    c.n_jobs = P / 2 + 1;
    c.n_frames = nf;
    c.sh1 = ntan + f0;
    if ((s = run_pass(ctx, c, kRowPass, "shear_x2", st)) != GRAPHIC_OK) return s;
    f0 += nf;
  }
  return GRAPHIC_OK;
}

// GRAPHIC_CHECK_FINITE: scan the float32 and float64 inputs on the stream,
// wait, and report whether any value is NaN or +-inf.
struct ScanF32 {
  const float* p;
  size_t n;
};
struct ScanF64 {
  const double* p;
  size_t n;
};

graphic_status check_finite(graphic_ctx ctx, hipStream_t st, std::initializer_list<ScanF32> f32,
                            std::initializer_list<ScanF64> f64) {
  if (launch_clear_flag(ctx->scan_flag, st) != hipSuccess) return GRAPHIC_ERR_HIP;
  for (const ScanF32& a : f32)
    if (a.p && launch_nonfinite_f32(a.p, a.n, ctx->scan_flag, st) != hipSuccess) return GRAPHIC_ERR_HIP;
  for (const ScanF64& a : f64)
    if (a.p && launch_nonfinite_f64(a.p, a.n, ctx->scan_flag, st) != hipSuccess) return GRAPHIC_ERR_HIP;
  int h = 0;
  if (hipMemcpyAsync(&h, ctx->scan_flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GRAPHIC_ERR_HIP;
  return h ? GRAPHIC_ERR_NONFINITE : GRAPHIC_OK;
}

graphic_status do_median(graphic_ctx ctx, long long T, int N, const float* stack, float* out, float* resid,
                         hipStream_t st, bool tm = false) {
  Timer t(ctx, st, "median");
  hipError_t e = tm ? launch_median_tile_major(stack, T, (long long)N * N, out, resid, tm_median_variant(ctx, T), st)
                    : launch_median(stack, T, (long long)N * N, out, resid, median_variant(ctx, T), st);
  t.done();
  return hip_ok(e);
}

graphic_status do_sums(graphic_ctx ctx, long long T, int N, const float* frames, double* flux, int slot,
                       hipStream_t st) {
  Timer t(ctx, st, "aux");
  hipError_t e = launch_frame_sums(frames, T, N, flux, slot, st);
  t.done();
  return hip_ok(e);
}

bool ws_ok(const void* ws, size_t have, size_t need) {
  if (need == 0) return true;
  if (!ws || have < need) return false;
  return (reinterpret_cast<uintptr_t>(ws) % kAlign) == 0;
}

// ---------------------------------------------------------------------------
// ADI reduction of a batch of cubes (Sect. 3.3 and 3.4)
// ---------------------------------------------------------------------------
struct BatchPlan {
  std::vector<int> P;                   // working size of every cube
  std::vector<std::vector<int>> classes;  // cube indices of every (N, P) class, in input order
  std::vector<size_t> stack_off, psf_off; // workspace offsets (SIZE_MAX: caller-provided)
  size_t fixed = 0;                     // bytes of stacks and PSFs
  size_t rot_min = 0, rot_default = 0;  // rotation workspace: minimum and default
};

graphic_status plan_batch(const graphic_cube_desc* d, int n, uint32_t flags, size_t chunk_bytes, BatchPlan* plan) {
  if (!d || n < 1) return GRAPHIC_ERR_ARG;
  if ((flags & ~GRAPHIC_BATCH_INPLACE) != 0) return GRAPHIC_ERR_ARG;
  plan->P.assign(n, 0);
  plan->stack_off.assign(n, SIZE_MAX);
  plan->psf_off.assign(n, SIZE_MAX);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    graphic_geom g{d[i].n_frames, d[i].n, d[i].pad, 0u};
    graphic_status s = check_geom(&g, &plan->P[i]);
    if (s != GRAPHIC_OK) return s;
    if (d[i].n_frames > kMaxT_Median) return GRAPHIC_ERR_UNSUPPORTED;
    if (!d[i].cube || !d[i].dx || !d[i].dy || !d[i].parang_deg || !d[i].final_img) return GRAPHIC_ERR_ARG;
    const size_t cube_b = (size_t)d[i].n_frames * d[i].n * d[i].n * sizeof(float);
    if (!d[i].residuals && !(flags & GRAPHIC_BATCH_INPLACE)) {
      plan->stack_off[i] = off;
      off += align_up(cube_b);
    }
    if (!d[i].psf) {
      plan->psf_off[i] = off;
      off += align_up((size_t)d[i].n * d[i].n * sizeof(float));
    }
    bool found = false;
    for (auto& c : plan->classes)
      if (d[c[0]].n == d[i].n && plan->P[c[0]] == plan->P[i]) {
        c.push_back(i);
        found = true;
        break;
      }
    if (!found) plan->classes.push_back({i});
  }
  plan->fixed = off;
  for (auto& c : plan->classes) {
    long long F = 0;
    for (int i : c) F += d[i].n_frames;
    const int N = d[c[0]].n, P = plan->P[c[0]];
    const RotLayout L = rot_layout(F, N, P, chunk_bytes, 0);
    plan->rot_min = std::max(plan->rot_min, L.params + align_up((size_t)N * P * sizeof(float)));
    plan->rot_default = std::max(plan->rot_default, L.total);
  }
  return GRAPHIC_OK;
}

// With check_fin, every cube and parameter array is scanned for non-finite
// values after the argument checks and before the reduction's launches.
graphic_status adi_batch(graphic_ctx ctx, const graphic_cube_desc* d, int n, uint32_t flags, void* ws,
                         size_t ws_bytes, hipStream_t st, bool check_fin = false) {
  BatchPlan plan;
  graphic_status s = plan_batch(d, n, flags, ctx->chunk_bytes, &plan);
  if (s != GRAPHIC_OK) return s;
  // argument checks: outputs must not overlap the inputs of any cube
  for (int i = 0; i < n; ++i) {
    const size_t cube_b = (size_t)d[i].n_frames * d[i].n * d[i].n * sizeof(float);
    const size_t img_b = (size_t)d[i].n * d[i].n * sizeof(float);
    const char* cb = static_cast<const char*>(static_cast<const void*>(d[i].cube));
    auto inside = [&](const void* p, size_t b) {
      const char* q = static_cast<const char*>(p);
      return q < cb + cube_b && cb < q + b;
    };
    if (inside(d[i].final_img, img_b)) return GRAPHIC_ERR_ARG;
    if (d[i].psf && (inside(d[i].psf, img_b) || d[i].psf == d[i].final_img)) return GRAPHIC_ERR_ARG;
    if (d[i].residuals && inside(d[i].residuals, cube_b)) return GRAPHIC_ERR_ARG;
  }
  if (!ws_ok(ws, ws_bytes, plan.fixed + plan.rot_min)) return GRAPHIC_ERR_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  for (int i = 0; i < n && check_fin; ++i) {
    const size_t T = (size_t)d[i].n_frames;
    s = check_finite(ctx, st, {{d[i].cube, T * d[i].n * d[i].n}},
                     {{d[i].dx, T}, {d[i].dy, T}, {d[i].parang_deg, T}});
    if (s != GRAPHIC_OK) return s;
  }
  char* w = static_cast<char*>(ws);
  std::vector<float*> stack(n), psf(n);
  for (int i = 0; i < n; ++i) {
    stack[i] = d[i].residuals ? d[i].residuals
               : (flags & GRAPHIC_BATCH_INPLACE) ? const_cast<float*>(d[i].cube)
                                                 : reinterpret_cast<float*>(w + plan.stack_off[i]);
    psf[i] = d[i].psf ? d[i].psf : reinterpret_cast<float*>(w + plan.psf_off[i]);
  }
  void* rot_ws = w + plan.fixed;
  const size_t rot_bytes = ws_bytes - plan.fixed;
  for (auto& c : plan.classes) {
    const int N = d[c[0]].n, P = plan.P[c[0]];
    std::vector<ShiftItem> sh;
    std::vector<RotItem> rot;
    // Stacks that only the workspace holds are kept tile-major when the
    // class has the geometry where that pays (P = 2N, N = 1024): the medians
    // then stream each 16-pixel run of the stack contiguously.  (At N = 2048
    // the row passes, which already spill, lose as much as the medians gain.)
    bool tm = ctx->tile_major && P == 2 * N && N == 1024;
    for (int i : c) {
      sh.push_back(ShiftItem{d[i].cube, stack[i], d[i].n_frames, d[i].dx, d[i].dy});
      rot.push_back(RotItem{stack[i], stack[i], d[i].n_frames, d[i].parang_deg});
      tm = tm && plan.stack_off[i] != SIZE_MAX && (long long)N * 4 * d[i].n_frames <= 0x7fffffffLL &&
           d[i].n_frames <= kMaxT_RegisterMedian;
    }
    // S_i = shift(cube_i): every cube of the class in the same launches
    if ((s = do_shift_batch(ctx, N, P, sh.data(), (int)sh.size(), st, tm)) != GRAPHIC_OK) return s;
    // PSF = median_i S_i; the median also rewrites the stack as S_i - PSF
    // (cheaper than subtracting the PSF in the first shear's loads: that
    // doubles the shear's reads, while the rewrite costs one streaming write)
    for (int i : c)
      if ((s = do_median(ctx, d[i].n_frames, N, stack[i], psf[i], stack[i], st, tm)) != GRAPHIC_OK) return s;
    // D_i = rotate(S_i - PSF, -parang_i), in place
    if ((s = do_rotate_batch(ctx, N, P, rot.data(), (int)rot.size(), -1.0, rot_ws, rot_bytes, st, tm)) !=
        GRAPHIC_OK)
      return s;
    // final = median_i D_i
    for (int i : c)
      if ((s = do_median(ctx, d[i].n_frames, N, stack[i], d[i].final_img, nullptr, st, tm)) != GRAPHIC_OK) return s;
  }
  return GRAPHIC_OK;
}

}  // namespace

// ===========================================================================
// Static scratch of graphic_rotate_noalloc
// ===========================================================================
// One array per GPU that the library runs on, held until the process ends.
// In host code its name is only a stand-in for the device variable: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device (with that device current) when a context is created on
// it, and only that address is handed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Resolve the calling device's copy of `scratch` (device `dev` is current).
hipError_t resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = ptr;
  return hipSuccess;
}

void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

}  // namespace

// ===========================================================================
// Public entry points
// ===========================================================================
extern "C" {

const char* graphic_status_string(graphic_status s) {
  // C callers may pass any int: read the bits as int, since a value outside
  // the enumerators is not a valid value of the C++ enum type
  int v;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case GRAPHIC_OK: return "GRAPHIC_OK";
    case GRAPHIC_ERR_ARG: return "GRAPHIC_ERR_ARG: invalid argument";
    case GRAPHIC_ERR_UNSUPPORTED: return "GRAPHIC_ERR_UNSUPPORTED: unsupported geometry";
    case GRAPHIC_ERR_WORKSPACE: return "GRAPHIC_ERR_WORKSPACE: workspace missing, too small or misaligned";
    case GRAPHIC_ERR_HIP: return "GRAPHIC_ERR_HIP: HIP runtime error";
    case GRAPHIC_ERR_NOMEM: return "GRAPHIC_ERR_NOMEM: out of device memory";
    case GRAPHIC_ERR_NONFINITE: return "GRAPHIC_ERR_NONFINITE: an input holds NaN or inf";
  }
  return "GRAPHIC: unknown status";
}

const char* graphic_version(void) { return "graphic-mi355x 0.1 (gfx950)"; }

int32_t graphic_resolved_pad(const graphic_geom* geom) {
  int P = 0;
  return check_geom(geom, &P, kAllFlags) == GRAPHIC_OK ? P : -1;
}

graphic_status graphic_create(graphic_ctx* out, int hip_device) {
  if (!out) return GRAPHIC_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return GRAPHIC_ERR_HIP;
  if (hipSetDevice(hip_device) != hipSuccess) return GRAPHIC_ERR_HIP;
  graphic_ctx c = new graphic_ctx_s();
  c->device = hip_device;
  if (const char* env = std::getenv("GRAPHIC_ROTATE_CHUNK_MB")) {
    long v = std::atol(env);
    if (v > 0) c->chunk_bytes = (size_t)v << 20;
  }
  if (const char* env = std::getenv("GRAPHIC_TILE_MAJOR")) c->tile_major = std::atoi(env) != 0;
  if (const char* env = std::getenv("GRAPHIC_FRAME_GROUP")) {   // every row pass
    const int v = std::atoi(env);
    if (v >= 1 && v <= 4096) c->frame_group = c->frame_group_shear = v;
  }
  if (const char* env = std::getenv("GRAPHIC_FRAME_GROUP_SHEAR")) {   // the two x-shears
    const int v = std::atoi(env);
    if (v >= 1 && v <= 4096) c->frame_group_shear = v;
  }
  graphic_status s = build_tables(c);
  if (s != GRAPHIC_OK) {
    graphic_destroy(c);
    return s;
  }
  // the no-allocation entry point's scratch on this device (its failure only
  // disables that entry point, which then returns GRAPHIC_ERR_HIP)
  (void)resolve_scratch(hip_device);
  *out = c;
  return GRAPHIC_OK;
}

void graphic_destroy(graphic_ctx ctx) {
  if (!ctx) return;
  for (auto& p : ctx->pending) {
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  if (ctx->tables) hipFree(ctx->tables);
  delete ctx;
}

graphic_status graphic_workspace_size(graphic_ctx ctx, int op, const graphic_geom* geom, size_t* bytes) {
  if (!bytes) return GRAPHIC_ERR_ARG;
  int P = 0;
  graphic_status s = check_geom(geom, &P, kAllFlags);
  if (s != GRAPHIC_OK) return s;
  const size_t chunk = ctx ? ctx->chunk_bytes : kDefaultChunkBytes;
  const long long T = geom->n_frames;
  const int N = geom->n;
  switch (op) {
    case GRAPHIC_OP_SHIFT: *bytes = shift_ws(T, N, P); return GRAPHIC_OK;
    case GRAPHIC_OP_ROTATE: *bytes = rot_layout(T, N, P, chunk, 0).total; return GRAPHIC_OK;
    case GRAPHIC_OP_ADI: {
      graphic_cube_desc d{};
      d.cube = reinterpret_cast<const float*>(kAlign);   // placeholders: only the geometry matters here
      d.n_frames = T;
      d.n = N;
      d.pad = geom->pad;
      d.dx = d.dy = d.parang_deg = reinterpret_cast<const double*>(kAlign);
      d.final_img = reinterpret_cast<float*>(kAlign);
      BatchPlan plan;
      if ((s = plan_batch(&d, 1, 0u, chunk, &plan)) != GRAPHIC_OK) return s;
      *bytes = plan.fixed + plan.rot_default;
      return GRAPHIC_OK;
    }
    case GRAPHIC_OP_MEDIAN: *bytes = 0; return T > kMaxT_Median ? GRAPHIC_ERR_UNSUPPORTED : GRAPHIC_OK;
    case GRAPHIC_OP_MEDIAN_WINDOW:
      if (T > kMaxT_Window) return GRAPHIC_ERR_UNSUPPORTED;
      *bytes = window_ws_bytes(T, (long long)N * N);
      return GRAPHIC_OK;
    case GRAPHIC_OP_BADPIX_MAP: *bytes = frame_stats_ws_bytes(); return GRAPHIC_OK;
    case GRAPHIC_OP_BADPIX_FIX:
      *bytes = align_up((size_t)T * N * N * sizeof(float)) + kAlign;
      return T > 65535 ? GRAPHIC_ERR_UNSUPPORTED : GRAPHIC_OK;
    case GRAPHIC_OP_ADI_WINDOW:
      if (T > kMaxT_Window) return GRAPHIC_ERR_UNSUPPORTED;
      *bytes = align_up((size_t)T * N * N * sizeof(float)) + window_ws_bytes(T, (long long)N * N) +
               rot_layout(T, N, P, chunk, 0).total;
      return GRAPHIC_OK;
    default: return GRAPHIC_ERR_ARG;
  }
}

graphic_status graphic_shift(graphic_ctx ctx, const graphic_geom* geom, const float* in, float* out,
                             const double* dx, const double* dy, double* flux, void* ws, size_t ws_bytes,
                             graphic_stream stream) {
  int P = 0;
  if (!ctx) return GRAPHIC_ERR_ARG;
  graphic_status s = check_geom(geom, &P, kAllFlags);
  if (s != GRAPHIC_OK) return s;
  if (!in || !out || !dx || !dy) return GRAPHIC_ERR_ARG;
  const long long T = geom->n_frames;
  const int N = geom->n;
  const bool padded = (geom->flags & GRAPHIC_KEEP_PADDED) != 0;
  const int No = padded ? P : N;             // output frame side
  const size_t bytes = (size_t)T * N * N * sizeof(float);
  if (padded ? padded_overlap_bad(in, out, T, N, P) : overlap_bad(in, out, bytes)) return GRAPHIC_ERR_ARG;
  if (!ws_ok(ws, ws_bytes, shift_ws(T, N, P))) return GRAPHIC_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  if ((geom->flags & GRAPHIC_CHECK_FINITE) &&
      (s = check_finite(ctx, st, {{in, (size_t)T * N * N}}, {{dx, (size_t)T}, {dy, (size_t)T}})) != GRAPHIC_OK)
    return s;
  if (flux && (s = do_sums(ctx, T, N, in, flux, 0, st)) != GRAPHIC_OK) return s;
  if (padded) {
    if ((s = do_shift_padded(ctx, N, P, T, in, out, dx, dy, st)) != GRAPHIC_OK) return s;
  } else {
    const ShiftItem item{in, out, T, dx, dy};
    if ((s = do_shift_batch(ctx, N, P, &item, 1, st)) != GRAPHIC_OK) return s;
  }
  if (flux && (s = do_sums(ctx, T, No, out, flux, 1, st)) != GRAPHIC_OK) return s;
  return GRAPHIC_OK;
}

graphic_status graphic_rotate(graphic_ctx ctx, const graphic_geom* geom, const float* in, float* out,
                              const double* theta_deg, double* flux, void* ws, size_t ws_bytes,
                              graphic_stream stream) {
  int P = 0;
  if (!ctx) return GRAPHIC_ERR_ARG;
  graphic_status s = check_geom(geom, &P, kAllFlags);
  if (s != GRAPHIC_OK) return s;
  if (!in || !out || !theta_deg) return GRAPHIC_ERR_ARG;
  const long long T = geom->n_frames;
  const int N = geom->n;
  const bool padded = (geom->flags & GRAPHIC_KEEP_PADDED) != 0;
  const int No = padded ? P : N;
  const size_t bytes = (size_t)T * N * N * sizeof(float);
  // the padded path reads every input frame of a chunk before its last pass
  // writes the output, so it needs disjoint arrays (or P == N, out == in)
  if (padded ? padded_overlap_bad(in, out, T, N, P) : overlap_bad(in, out, bytes)) return GRAPHIC_ERR_ARG;
  RotLayout need = rot_layout(T, N, P, ctx->chunk_bytes, 0);
  const size_t minimum = need.params + align_up((size_t)N * P * sizeof(float));
  if (!ws_ok(ws, ws_bytes, minimum)) return GRAPHIC_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  if ((geom->flags & GRAPHIC_CHECK_FINITE) &&
      (s = check_finite(ctx, st, {{in, (size_t)T * N * N}}, {{theta_deg, (size_t)T}})) != GRAPHIC_OK)
    return s;
  if (flux && (s = do_sums(ctx, T, N, in, flux, 0, st)) != GRAPHIC_OK) return s;
  if (padded) {
    if ((s = do_rotate_padded(ctx, N, P, T, in, out, theta_deg, ws, ws_bytes, st)) != GRAPHIC_OK) return s;
  } else {
    const RotItem item{in, out, T, theta_deg};
    if ((s = do_rotate_batch(ctx, N, P, &item, 1, 1.0, ws, ws_bytes, st)) != GRAPHIC_OK) return s;
  }
  if (flux && (s = do_sums(ctx, T, No, out, flux, 1, st)) != GRAPHIC_OK) return s;
  return GRAPHIC_OK;
}

graphic_status graphic_rotate_noalloc(graphic_ctx ctx, const graphic_geom* geom, const float* in, float* out,
                                      const double* theta_deg, double* flux, graphic_stream stream) {
  int P = 0;
  if (!ctx) return GRAPHIC_ERR_ARG;
  graphic_status s = check_geom(geom, &P, GRAPHIC_KEEP_PADDED);
  if (s != GRAPHIC_OK) return s;
  const long long T = geom->n_frames;
  const int N = geom->n;
  // the static scratch must hold the per-frame parameters and one working frame
  const RotLayout need = rot_layout(T, N, P, ctx->chunk_bytes, 0);
  if (need.params + align_up((size_t)N * P * sizeof(float)) > kNoAllocScratchBytes) return GRAPHIC_ERR_UNSUPPORTED;
  if (!in || !out || !theta_deg) return GRAPHIC_ERR_ARG;
  const bool padded = (geom->flags & GRAPHIC_KEEP_PADDED) != 0;
  if (padded ? padded_overlap_bad(in, out, T, N, P) : overlap_bad(in, out, (size_t)T * N * N * sizeof(float)))
    return GRAPHIC_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  void* ws = scratch_ptr(ctx->device);
  if (!ws) return GRAPHIC_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool timing = ctx->timing;        // event timing would create events: off for this call
  ctx->timing = false;
  if (flux) s = do_sums(ctx, T, N, in, flux, 0, st);
  if (s == GRAPHIC_OK) {
    if (padded) {
      s = do_rotate_padded(ctx, N, P, T, in, out, theta_deg, ws, kNoAllocScratchBytes, st);
    } else {
      const RotItem item{in, out, T, theta_deg};
      s = do_rotate_batch(ctx, N, P, &item, 1, 1.0, ws, kNoAllocScratchBytes, st);
    }
  }
  if (s == GRAPHIC_OK && flux) s = do_sums(ctx, T, padded ? P : N, out, flux, 1, st);
  ctx->timing = timing;
  return s;
}

graphic_status graphic_median(graphic_ctx ctx, const graphic_geom* geom, const float* stack, float* out,
                              void* ws, size_t ws_bytes, graphic_stream stream) {
  (void)ws;
  (void)ws_bytes;
  if (!ctx || !geom || !stack || !out) return GRAPHIC_ERR_ARG;
  if (geom->n_frames < 1 || geom->n < 1 || (geom->flags & ~GRAPHIC_CHECK_FINITE) != 0) return GRAPHIC_ERR_ARG;
  if (geom->n_frames > kMaxT_Median) return GRAPHIC_ERR_UNSUPPORTED;
  const long long T = geom->n_frames;
  const int N = geom->n;
  if (overlap_bad(stack, out, (size_t)N * N * sizeof(float)) ||
      (out >= stack && out < stack + (size_t)T * N * N))
    return GRAPHIC_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (geom->flags & GRAPHIC_CHECK_FINITE) {
    graphic_status s = check_finite(ctx, st, {{stack, (size_t)T * N * N}}, {});
    if (s != GRAPHIC_OK) return s;
  }
  return do_median(ctx, T, N, stack, out, nullptr, st);
}

graphic_status graphic_adi_reduce(graphic_ctx ctx, const graphic_geom* geom, const float* cube, const double* dx,
                                  const double* dy, const double* parang_deg, float* final_img, float* psf,
                                  float* residuals, void* ws, size_t ws_bytes, graphic_stream stream) {
  if (!ctx || !geom) return GRAPHIC_ERR_ARG;
  if ((geom->flags & ~GRAPHIC_CHECK_FINITE) != 0) return GRAPHIC_ERR_ARG;
  graphic_cube_desc d;
  d.cube = cube;
  d.n_frames = geom->n_frames;
  d.n = geom->n;
  d.pad = geom->pad;
  d.dx = dx;
  d.dy = dy;
  d.parang_deg = parang_deg;
  d.final_img = final_img;
  d.psf = psf;
  d.residuals = residuals;
  return adi_batch(ctx, &d, 1, 0u, ws, ws_bytes, static_cast<hipStream_t>(stream),
                   (geom->flags & GRAPHIC_CHECK_FINITE) != 0);
}

}  // extern "C"

namespace {

graphic_status window_args(graphic_ctx ctx, const graphic_geom* geom, const void* times, const void* parang,
                           double t_max, double alpha_min, int* P) {
  if (!ctx || !geom || !times || !parang) return GRAPHIC_ERR_ARG;
  graphic_status s = check_geom(geom, P, GRAPHIC_CHECK_FINITE);
  if (s != GRAPHIC_OK) return s;
  if (geom->n_frames > kMaxT_Window) return GRAPHIC_ERR_UNSUPPORTED;
  if (std::isnan(t_max) || std::isnan(alpha_min)) return GRAPHIC_ERR_ARG;
  return GRAPHIC_OK;
}

// Row groups of a long sequence (T > kWinKeys).  The plan is read back to the
// host (one stream synchronisation): it rejects a group that selects more
// than kWinKeys frames and, with the residuals written over the stack, fixes
// when each group's residuals may be written: after the last group that
// reads any of its frames.  A row that selects nothing takes the median of
// all frames (computed only when such a row exists).
graphic_status do_median_window_groups(graphic_ctx ctx, long long T, int N, const float* stack,
                                       const double* times, const double* parang, double t_max, double alpha_min,
                                       float* psf, float* resid, char* ws, hipStream_t st) {
  const long long npix = (long long)N * N;
  const WindowLayout L = window_layout(T, npix);
  auto* sel = reinterpret_cast<unsigned long long*>(ws + L.sel);
  int* list = reinterpret_cast<int*>(ws + L.list);
  int* gcount = reinterpret_cast<int*>(ws + L.gcount);
  int* need = reinterpret_cast<int*>(ws + L.need);
  int* flags = reinterpret_cast<int*>(ws + L.flags);
  float* psf_all = reinterpret_cast<float*>(ws + L.psf_all);
  float* ring = reinterpret_cast<float*>(ws + L.ring);
  const long long groups = (T + kWinRows - 1) / kWinRows;
  std::vector<int> h_count((size_t)groups), h_need((size_t)groups);
  int h_flags = 0;
  {
    Timer t(ctx, st, "aux");
    hipError_t e = launch_window_plan(times, parang, T, t_max, alpha_min, list, gcount, need, sel, flags, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h_count.data(), gcount, groups * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h_need.data(), need, groups * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_flags, flags, sizeof(int), hipMemcpyDeviceToHost, st);
    t.done();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return GRAPHIC_ERR_HIP;
  }
  const bool in_place = resid == stack;
  const bool use_ring = resid != nullptr && psf == nullptr;
  // group g's residuals are written after group fin[g]
  std::vector<std::vector<int>> write_after((size_t)groups);
  for (long long g = 0; g < groups; ++g) {
    if (h_count[g] > kWinKeys) return GRAPHIC_ERR_UNSUPPORTED;
    const long long fin = in_place ? std::max<long long>(g, h_need[g]) : g;
    if (use_ring && fin - g >= kWinRing) return GRAPHIC_ERR_UNSUPPORTED;
    write_after[(size_t)fin].push_back((int)g);
  }
  auto psf_rows = [&](long long g) -> float* {
    return psf ? psf + g * kWinRows * npix : ring + (g % kWinRing) * kWinRows * npix;
  };
  Timer t(ctx, st, "median");
  hipError_t e = hipSuccess;
  if (h_flags & 1) e = launch_median(stack, T, npix, psf_all, nullptr, median_variant(ctx, T), st);
  for (long long g = 0; g < groups && e == hipSuccess; ++g) {
    const long long f0 = g * kWinRows;
    const int rows = (int)std::min<long long>(kWinRows, T - f0);
    e = launch_median_window_rows(stack, npix, list + g * kWinKeys, h_count[g], rows, sel + f0 * 64, psf_all,
                                  psf_rows(g), st);
    if (!resid) continue;
    for (int d : write_after[(size_t)g]) {
      if (e != hipSuccess) break;
      const long long d0 = (long long)d * kWinRows;
      const long long n = std::min<long long>(kWinRows, T - d0) * npix;
      e = launch_window_resid(stack + d0 * npix, psf_rows(d), resid + d0 * npix, n, st);
    }
  }
  t.done();
  return hip_ok(e);
}

// Selection, then the per-frame medians (Sect. 3.3); ws holds the selection
// rows and counts (window_layout).
graphic_status do_median_window(graphic_ctx ctx, long long T, int N, const float* stack, const double* times,
                                const double* parang, double t_max, double alpha_min, float* psf, float* resid,
                                char* ws, hipStream_t st) {
  if (T > kWinKeys)
    return do_median_window_groups(ctx, T, N, stack, times, parang, t_max, alpha_min, psf, resid, ws, st);
  const WindowLayout L = window_layout(T, (long long)N * N);
  auto* sel = reinterpret_cast<unsigned long long*>(ws + L.sel);
  auto* counts = reinterpret_cast<int*>(ws + L.counts);
  Timer t(ctx, st, "median");
  hipError_t e = launch_select_frames(times, parang, T, t_max, alpha_min, sel, counts, st);
  if (e == hipSuccess) e = launch_median_window(stack, T, (long long)N * N, sel, psf, resid, st);
  t.done();
  return hip_ok(e);
}

}  // namespace

extern "C" {

graphic_status graphic_median_window(graphic_ctx ctx, const graphic_geom* geom, const float* stack,
                                     const double* times, const double* parang_deg, double t_max,
                                     double alpha_min_deg, float* psf_cube, float* resid, void* ws,
                                     size_t ws_bytes, graphic_stream stream) {
  int P = 0;
  graphic_status s = window_args(ctx, geom, times, parang_deg, t_max, alpha_min_deg, &P);
  if (s != GRAPHIC_OK) return s;
  if (!stack || (!psf_cube && !resid)) return GRAPHIC_ERR_ARG;
  const long long T = geom->n_frames;
  const int N = geom->n;
  const size_t cube_b = (size_t)T * N * N * sizeof(float);
  if (psf_cube && (overlap_bad(stack, psf_cube, cube_b) || psf_cube == stack)) return GRAPHIC_ERR_ARG;
  if (resid && overlap_bad(stack, resid, cube_b)) return GRAPHIC_ERR_ARG;
  if (psf_cube && resid && (overlap_bad(psf_cube, resid, cube_b) || psf_cube == resid)) return GRAPHIC_ERR_ARG;
  if (!ws_ok(ws, ws_bytes, window_ws_bytes(T, (long long)N * N))) return GRAPHIC_ERR_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  if ((geom->flags & GRAPHIC_CHECK_FINITE) &&
      (s = check_finite(ctx, static_cast<hipStream_t>(stream), {{stack, (size_t)T * N * N}},
                        {{times, (size_t)T}, {parang_deg, (size_t)T}})) != GRAPHIC_OK)
    return s;
  return do_median_window(ctx, T, N, stack, times, parang_deg, t_max, alpha_min_deg, psf_cube, resid,
                          static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

graphic_status graphic_alpha_min_deg(double n_fwhm, double fwhm, double r_min, double* out_deg) {
  if (!out_deg || !std::isfinite(n_fwhm) || !std::isfinite(fwhm) || !std::isfinite(r_min) || !(r_min > 0.0))
    return GRAPHIC_ERR_ARG;
  const double x = n_fwhm * fwhm / (2.0 * r_min);
  if (!(x >= 0.0 && x <= 1.0)) return GRAPHIC_ERR_ARG;
  *out_deg = 2.0 * std::asin(x) * (180.0 / 3.14159265358979323846);
  return GRAPHIC_OK;
}

graphic_status graphic_adi_reduce_window(graphic_ctx ctx, const graphic_geom* geom, const float* cube,
                                         const double* dx, const double* dy, const double* parang_deg,
                                         const double* times, double t_max, double alpha_min_deg,
                                         float* final_img, float* psf_cube, float* residuals, void* ws,
                                         size_t ws_bytes, graphic_stream stream) {
  int P = 0;
  graphic_status s = window_args(ctx, geom, times, parang_deg, t_max, alpha_min_deg, &P);
  if (s != GRAPHIC_OK) return s;
  if (!cube || !dx || !dy || !final_img) return GRAPHIC_ERR_ARG;
  const long long T = geom->n_frames;
  const int N = geom->n;
  const size_t cube_b = (size_t)T * N * N * sizeof(float);
  const size_t img_b = (size_t)N * N * sizeof(float);
  auto inside = [&](const void* p, size_t b) {
    const char* q = static_cast<const char*>(p);
    const char* c = static_cast<const char*>(static_cast<const void*>(cube));
    return q < c + cube_b && c < q + b;
  };
  if (inside(final_img, img_b)) return GRAPHIC_ERR_ARG;
  if (psf_cube && (inside(psf_cube, cube_b) || overlap_bad(psf_cube, final_img, img_b))) return GRAPHIC_ERR_ARG;
  if (residuals && (inside(residuals, cube_b) || overlap_bad(residuals, final_img, img_b))) return GRAPHIC_ERR_ARG;
  if (psf_cube && residuals && overlap_bad(psf_cube, residuals, cube_b)) return GRAPHIC_ERR_ARG;
  const size_t stack_b = residuals ? 0 : align_up(cube_b);
  const size_t fixed = stack_b + window_ws_bytes(T, (long long)N * N);
  const RotLayout L = rot_layout(T, N, P, ctx->chunk_bytes, 0);
  if (!ws_ok(ws, ws_bytes, fixed + L.params + align_up((size_t)N * P * sizeof(float)))) return GRAPHIC_ERR_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((geom->flags & GRAPHIC_CHECK_FINITE) &&
      (s = check_finite(ctx, st, {{cube, (size_t)T * N * N}},
                        {{dx, (size_t)T}, {dy, (size_t)T}, {parang_deg, (size_t)T}, {times, (size_t)T}})) !=
          GRAPHIC_OK)
    return s;
  char* w = static_cast<char*>(ws);
  float* stack = residuals ? residuals : reinterpret_cast<float*>(w);
  ShiftItem sh{cube, stack, T, dx, dy};
  if ((s = do_shift_batch(ctx, N, P, &sh, 1, st)) != GRAPHIC_OK) return s;
  if ((s = do_median_window(ctx, T, N, stack, times, parang_deg, t_max, alpha_min_deg, psf_cube, stack,
                            w + stack_b, st)) != GRAPHIC_OK)
    return s;
  RotItem rot{stack, stack, T, parang_deg};
  if ((s = do_rotate_batch(ctx, N, P, &rot, 1, -1.0, w + fixed, ws_bytes - fixed, st)) != GRAPHIC_OK) return s;
  return do_median(ctx, T, N, stack, final_img, nullptr, st);
}

graphic_status graphic_parallactic_angles(graphic_ctx ctx, const double* lst_s, int64_t n_frames, double ra_deg,
                                          double dec_deg, double lat_deg, double* out_deg, graphic_stream stream) {
  if (!ctx || !lst_s || !out_deg || n_frames < 1) return GRAPHIC_ERR_ARG;
  if (!std::isfinite(ra_deg) || !std::isfinite(dec_deg) || !std::isfinite(lat_deg)) return GRAPHIC_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Timer t(ctx, st, "aux");
  hipError_t e = launch_parallactic(lst_s, n_frames, ra_deg, dec_deg, lat_deg, out_deg, st);
  t.done();
  return hip_ok(e);
}

graphic_status graphic_register(graphic_ctx ctx, const graphic_geom* geom, const float* cube,
                                const graphic_register_params* params, double* out, int32_t* flags,
                                graphic_stream stream) {
  if (!ctx || !geom || !cube || !params || !out || !flags) return GRAPHIC_ERR_ARG;
  int P = 0;
  graphic_status s = check_geom(geom, &P);
  if (s != GRAPHIC_OK) return s;
  const graphic_register_params& q = *params;
  if (q.half < 1 || q.half > 32 || q.min_size > q.max_size || q.max_iter < 1 || std::isnan(q.threshold) ||
      std::isnan(q.saturation))
    return GRAPHIC_ERR_ARG;
  if (geom->n_frames > 0x7fffffffLL) return GRAPHIC_ERR_UNSUPPORTED;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  RegisterParams prm{q.threshold, q.min_size, q.max_size, q.half, q.saturation, q.max_iter};
  hipStream_t st = static_cast<hipStream_t>(stream);
  Timer t(ctx, st, "register");
  hipError_t e = launch_register(cube, geom->n_frames, geom->n, prm, out, flags, st);
  t.done();
  return hip_ok(e);
}

graphic_status graphic_median_nan(graphic_ctx ctx, const graphic_geom* geom, const float* stack, float* out,
                                  graphic_stream stream) {
  if (!ctx || !geom || !stack || !out) return GRAPHIC_ERR_ARG;
  if (geom->n_frames < 1 || geom->n < 1 || geom->flags != 0) return GRAPHIC_ERR_ARG;
  if (geom->n_frames > kMaxT_NanMedian) return GRAPHIC_ERR_UNSUPPORTED;
  const long long T = geom->n_frames;
  const int N = geom->n;
  if (overlap_bad(stack, out, (size_t)N * N * sizeof(float)) || (out >= stack && out < stack + (size_t)T * N * N))
    return GRAPHIC_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Timer t(ctx, st, "median");
  hipError_t e = launch_median_nan(stack, T, (long long)N * N, out, st);
  t.done();
  return hip_ok(e);
}

namespace {
graphic_status frames_args(graphic_ctx ctx, const graphic_geom* geom, const void* cube) {
  if (!ctx || !geom || !cube) return GRAPHIC_ERR_ARG;
  if (geom->n_frames < 1 || geom->n < 1 || geom->flags != 0) return GRAPHIC_ERR_ARG;
  if (geom->n_frames > 65535) return GRAPHIC_ERR_UNSUPPORTED;
  return hipSetDevice(ctx->device) == hipSuccess ? GRAPHIC_OK : GRAPHIC_ERR_HIP;
}
}  // namespace

graphic_status graphic_mask_disk(graphic_ctx ctx, const graphic_geom* geom, float* cube, const double* xs,
                                 const double* ys, double radius, graphic_stream stream) {
  graphic_status s = frames_args(ctx, geom, cube);
  if (s != GRAPHIC_OK) return s;
  if (!xs || !ys || std::isnan(radius)) return GRAPHIC_ERR_ARG;
  return hip_ok(launch_mask_disk(cube, geom->n_frames, geom->n, xs, ys, radius, static_cast<hipStream_t>(stream)));
}

graphic_status graphic_subtract_nearest(graphic_ctx ctx, const graphic_geom* geom, float* cube, const double* times,
                                        const float* skies, const double* sky_times, int32_t n_skies,
                                        graphic_stream stream) {
  graphic_status s = frames_args(ctx, geom, cube);
  if (s != GRAPHIC_OK) return s;
  if (!times || !skies || !sky_times || n_skies < 1) return GRAPHIC_ERR_ARG;
  const size_t fb = (size_t)geom->n * geom->n * sizeof(float);
  const char* c0 = reinterpret_cast<const char*>(cube);
  const char* s0 = reinterpret_cast<const char*>(skies);
  if (c0 < s0 + fb * (size_t)n_skies && s0 < c0 + fb * (size_t)geom->n_frames) return GRAPHIC_ERR_ARG;
  return hip_ok(launch_subtract_nearest(cube, geom->n_frames, geom->n, times, skies, sky_times, n_skies,
                                        static_cast<hipStream_t>(stream)));
}

graphic_status graphic_badpix_map(graphic_ctx ctx, int32_t n, const float* frame, double c_sigma, uint8_t* map,
                                  double* stats, void* ws, size_t ws_bytes, graphic_stream stream) {
  if (!ctx || !frame || !map || n < 1 || std::isnan(c_sigma)) return GRAPHIC_ERR_ARG;
  if (!ws_ok(ws, ws_bytes, frame_stats_ws_bytes())) return GRAPHIC_ERR_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  return hip_ok(launch_badpix_map(frame, n, c_sigma, map, stats, ws, static_cast<hipStream_t>(stream)));
}

graphic_status graphic_badpix_fix(graphic_ctx ctx, const graphic_geom* geom, float* cube, const uint8_t* map,
                                  int32_t max_passes, int32_t* passes, void* ws, size_t ws_bytes,
                                  graphic_stream stream) {
  graphic_status s = frames_args(ctx, geom, cube);
  if (s != GRAPHIC_OK) return s;
  if (max_passes < 0) return GRAPHIC_ERR_ARG;
  const long long T = geom->n_frames;
  const int N = geom->n;
  const size_t cube_b = align_up((size_t)T * N * N * sizeof(float));
  if (!ws_ok(ws, ws_bytes, cube_b + kAlign)) return GRAPHIC_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* alt = static_cast<float*>(ws);
  int* dflags = reinterpret_cast<int*>(static_cast<char*>(ws) + cube_b);
  if (map && launch_apply_map(cube, T, N, map, st) != hipSuccess) return GRAPHIC_ERR_HIP;
  float* src = cube;
  float* dst = alt;
  int done = 0;
  int hflags[2] = {0, 0};
  for (int p = 0; p < max_passes; ++p) {
    if (hipMemsetAsync(dflags, 0, 2 * sizeof(int), st) != hipSuccess) return GRAPHIC_ERR_HIP;
    if (launch_repair_pass(src, dst, T, N, dflags, st) != hipSuccess) return GRAPHIC_ERR_HIP;
    if (hipMemcpyAsync(hflags, dflags, 2 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return GRAPHIC_ERR_HIP;
    std::swap(src, dst);                     // src now holds the pass's result
    const bool left = hflags[0] != 0, changed = hflags[1] != 0;
    if (!left && !changed) break;            // no NaN was there
    ++done;
    if (!left || !changed) break;
  }
  if (src != cube &&
      hipMemcpyAsync(cube, src, (size_t)T * N * N * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
    return GRAPHIC_ERR_HIP;
  if (passes) *passes = done;
  return GRAPHIC_OK;
}

graphic_status graphic_annular_rms(graphic_ctx ctx, const graphic_geom* geom, const float* a, const float* b,
                                   double cx, double cy, double width, int32_t n_rings, double* rms, int64_t* counts,
                                   graphic_stream stream) {
  graphic_status s = frames_args(ctx, geom, a);
  if (s != GRAPHIC_OK) return s;
  if (!rms || !counts || n_rings < 1 || n_rings > kMaxRings) return GRAPHIC_ERR_ARG;
  if (!std::isfinite(width) || !std::isfinite(cx) || !std::isfinite(cy) || !(width > 0.0)) return GRAPHIC_ERR_ARG;
  if ((std::fabs(cx) + std::fabs(cy) + 2.0 * geom->n) / width >= 1073741824.0) return GRAPHIC_ERR_ARG;
  const long long T = geom->n_frames;
  const int N = geom->n;
  const size_t frames_b = (size_t)T * N * N * sizeof(float);
  const char* ra = reinterpret_cast<const char*>(rms);
  const size_t rms_b = (size_t)T * n_rings * sizeof(double);
  auto overlaps = [&](const void* x, size_t xb) {
    const char* q = static_cast<const char*>(x);
    return q < ra + rms_b && ra < q + xb;
  };
  if (overlaps(a, frames_b) || (b && overlaps(b, frames_b)) || overlaps(counts, (size_t)n_rings * sizeof(int64_t)))
    return GRAPHIC_ERR_ARG;
  return hip_ok(launch_annular_rms(a, b, T, N, cx, cy, width, n_rings, rms, reinterpret_cast<long long*>(counts),
                                   static_cast<hipStream_t>(stream)));
}

graphic_status graphic_batch_workspace_size(graphic_ctx ctx, const graphic_cube_desc* descs, int n_cubes,
                                            uint32_t flags, size_t* bytes) {
  if (!bytes) return GRAPHIC_ERR_ARG;
  BatchPlan plan;
  graphic_status s = plan_batch(descs, n_cubes, flags, ctx ? ctx->chunk_bytes : kDefaultChunkBytes, &plan);
  if (s != GRAPHIC_OK) return s;
  *bytes = plan.fixed + plan.rot_default;
  return GRAPHIC_OK;
}

graphic_status graphic_adi_reduce_batch(graphic_ctx ctx, const graphic_cube_desc* descs, int n_cubes,
                                        uint32_t flags, void* ws, size_t ws_bytes, graphic_stream stream) {
  if (!ctx) return GRAPHIC_ERR_ARG;
  return adi_batch(ctx, descs, n_cubes, flags, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"

struct graphic_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

extern "C" {

graphic_status graphic_adi_graph_create(graphic_ctx ctx, const graphic_cube_desc* descs, int n_cubes,
                                        uint32_t flags, void* ws, size_t ws_bytes, graphic_graph* graph) {
  if (!ctx || !graph) return GRAPHIC_ERR_ARG;
  *graph = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return GRAPHIC_ERR_HIP;
  const bool timing = ctx->timing;
  ctx->timing = false;                     // no event nodes inside the graph
  graphic_status s = GRAPHIC_ERR_HIP;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    s = adi_batch(ctx, descs, n_cubes, flags, ws, ws_bytes, cs);
    if (hipStreamEndCapture(cs, &g) != hipSuccess && s == GRAPHIC_OK) s = GRAPHIC_ERR_HIP;
  }
  ctx->timing = timing;
  hipStreamDestroy(cs);
  if (s == GRAPHIC_OK && !g) s = GRAPHIC_ERR_HIP;
  hipGraphExec_t x = nullptr;
  if (s == GRAPHIC_OK && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) s = GRAPHIC_ERR_HIP;
  if (s != GRAPHIC_OK) {
    if (g) hipGraphDestroy(g);
    return s;
  }
  graphic_graph out = new (std::nothrow) graphic_graph_s();
  if (!out) {
    hipGraphExecDestroy(x);
    hipGraphDestroy(g);
    return GRAPHIC_ERR_NOMEM;
  }
  out->graph = g;
  out->exec = x;
  out->device = ctx->device;
  *graph = out;
  return GRAPHIC_OK;
}

graphic_status graphic_graph_launch(graphic_graph graph, graphic_stream stream) {
  if (!graph) return GRAPHIC_ERR_ARG;
  if (hipSetDevice(graph->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  return hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)) == hipSuccess ? GRAPHIC_OK
                                                                                    : GRAPHIC_ERR_HIP;
}

void graphic_graph_destroy(graphic_graph graph) {
  if (!graph) return;
  hipSetDevice(graph->device);
  if (graph->exec) hipGraphExecDestroy(graph->exec);
  if (graph->graph) hipGraphDestroy(graph->graph);
  delete graph;
}

}  // extern "C"

namespace {

// Mean device milliseconds of `reps` back-to-back launches after one warm-up.
template <class F>
double time_launches(hipStream_t st, int reps, F&& launch, bool* ok) {
  hipEvent_t a = nullptr, b = nullptr;
  *ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
  float ms = 0.f;
  if (*ok) *ok = launch() == hipSuccess;
  if (*ok) *ok = hipEventRecord(a, st) == hipSuccess;
  for (int r = 0; r < reps && *ok; ++r) *ok = launch() == hipSuccess;
  if (*ok) *ok = hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
                 hipEventElapsedTime(&ms, a, b) == hipSuccess;
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  return (double)ms / reps;
}

}  // namespace

extern "C" {

graphic_status graphic_autotune(graphic_ctx ctx, const graphic_geom* geom, void* ws, size_t ws_bytes,
                                graphic_stream stream) {
  if (!ctx) return GRAPHIC_ERR_ARG;
  int P = 0;
  graphic_status s = check_geom(geom, &P);
  if (s != GRAPHIC_OK) return s;
  if (geom->n_frames > kMaxT_Median) return GRAPHIC_ERR_UNSUPPORTED;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return GRAPHIC_ERR_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return GRAPHIC_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int N = geom->n, o = (P - N) / 2;
  const long long T = geom->n_frames;
  float* buf = static_cast<float*>(ws);
  // synthetic frames: the timings do not depend on the values, but the
  // median's early stop does, so the data is spread like sky frames
  if (launch_fill_noise(buf, ws_bytes / sizeof(float), 0x2545F491u, st) != hipSuccess) return GRAPHIC_ERR_HIP;
  bool ok = true;
  // staged column passes of both pairings (only the canonical geometry has a
  // second variant), over as many frames as one launch of the pipeline
  // takes: the whole cube for the shift's y-pass, one rotation chunk for the
  // y-shear (the tile choice depends on the launch size through its tail)
  if (P == 2 * N && P / 2 >= 256) {
    for (int mir = 0; mir < 2; ++mir) {
      const size_t fb = (size_t)N * (mir ? P : N) * sizeof(float);
      long long F = std::min<long long>(T, (long long)(ws_bytes / fb));
      if (mir) F = std::min<long long>(F, std::max<long long>(1, (long long)(ctx->chunk_bytes / fb)));
      if (F < std::min<long long>(T, 8)) continue;
      LinePass c = base_pass(ctx, P);
      c.src = buf;
      c.dst = buf;
      c.src_fs = c.dst_fs = (long long)N * (mir ? P : N);
      c.src_ls = c.dst_ls = 1;
      c.src_ps = c.dst_ps = mir ? P : N;
      c.line_lo = mir ? 0 : o;
      c.n_lines = mir ? P : N;
      c.in_off = o;
      c.in_len = N;
      c.out_off = o;
      c.out_len = N;
      c.dst_line_lo = mir ? 0 : o;
      c.mirror = mir;
      c.n_jobs = mir ? P / 2 + 1 : N / 2;
      c.n_frames = F;
      double best = 0.0;
      int pick = 0;
      for (int v = 0; v < 2 && ok; ++v) {
        const double ms = time_launches(st, 3, [&] { return launch_line_pass(c, kColPass, v, st); }, &ok);
        if (ok && (v == 0 || ms < best)) {
          best = ms;
          pick = v;
        }
      }
      if (!ok) return GRAPHIC_ERR_HIP;
      ctx->col_var[ilog2(P / 2)][mir] = pick;
    }
  }
  // median: the pipeline runs it twice per cube, once rewriting the stack as
  // residuals and once read-only; both are timed, on as many pixels of this
  // frame count as the workspace holds
  // (deep stacks take the streaming select, which has no variants)
  long long npix = T > kMaxT_RegisterMedian
                       ? 0
                       : std::min<long long>((long long)N * N, (long long)(ws_bytes / sizeof(float)) / (T + 1));
  npix -= npix % 128;
  if (npix >= std::min<long long>(16384, (long long)N * N - ((long long)N * N) % 128)) {
    float* out = buf + (size_t)T * npix;
    double best = 0.0;
    int pick = 0;
    for (int v = 0; v < 2 && ok; ++v) {
      const double ms = time_launches(st, 2, [&] {
        hipError_t e = launch_median(buf, T, npix, out, buf, v, st);
        return e != hipSuccess ? e : launch_median(buf, T, npix, out, nullptr, v, st);
      }, &ok);
      if (ok && (v == 0 || ms < best)) {
        best = ms;
        pick = v;
      }
    }
    if (!ok) return GRAPHIC_ERR_HIP;
    ctx->med_var[median_class(T)] = pick;
    // the tile-major median of the large canonical sizes, the same way
    if (P == 2 * N && N == 1024) {
      for (int v = 0; v < 2 && ok; ++v) {
        const double ms = time_launches(st, 2, [&] {
          hipError_t e = launch_median_tile_major(buf, T, npix, out, buf, v, st);
          return e != hipSuccess ? e : launch_median_tile_major(buf, T, npix, out, nullptr, v, st);
        }, &ok);
        if (ok && (v == 0 || ms < best)) {
          best = ms;
          pick = v;
        }
      }
      if (!ok) return GRAPHIC_ERR_HIP;
      ctx->tmm_var[median_class(T)] = pick;
    }
  }
  return GRAPHIC_OK;
}

graphic_status graphic_tuning_export(graphic_ctx ctx, char* buf, size_t buf_len, size_t* needed) {
  if (!ctx) return GRAPHIC_ERR_ARG;
  std::string t;
  for (int l = 0; l < 16; ++l)
    for (int m = 0; m < 2; ++m)
      if (ctx->col_var[l][m] >= 0)
        t += "col " + std::to_string(1 << l) + " " + std::to_string(m) + " " + std::to_string(ctx->col_var[l][m]) + "\n";
  for (int c = 0; c < 8; ++c)
    if (ctx->med_var[c] >= 0) t += "med " + std::to_string(c) + " " + std::to_string(ctx->med_var[c]) + "\n";
  for (int c = 0; c < 8; ++c)
    if (ctx->tmm_var[c] >= 0) t += "tmm " + std::to_string(c) + " " + std::to_string(ctx->tmm_var[c]) + "\n";
  if (needed) *needed = t.size() + 1;
  if (buf && buf_len > 0) {
    const size_t n = std::min(buf_len - 1, t.size());
    std::memcpy(buf, t.data(), n);
    buf[n] = '\0';
    if (buf_len < t.size() + 1) return GRAPHIC_ERR_ARG;
  }
  return GRAPHIC_OK;
}

graphic_status graphic_tuning_import(graphic_ctx ctx, const char* text) {
  if (!ctx || !text) return GRAPHIC_ERR_ARG;
  int col[16][2], med[8], tmm[8];
  std::memcpy(col, ctx->col_var, sizeof(col));
  std::memcpy(med, ctx->med_var, sizeof(med));
  std::memcpy(tmm, ctx->tmm_var, sizeof(tmm));
  const char* q = text;
  while (*q) {
    while (*q == '\n' || *q == ' ') ++q;
    if (!*q) break;
    char kind[4] = {0};
    int a = 0, b = 0, v = 0, used = 0;
    if (std::sscanf(q, "%3s %d %d %d%n", kind, &a, &b, &v, &used) == 4 && std::strcmp(kind, "col") == 0) {
      if (a < 8 || a > 2048 || (a & (a - 1)) || (b != 0 && b != 1) || v < 0 || v > 1) return GRAPHIC_ERR_ARG;
      col[ilog2(a)][b] = v;
    } else if (std::sscanf(q, "%3s %d %d%n", kind, &a, &v, &used) == 3 &&
               (std::strcmp(kind, "med") == 0 || std::strcmp(kind, "tmm") == 0)) {
      if (a < 0 || a > 7 || v < 0 || v > 1) return GRAPHIC_ERR_ARG;
      (kind[0] == 'm' ? med : tmm)[a] = v;
    } else {
      return GRAPHIC_ERR_ARG;
    }
    q += used;
    while (*q && *q != '\n') {
      if (*q != ' ') return GRAPHIC_ERR_ARG;
      ++q;
    }
  }
  std::memcpy(ctx->col_var, col, sizeof(col));
  std::memcpy(ctx->med_var, med, sizeof(med));
  std::memcpy(ctx->tmm_var, tmm, sizeof(tmm));
  return GRAPHIC_OK;
}

graphic_status graphic_timing_enable(graphic_ctx ctx, int enable) {
  if (!ctx) return GRAPHIC_ERR_ARG;
  for (auto& p : ctx->pending) {
    hipEventSynchronize(p.stop);
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  ctx->pending.clear();
  ctx->acc.clear();
  ctx->timing = enable != 0;
  return GRAPHIC_OK;
}

graphic_status graphic_timing_read(graphic_ctx ctx, const char* family, double* total_ms, int64_t* launches) {
  if (!ctx || !family || !total_ms || !launches) return GRAPHIC_ERR_ARG;
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.stop) != hipSuccess) return GRAPHIC_ERR_HIP;
    hipEventElapsedTime(&ms, p.start, p.stop);
    bool found = false;
    for (auto& a : ctx->acc)
      if (a.family == p.family) {
        a.ms += ms;
        a.n += 1;
        found = true;
      }
    if (!found) ctx->acc.push_back({p.family, (double)ms, 1});
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  ctx->pending.clear();
  *total_ms = 0.0;
  *launches = 0;
  for (auto& a : ctx->acc)
    if (a.family == family) {
      *total_ms = a.ms;
      *launches = a.n;
    }
  return GRAPHIC_OK;
}

}  // extern "C"
