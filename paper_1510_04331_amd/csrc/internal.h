// Internal declarations shared by the C ABI (graphic.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace graphic {

constexpr int kMinM = 8;      // smallest half working size (P = 16)
constexpr int kMaxM = 2048;   // largest half working size (P = 4096)

// Twiddle tables of one half size M = P/2, in device memory.
//   fwd[k2*Ma + n1]  = exp(-2 pi i n1 k2 / M)          (four-step, forward)
//   inv[n1*Mb + k2]  = exp(+2 pi i n1 k2 / M)          (four-step, inverse)
//   fold[h*M + m]    = 1 (h = 0) or exp(-2 pi i m / P) (h = 1)
//   split[((h*2 + e)*Ma + j)*Ma + n1] = exp(-2 pi i (h (n1 + Ma j) / P + j e / Mb))
//                                     (M = 2048 only: the two-wave jobs)
struct TwiddleTables {
  const float2* fwd;
  const float2* inv;
  const float2* fold;
  const float2* split;
};

constexpr int kMaxCubesPerLaunch = 16;

// Tile-major stack layout: the value of frame t at pixel p (row-major pixel
// index of an N x N frame) of a T-frame stack sits at float index
// ((p / 16) * T + t) * 16 + p % 16, so the T values of 16 neighbouring pixels
// are one contiguous run of 64 T bytes.  The ADI reduction keeps its
// workspace stack in this layout for the large canonical sizes.
constexpr int kTilePix = 16;

// One cube of a batched launch: frames [frame0, frame0 + n) of the launch
// belong to it (frame0 may be negative when the launch starts inside it).
// A null member means "the launch's own array, indexed by the launch frame".
struct CubeRef {
  const float* src;       // the cube's frame 0 in the pass's source, or null
  float* dst;             // the cube's frame 0 in the pass's destination, or null
  const double* sh0;      // the cube's per-frame constant shift (local frame index), or null
  long long frame0;
  long long tm_T;         // frames of the cube (tile-major source or destination only)
};

// One pass of one-dimensional Fourier shifts over the lines of a stack of
// 2-D arrays.  Coordinates along and across the lines are those of the
// zero-padded P x P frame; the mapping to array indices is described by the
// offsets below.  See line_pass.hip for the algorithm.
struct LinePass {
  // memory: element (frame f, line li, position pi) at base + f*fs + li*ls + pi*ps
  const float* src;
  float* dst;
  long long src_fs, dst_fs;
  int src_ls, src_ps, dst_ls, dst_ps;

  int P;                  // working size
  int line_lo;            // first line (padded coordinate) of the line set
  int n_lines;            // number of lines in the set (source and destination)
  int in_off, in_len;     // source support along the line: [in_off, in_off+in_len)
  int out_off, out_len;   // destination window along the line
  int dst_line_lo;        // destination array line index = line - dst_line_lo

  int mirror;             // 0: pair lines (l, l+1) with one shift; 1: pair (c-d, c+d)
  int n_jobs;             // jobs (line pairs) per frame
  long long n_frames;
  int blocks_per_frame;   // set by the launcher: blocks never straddle frames
  int frame_group;        // block order: 0 or 1 = frame by frame; g > 1 = the blocks of g
                          // consecutive frames interleaved, frame fastest

  // Tile-major cube arrays (cube launches only, rows of N = P/2 = 1024
  // pixels, window-to-window or window-to-full index patterns): the source
  // (src_tm) or destination (dst_tm) of every cube is a tile-major stack of
  // cubes[i].tm_T frames; *_fs, *_ls and *_ps are ignored for it.
  int src_tm, dst_tm;

  // Batched launches: with n_cubes > 0, frame f of the launch lives in the
  // cube with the largest frame0 <= f, and src/dst/sh0 come from that cube
  // (sh1 and flip stay indexed by the launch's frame f).
  int n_cubes;
  CubeRef cubes[kMaxCubesPerLaunch];

  // shift of line l in frame f: sh0[f] + sh1[f] * (l - P/2)   (either may be null)
  const double* sh0;
  const double* sh1;

  // per-frame half-turn flag (nullable) and where it acts
  const int* flip;
  const int* flip_list;   // indices of the half-turned frames (relative to this pass's frames)
  const int* flip_count;  // their number (device memory)
  int flip_src_reverse;   // source array read reversed along and across lines
  int flip_lines;         // line set and destination lines start one later
  int flip_in_off;        // source support starts one later

  TwiddleTables tw;
};

enum PassKind { kRowPass = 0, kColPass = 1 };

// Raises a kernel's dynamic LDS limit to `bytes` before its launch; returns
// the runtime's status so that a refused size stops the launch.
template <typename Kernel>
inline hipError_t set_dynamic_lds(Kernel* kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// Index patterns of a pass (input support -> output window), see line_pass.hip.
enum IoKind { kIoGeneric = 0, kIoWinWin = 1, kIoWinFull = 2, kIoFullWin = 3 };

// variant: 0 = default launch shape; 1 = the alternative tile width of the
// staged column pass (rows and other geometries ignore it).
hipError_t launch_line_pass(const LinePass& p, int kind, int variant, hipStream_t s);

// Per-frame rotation parameters from angles: flip (|theta| > 90), -tan(theta'/2), sin(theta').
hipError_t launch_rotation_params(const double* theta_deg, double sign, long long T,
                                  int* flip, double* neg_tan_half, double* sin_theta,
                                  hipStream_t s);

// Compacted list of the frames f0 <= f < f0 + n with flip[f] != 0, as indices
// relative to f0, and their count.
hipError_t launch_flip_list(const int* flip, long long f0, long long n, int* list, int* count,
                            hipStream_t s);

// Exact per-pixel median of a [T][npix] stack -> [npix]; with resid non-null,
// every value is also written back as value - median (resid may be stack).
// variant: 0 = 16-pixel tiles, 1 = 8-pixel tiles (same result).
hipError_t launch_median(const float* stack, long long T, long long npix, float* out, float* resid,
                         int variant, hipStream_t s);
// The same on a tile-major stack (npix a multiple of 16; resid, if non-null,
// is tile-major too and may be stack); variant as above.
hipError_t launch_median_tile_major(const float* stack, long long T, long long npix, float* out, float* resid,
                                    int variant, hipStream_t s);

// Frame selection of the per-frame PSF (sel: [T][64] bit rows, counts: [T]).
hipError_t launch_select_frames(const double* times, const double* parang, long long T, double t_max,
                                double alpha_min, unsigned long long* sel, int* counts, hipStream_t s);

// Per-frame medians over selected frames of a [T][npix] stack (T <= 2048):
// psf[f] (nullable) and resid[f] = stack[f] - psf[f] (nullable, may be stack).
hipError_t launch_median_window(const float* stack, long long T, long long npix, const unsigned long long* sel,
                                float* psf, float* resid, hipStream_t s);

// Longer sequences run in groups of kWinRows consecutive rows; a group may
// select at most kWinKeys distinct frames.
constexpr int kWinRows = 256;
constexpr int kWinKeys = 2048;
// Per group g (one block each): the frames that any row of g selects, in
// frame order, list[g][0..counts[g]) (counts[g] may exceed kWinKeys: then
// only the count is meaningful); need[f / kWinRows] = the last group that
// selects frame f (-1 if none); sel[f] = the selection of row f as bits over
// its group's list (bit i of word j: entry j + 64 i); flags bit 0 set when a
// row selects nothing.
hipError_t launch_window_plan(const double* times, const double* parang, long long T, double t_max,
                              double alpha_min, int* list, int* counts, int* need, unsigned long long* sel,
                              int* flags, hipStream_t s);
// Per-frame medians of one group: n_rows rows of sel over the n_keys frames
// of list -> psf[0..n_rows) ([n_rows][npix]); an empty row takes psf_all.
hipError_t launch_median_window_rows(const float* stack, long long npix, const int* list, int n_keys, int n_rows,
                                     const unsigned long long* sel, const float* psf_all, float* psf,
                                     hipStream_t s);
// resid[i] = stack[i] - psf[i] for i < n (resid may be stack).
hipError_t launch_window_resid(const float* stack, const float* psf, float* resid, long long n, hipStream_t s);

// Registration (Sect. 3.1).  Per frame, out[f * kRegisterOut + k]: centroid x,
// y, fitted x0, y0, I0, alpha, beta, Bg, final half sum of squared
// residuals, Moffat FWHM, recentring shift dx = N/2 - x0, dy = N/2 - y0;
// flags[f]: bit 0 centroid patch found, bit 1 fit converged.
struct RegisterParams {
  double threshold;      // patch threshold
  int min_size, max_size;  // accepted patch sizes (pixels)
  int half;              // fit box half side (1..32)
  double saturation;     // pixels at or above it are masked in the fit
  int max_iter;          // Levenberg-Marquardt iterations
};
constexpr int kRegisterOut = 12;
hipError_t launch_register(const float* cube, long long T, int n, const RegisterParams& prm, double* out,
                           int* flags, hipStream_t s);
hipError_t launch_parallactic(const double* lst_s, long long T, double ra_deg, double dec_deg, double lat_deg,
                              double* out, hipStream_t s);

// NaN-ignoring per-pixel median (NaN where no value is left), T <= 4096.
hipError_t launch_median_nan(const float* stack, long long T, long long npix, float* out, hipStream_t s);

// Pre-processing (Sect. 3.2); frames are indexed by the grid's y, T <= 65535.
hipError_t launch_mask_disk(float* cube, long long T, int n, const double* xs, const double* ys, double radius,
                            hipStream_t s);
hipError_t launch_subtract_nearest(float* cube, long long T, int n, const double* times, const float* skies,
                                   const double* sky_times, int S, hipStream_t s);
size_t frame_stats_ws_bytes();
hipError_t launch_badpix_map(const float* frame, int n, double c_sigma, unsigned char* map, double* stats, void* ws,
                             hipStream_t s);
hipError_t launch_apply_map(float* cube, long long T, int n, const unsigned char* map, hipStream_t s);
hipError_t launch_repair_pass(const float* src, float* dst, long long T, int n, int* flags, hipStream_t s);

// Image-quality test (Sect. 4.1): RMS of a - b (b nullable) in n_rings annuli
// of width `width` around (cx, cy), per frame of [T][N][N] stacks, into
// rms[T][n_rings] (NaN: empty annulus) and counts[n_rings] (pixels per
// annulus); n_rings <= kMaxRings, T <= 65535.
constexpr int kMaxRings = 4096;
hipError_t launch_annular_rms(const float* a, const float* b, long long T, int N, double cx, double cy, double width,
                              int n_rings, double* rms, long long* counts, hipStream_t s);

// n floats of seeded noise around a sky level (for timing runs on scratch).
hipError_t launch_fill_noise(float* p, size_t n, unsigned seed, hipStream_t s);

// Non-finite scan: launch_clear_flag sets *flag = 0; the scans set it to 1
// if any of the n values is NaN or +-inf.
hipError_t launch_clear_flag(int* flag, hipStream_t s);
hipError_t launch_nonfinite_f32(const float* p, size_t n, int* flag, hipStream_t s);
hipError_t launch_nonfinite_f64(const double* p, size_t n, int* flag, hipStream_t s);

// Per-frame float64 sums of [T][N][N] frames into flux[2*t + slot].
hipError_t launch_frame_sums(const float* frames, long long T, int N, double* flux, int slot,
                             hipStream_t s);

}  // namespace graphic
