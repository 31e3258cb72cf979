/*
 * graphic.h -- C ABI of the MI355X Fourier ADI library (libgraphic.so).
 *
 * The operations follow Hagelberg et al. 2016, "The Geneva Reduction and
 * Analysis Pipeline for High-contrast Imaging of planetary Companions"
 * (MNRAS, arXiv:1510.04331):
 *   - graphic_shift:      Sect. 3.3.1, Fourier shift (2-D shift equation):
 *                         FT of the zero-padded frame, multiplication by the
 *                         phasor exp(-i 2 pi (nu_x a + nu_y b)), inverse FT.
 *   - graphic_rotate:     Sect. 3.4, rotation as three Fourier shears
 *                         R = S_x(-tan(theta/2)) S_y(sin theta) S_x(-tan(theta/2)).
 *   - graphic_median:     Sect. 3.3 and 3.4, per-pixel median of a stack.
 *   - graphic_adi_reduce: Sect. 3 (classical ADI): recentre every frame,
 *                         take the per-pixel median PSF, subtract it,
 *                         derotate by minus the parallactic angle and merge
 *                         the frames with a per-pixel median.
 *
 * Conventions
 *   - Frames are float32, row-major, x (column) fastest: cube[t][y][x].
 *   - Frames are square, N x N, N even.  The working size P is a power of two
 *     with N <= P <= 4096 (default: smallest power of two >= 2N).  The frame
 *     sits at offset (P-N)/2 of the zero-padded P x P frame, so the centre of
 *     rotation c = P/2 is frame pixel (N/2, N/2).
 *   - A shift (dx, dy) moves the content toward larger x and y.
 *   - A rotation by theta (degrees) turns the content counter-clockwise in the
 *     (x right, y up) frame: content at c + u ends at c + R(theta) u.  For
 *     |theta| > 90 an exact half-turn is applied first.
 *   - The Nyquist bin of every one-dimensional transform gets the real phasor
 *     cos(pi s), so every pass maps real lines to real lines.
 *   - Arithmetic: float32 transforms; the phase arguments k*s/P are reduced
 *     modulo one in float64; flux sums are float64.
 *
 * Memory and ownership
 *   - Every data pointer is DEVICE memory owned by the caller (for example a
 *     torch tensor's data_ptr()).  The library never allocates, frees or keeps
 *     caller memory.  Scratch memory ("workspace") is caller-provided device
 *     memory of at least graphic_workspace_size() bytes, 256-byte aligned.
 *   - A context owns only its twiddle tables and the device it was made on.
 *     It is not thread-safe: use one context per host thread.
 *
 * Execution and errors
 *   - Calls enqueue work on the given HIP stream and return without waiting.
 *   - Arguments are checked on the host before anything is enqueued: a null
 *     required pointer, odd or out-of-range N, an invalid P, T < 1, a too-small
 *     or misaligned workspace, or partially overlapping input and output
 *     return an error and launch nothing.  out == in is allowed where stated.
 *   - A failed launch returns GRAPHIC_ERR_HIP.  Device-side faults surface at
 *     the caller's next synchronisation.
 *   - Non-finite input values are a precondition violation; the output is then
 *     unspecified.  The GRAPHIC_CHECK_FINITE geometry flag validates them.
 */
#ifndef GRAPHIC_H
#define GRAPHIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct graphic_ctx_s* graphic_ctx;

/* An opaque HIP stream (hipStream_t); NULL is the default stream. */
typedef void* graphic_stream;

typedef enum {
    GRAPHIC_OK = 0,
    GRAPHIC_ERR_ARG = 1,          /* invalid argument; nothing launched */
    GRAPHIC_ERR_UNSUPPORTED = 2,  /* valid but unsupported geometry */
    GRAPHIC_ERR_WORKSPACE = 3,    /* workspace null, too small or misaligned */
    GRAPHIC_ERR_HIP = 4,          /* a HIP runtime call failed */
    GRAPHIC_ERR_NOMEM = 5,        /* the context could not allocate its tables */
    GRAPHIC_ERR_NONFINITE = 6     /* GRAPHIC_CHECK_FINITE found a NaN or inf input */
} graphic_status;

/* Operation codes for graphic_workspace_size. */
enum {
    GRAPHIC_OP_SHIFT = 0,
    GRAPHIC_OP_ROTATE = 1,
    GRAPHIC_OP_ADI = 2,
    GRAPHIC_OP_MEDIAN = 3,
    GRAPHIC_OP_MEDIAN_WINDOW = 4,
    GRAPHIC_OP_ADI_WINDOW = 5,
    GRAPHIC_OP_BADPIX_MAP = 6,
    GRAPHIC_OP_BADPIX_FIX = 7
};

/* Geometry of one cube. */
typedef struct {
    int64_t n_frames;   /* T >= 1 */
    int32_t n;          /* N: even, 4 <= N <= 4096 */
    int32_t pad;        /* P: power of two, N <= P <= 4096, 16 <= P; 0 => default */
    uint32_t flags;     /* GRAPHIC_KEEP_PADDED | GRAPHIC_CHECK_FINITE, as each entry point allows; else 0 */
} graphic_geom;

/* Flags of graphic_geom.
 *
 * GRAPHIC_KEEP_PADDED (graphic_shift, graphic_rotate): the output is the
 *   whole zero-padded working frame, out[T][P][P], instead of its N x N
 *   window; the input stays [T][N][N] and must not overlap the output unless
 *   P == N and out == in.  The operations of Sect. 3.3.1 and 3.4 are defined
 *   on the padded frame: with this flag an integer shift is an exact circular
 *   roll of it, a quarter turn an exact permutation, and the sum over the
 *   padded frame (the DC term of every line) is kept.  The flux sums of the
 *   output then run over the P x P frame.
 *
 * GRAPHIC_CHECK_FINITE (graphic_shift, graphic_rotate, graphic_median,
 *   graphic_adi_reduce, graphic_median_window, graphic_adi_reduce_window):
 *   before any other launch the call scans every float input (frames and
 *   per-frame parameters) for NaN and +-inf on `stream`, waits for the scan
 *   (the call synchronises `stream`, so it cannot be captured into a graph)
 *   and returns GRAPHIC_ERR_NONFINITE, with nothing else launched, if it
 *   found one.  The scan reads each input once more. */
#define GRAPHIC_KEEP_PADDED 1u
#define GRAPHIC_CHECK_FINITE 2u

/* Create a context on HIP device `hip_device` (builds the twiddle tables on
 * that device).  Returns GRAPHIC_ERR_HIP if the device is unusable. */
graphic_status graphic_create(graphic_ctx* ctx, int hip_device);

/* Release a context and its tables (NULL is ignored).  Work already enqueued
 * with the context must have completed. */
void graphic_destroy(graphic_ctx ctx);

/* Static, human-readable name of a status code. */
const char* graphic_status_string(graphic_status s);

/* Library version string (static). */
const char* graphic_version(void);

/* Working size P that a geometry resolves to (pad, or the default for pad=0),
 * or -1 if the geometry is invalid.  Host-only; needs no context. */
int32_t graphic_resolved_pad(const graphic_geom* geom);

/* Bytes of workspace that operation `op` (GRAPHIC_OP_*) needs for `geom`.
 * Host-only; `ctx` may be NULL. */
graphic_status graphic_workspace_size(graphic_ctx ctx, int op, const graphic_geom* geom,
                                      size_t* bytes);

/*
 * Fourier shift of every frame (Sect. 3.3.1, 2-D shift equation).
 *   in, out : [T][N][N] float32 device arrays; out == in is allowed.  With
 *             GRAPHIC_KEEP_PADDED, out is [T][P][P] (see the flag).
 *   dx, dy  : [T] float64 device arrays, content displacement in pixels.
 *   flux    : NULL, or a [T][2] float64 device array receiving, per frame, the
 *             sum of the input frame and the sum of the output frame.
 *   ws      : device workspace of graphic_workspace_size(GRAPHIC_OP_SHIFT) bytes.
 * Work: a column pass then a row pass, each a one-dimensional transform of the
 * zero-extended line, a phase ramp and an inverse transform.
 */
graphic_status graphic_shift(graphic_ctx ctx, const graphic_geom* geom,
                             const float* in, float* out,
                             const double* dx, const double* dy,
                             double* flux, void* ws, size_t ws_bytes,
                             graphic_stream stream);

/*
 * Three-shear Fourier rotation of every frame (Sect. 3.4).
 *   in, out   : [T][N][N] float32 device arrays; out == in is allowed.  With
 *               GRAPHIC_KEEP_PADDED, out is [T][P][P] (see the flag).
 *   theta_deg : [T] float64 device array, counter-clockwise angle in degrees;
 *               any finite angle (the rotation has period 360 degrees, and
 *               the angle is first reduced to [-180, 180]).
 *   flux      : NULL or [T][2] float64 (input sum, output sum) per frame.
 *   ws        : graphic_workspace_size(GRAPHIC_OP_ROTATE) bytes.
 */
graphic_status graphic_rotate(graphic_ctx ctx, const graphic_geom* geom,
                              const float* in, float* out,
                              const double* theta_deg, double* flux,
                              void* ws, size_t ws_bytes, graphic_stream stream);

/*
 * graphic_rotate without a workspace, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc.  It makes no hipMalloc, hipFree or other
 * allocating call (and creates no timing events).  Its scratch -- the
 * per-frame shear factors, the half-turn list and a chunk of x-sheared
 * frames -- is a library-owned static device array of
 * GRAPHIC_NOALLOC_SCRATCH_BYTES (128 MiB) on each GPU the library runs on,
 * held until the process ends; its address on a device is taken once, when
 * the first context is created on that device.
 *   Arguments, results and geom flags as graphic_rotate (GRAPHIC_KEEP_PADDED
 *   is allowed; GRAPHIC_CHECK_FINITE, which synchronises, is not).
 *   Limit: about 24 T bytes of parameters plus one N x P float32 frame must
 *   fit the array, else GRAPHIC_ERR_UNSUPPORTED (checked first, nothing
 *   launched); the frames run in chunks of as many as fit.
 *   Every call on one GPU shares that GPU's array and leaves its contents
 *   behind (nothing in it needs to start at zero): calls that overlap on
 *   one device -- other streams, host threads or contexts -- race on it and
 *   must be ordered by the caller.  GRAPHIC_ERR_HIP if the array's address
 *   could not be taken on this device.
 */
#define GRAPHIC_NOALLOC_SCRATCH_BYTES (128u << 20)
graphic_status graphic_rotate_noalloc(graphic_ctx ctx, const graphic_geom* geom,
                                      const float* in, float* out,
                                      const double* theta_deg, double* flux,
                                      graphic_stream stream);

/*
 * Exact per-pixel median over the T frames of a float32 stack (the combiner
 * of Sect. 3.3 and 3.4).  Values are ordered by IEEE totalOrder (-0 < +0);
 * with lo and hi the elements of rank (T-1)/2 and T/2, the result is
 * (lo + hi) * 0.5 in float32, which is lo when T is odd.  NaN input is a
 * precondition violation.  T <= 2^24: up to 4096 frames each pixel's values
 * are read once into registers; deeper stacks are read once per 8-bit digit
 * of the select (four to six passes over the stack).
 *   stack : [T][N][N] float32 (only T and N of geom are used).
 *   out   : [N][N] float32.
 *   ws    : graphic_workspace_size(GRAPHIC_OP_MEDIAN) bytes (may be 0; then ws may be NULL).
 */
graphic_status graphic_median(graphic_ctx ctx, const graphic_geom* geom,
                              const float* stack, float* out,
                              void* ws, size_t ws_bytes, graphic_stream stream);

/*
 * Classical ADI reduction (Sect. 3.3 and 3.4): S_i = shift(cube_i, dx_i, dy_i);
 * PSF = median_i S_i; D_i = rotate(S_i - PSF, -parang_i); final = median_i D_i.
 *   cube       : [T][N][N] float32 input (not modified).
 *   dx, dy     : [T] float64 recentring shifts; parang_deg : [T] float64.
 *   final_img  : [N][N] float32 output.
 *   psf        : NULL or [N][N] float32, receives the median PSF.
 *   residuals  : NULL or [T][N][N] float32, receives the derotated residuals D_i.
 *   ws         : graphic_workspace_size(GRAPHIC_OP_ADI) bytes.
 */
graphic_status graphic_adi_reduce(graphic_ctx ctx, const graphic_geom* geom,
                                  const float* cube, const double* dx, const double* dy,
                                  const double* parang_deg, float* final_img,
                                  float* psf, float* residuals,
                                  void* ws, size_t ws_bytes, graphic_stream stream);

/*
 * Per-frame PSF with the frame selection of Sect. 3.3: the PSF of frame i is
 * the median (as in graphic_median) of the frames k with
 *   |times_k - times_i| < t_max   and   |parang_k - parang_i| > alpha_min_deg,
 * and a frame whose selection is empty takes the median of all frames.  (The
 * paper prints the minimum rotation as 2 sin(n FWHM / (2 r_min)); callers
 * derive alpha_min_deg as the chord angle 2 arcsin(n FWHM / (2 r_min)).)
 * Frame i never selects itself unless alpha_min_deg < 0 or the fallback applies.
 * graphic_alpha_min_deg gives alpha_min_deg from the paper's parameters.
 *   stack     : [T][N][N] float32, T <= 262144.
 *   times     : [T] float64 observing times (any unit, the unit of t_max).
 *   parang_deg: [T] float64 parallactic angles.
 *   psf_cube  : NULL or [T][N][N] float32, receives PSF_i.
 *   resid     : NULL or [T][N][N] float32, receives stack_i - PSF_i (may be
 *               stack itself; otherwise it must not overlap it).  At least
 *               one of psf_cube and resid is given.
 *   ws        : graphic_workspace_size(GRAPHIC_OP_MEDIAN_WINDOW) bytes (the
 *               selection: T x 512 bytes plus T ints; for T > 2048 also the
 *               row-group plan, one [N][N] image and, for residuals written
 *               with no PSF cube, 2304 [N][N] frames of PSF in waiting).
 * Cost (T <= 2048): one sort of every pixel's T values, then per frame
 * O(T / 64) work per pixel plus the frames that enter or leave the selection.
 * Longer sequences (T > 2048) run in groups of 256 consecutive frames, each
 * sorting only the frames its rows select; the call then waits once for the
 * selection plan (a synchronisation of the stream) and returns
 * GRAPHIC_ERR_UNSUPPORTED, before any output is written, when a group's
 * frames select more than 2048 distinct frames, or, with resid given and
 * psf_cube NULL, when a frame is selected by a frame of a group more than
 * eight groups after its own (local windows, the paper's case, meet both).
 * The plan compares every frame with every other, O(T^2).
 */
graphic_status graphic_median_window(graphic_ctx ctx, const graphic_geom* geom, const float* stack,
                                     const double* times, const double* parang_deg, double t_max,
                                     double alpha_min_deg, float* psf_cube, float* resid,
                                     void* ws, size_t ws_bytes, graphic_stream stream);

/*
 * Minimum field rotation of the frame selection (Sect. 3.3): the angle, in
 * degrees, through which a point at radius r_min (px) turns to move n_fwhm
 * times fwhm (px) along its chord, 2 arcsin(n_fwhm fwhm / (2 r_min)).  (The
 * paper prints 2 sin(...); the chord angle is the reading taken.)  Host-only,
 * needs no context.  Errors: GRAPHIC_ERR_ARG for a null out_deg, non-finite
 * arguments, r_min <= 0, or n_fwhm fwhm outside [0, 2 r_min].
 */
graphic_status graphic_alpha_min_deg(double n_fwhm, double fwhm, double r_min, double* out_deg);

/*
 * ADI reduction with the per-frame PSF of graphic_median_window:
 * S_i = shift(cube_i), R_i = S_i - PSF_i, D_i = rotate(R_i, -parang_i),
 * final = median_i D_i.  Arguments as graphic_adi_reduce, plus the selection
 * (times, t_max, alpha_min_deg) and psf_cube (NULL or [T][N][N]).  T <= 262144,
 * with the same conditions for T > 2048 as graphic_median_window.
 *   ws : graphic_workspace_size(GRAPHIC_OP_ADI_WINDOW) bytes.
 */
graphic_status graphic_adi_reduce_window(graphic_ctx ctx, const graphic_geom* geom, const float* cube,
                                         const double* dx, const double* dy, const double* parang_deg,
                                         const double* times, double t_max, double alpha_min_deg,
                                         float* final_img, float* psf_cube, float* residuals,
                                         void* ws, size_t ws_bytes, graphic_stream stream);

/*
 * Registration (Sect. 3.1).
 *
 * graphic_parallactic_angles: per-frame parallactic angle in degrees from the
 * local sidereal time (seconds), with hour angle h = 15 LST / 3600 - ra_deg:
 *   atan2(cos(lat) sin(h), cos(dec) sin(lat) - sin(dec) cos(lat) cos(h))
 * (the two-argument arctangent fixes the quadrant).  lst_s, out: [T] float64.
 *
 * graphic_register: per frame (one block each), the star centroid and a
 * Moffat fit (Sect. 3.1.2).  The centroid is the centre of mass, weighted by
 * pixel values, of the 4-connected patch of pixels above `threshold` that
 * holds the brightest pixel, grown inside a 64 x 64 box around it; a patch
 * whose size lies outside [min_size, max_size] fails and the brightest pixel
 * stands in.  The fit is least squares of
 *   I0 (beta - 1) / (pi alpha^2) (1 + ((x-x0)^2 + (y-y0)^2) / alpha^2)^-beta + Bg
 * over the (2 half)^2 box around the rounded centroid (clipped to the frame),
 * pixels at or above `saturation` and non-finite pixels masked, by
 * Levenberg-Marquardt in float64 from: Bg = mean of the unmasked box-border
 * pixels, alpha = beta = 2.5, (x0, y0) = centroid, I0 matching the brightest
 * unmasked pixel.  Pixel (x, y) is column x, row y; the recentring shift of
 * graphic_shift is (N/2 - x0, N/2 - y0).  FWHM = 2 alpha sqrt(2^(1/beta) - 1).
 *   cube  : [T][N][N] float32.
 *   out   : [T][12] float64: centroid x, y; x0, y0, I0, alpha, beta, Bg; the
 *           final half sum of squared residuals; the FWHM of the fitted
 *           profile; the recentring shift dx = N/2 - x0, dy = N/2 - y0.
 *   flags : [T] int32: bit 0 centroid patch found, bit 1 fit converged.
 * Errors: GRAPHIC_ERR_ARG for null pointers, half outside 1..32, min_size >
 * max_size or max_iter < 1; geometry errors as graphic_shift.
 */
typedef struct {
    double threshold;            /* patch threshold (frame units) */
    int32_t min_size, max_size;  /* accepted patch sizes in pixels */
    int32_t half;                /* fit box half side, 1..32 */
    int32_t max_iter;            /* Levenberg-Marquardt iterations, >= 1 */
    double saturation;           /* mask level (use +inf for none) */
} graphic_register_params;

graphic_status graphic_parallactic_angles(graphic_ctx ctx, const double* lst_s, int64_t n_frames, double ra_deg,
                                          double dec_deg, double lat_deg, double* out_deg, graphic_stream stream);
graphic_status graphic_register(graphic_ctx ctx, const graphic_geom* geom, const float* cube,
                                const graphic_register_params* params, double* out, int32_t* flags,
                                graphic_stream stream);

/*
 * Image pre-processing (Sect. 3.2).  Frames as graphic_geom (T <= 65535).
 *
 * graphic_median_nan: per-pixel median of a stack ignoring NaN values, as
 *   graphic_median over the values left (the master sky of Sect. 3.2.1 after
 *   the star is masked); a pixel with no value left is NaN.  T <= 4096.
 * graphic_mask_disk: sets to NaN, in place, the pixels of frame i with
 *   (x - xs[i])^2 + (y - ys[i])^2 <= radius^2 (x column, y row; xs, ys [T]
 *   float64).
 * graphic_subtract_nearest: frame_i -= skies[s] in place, s the sky whose
 *   time is closest to times[i] (the earliest on a tie); skies [S][N][N]
 *   float32, sky_times [S] float64, times [T] float64, S >= 1.
 * graphic_badpix_map: bad pixels of one N x N frame (a master dark or sky):
 *   non-finite, or differing from the median of the finite pixels by more
 *   than c_sigma times their standard deviation (float64).  map [N][N] uint8
 *   (1 = bad); stats NULL or [3] float64 (median, mean, sigma).
 *   ws: graphic_workspace_size(GRAPHIC_OP_BADPIX_MAP) bytes (geometry T = 1).
 * graphic_badpix_fix: sets the pixels of `map` (NULL: none) to NaN in every
 *   frame, then fills, pass after pass, every NaN pixel that has non-NaN
 *   8-neighbours with their float32 median, each pass reading the previous
 *   one, until no NaN is left, a pass changes nothing, or max_passes.  The
 *   number of passes that met a NaN goes to *passes (host int, nullable).
 *   Synchronises `stream` after every pass.
 *   ws: graphic_workspace_size(GRAPHIC_OP_BADPIX_FIX) bytes (T N^2 floats
 *   plus flags).
 */
graphic_status graphic_median_nan(graphic_ctx ctx, const graphic_geom* geom, const float* stack, float* out,
                                  graphic_stream stream);
graphic_status graphic_mask_disk(graphic_ctx ctx, const graphic_geom* geom, float* cube, const double* xs,
                                 const double* ys, double radius, graphic_stream stream);
graphic_status graphic_subtract_nearest(graphic_ctx ctx, const graphic_geom* geom, float* cube, const double* times,
                                        const float* skies, const double* sky_times, int32_t n_skies,
                                        graphic_stream stream);
graphic_status graphic_badpix_map(graphic_ctx ctx, int32_t n, const float* frame, double c_sigma, uint8_t* map,
                                  double* stats, void* ws, size_t ws_bytes, graphic_stream stream);
graphic_status graphic_badpix_fix(graphic_ctx ctx, const graphic_geom* geom, float* cube, const uint8_t* map,
                                  int32_t max_passes, int32_t* passes, void* ws, size_t ws_bytes,
                                  graphic_stream stream);

/*
 * Image-quality test (Sect. 4.1): the paper shifts an image by (3.5, 2.7) px
 * and back, or rotates it by 11.3 deg and back, subtracts the original and
 * plots the root mean square of the difference in concentric annuli.  The
 * round trips are graphic_shift / graphic_rotate calls; this entry point
 * measures the difference.
 *
 * graphic_annular_rms: for every frame t of the [T][N][N] float32 stack a
 *   (geometry as graphic_geom, pad ignored; T <= 65535), the RMS of
 *   a[t] - b[t] (b NULL: of a[t]; else the same shape as a) over each annulus
 *   k = 0 .. n_rings - 1 of width `width` px around (cx, cy): the pixels
 *   (x, y), x the column, with (k width)^2 <= (x - cx)^2 + (y - cy)^2 <
 *   ((k + 1) width)^2, compared in float64 without a square root.  Sums are
 *   float64.  rms [T][n_rings] float64 device memory (NaN for an annulus
 *   with no pixel); counts [n_rings] int64 device memory (pixels per
 *   annulus).  1 <= n_rings <= 4096; width, cx and cy finite, width > 0 and
 *   (|cx| + |cy| + 2N) / width < 2^30.  The sums are float64 atomics, so
 *   repeated calls agree to rounding, not bit for bit.
 */
graphic_status graphic_annular_rms(graphic_ctx ctx, const graphic_geom* geom, const float* a, const float* b,
                                   double cx, double cy, double width, int32_t n_rings, double* rms, int64_t* counts,
                                   graphic_stream stream);

/*
 * Batched ADI reduction of cubes of uneven frame count and size (the
 * classical reduction of graphic_adi_reduce applied to every cube).  Cubes
 * with the same N and P form a size class; every line pass of a class runs
 * over the frames of up to 16 of its cubes in one launch, and the rotation
 * works through the concatenated frames of the class in chunks that may span
 * cubes.  The results are bitwise identical to one graphic_adi_reduce call
 * per cube.  Each cube is described by a graphic_cube_desc (host array,
 * device pointers).
 *   flags : 0, or GRAPHIC_BATCH_INPLACE to use each cube's input array as its
 *           working stack (the input is overwritten with the derotated
 *           residuals); otherwise the stack goes to `residuals` if given, or
 *           to the workspace.
 *   ws    : graphic_batch_workspace_size() bytes; a smaller workspace (down
 *           to the stacks, PSFs and one working frame) makes the rotation
 *           use smaller chunks.
 */
#define GRAPHIC_BATCH_INPLACE 1u

typedef struct {
    const float* cube;          /* [T][N][N] float32 */
    int64_t n_frames;           /* T, 1 <= T <= 2^24 */
    int32_t n, pad;             /* N and P as in graphic_geom */
    const double* dx;           /* [T] recentring shifts */
    const double* dy;           /* [T] */
    const double* parang_deg;   /* [T] parallactic angles; frames are derotated by -parang */
    float* final_img;           /* [N][N] output */
    float* psf;                 /* NULL or [N][N] output */
    float* residuals;           /* NULL or [T][N][N] output (derotated residuals) */
} graphic_cube_desc;

graphic_status graphic_batch_workspace_size(graphic_ctx ctx, const graphic_cube_desc* descs, int n_cubes,
                                            uint32_t flags, size_t* bytes);

graphic_status graphic_adi_reduce_batch(graphic_ctx ctx, const graphic_cube_desc* descs, int n_cubes,
                                        uint32_t flags, void* ws, size_t ws_bytes, graphic_stream stream);

/* Captured pipelines (HIP graphs).
 *
 * graphic_adi_graph_create records every launch that graphic_adi_reduce_batch
 * would make for these descriptors, workspace and flags into a HIP graph
 * (stream capture on a library-owned stream), and instantiates it.
 * graphic_graph_launch replays the whole reduction on `stream` with one call:
 * same shapes, same device pointers, current contents.  To reduce new data,
 * write it into the same cube buffers (and parameter arrays) before the
 * launch.  The caller keeps every buffer named by the descriptors and the
 * workspace alive and unmoved until graphic_graph_destroy; replays that
 * overlap on the device race on those buffers.  Errors: the argument checks
 * of graphic_adi_reduce_batch, made before anything is captured;
 * GRAPHIC_ERR_HIP if capture or instantiation fails.  Kernel timing is off
 * inside a captured graph.  The graph holds no memsets. */
typedef struct graphic_graph_s* graphic_graph;

graphic_status graphic_adi_graph_create(graphic_ctx ctx, const graphic_cube_desc* descs, int n_cubes,
                                        uint32_t flags, void* ws, size_t ws_bytes, graphic_graph* graph);
graphic_status graphic_graph_launch(graphic_graph graph, graphic_stream stream);
void graphic_graph_destroy(graphic_graph graph);

/* Autotuning of launch shapes.
 *
 * graphic_autotune times the library's alternative launch shapes for a
 * geometry on the caller's device -- the tile width (jobs per block) of the
 * column passes for both line pairings, and the pixel tile (16 or 8) of the
 * median for this frame count, in the frame-major layout and, for the sizes
 * whose ADI workspace stack is tile-major (P = 2N, N = 1024), in that
 * layout too -- and keeps the fastest in the context; later
 * calls with that geometry use them.  Every variant computes bit-identical
 * results.  It overwrites `ws` with synthetic frames and synchronises
 * `stream`.  Each kernel is timed at the size of one launch of the pipeline
 * (the whole cube for the shift's column pass, one rotation chunk for the
 * y-shear, the whole stack for the median, with and without the residual
 * rewrite), or on as much of it as `ws` holds; a kernel whose data does not
 * fit (fewer than 8 frames, or 16384 pixels) keeps its default.  The ADI
 * workspace of the same geometry (graphic_workspace_size) covers every
 * kernel at full size.  Errors: GRAPHIC_ERR_ARG / _UNSUPPORTED for the geometry,
 * GRAPHIC_ERR_WORKSPACE for a null or misaligned `ws`, GRAPHIC_ERR_HIP.
 *
 * graphic_tuning_export writes the tuned choices as text (one "col M pairing
 * variant", "med class variant" or "tmm class variant" line each, class =
 * ceil(log2(ceil(T / 64)))) into buf (with its NUL; the
 * length needed, NUL included, goes to *needed; a short buffer gets a
 * truncated copy and GRAPHIC_ERR_ARG); graphic_tuning_import reads such text
 * back (all or nothing: a malformed line leaves the context unchanged and
 * returns GRAPHIC_ERR_ARG), so that choices can be cached across processes. */
graphic_status graphic_autotune(graphic_ctx ctx, const graphic_geom* geom, void* ws, size_t ws_bytes,
                                graphic_stream stream);
graphic_status graphic_tuning_export(graphic_ctx ctx, char* buf, size_t buf_len, size_t* needed);
graphic_status graphic_tuning_import(graphic_ctx ctx, const char* text);

/* Per-kernel timing with HIP events on the caller's stream (for benchmarks).
 * When enabled, every library kernel launch is bracketed by events; the
 * accumulated milliseconds and launch counts per kernel family are read with
 * graphic_timing_read after the stream has been synchronised.  Families:
 * "shift_y", "shift_x" (the two shift passes), "shear_x1", "shear_y",
 * "shear_x2" (the three rotation passes), "median" and "aux" (per-frame
 * parameters and flux sums).  Enabling (or disabling) clears the counters. */
graphic_status graphic_timing_enable(graphic_ctx ctx, int enable);
graphic_status graphic_timing_read(graphic_ctx ctx, const char* family,
                                   double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GRAPHIC_H */
