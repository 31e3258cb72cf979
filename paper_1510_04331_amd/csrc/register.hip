// Registration (Sect. 3.1): parallactic angles, star centroid and Moffat fit.
//
// One block of 256 threads registers one frame:
//   1. the brightest pixel (non-finite values never win; ties go to the first
//      pixel in row-major order);
//   2. the 4-connected patch of pixels above the threshold that holds it,
//      grown inside a 64 x 64 box in LDS, and the patch's centre of mass
//      weighted by pixel values (a patch size outside [min, max] fails and
//      the brightest pixel stands in);
//   3. a least-squares fit of the Moffat profile of Sect. 3.1.2,
//        I0 (beta - 1) / (pi alpha^2) (1 + r^2 / alpha^2)^-beta + Bg,
//      over a (2 half)^2 box around the rounded centroid, saturated and
//      non-finite pixels masked, by Levenberg-Marquardt in float64 with
//      analytic derivatives (Marquardt's diagonal scaling of the damping).
// The starting point: background = mean of the unmasked box-border pixels,
// alpha = beta = 2.5, centre = centroid, I0 matching the brightest unmasked
// pixel above the background.

#include <cmath>

#include "internal.h"

namespace graphic {

namespace {

constexpr int kRegThreads = 256;
constexpr int kBox = 64;                 // centroid search box
constexpr int kMaxFit = 64;              // largest fit box side (half <= 32)
constexpr int kNJ = 6;                   // fit parameters
constexpr int kNSum = 21 + 6 + 1;        // upper triangle of J^T J, J^T r, cost

__device__ __forceinline__ void box_range(int n, int c, int side, int& lo, int& hi) {
  lo = c - side / 2;
  if (side <= n) {
    lo = lo < 0 ? 0 : lo;
    lo = lo > n - side ? n - side : lo;
  } else {
    lo = 0;
  }
  hi = lo + side < n ? lo + side : n;
}

// Block sum of K doubles per thread (result valid in thread 0).
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red /* [4][K] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    v[k] = x;
  }
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = red[k] + red[K + k] + red[2 * K + k] + red[3 * K + k];
  __syncthreads();
}

struct FitPixel {
  float x, y, v;                           // x < 0 marks a masked pixel
};

// Model value and derivatives with respect to (I0, x0, y0, alpha, beta, Bg).
__device__ __forceinline__ double moffat_grad(const double* p, double x, double y, double* d) {
  const double i0 = p[0], xc = p[1], yc = p[2], a = p[3], b = p[4], bg = p[5];
  const double dx = xc - x, dy = yc - y;
  const double r2 = dx * dx + dy * dy;
  const double a2 = a * a;
  const double u = 1.0 + r2 / a2;
  const double upb = pow(u, -b);
  const double A = (b - 1.0) / (M_PI * a2);
  const double f = i0 * A * upb;
  d[0] = A * upb;
  d[1] = -2.0 * b * f * dx / (a2 * u);
  d[2] = -2.0 * b * f * dy / (a2 * u);
  d[3] = f * (-2.0 / a + 2.0 * b * r2 / (a2 * a * u));
  d[4] = f * (1.0 / (b - 1.0) - log(u));
  d[5] = 1.0;
  return f + bg;
}

__device__ __forceinline__ double moffat_val(const double* p, double x, double y) {
  const double dx = p[1] - x, dy = p[2] - y;
  const double a2 = p[3] * p[3];
  return p[0] * (p[4] - 1.0) / (M_PI * a2) * pow(1.0 + (dx * dx + dy * dy) / a2, -p[4]) + p[5];
}

// Solves (A + lam diag(A)) x = -g for a symmetric 6 x 6 A (upper triangle
// packed row by row) by Cholesky; false if not positive definite.
__device__ bool damped_solve(const double* Ap, const double* g, double lam, double* x) {
  double L[kNJ][kNJ];
  int k = 0;
  for (int i = 0; i < kNJ; ++i)
    for (int j = i; j < kNJ; ++j) {
      L[i][j] = Ap[k];
      L[j][i] = Ap[k];
      ++k;
    }
  for (int i = 0; i < kNJ; ++i) L[i][i] *= 1.0 + lam;
  for (int j = 0; j < kNJ; ++j) {
    double s = L[j][j];
    for (int m = 0; m < j; ++m) s -= L[j][m] * L[j][m];
    if (!(s > 0.0)) return false;
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < kNJ; ++i) {
      double t = L[i][j];
      for (int m = 0; m < j; ++m) t -= L[i][m] * L[j][m];
      L[i][j] = t / L[j][j];
    }
  }
  double y[kNJ];
  for (int i = 0; i < kNJ; ++i) {
    double t = -g[i];
    for (int m = 0; m < i; ++m) t -= L[i][m] * y[m];
    y[i] = t / L[i][i];
  }
  for (int i = kNJ - 1; i >= 0; --i) {
    double t = y[i];
    for (int m = i + 1; m < kNJ; ++m) t -= L[m][i] * x[m];
    x[i] = t / L[i][i];
  }
  return true;
}

__global__ void __launch_bounds__(kRegThreads)
register_kernel(const float* __restrict__ cube, long long T, int n, RegisterParams prm, double* __restrict__ out,
                int* __restrict__ flags) {
  // the centroid box and labels are dead once the fit pixels are loaded
  __shared__ __align__(16) unsigned char s_raw[kMaxFit * kMaxFit * sizeof(FitPixel)];
  float* s_box = reinterpret_cast<float*>(s_raw);
  unsigned char* s_lab = s_raw + kBox * kBox * sizeof(float);
  FitPixel* s_fit = reinterpret_cast<FitPixel*>(s_raw);
  static_assert(kBox * kBox * (sizeof(float) + 1) <= sizeof(s_raw), "centroid box fits the shared buffer");
  __shared__ double s_red[4 * kNSum];
  __shared__ float s_bv[4];
  __shared__ int s_bi[4];
  __shared__ int s_changed[3];
  __shared__ double s_p[kNJ], s_trial[kNJ];
  __shared__ int s_ctl[2];               // [0]: iteration go on, [1]: accepted

  const long long f = blockIdx.x;
  const float* fr = cube + (size_t)f * n * n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long npix = (long long)n * n;

  // ---- 1. brightest pixel (first in row-major order among equals) ----
  float bv = -INFINITY;
  int bi = 0x7fffffff;
  for (long long i = tid; i < npix; i += kRegThreads) {
    float v = fr[i];
    v = isfinite(v) ? v : -INFINITY;
    if (v > bv || (v == bv && (int)i < bi)) {
      bv = v;
      bi = (int)i;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(bv, o);
    const int oi = __shfl_xor(bi, o);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    s_bv[wave] = bv;
    s_bi[wave] = bi;
  }
  __syncthreads();
  bv = s_bv[0];
  bi = s_bi[0];
  for (int w = 1; w < 4; ++w)
    if (s_bv[w] > bv || (s_bv[w] == bv && s_bi[w] < bi)) {
      bv = s_bv[w];
      bi = s_bi[w];
    }
  if (bi == 0x7fffffff) bi = 0;          // every pixel non-finite
  const int iy = bi / n, ix = bi % n;

  // ---- 2. patch above the threshold holding the brightest pixel ----
  int by0, by1, bx0, bx1;
  box_range(n, iy, kBox, by0, by1);
  box_range(n, ix, kBox, bx0, bx1);
  const int bw = bx1 - bx0, bh = by1 - by0;
  for (int i = tid; i < kBox * kBox; i += kRegThreads) {
    const int r = i / kBox, c = i % kBox;
    float v = -INFINITY;
    if (r < bh && c < bw) {
      v = fr[(size_t)(by0 + r) * n + (bx0 + c)];
      v = isfinite(v) ? v : -INFINITY;
    }
    s_box[i] = v;
    s_lab[i] = 0;
  }
  if (tid < 3) s_changed[tid] = 0;
  __syncthreads();
  const int seed = (iy - by0) * kBox + (ix - bx0);
  const bool seeded = (double)s_box[seed] > prm.threshold;
  if (tid == 0 && seeded) s_lab[seed] = 1;
  __syncthreads();
  // grow to the fixed point (labels only turn on, so concurrent updates only
  // delay convergence); bounded by the box size
  if (seeded) {
    for (int it = 0; it < kBox * kBox; ++it) {
      if (tid == 0) s_changed[(it + 1) % 3] = 0;
      bool ch = false;
      for (int i = tid; i < kBox * kBox; i += kRegThreads) {
        if (s_lab[i] || !((double)s_box[i] > prm.threshold)) continue;
        const int r = i / kBox, c = i % kBox;
        const bool nb = (c > 0 && s_lab[i - 1]) || (c + 1 < kBox && s_lab[i + 1]) || (r > 0 && s_lab[i - kBox]) ||
                        (r + 1 < kBox && s_lab[i + kBox]);
        if (nb) {
          s_lab[i] = 1;
          ch = true;
        }
      }
      if (ch) s_changed[it % 3] = 1;
      __syncthreads();
      const bool any = s_changed[it % 3] != 0;
      __syncthreads();
      if (!any) break;
    }
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};   // size, sum v, sum v x, sum v y
  for (int i = tid; i < kBox * kBox; i += kRegThreads)
    if (s_lab[i]) {
      const double v = s_box[i];
      acc[0] += 1.0;
      acc[1] += v;
      acc[2] += v * (double)(bx0 + i % kBox);
      acc[3] += v * (double)(by0 + i / kBox);
    }
  block_sum<4>(acc, s_red);
  __shared__ double s_c[2];
  __shared__ int s_cok;
  if (tid == 0) {
    const bool ok = seeded && acc[0] >= (double)prm.min_size && acc[0] <= (double)prm.max_size;
    s_c[0] = ok ? acc[2] / acc[1] : (double)ix;
    s_c[1] = ok ? acc[3] / acc[1] : (double)iy;
    s_cok = ok ? 1 : 0;
  }
  __syncthreads();
  const double cx = s_c[0], cy = s_c[1];

  // ---- 3. Moffat fit ----
  const int side = 2 * prm.half;
  int fy0, fy1, fx0, fx1;
  box_range(n, (int)rint(cx), side, fx0, fx1);
  box_range(n, (int)rint(cy), side, fy0, fy1);
  const int fw = fx1 - fx0, fh = fy1 - fy0;
  __syncthreads();                         // the centroid box is dead from here
  double st[3] = {0.0, 0.0, 0.0};          // border count, border sum
  double vmax = -INFINITY;
  for (int i = tid; i < fw * fh; i += kRegThreads) {
    const int r = i / fw, c = i % fw;
    const float v = fr[(size_t)(fy0 + r) * n + (fx0 + c)];
    const bool masked = !isfinite(v) || (double)v >= prm.saturation;
    s_fit[i] = FitPixel{masked ? -1.0f : (float)(fx0 + c), (float)(fy0 + r), v};
    if (masked) continue;
    if (r == 0 || r == fh - 1 || c == 0 || c == fw - 1) {
      st[0] += 1.0;
      st[1] += v;
    }
    vmax = v > vmax ? v : vmax;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(vmax, o);
    vmax = ov > vmax ? ov : vmax;
  }
  __shared__ double s_vmax[4];
  if (lane == 0) s_vmax[wave] = vmax;
  block_sum<3>(st, s_red);
  if (tid == 0) {
    double m = s_vmax[0];
    for (int w = 1; w < 4; ++w) m = s_vmax[w] > m ? s_vmax[w] : m;
    const double bg = st[0] > 0.0 ? st[1] / st[0] : 0.0;
    s_p[0] = (m - bg) * M_PI * 2.5 * 2.5 / 1.5;
    s_p[1] = cx;
    s_p[2] = cy;
    s_p[3] = 2.5;
    s_p[4] = 2.5;
    s_p[5] = bg;
    s_ctl[0] = 1;
    s_ctl[1] = 1;
  }
  __syncthreads();
  const int nfit = fw * fh;
  double lam = 1e-3, cost = 0.0;            // thread 0's solver state
  double Ap[21], g[kNJ];
  bool converged = false;
  for (int it = 0; it < prm.max_iter; ++it) {
    if (s_ctl[1]) {                         // accepted step (or start): normal equations at s_p
      double sum[kNSum];
#pragma unroll
      for (int k = 0; k < kNSum; ++k) sum[k] = 0.0;
      for (int i = tid; i < nfit; i += kRegThreads) {
        double d[kNJ];
        const FitPixel q = s_fit[i];
        if (q.x < 0.0f) continue;
        const double r = moffat_grad(s_p, q.x, q.y, d) - q.v;
        int k = 0;
#pragma unroll
        for (int a = 0; a < kNJ; ++a)
#pragma unroll
          for (int b = a; b < kNJ; ++b) sum[k++] += d[a] * d[b];
#pragma unroll
        for (int a = 0; a < kNJ; ++a) sum[21 + a] += d[a] * r;
        sum[27] += 0.5 * r * r;
      }
      block_sum<kNSum>(sum, s_red);
      if (tid == 0) {
        for (int k = 0; k < 21; ++k) Ap[k] = sum[k];
        for (int a = 0; a < kNJ; ++a) g[a] = sum[21 + a];
        cost = sum[27];
      }
    }
    if (tid == 0) {
      double dx[kNJ] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      bool solved = damped_solve(Ap, g, lam, dx);
      while (!solved && lam < 1e30) {
        lam *= 10.0;
        solved = damped_solve(Ap, g, lam, dx);
      }
      if (!solved)
        for (int a = 0; a < kNJ; ++a) dx[a] = 0.0;
      for (int a = 0; a < kNJ; ++a) s_trial[a] = s_p[a] + dx[a];
    }
    __syncthreads();
    double tc[1] = {0.0};
    for (int i = tid; i < nfit; i += kRegThreads) {
      const FitPixel q = s_fit[i];
      if (q.x < 0.0f) continue;
      const double r = moffat_val(s_trial, q.x, q.y) - q.v;
      tc[0] += 0.5 * r * r;
    }
    block_sum<1>(tc, s_red);
    if (tid == 0) {
      const bool better = tc[0] < cost && isfinite(tc[0]);
      double step = 0.0, size = 0.0;
      for (int a = 0; a < kNJ; ++a) {
        step = fmax(step, fabs(s_trial[a] - s_p[a]));
        size = fmax(size, fabs(s_p[a]));
      }
      if (better) {
        const double gain = cost - tc[0];
        for (int a = 0; a < kNJ; ++a) s_p[a] = s_trial[a];
        lam = fmax(lam * 0.1, 1e-15);
        if (gain <= 1e-15 * cost || step <= 1e-13 * (size + 1e-300)) converged = true;
        cost = tc[0];
      } else {
        lam *= 10.0;
        if (lam > 1e20 || step <= 1e-13 * (size + 1e-300)) converged = true;
      }
      s_ctl[0] = converged ? 0 : 1;
      s_ctl[1] = better ? 1 : 0;
    }
    __syncthreads();
    if (!s_ctl[0]) break;
  }
  if (tid == 0) {
    double* o = out + f * kRegisterOut;
    o[0] = cx;
    o[1] = cy;
    o[2] = s_p[1];
    o[3] = s_p[2];
    o[4] = s_p[0];
    o[5] = s_p[3];
    o[6] = s_p[4];
    o[7] = s_p[5];
    o[8] = cost;
    // FWHM of the fitted Moffat profile (Sect. 3.1.2): the radius where the
    // profile falls to half its peak, doubled
    o[9] = 2.0 * s_p[3] * sqrt(exp2(1.0 / s_p[4]) - 1.0);
    // recentring shift that brings the fitted centre to pixel (N/2, N/2)
    o[10] = 0.5 * (double)n - s_p[1];
    o[11] = 0.5 * (double)n - s_p[2];
    flags[f] = (s_cok ? 1 : 0) | (converged ? 2 : 0);
  }
}

__global__ void parallactic_kernel(const double* __restrict__ lst_s, long long T, double ra_deg, double dec_deg,
                                   double lat_deg, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const double d2r = M_PI / 180.0;
  const double h = (15.0 * lst_s[i] / 3600.0 - ra_deg) * d2r;
  const double d = dec_deg * d2r, p = lat_deg * d2r;
  out[i] = atan2(cos(p) * sin(h), cos(d) * sin(p) - sin(d) * cos(p) * cos(h)) / d2r;
}

}  // namespace

hipError_t launch_register(const float* cube, long long T, int n, const RegisterParams& prm, double* out,
                           int* flags, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(register_kernel, dim3((unsigned)T), dim3(kRegThreads), 0, s, cube, T, n, prm, out, flags);
  return hipGetLastError();
}

hipError_t launch_parallactic(const double* lst_s, long long T, double ra_deg, double dec_deg, double lat_deg,
                              double* out, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(parallactic_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, lst_s, T, ra_deg,
                     dec_deg, lat_deg, out);
  return hipGetLastError();
}

}  // namespace graphic
