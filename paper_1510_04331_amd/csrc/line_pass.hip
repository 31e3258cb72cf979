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
// Ma lanes; every lane holds Mb complex values.
//
// Phasor: bin k of the length-P transform (signed index kt) gets
// exp(-2 pi i kt s / P); the Nyquist bin gets cos(pi s).  The phase kt*s/P is
// formed and reduced modulo one in float64 as kt = (2 k2 + h) + 2 Mb k1' with
// a per-lane factor for (2 k2 + h) and a per-job table over k1', each entry
// evaluated from its own float64-reduced phase.

#include "dft_codelets.h"
#include "internal.h"

namespace graphic {

template <int M>
struct Shape {
  static constexpr int lg = __builtin_ctz(M);
  static constexpr int Ma = 1 << (lg / 2);
  static constexpr int Mb = M / Ma;
  static constexpr int JOB = 2 * Ma;
  static constexpr int ROWP = Ma + 1;                  // padded LDS row (complex)
  static constexpr int HALF = Mb * ROWP;               // complex per half-job
  static constexpr int PER_JOB = 2 * HALF + Ma;        // + phasor table
  static_assert(Mb == Ma || Mb == 2 * Ma, "square or 1:2 four-step split");
};

// float64 reduction of kk * q modulo one, then float32 sin/cos of the residue.
__device__ __forceinline__ cf phase_exp(double kk, double q, float scale) {
  double ph = kk * q;
  ph = ph - rint(ph);                       // |ph| <= 1/2 cycle
  float a = (float)(ph * -6.283185307179586476925);
  float sn, cs;
  sincosf(a, &sn, &cs);
  return {cs * scale, sn * scale};
}

// Occupancy target (waves per SIMD) that bounds the register budget; the LDS
// footprint (about 17 KB per wave for M >= 512) allows no more than this.
template <int M>
constexpr int waves_per_eu() {
  return M <= 1024 ? 4 : 2;
}

template <int M, int KIND, int G>
__global__ void __launch_bounds__(G * Shape<M>::JOB, waves_per_eu<M>())
line_pass_kernel(const LinePass p) {
  using S = Shape<M>;
  constexpr int Ma = S::Ma, Mb = S::Mb, JOB = S::JOB;
  extern __shared__ float2 lds_raw[];
  cf* lds = reinterpret_cast<cf*>(lds_raw);

  const int tid = threadIdx.x;
  int jl, r;
  if constexpr (KIND == kRowPass) {
    jl = tid / JOB;
    r = tid % JOB;
  } else {
    jl = tid % G;
    r = tid / G;
  }
  const int h = r / Ma;        // 0: even bins, 1: odd bins
  const int n1 = r % Ma;

  // LDS addressing: (job, half, row k2, column n1); the column kernel keeps the
  // job index fastest so that lanes of one wave (consecutive jobs) hit
  // consecutive words.
  auto lidx = [&](int hh, int k2, int c) -> int {
    if constexpr (KIND == kRowPass)
      return (jl * 2 + hh) * S::HALF + k2 * S::ROWP + c;
    else
      return ((hh * Mb + k2) * S::ROWP + c) * G + jl;
  };
  auto tidx = [&](int k1) -> int {   // phasor table of the job
    if constexpr (KIND == kRowPass)
      return G * 2 * S::HALF + jl * Ma + k1;
    else
      return G * 2 * S::HALF + k1 * G + jl;
  };

  // XCD-aware block order: the hardware deals consecutive block ids to the
  // eight XCDs in turn; remap so that each XCD walks a contiguous range of jobs
  // (neighbouring lines share cache lines in its L2).
  long long nb = gridDim.x;
  long long b = blockIdx.x;
  long long per = (nb + 7) / 8;
  long long lb = (b % 8) * per + b / 8;
  if (nb % 8 != 0) lb = b;   // keep it simple when the grid does not split evenly

  const long long total = p.n_frames * (long long)p.n_jobs;
  const long long gj = lb * G + jl;
  const bool job_ok = gj < total;
  const long long f = job_ok ? gj / p.n_jobs : 0;
  const int j = job_ok ? (int)(gj % p.n_jobs) : 0;

  const int P = p.P;
  const int c = P / 2;
  const int flipf = (p.flip != nullptr && job_ok) ? (p.flip[f] != 0) : 0;
  const int line_lo = p.line_lo + (p.flip_lines ? flipf : 0);
  // Line coordinates are periodic (mod P): with P = N a half-turned frame's
  // support wraps, and padded line P is line 0 (shift -c * coef).
  int la, lb2;
  bool b_exists = true;
  if (p.mirror) {
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
  double s = 0.0;
  if (job_ok) {
    if (p.sh0) s += p.sh0[f];
    if (p.sh1) s += p.sh1[f] * (double)(la - c);
  }
  const double q = s / (double)P;

  const int in_off = p.in_off + (p.flip_in_off ? flipf : 0);
  const int L = p.in_len;
  const int R = 2 * in_off + L - 1;
  const bool rev = p.flip_src_reverse && flipf;
  const int lia = rev ? (p.n_lines - 1 - ra) : ra;
  const int lib = rev ? (p.n_lines - 1 - rb) : rb;
  const float* srcf = p.src + f * p.src_fs;
  const float* rowa = srcf + (long long)lia * p.src_ls;
  const float* rowb = srcf + (long long)lib * p.src_ls;
  const float* suba = p.sub ? p.sub + (long long)lia * p.sub_ls : nullptr;
  const float* subb = p.sub ? p.sub + (long long)lib * p.sub_ls : nullptr;
  const bool rev_b = p.mirror ? !rev : rev;

  // ---- per-job phasor table over k1 (written now, read after the transpose) ----
  if (h == 0) {
    const int k1s = n1 < Ma / 2 ? n1 : n1 - Ma;
    lds[tidx(n1)] = phase_exp((double)(2 * Mb) * (double)k1s, q, 1.0f / (float)P);
  }

  // ---- load, pack and fold into this half's branch ----
  cf v[Mb];
#pragma unroll
  for (int n2 = 0; n2 < Mb; ++n2) {
    const int m = n1 + Ma * n2;
    cf z[2];
#pragma unroll
    for (int cnd = 0; cnd < 2; ++cnd) {
      const int n = m + cnd * M;
      const int u = (n - in_off + P) & (P - 1);
      float av = 0.f, bv = 0.f;
      if (u < L) {
        const int pa = rev ? (L - 1 - u) : u;
        const int pb = rev_b ? (L - 1 - u) : u;
        if (a_ok) {
          av = rowa[(long long)pa * p.src_ps];
          if (suba) av -= suba[(long long)pa * p.sub_ps];
        }
        if (b_ok) {
          bv = rowb[(long long)pb * p.src_ps];
          if (subb) bv -= subb[(long long)pb * p.sub_ps];
        }
      }
      z[cnd] = {av, bv};
    }
    const float2 w = p.tw.fold[h * M + m];
    const cf x = h ? csub(z[0], z[1]) : cadd(z[0], z[1]);
    v[n2] = cmul(x, {w.x, w.y});
  }

  // ---- step A: length-Mb transforms over n2, twiddle, transpose ----
  Dft<Mb, -1>::run(v);
#pragma unroll
  for (int k2 = 0; k2 < Mb; ++k2) {
    const float2 w = p.tw.fwd[k2 * Ma + n1];
    lds[lidx(h, k2, n1)] = cmul(v[k2], {w.x, w.y});
  }
  __syncthreads();

  // ---- step C: length-Ma transforms over n1, phasor, inverse, twiddle ----
  constexpr int NQ = Mb / Ma;
#pragma unroll
  for (int qq = 0; qq < NQ; ++qq) {
    const int k2 = n1 + Ma * qq;
    cf w[Ma];
#pragma unroll
    for (int c1 = 0; c1 < Ma; ++c1) w[c1] = lds[lidx(h, k2, c1)];
    Dft<Ma, -1>::run(w);
    const cf tlo = phase_exp((double)(2 * k2 + h), q, 1.0f);
    const bool nyq_lane = (h == 0) && (k2 == 0);
#pragma unroll
    for (int k1 = 0; k1 < Ma; ++k1) {
      cf ph = cmul(tlo, lds[tidx(k1)]);
      if (k1 == Ma / 2 && nyq_lane) ph.y = 0.f;   // real, symmetric Nyquist term
      w[k1] = cmul(w[k1], ph);
    }
    Dft<Ma, +1>::run(w);
#pragma unroll
    for (int c1 = 0; c1 < Ma; ++c1) v[qq * Ma + c1] = w[c1];
  }
  __syncthreads();
#pragma unroll
  for (int qq = 0; qq < NQ; ++qq) {
    const int k2 = n1 + Ma * qq;
#pragma unroll
    for (int c1 = 0; c1 < Ma; ++c1) {
      const float2 t = p.tw.inv[c1 * Mb + k2];
      lds[lidx(h, k2, c1)] = cmul(v[qq * Ma + c1], {t.x, t.y});
    }
  }
  __syncthreads();

  // ---- step A': length-Mb inverse transforms over k2 ----
#pragma unroll
  for (int k2 = 0; k2 < Mb; ++k2) v[k2] = lds[lidx(h, k2, n1)];
  Dft<Mb, +1>::run(v);
  __syncthreads();

  // ---- unfold: combine the even- and odd-bin halves ----
#pragma unroll
  for (int n2 = 0; n2 < Mb; ++n2) lds[lidx(h, n2, n1)] = v[n2];
  __syncthreads();

  const int dst_lo = p.dst_line_lo + (p.flip_lines ? flipf : 0);
  const int out_line_a = (la - dst_lo + P) & (P - 1);
  const int out_line_b = (lb2 - dst_lo + P) & (P - 1);
  float* dstf = p.dst + f * p.dst_fs;
  float* oa = dstf + (long long)out_line_a * p.dst_ls;
  float* ob = dstf + (long long)out_line_b * p.dst_ls;
#pragma unroll
  for (int n2 = 0; n2 < Mb; ++n2) {
    const int m = n1 + Ma * n2;
    const cf oth = lds[lidx(1 - h, n2, n1)];
    const cf own = v[n2];
    const float2 t = p.tw.fold[M + m];
    const cf e = h ? oth : own;
    const cf o = h ? own : oth;
    const cf wo = cmulc(o, {t.x, t.y});               // o * exp(+2 pi i m / P)
    const cf y = h ? csub(e, wo) : cadd(e, wo);
    const int n = m + h * M;
    const int ua = n - p.out_off;
    if (a_ok && ua >= 0 && ua < p.out_len) oa[(long long)ua * p.dst_ps] = y.x;
    if (b_ok) {
      const int nb_ = p.mirror ? ((R - n) % P + P) % P : n;
      const int ub = nb_ - p.out_off;
      if (ub >= 0 && ub < p.out_len) ob[(long long)ub * p.dst_ps] = y.y;
    }
  }
}

// ---------------------------------------------------------------------------
// Launch
// ---------------------------------------------------------------------------

template <int M>
constexpr int col_jobs_per_block() {
  using S = Shape<M>;
  constexpr int budget = 140 * 1024;
  int g = 16;
  while (g > 1 && (g * S::PER_JOB * 8 > budget || g * S::JOB > 1024)) g /= 2;
  return g;
}

template <int M>
constexpr int row_jobs_per_block() {
  return 64 / Shape<M>::JOB > 0 ? 64 / Shape<M>::JOB : 1;
}

template <int M>
static hipError_t launch_m(const LinePass& p, int kind, hipStream_t st) {
  using S = Shape<M>;
  const long long total = p.n_frames * (long long)p.n_jobs;
  if (kind == kRowPass) {
    constexpr int G = row_jobs_per_block<M>();
    const long long blocks = (total + G - 1) / G;
    const size_t lds = (size_t)G * S::PER_JOB * sizeof(cf);
    hipFuncSetAttribute((const void*)line_pass_kernel<M, kRowPass, G>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((line_pass_kernel<M, kRowPass, G>), dim3((unsigned)blocks), dim3(G * S::JOB),
                       lds, st, p);
  } else {
    constexpr int G = col_jobs_per_block<M>();
    const long long blocks = (total + G - 1) / G;
    const size_t lds = (size_t)G * S::PER_JOB * sizeof(cf);
    hipFuncSetAttribute((const void*)line_pass_kernel<M, kColPass, G>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((line_pass_kernel<M, kColPass, G>), dim3((unsigned)blocks), dim3(G * S::JOB),
                       lds, st, p);
  }
  return hipGetLastError();
}

hipError_t launch_line_pass(const LinePass& p, int kind, int /*jobs_per_block*/, hipStream_t s) {
  const long long total = p.n_frames * (long long)p.n_jobs;
  if (total <= 0) return hipSuccess;
  switch (p.P / 2) {
    case 8: return launch_m<8>(p, kind, s);
    case 16: return launch_m<16>(p, kind, s);
    case 32: return launch_m<32>(p, kind, s);
    case 64: return launch_m<64>(p, kind, s);
    case 128: return launch_m<128>(p, kind, s);
    case 256: return launch_m<256>(p, kind, s);
    case 512: return launch_m<512>(p, kind, s);
    case 1024: return launch_m<1024>(p, kind, s);
    case 2048: return launch_m<2048>(p, kind, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace graphic
