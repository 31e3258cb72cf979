// Register-resident DFT codelets for gfx950 (wave64).
//
// A codelet transforms L complex float32 values held in one lane's VGPRs,
// natural order in and out, with compile-time twiddles.  It is a mixed
// radix-4 / radix-2 decimation-in-time recursion; twiddles that are
// multiples of pi/4 are applied with sign changes, swaps or one scaling.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace graphic {

struct cf {
  float x, y;
};

__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cf cmul(cf a, cf b) {
  return {fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
__device__ __forceinline__ cf cmulc(cf a, cf b) {
  return {fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y)};
}
__device__ __forceinline__ cf cscale(cf a, float s) { return {a.x * s, a.y * s}; }
// multiply by -i (SIGN = -1) or +i (SIGN = +1)
template <int SIGN>
__device__ __forceinline__ cf mul_i(cf a) {
  if constexpr (SIGN < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

// ---------------------------------------------------------------------------
// Compile-time cos / sin of 2*pi*num/den (octant reduction + Taylor series in
// double precision; the float rounding of the result is then exact to half
// an ulp for every angle used here).
// ---------------------------------------------------------------------------
namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int i = 1; i < 24; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int i = 1; i < 24; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
// r in [0, den): angle 2*pi*r/den.  Returns cos (which==0) or sin (which==1).
constexpr double cs(long num, long den, int which) {
  long r = ((num % den) + den) % den;
  double sgn_s = 1.0, sgn_c = 1.0;
  double rr = (double)r;
  double dd = (double)den;
  if (2.0 * rr > dd) {  // theta > pi: reflect, sin changes sign
    rr = dd - rr;
    sgn_s = -1.0;
  }
  if (4.0 * rr > dd) {  // theta > pi/2: theta = pi - t
    rr = dd / 2.0 - rr;
    sgn_c = -sgn_c;
  }
  bool swap = false;
  if (8.0 * rr > dd) {  // theta > pi/4: theta = pi/2 - t
    rr = dd / 4.0 - rr;
    swap = true;
  }
  double t = 2.0 * kPi * rr / dd;
  double c = taylor_cos(t), s = taylor_sin(t);
  if (swap) {
    double tmp = c;
    c = s;
    s = tmp;
  }
  return which == 0 ? sgn_c * c : sgn_s * s;
}
}  // namespace ct

// Multiply by the compile-time twiddle exp(SIGN * 2*pi*i * E / L).
template <long E, long L, int SIGN>
__device__ __forceinline__ cf twiddle(cf a) {
  constexpr long e = ((E % L) + L) % L;
  if constexpr (e == 0) {
    return a;
  } else if constexpr ((4 * e) % L == 0) {
    constexpr long q = (4 * e) / L;  // quarter turns (SIGN applied below)
    constexpr long qs = SIGN > 0 ? q : (4 - q) % 4;
    if constexpr (qs == 1) return {-a.y, a.x};
    else if constexpr (qs == 2) return {-a.x, -a.y};
    else return {a.y, -a.x};
  } else if constexpr ((8 * e) % L == 0) {
    constexpr float h = 0.70710678118654752440f;
    constexpr long o = (8 * e) / L;            // odd octant 1,3,5,7
    constexpr long os = SIGN > 0 ? o : (8 - o);
    // exp(i*pi*os/4) = (cx, sy) * h with signs
    constexpr float cx = (os == 1 || os == 7) ? 1.0f : -1.0f;
    constexpr float sy = (os == 1 || os == 3) ? 1.0f : -1.0f;
    // (a.x + i a.y)(cx + i sy) h
    return {(cx * a.x - sy * a.y) * h, (cx * a.y + sy * a.x) * h};
  } else {
    constexpr float c = (float)ct::cs(e, L, 0);
    constexpr float s = (float)(SIGN * ct::cs(e, L, 1));
    return {fmaf(a.x, c, -a.y * s), fmaf(a.x, s, a.y * c)};
  }
}

template <int L, int SIGN>
struct Dft;

template <int SIGN>
struct Dft<1, SIGN> {
  static __device__ __forceinline__ void run(cf*) {}
};

template <int SIGN>
struct Dft<2, SIGN> {
  static __device__ __forceinline__ void run(cf* v) {
    cf a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN>
__device__ __forceinline__ void radix4(cf b0, cf b1, cf b2, cf b3, cf& y0, cf& y1, cf& y2, cf& y3) {
  cf t0 = cadd(b0, b2), t1 = csub(b0, b2);
  cf t2 = cadd(b1, b3), t3 = mul_i<SIGN>(csub(b1, b3));
  y0 = cadd(t0, t2);
  y2 = csub(t0, t2);
  y1 = cadd(t1, t3);
  y3 = csub(t1, t3);
}

template <int SIGN>
struct Dft<4, SIGN> {
  static __device__ __forceinline__ void run(cf* v) {
    radix4<SIGN>(v[0], v[1], v[2], v[3], v[0], v[1], v[2], v[3]);
  }
};

// Twiddle with a deferred scale: exp(SIGN * 2*pi*i * E / L) = scale * (1 + i r)
// or scale * (r + i), so a * twiddle = scale * apply(a) where apply costs two
// fused multiply-adds (or two additions for the odd octants, nothing for
// quarter turns).  The compile-time scale is left to the caller, who folds it
// into the additions of the next butterfly (x + scale * y is one FMA), which
// saves the two multiplications of a plain complex product.
template <long E, long L, int SIGN>
struct ScaledTwiddle {
  static constexpr long e = ((E % L) + L) % L;
  static constexpr bool trivial = e == 0 || (4 * e) % L == 0;
  static constexpr bool octant = !trivial && (8 * e) % L == 0;
  static constexpr double c = ct::cs(e, L, 0);
  static constexpr double sn = SIGN * ct::cs(e, L, 1);
  static constexpr bool cos_major = (c < 0 ? -c : c) >= (sn < 0 ? -sn : sn);
  // the scale, in double (its float rounding is taken where it is used)
  static constexpr double scale_d = trivial ? 1.0
                                    : octant ? 0.70710678118654752440
                                             : (cos_major ? c : sn);
  static __device__ __forceinline__ cf apply(cf a) {
    if constexpr (trivial) {
      return twiddle<E, L, SIGN>(a);
    } else if constexpr (octant) {
      constexpr long o = (8 * e) / L;            // odd octant 1,3,5,7
      constexpr long os = SIGN > 0 ? o : (8 - o);
      constexpr float cx = (os == 1 || os == 7) ? 1.0f : -1.0f;
      constexpr float sy = (os == 1 || os == 3) ? 1.0f : -1.0f;
      return {cx * a.x - sy * a.y, cx * a.y + sy * a.x};
    } else if constexpr (cos_major) {
      constexpr float r = (float)(sn / c);       // |r| <= 1
      return {fmaf(-a.y, r, a.x), fmaf(a.x, r, a.y)};
    } else {
      constexpr float r = (float)(c / sn);       // |r| < 1
      return {fmaf(a.x, r, -a.y), fmaf(a.y, r, a.x)};
    }
  }
};

namespace detail {
// One radix-4 butterfly of the decimation in time, with the three twiddles'
// scales folded into its additions: with b_k = c_k u_k (c_0 = 1),
//   t0, t1 = b0 +- c2 u2;  t2 = c1 (u1 + (c3/c1) u3);  t3 = c1 (u1 - (c3/c1) u3) (-+i)
// and every output is t0 or t1 plus or minus c1 times a term: twelve fused
// multiply-adds or additions per component pair, as the plain butterfly.
template <int L, int SIGN, int Q, int K>
__device__ __forceinline__ void combine4(cf (&s)[4][Q], cf* v) {
  using T1 = ScaledTwiddle<K, L, SIGN>;
  using T2 = ScaledTwiddle<2 * K, L, SIGN>;
  using T3 = ScaledTwiddle<3 * K, L, SIGN>;
  constexpr float c1 = (float)T1::scale_d;
  constexpr float c2 = (float)T2::scale_d;
  constexpr float r3 = (float)(T3::scale_d / T1::scale_d);
  const cf b0 = s[0][K];
  const cf u1 = T1::apply(s[1][K]);
  const cf u2 = T2::apply(s[2][K]);
  const cf u3 = T3::apply(s[3][K]);
  const cf t0 = {fmaf(c2, u2.x, b0.x), fmaf(c2, u2.y, b0.y)};
  const cf t1 = {fmaf(-c2, u2.x, b0.x), fmaf(-c2, u2.y, b0.y)};
  const cf p = {fmaf(r3, u3.x, u1.x), fmaf(r3, u3.y, u1.y)};
  const cf m = mul_i<SIGN>(cf{fmaf(-r3, u3.x, u1.x), fmaf(-r3, u3.y, u1.y)});
  v[K] = {fmaf(c1, p.x, t0.x), fmaf(c1, p.y, t0.y)};
  v[K + 2 * Q] = {fmaf(-c1, p.x, t0.x), fmaf(-c1, p.y, t0.y)};
  v[K + Q] = {fmaf(c1, m.x, t1.x), fmaf(c1, m.y, t1.y)};
  v[K + 3 * Q] = {fmaf(-c1, m.x, t1.x), fmaf(-c1, m.y, t1.y)};
}
template <int L, int SIGN, int Q, int... Ks>
__device__ __forceinline__ void combine4_all(cf (&s)[4][Q], cf* v, std::integer_sequence<int, Ks...>) {
  (combine4<L, SIGN, Q, Ks>(s, v), ...);
}
template <int L, int SIGN, int Q, int K>
__device__ __forceinline__ void combine2(cf (&s)[2][Q], cf* v) {
  cf b0 = s[0][K];
  cf b1 = twiddle<K, L, SIGN>(s[1][K]);
  v[K] = cadd(b0, b1);
  v[K + Q] = csub(b0, b1);
}
template <int L, int SIGN, int Q, int... Ks>
__device__ __forceinline__ void combine2_all(cf (&s)[2][Q], cf* v, std::integer_sequence<int, Ks...>) {
  (combine2<L, SIGN, Q, Ks>(s, v), ...);
}
}  // namespace detail

// L >= 8: decimation in time by 4 (or by 2 when L/4 would not be a power of 4
// times {1,2}: every power of two is handled).
template <int L, int SIGN>
struct Dft {
  static_assert((L & (L - 1)) == 0 && L >= 8, "power-of-two length");
  static __device__ __forceinline__ void run(cf* v) {
    constexpr int Q = L / 4;
    cf s[4][Q];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < Q; ++j) s[r][j] = v[4 * j + r];
#pragma unroll
    for (int r = 0; r < 4; ++r) Dft<Q, SIGN>::run(s[r]);
    detail::combine4_all<L, SIGN, Q>(s, v, std::make_integer_sequence<int, Q>{});
  }
};

}  // namespace graphic
