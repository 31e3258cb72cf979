// Measurement program (not part of the library): one 32-point DFT stage of the
// line passes' four-step transforms, computed
//   (a) by the register codelet the line passes use (each lane transforms one
//       vector held in its VGPRs, radix-4 decimation in time), and
//   (b) as a DFT-as-GEMM on the matrix cores: a wave holds 32 vectors as the
//       rows of a 32 x 32 complex matrix X and computes Y = X G with
//       v_mfma_f32_32x32x2f32 (four real products per complex product, 64
//       instructions per wave and stage), G the DFT matrix exp(-+2 pi i k n / 32);
//       between stages X goes through LDS, because the product's output layout
//       is not its input layout.
// Both apply the stage `reps` times, forward and inverse in turn, to vectors
// resident in HBM (read once, written once).  The program checks both against a
// float64 direct DFT (two stages: forward then inverse, which gives 32 x) and
// prints one JSON line with the time per vector and stage.
//
// usage: dft32_mfma [n_vectors] [reps]
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../dft_codelets.h"

using graphic::cf;
using graphic::Dft;

typedef float v16f __attribute__((ext_vector_type(16)));

// (a) one vector per lane; element k of vector v at in[k * n + v] (coalesced)
__global__ void __launch_bounds__(256) valu_kernel(const float2* __restrict__ in, float2* __restrict__ out, int n,
                                                   int reps) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n) return;
  cf x[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    const float2 t = in[(size_t)k * n + v];
    x[k] = {t.x, t.y};
  }
  for (int r = 0; r < reps; r += 2) {
    Dft<32, -1>::run(x);
    Dft<32, +1>::run(x);
  }
#pragma unroll
  for (int k = 0; k < 32; ++k) out[(size_t)k * n + v] = make_float2(x[k].x, x[k].y);
}

// (b) 32 vectors per wave, 4 waves per block; the same memory layout.
// v_mfma_f32_32x32x2f32: lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32];
// accumulator v of lane l is D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
__global__ void __launch_bounds__(256) mfma_kernel(const float2* __restrict__ in, float2* __restrict__ out, int n,
                                                   int reps) {
  __shared__ float xs[4][2][32][33];                   // per wave: re / im of X[row][col]
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + w) * 32;           // first vector of the wave
  const int c = l % 32, hi = l / 32;
  // load X (rows = vectors, cols = k): lanes over vectors for coalescing
  for (int k = hi; k < 32; k += 2) {
    const int v = row0 + c;
    const float2 t = v < n ? in[(size_t)k * n + v] : make_float2(0.f, 0.f);
    xs[w][0][c][k] = t.x;
    xs[w][1][c][k] = t.y;
  }
  // B operands: G[k][j] = exp(-2 pi i k j / 32), k = 2 kp + hi, j = c
  float gr[16], gi[16], ngi[16];
#pragma unroll
  for (int kp = 0; kp < 16; ++kp) {
    const int k = 2 * kp + hi;
    const int e = (k * c) & 31;
    const float a = -6.283185307179586f * (float)e / 32.0f;
    gr[kp] = cosf(a);
    gi[kp] = sinf(a);
    ngi[kp] = -gi[kp];
  }
  __syncthreads();
  for (int r = 0; r < reps; ++r) {
    const bool inv = (r & 1) != 0;
    v16f yr = {}, yi = {};
#pragma unroll
    for (int kp = 0; kp < 16; ++kp) {
      const float ar = xs[w][0][c][2 * kp + hi], ai = xs[w][1][c][2 * kp + hi];
      // forward (Gi = gi): Yr = Xr Gr - Xi Gi, Yi = Xr Gi + Xi Gr; inverse: Gi = -gi
      const float bi = inv ? ngi[kp] : gi[kp], nbi = inv ? gi[kp] : ngi[kp];
      yr = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, gr[kp], yr, 0, 0, 0);
      yr = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, nbi, yr, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, yi, 0, 0, 0);
      yi = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, gr[kp], yi, 0, 0, 0);
    }
    __syncthreads();                                    // every lane has read X
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v / 4) + 4 * hi + (v % 4);
      xs[w][0][i][c] = yr[v];
      xs[w][1][i][c] = yi[v];
    }
    __syncthreads();
  }
  for (int k = hi; k < 32; k += 2) {
    const int v = row0 + c;
    if (v < n) out[(size_t)k * n + v] = make_float2(xs[w][0][c][k], xs[w][1][c][k]);
  }
}

static void direct_dft(const double* xr, const double* xi, double* yr, double* yi, int sign) {
  for (int k = 0; k < 32; ++k) {
    double sr = 0, si = 0;
    for (int m = 0; m < 32; ++m) {
      const double a = sign * 2.0 * M_PI * (double)((k * m) % 32) / 32.0;
      sr += xr[m] * cos(a) - xi[m] * sin(a);
      si += xr[m] * sin(a) + xi[m] * cos(a);
    }
    yr[k] = sr;
    yi[k] = si;
  }
}

#define CHECK(x)                                                  \
  do {                                                            \
    if ((x) != hipSuccess) {                                      \
      fprintf(stderr, "HIP error at %s:%d\n", __FILE__, __LINE__); \
      return 1;                                                   \
    }                                                             \
  } while (0)

int main(int argc, char** argv) {
  const int n = argc > 1 ? atoi(argv[1]) : (1 << 20);
  const int reps = argc > 2 ? atoi(argv[2]) : 64;
  if (n < 128 || n % 128 != 0 || reps < 2 || reps % 2 != 0) {
    fprintf(stderr, "n must be a multiple of 128, reps even\n");
    return 2;
  }
  std::vector<float2> h((size_t)32 * n);
  unsigned s = 12345u;
  for (auto& t : h) {
    s = s * 1664525u + 1013904223u;
    const float a = (float)(s >> 8) / 16777216.0f - 0.5f;
    s = s * 1664525u + 1013904223u;
    const float b = (float)(s >> 8) / 16777216.0f - 0.5f;
    t = make_float2(a * 1e-30f, b * 1e-30f);       // bounded after reps stages (32^(reps/2) growth)
  }
  float2 *din, *dout;
  CHECK(hipMalloc(&din, h.size() * sizeof(float2)));
  CHECK(hipMalloc(&dout, h.size() * sizeof(float2)));
  CHECK(hipMemcpy(din, h.data(), h.size() * sizeof(float2), hipMemcpyHostToDevice));
  double err[2] = {0, 0}, ms[2] = {0, 0};
  for (int method = 0; method < 2; ++method) {
    // parity: two stages (forward, inverse) on every vector, sampled check
    auto launch = [&](int r) {
      if (method == 0) hipLaunchKernelGGL(valu_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, din, dout, n, r);
      else hipLaunchKernelGGL(mfma_kernel, dim3(n / 128), dim3(256), 0, 0, din, dout, n, r);
    };
    launch(2);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    std::vector<float2> o(h.size());
    CHECK(hipMemcpy(o.data(), dout, o.size() * sizeof(float2), hipMemcpyDeviceToHost));
    double num = 0, den = 0;
    for (int v = 0; v < n; v += 997) {
      double xr[32], xi[32], yr[32], yi[32], zr[32], zi[32];
      for (int k = 0; k < 32; ++k) {
        xr[k] = h[(size_t)k * n + v].x;
        xi[k] = h[(size_t)k * n + v].y;
      }
      direct_dft(xr, xi, yr, yi, -1);
      direct_dft(yr, yi, zr, zi, +1);
      for (int k = 0; k < 32; ++k) {
        const double dr = o[(size_t)k * n + v].x - zr[k], di = o[(size_t)k * n + v].y - zi[k];
        num += dr * dr + di * di;
        den += zr[k] * zr[k] + zi[k] * zi[k];
      }
    }
    err[method] = sqrt(num / den);
    if (getenv("DFT32_DEBUG"))
      for (int k = 0; k < 4; ++k)
        fprintf(stderr, "method %d k %d: got (%g, %g) want (%g, %g)\n", method, k, o[(size_t)k * n].x,
                o[(size_t)k * n].y, 32.0 * h[(size_t)k * n].x, 32.0 * h[(size_t)k * n].y);
    // timing
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    launch(reps);
    CHECK(hipEventRecord(a, 0));
    for (int it = 0; it < 5; ++it) launch(reps);
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float t = 0;
    CHECK(hipEventElapsedTime(&t, a, b));
    ms[method] = t / 5.0;
  }
  const double stages = (double)n * reps;
  printf("{\"what\": \"32-point complex DFT stage, %d vectors x %d stages\", "
         "\"valu_codelet\": {\"ms\": %.3f, \"ns_per_vector_stage\": %.4f, \"rel_l2_vs_direct_dft\": %.2e}, "
         "\"mfma_32x32x2_f32\": {\"ms\": %.3f, \"ns_per_vector_stage\": %.4f, \"rel_l2_vs_direct_dft\": %.2e}, "
         "\"mfma_over_valu_time\": %.2f}\n",
         n, reps, ms[0], ms[0] * 1e6 / stages, err[0], ms[1], ms[1] * 1e6 / stages, err[1], ms[1] / ms[0]);
  return (err[0] < 1e-5 && err[1] < 1e-5) ? 0 : 3;
}
