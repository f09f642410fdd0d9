// Device helpers shared by the HIP kernels of the layered-media TE-FMM.
#pragma once
#include <hip/hip_runtime.h>

namespace tefmm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct dc {
  double x, y;
};

__device__ __forceinline__ dc cmul(dc a, dc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ dc cadd(dc a, dc b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ dc csub(dc a, dc b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ dc cscale(dc a, double s) { return {a.x * s, a.y * s}; }
__device__ __forceinline__ dc cdiv(dc a, dc b) {
  // scaled division (Smith's method)
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return {(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  }
  double r = b.x / b.y, den = b.x * r + b.y;
  return {(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}
__device__ __forceinline__ dc csqrt_pr(dc z) {
  // principal square root, Re >= 0
  double r = hypot(z.x, z.y);
  if (r == 0.0) return {0.0, 0.0};
  if (z.x >= 0) {
    double t = sqrt(0.5 * (r + z.x));
    return {t, z.y / (2.0 * t)};
  }
  double t = sqrt(0.5 * (r - z.x));
  return {fabs(z.y) / (2.0 * t), copysign(t, z.y)};
}
__device__ __forceinline__ dc cexp_i(dc z, double k) {
  // exp(i k z)
  double s, c;
  sincos(k * z.x, &s, &c);
  double m = exp(-k * z.y);
  return {m * c, m * s};
}

// Graded multi-index order used everywhere: |g| ascending, then g1 descending,
// then g2 descending.  Index of g = (a, b, c), m = a + b + c:
//   C(m+2, 3) + (m-a)(m-a+1)/2 + (m-a-b).
__host__ __device__ __forceinline__ int mi_index(int a, int b, int c) {
  int m = a + b + c;
  return (m * (m + 1) * (m + 2)) / 6 + ((m - a) * (m - a + 1)) / 2 + (m - a - b);
}
__host__ __device__ __forceinline__ int mi_count(int n) { return ((n + 1) * (n + 2) * (n + 3)) / 6; }

}  // namespace tefmm

namespace tefmm {
// Compact derivative-table layout: only g with g1 <= 2 are kept (the Helmholtz
// equation gives every other entry from these), ordered by |g| = n, then g1,
// then g3:  idx = off(n) + [g1>=1](n+1) + [g1>=2] n + g3,  off(0) = 0,
// off(n) = 1 + 3 n (n-1) / 2.  Count up to order N: off(N+1) = 1 + 3 N (N+1)/2.
__host__ __device__ __forceinline__ int g_offset(int n) { return n == 0 ? 0 : 1 + (3 * n * (n - 1)) / 2; }
__host__ __device__ __forceinline__ int g_index(int g1, int g2, int g3) {
  const int n = g1 + g2 + g3;
  return g_offset(n) + (g1 >= 1 ? n + 1 : 0) + (g1 >= 2 ? n : 0) + g3;
}
__host__ __device__ __forceinline__ int g_count(int N) { return g_offset(N + 1); }
}  // namespace tefmm
