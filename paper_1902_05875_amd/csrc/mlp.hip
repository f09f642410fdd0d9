// Fully connected tanh network on the matrix cores, with its training step
// (the surrogate for the reaction derivative tables).
//
//   a_0 = x,  a_{l+1} = tanh(W_l a_l + b_l) (l < n_hidden),  y = W_out a_H + b_out,
//   L = mean over samples and outputs of (y - t)^2,  Adam updates.
//
// The hidden products run as a BF16 MFMA GEMM (v_mfma_f32_16x16x16_bf16: operands
// rounded to BF16 when staged into LDS, FP32 accumulation).  With `split` set, each
// FP32 operand is carried as two BF16 values, x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi), and a product takes three MFMAs (lo hi + hi lo + hi hi, the
// small terms first; lo lo is below FP32 rounding of the sum), which keeps about
// 16 mantissa bits of each operand instead of 8.  The first layer
// (a few inputs) and its weight gradient stay in FP32 on the vector units, since
// rounding the coordinates themselves to 8 mantissa bits would cost more
// accuracy than all later layers, and so does the output layer (forward and its
// two backward products), whose values are the results.  Master weights, gradients and Adam moments
// are FP32.  Activations are stored row-major, one row per sample.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tefmm.h"
#include "kernels.hpp"
#include "mlp.hpp"

namespace tefmm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// C(i, j) = sum_k A(i, k) B(k, j) over this block's K range, then either
//   store: C = act(acc + bias[j])   or   atomic: C += acc   (split K)
// A(i, k) = A[i sai + k sak], B(k, j) = B[k sbk + j sbj], C(i, j) = C[i ldc + j].
struct GemmArgs {
  int M, N, K;
  const float* A;
  int64_t sai, sak;
  const float* B;
  int64_t sbk, sbj;
  float* C;
  int64_t ldc;
  const float* bias;
  int act;     // 0: none, 1: tanh
  int atomic;  // 1: accumulate atomically
  int kps;     // K per blockIdx.z
  int split;   // 1: operands as BF16 hi + lo pairs, three MFMAs per product
};

// 64 x 64 output tile per workgroup, four waves of 32 x 32 (2 x 2 MFMA tiles).
// MFMA 16x16x16 BF16 operand layout: lane l holds A[l & 15][4 (l >> 4) + 0..3]
// and B[4 (l >> 4) + 0..3][l & 15]; result register r of lane l is
// C[4 (l >> 4) + r][l & 15].
template <bool SPLIT>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __align__(16) unsigned short sA[64][36];  // [row][k]
  __shared__ __align__(16) unsigned short sB[64][36];  // [col][k]
  __shared__ __align__(16) unsigned short sAl[SPLIT ? 64 : 1][36];  // low parts (SPLIT)
  __shared__ __align__(16) unsigned short sBl[SPLIT ? 64 : 1][36];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kbeg = blockIdx.z * g.kps;
  const int kend = min(g.K, kbeg + g.kps);
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + 256 * r;
      int row, kk;
      if (g.sak == 1) {
        row = e >> 5, kk = e & 31;
      } else {
        row = e & 63, kk = e >> 6;
      }
      const int i = i0 + row, k = k0 + kk;
      const float v = (i < g.M && k < kend) ? g.A[(int64_t)i * g.sai + (int64_t)k * g.sak] : 0.f;
      const unsigned short hi = f2bf(v);
      sA[row][kk] = hi;
      if (SPLIT) sAl[row][kk] = f2bf(v - __uint_as_float((unsigned)hi << 16));
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tid + 256 * r;
      int col, kk;
      if (g.sbj == 1) {
        col = e & 63, kk = e >> 6;
      } else {
        col = e >> 5, kk = e & 31;
      }
      const int j = j0 + col, k = k0 + kk;
      const float v = (j < g.N && k < kend) ? g.B[(int64_t)k * g.sbk + (int64_t)j * g.sbj] : 0.f;
      const unsigned short hi = f2bf(v);
      sB[col][kk] = hi;
      if (SPLIT) sBl[col][kk] = f2bf(v - __uint_as_float((unsigned)hi << 16));
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 32; ks += 16) {
      bf16x4 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = *(const bf16x4*)&sA[wr + 16 * t + (lane & 15)][ks + 4 * (lane >> 4)];
        bv[t] = *(const bf16x4*)&sB[wc + 16 * t + (lane & 15)][ks + 4 * (lane >> 4)];
      }
      if (SPLIT) {
        bf16x4 al[2], bl[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          al[t] = *(const bf16x4*)&sAl[wr + 16 * t + (lane & 15)][ks + 4 * (lane >> 4)];
          bl[t] = *(const bf16x4*)&sBl[wc + 16 * t + (lane & 15)][ks + 4 * (lane >> 4)];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[a], bv[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bl[b], acc[a][b], 0, 0, 0);
          }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + 16 * a + 4 * (lane >> 4) + r, j = j0 + wc + 16 * b + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        float v = acc[a][b][r];
        float* c = g.C + (int64_t)i * g.ldc + j;
        if (g.atomic) {
          atomicAdd(c, v);
        } else {
          if (g.bias) v += g.bias[j];
          if (g.act == 1) v = tanhf(v);
          *c = v;
        }
      }
}

// The same product in FP32 on the vector units (the output layer, whose values are the
// surrogate's results: BF16 operands there would cost ~3e-3 of their accuracy).  64 x 64
// output tile per workgroup of 256, 4 x 4 per thread, K in steps of 16 through LDS.
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs g) {
  __shared__ float sA[16][65];  // [k][row]
  __shared__ float sB[16][65];  // [k][col]
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int kbeg = blockIdx.z * g.kps;
  const int kend = min(g.K, kbeg + g.kps);
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + 256 * r;  // 1024 = 64 x 16 entries of each operand
      const int row = e & 63, kk = e >> 6;
      const int i = i0 + row, j = j0 + row, k = k0 + kk;
      sA[kk][row] = (i < g.M && k < kend) ? g.A[(int64_t)i * g.sai + (int64_t)k * g.sak] : 0.f;
      sB[kk][row] = (j < g.N && k < kend) ? g.B[(int64_t)k * g.sbk + (int64_t)j * g.sbj] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[kk][tr + 16 * a], bv[a] = sB[kk][tc + 16 * a];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + tr + 16 * a, j = j0 + tc + 16 * b;
      if (i >= g.M || j >= g.N) continue;
      float v = acc[a][b];
      float* c = g.C + (int64_t)i * g.ldc + j;
      if (g.atomic) {
        atomicAdd(c, v);
      } else {
        if (g.bias) v += g.bias[j];
        if (g.act == 1) v = tanhf(v);
        *c = v;
      }
    }
}

// first layer in FP32: a1[s][j] = tanh(sum_i W0[j][i] x[s][i] + b0[j])
__global__ void k_mlp_in(const float* x, int64_t n, int nin, int width, const float* W0, const float* b0, float* a1) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * width) return;
  const int64_t s = e / width;
  const int j = (int)(e - s * width);
  float v = b0[j];
  for (int i = 0; i < nin; ++i) v += W0[j * nin + i] * x[s * nin + i];
  a1[e] = tanhf(v);
}

// dW0[j][i] += sum_s d[s][j] x[s][i]  (FP32; one block per 256 samples)
__global__ void k_mlp_in_grad(const float* x, const float* d, int64_t n, int nin, int width, float* dW0) {
  __shared__ float sx[256 * 4];
  const int64_t s0 = (int64_t)blockIdx.x * 256;
  const int cnt = (int)min<int64_t>(256, n - s0);
  for (int e = threadIdx.x; e < cnt * nin; e += blockDim.x) sx[e] = x[s0 * nin + e];
  __syncthreads();
  for (int e = threadIdx.x; e < width * nin; e += blockDim.x) {
    const int j = e / nin, i = e - j * nin;
    float acc = 0.f;
    for (int s = 0; s < cnt; ++s) acc += d[(s0 + s) * width + j] * sx[s * nin + i];
    atomicAdd(&dW0[e], acc);
  }
}

// d = 2 (y - t) / (n n_out) in place of y; loss += sum (y - t)^2 / (n n_out)
__global__ void k_mlp_loss(float* y, const float* t, int64_t cnt, float scale, double* loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * blockDim.x) {
    const float r = y[e] - t[e];
    acc += (double)r * r;
    y[e] = 2.f * r * scale;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] * scale);
}

// d[s][j] *= 1 - a[s][j]^2
__global__ void k_mlp_tanh_back(float* d, const float* a, int64_t cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) d[e] *= 1.f - a[e] * a[e];
}

// db[j] += sum_s d[s][j]: block (column chunk of 64, row chunk of 256)
__global__ void k_mlp_colsum(const float* d, int64_t n, int ncol, float* db) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t s0 = (int64_t)blockIdx.y * 256;
  if (j >= ncol) return;
  float acc = 0.f;
  for (int64_t s = s0 + (threadIdx.x >> 6); s < min<int64_t>(n, s0 + 256); s += 4) acc += d[s * ncol + j];
  atomicAdd(&db[j], acc);
}

__global__ void k_mlp_adam(float* th, const float* g, float* m, float* v, int64_t P, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi, v[e] = vi;
  th[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_mlp_gather(const float* src, const int* idx, int64_t cnt, int cols, float* dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt * cols) return;
  const int64_t r = e / cols;
  dst[e] = src[(int64_t)idx[r] * cols + (e - r * cols)];
}

// f32: the FP32 vector-unit product (output layer) instead of the BF16 MFMA one
static hipError_t gemm(const GemmArgs& g0, hipStream_t s, bool f32 = false) {
  GemmArgs g = g0;
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return hipSuccess;
  int splits = 1;
  if (g.atomic) {
    g.kps = 256;
    splits = (g.K + 255) / 256;
  } else {
    g.kps = ((g.K + 31) / 32) * 32;
  }
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
  if (f32)
    hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, s, g);
  else if (g.split)
    hipLaunchKernelGGL(k_gemm_bf16<true>, grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(k_gemm_bf16<false>, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

static inline unsigned nblk(int64_t cnt, int b = 256) { return (unsigned)((cnt + b - 1) / b); }

Mlp::~Mlp() {
  for (float* p : {theta, grad, m, v, acts, y, d0, d1, xb, tb})
    if (p) (void)hipFree(p);
  if (d_loss) (void)hipFree(d_loss);
  if (d_idx) (void)hipFree(d_idx);
}

void Mlp::layout() {
  off_W.clear(), off_b.clear(), rows.clear(), cols.clear();
  int64_t o = 0;
  for (int l = 0; l <= n_hidden; ++l) {
    const int r = l == n_hidden ? n_out : width, c = l == 0 ? n_in : width;
    rows.push_back(r), cols.push_back(c);
    off_W.push_back(o);
    o += (int64_t)r * c;
    off_b.push_back(o);
    o += r;
  }
  P = o;
}

hipError_t Mlp::reserve(int64_t n) {
  if (n <= cap) return hipSuccess;
  for (float** p : {&acts, &y, &d0, &d1, &xb, &tb})
    if (*p) (void)hipFree(*p), *p = nullptr;
  if (d_idx) (void)hipFree(d_idx), d_idx = nullptr;
  hipError_t e;
  if ((e = hipMalloc(&acts, sizeof(float) * n * width * n_hidden)) != hipSuccess) return e;
  if ((e = hipMalloc(&y, sizeof(float) * n * n_out)) != hipSuccess) return e;
  if ((e = hipMalloc(&d0, sizeof(float) * n * width)) != hipSuccess) return e;
  if ((e = hipMalloc(&d1, sizeof(float) * n * width)) != hipSuccess) return e;
  if ((e = hipMalloc(&xb, sizeof(float) * n * n_in)) != hipSuccess) return e;
  if ((e = hipMalloc(&tb, sizeof(float) * n * n_out)) != hipSuccess) return e;
  if ((e = hipMalloc(&d_idx, sizeof(int) * n)) != hipSuccess) return e;
  cap = n;
  return hipSuccess;
}

// forward of n <= cap rows; activations a_1..a_H kept in acts, outputs in out
hipError_t Mlp::forward(const float* x, int64_t n, float* out, hipStream_t s) {
  return forward_in(x, n, out, s, acts, cap * width, n_hidden);
}

// forward of n rows with the hidden activation a_{l+1} in slab l % nslab of buf (slabs
// `stride` floats apart, each holding n x width): nslab = n_hidden keeps every layer (for
// the backward pass), nslab = 2 only the two a product reads and writes
hipError_t Mlp::forward_in(const float* x, int64_t n, float* out, hipStream_t s, float* buf, int64_t stride,
                           int nslab) {
  hipError_t e;
  hipLaunchKernelGGL(k_mlp_in, dim3(nblk(n * width)), dim3(256), 0, s, x, n, n_in, width, theta + off_W[0],
                     theta + off_b[0], buf);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int l = 1; l <= n_hidden; ++l) {
    const float* ain = buf + (int64_t)((l - 1) % nslab) * stride;
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.M = (int)n, g.N = rows[l], g.K = cols[l];
    g.split = split;
    g.A = ain, g.sai = width, g.sak = 1;
    g.B = theta + off_W[l], g.sbk = 1, g.sbj = cols[l];  // B(k, j) = W[j][k]
    g.bias = theta + off_b[l];
    if (l < n_hidden) {
      g.C = buf + (int64_t)(l % nslab) * stride, g.ldc = width, g.act = 1;
    } else {
      g.C = out, g.ldc = n_out, g.act = 0;
    }
    if ((e = gemm(g, s, l == n_hidden)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// gradient of the mean-squared loss over rows [x, t) (n <= cap) into grad (zeroed here)
hipError_t Mlp::loss_grad(const float* x, const float* t, int64_t n, hipStream_t s) {
  hipError_t e;
  if ((e = hipMemsetAsync(grad, 0, sizeof(float) * P, s)) != hipSuccess) return e;
  if ((e = forward(x, n, y, s)) != hipSuccess) return e;
  const int64_t cnt = n * n_out;
  hipLaunchKernelGGL(k_mlp_loss, dim3((unsigned)std::min<int64_t>(1024, nblk(cnt))), dim3(256), 0, s, y, t, cnt,
                     1.f / (float)cnt, d_loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // y now holds dL/dy; walk back through the layers
  const float* d = y;
  int ld = n_out;
  float* dn = d0;
  for (int l = n_hidden; l >= 1; --l) {
    const float* ain = acts + (int64_t)(l - 1) * cap * width;  // a_l (input of layer l)
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    // dW_l += d^T a_l : (rows x n)(n x cols)
    g.M = rows[l], g.N = cols[l], g.K = (int)n;
    g.split = split;
    g.A = d, g.sai = 1, g.sak = ld;
    g.B = ain, g.sbk = width, g.sbj = 1;
    g.C = grad + off_W[l], g.ldc = cols[l], g.atomic = 1;
    if ((e = gemm(g, s, l == n_hidden)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_colsum, dim3((unsigned)((rows[l] + 63) / 64), nblk(n)), dim3(256), 0, s, d, n, rows[l],
                       grad + off_b[l]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // d_prev = (d W_l) * (1 - a_l^2)
    std::memset(&g, 0, sizeof(g));
    g.M = (int)n, g.N = cols[l], g.K = rows[l];
    g.split = split;
    g.A = d, g.sai = ld, g.sak = 1;
    g.B = theta + off_W[l], g.sbk = cols[l], g.sbj = 1;
    g.C = dn, g.ldc = width;
    if ((e = gemm(g, s, l == n_hidden)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_tanh_back, dim3(nblk(n * width)), dim3(256), 0, s, dn, ain, n * width);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    d = dn, ld = width;
    dn = (dn == d0) ? d1 : d0;
  }
  hipLaunchKernelGGL(k_mlp_in_grad, dim3(nblk(n)), dim3(256), 0, s, x, d, n, n_in, width, grad + off_W[0]);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_colsum, dim3((unsigned)((width + 63) / 64), nblk(n)), dim3(256), 0, s, d, n, width,
                     grad + off_b[0]);
  return hipGetLastError();
}

hipError_t Mlp::adam(float lr, hipStream_t s) {
  ++step;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3(nblk(P)), dim3(256), 0, s, theta, grad, m, v, P, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

// 64-bit mixing for seeded host random numbers (splitmix64 finaliser)
static uint64_t mix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

hipError_t Mlp::train(const float* X, const float* T, int64_t n, int epochs, int batch, float lr, uint64_t seed,
                      std::vector<double>& losses, hipStream_t s) {
  hipError_t e;
  if ((e = reserve(batch)) != hipSuccess) return e;
  std::vector<int> perm(n);
  int* d_perm = nullptr;
  if ((e = hipMalloc(&d_perm, sizeof(int) * n)) != hipSuccess) return e;
  uint64_t st = seed;
  losses.clear();
  for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
    // Fisher-Yates shuffle of the sample order
    for (int64_t i = 0; i < n; ++i) perm[i] = (int)i;
    for (int64_t i = n - 1; i > 0; --i) {
      st = mix64(st);
      std::swap(perm[i], perm[st % (uint64_t)(i + 1)]);
    }
    if ((e = hipMemcpyAsync(d_perm, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, s)) != hipSuccess) break;
    if ((e = hipMemsetAsync(d_loss, 0, sizeof(double), s)) != hipSuccess) break;
    int nb = 0;
    for (int64_t b0 = 0; b0 < n && e == hipSuccess; b0 += batch, ++nb) {
      const int64_t cnt = std::min<int64_t>(batch, n - b0);
      hipLaunchKernelGGL(k_mlp_gather, dim3(nblk(cnt * n_in)), dim3(256), 0, s, X, d_perm + b0, cnt, n_in, xb);
      hipLaunchKernelGGL(k_mlp_gather, dim3(nblk(cnt * n_out)), dim3(256), 0, s, T, d_perm + b0, cnt, n_out, tb);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = loss_grad(xb, tb, cnt, s)) != hipSuccess) break;
      // cosine decay of the step size over the run, down to 2% of lr
      const double prog = (double)ep / std::max(1, epochs);
      e = adam((float)(lr * (0.02 + 0.98 * 0.5 * (1.0 + std::cos(3.14159265358979 * prog)))), s);
    }
    if (e != hipSuccess) break;
    double L = 0;
    // the host permutation is rewritten next epoch: wait for its upload (and the epoch)
    if ((e = hipMemcpyAsync(&L, d_loss, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
    losses.push_back(L / nb);
  }
  (void)hipFree(d_perm);
  return e;
}

hipError_t Mlp::init(int ni, int w, int nh, int no, uint64_t seed) {
  n_in = ni, width = w, n_hidden = nh, n_out = no;
  layout();
  hipError_t e;
  for (float** p : {&theta, &grad, &m, &v})
    if ((e = hipMalloc(p, sizeof(float) * P)) != hipSuccess) return e;
  if ((e = hipMalloc(&d_loss, sizeof(double))) != hipSuccess) return e;
  if ((e = hipMemset(m, 0, sizeof(float) * P)) != hipSuccess) return e;
  if ((e = hipMemset(v, 0, sizeof(float) * P)) != hipSuccess) return e;
  // Glorot-uniform weights, zero biases
  std::vector<float> th(P, 0.f);
  uint64_t st = seed;
  for (int l = 0; l <= n_hidden; ++l) {
    const double a = std::sqrt(6.0 / (rows[l] + cols[l]));
    for (int64_t i = 0; i < (int64_t)rows[l] * cols[l]; ++i) {
      st = mix64(st);
      const double u = (double)(st >> 11) * (1.0 / 9007199254740992.0);
      th[off_W[l] + i] = (float)(a * (2.0 * u - 1.0));
    }
  }
  step = 0;
  return hipMemcpy(theta, th.data(), sizeof(float) * P, hipMemcpyHostToDevice);
}

}  // namespace tefmm

using tefmm::Mlp;

struct tefmm_mlp {
  Mlp net;
  std::string err;
};

#define MLPCHK(x)                                     \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) {                           \
      m->err = std::string(#x) + ": " + hipGetErrorString(e_); \
      return TEFMM_ERR_HIP;                           \
    }                                                 \
  } while (0)

extern "C" int tefmm_mlp_create(tefmm_mlp_t* out, int n_in, int width, int n_hidden, int n_out, uint64_t seed) {
  if (!out) return TEFMM_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_in < 1 || n_in > 4 || width < 1 || width > 4096 || n_hidden < 1 || n_hidden > 16 || n_out < 1 ||
      n_out > 65536)
    return TEFMM_ERR_INVALID_ARG;
  tefmm_mlp* m = new tefmm_mlp();
  if (m->net.init(n_in, width, n_hidden, n_out, seed) != hipSuccess) {
    delete m;
    return TEFMM_ERR_HIP;
  }
  *out = m;
  return TEFMM_OK;
}

extern "C" void tefmm_mlp_destroy(tefmm_mlp_t m) { delete m; }

extern "C" int64_t tefmm_mlp_num_params(tefmm_mlp_t m) { return m ? m->net.P : -1; }

extern "C" const char* tefmm_mlp_last_error(tefmm_mlp_t m) { return m ? m->err.c_str() : "null handle"; }

extern "C" int tefmm_mlp_set_params(tefmm_mlp_t m, const float* theta) {
  if (!m || !theta) return TEFMM_ERR_INVALID_ARG;
  MLPCHK(hipMemcpy(m->net.theta, theta, sizeof(float) * m->net.P, hipMemcpyHostToDevice));
  MLPCHK(hipMemset(m->net.m, 0, sizeof(float) * m->net.P));
  MLPCHK(hipMemset(m->net.v, 0, sizeof(float) * m->net.P));
  m->net.step = 0;
  return TEFMM_OK;
}

extern "C" int tefmm_mlp_get_params(tefmm_mlp_t m, float* theta) {
  if (!m || !theta) return TEFMM_ERR_INVALID_ARG;
  MLPCHK(hipMemcpy(theta, m->net.theta, sizeof(float) * m->net.P, hipMemcpyDeviceToHost));
  return TEFMM_OK;
}

extern "C" int tefmm_mlp_set_split(tefmm_mlp_t m, int split) {
  if (!m || (split != 0 && split != 1)) return TEFMM_ERR_INVALID_ARG;
  m->net.split = split;
  return TEFMM_OK;
}

extern "C" int tefmm_mlp_forward(tefmm_mlp_t m, const float* x, int64_t n, float* y, void* stream) {
  if (!m || n < 0 || (n > 0 && (!x || !y))) return TEFMM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int64_t chunk = 65536;
  MLPCHK(m->net.reserve(std::min<int64_t>(chunk, std::max<int64_t>(n, 1))));
  for (int64_t r0 = 0; r0 < n; r0 += m->net.cap) {
    const int64_t cnt = std::min<int64_t>(m->net.cap, n - r0);
    MLPCHK(m->net.forward(x + r0 * m->net.n_in, cnt, y + r0 * m->net.n_out, s));
  }
  return TEFMM_OK;
}

// Fixed device workspace of the forward pass that allocates nothing: two activation
// slabs of n x width floats.  Each GPU the library runs on holds its own copy until the
// process ends.  Host code never passes `scratch` itself (its host-side name is not a
// device address): the entry point looks up each device's address once.
static constexpr int64_t MLP_SCRATCH_FLOATS = (int64_t)TEFMM_MLP_SCRATCH_BYTES / sizeof(float);
static __device__ __align__(256) float scratch[MLP_SCRATCH_FLOATS];

static constexpr int MAX_DEVICES = 64;
static float* g_scratch_ptr[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Address of this device's copy of `scratch` (looked up on the first call per device).
static hipError_t scratch_address(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = (float*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

extern "C" int tefmm_mlp_forward_noalloc(tefmm_mlp_t m, const float* x, int64_t n, float* y, void* stream) {
  if (!m || n < 0 || (n > 0 && (!x || !y))) return TEFMM_ERR_INVALID_ARG;
  const int64_t need = 2 * n * (int64_t)m->net.width;  // two slabs of n x width
  if (need > MLP_SCRATCH_FLOATS) {
    m->err = "tefmm_mlp_forward_noalloc: " + std::to_string(n) + " rows x width " +
             std::to_string(m->net.width) + " need " + std::to_string(need * sizeof(float)) +
             " bytes of workspace, more than the fixed " + std::to_string((int64_t)TEFMM_MLP_SCRATCH_BYTES) +
             " (at most " + std::to_string(MLP_SCRATCH_FLOATS / (2 * m->net.width)) + " rows per call)";
    return TEFMM_ERR_INVALID_ARG;
  }
  float* buf = nullptr;
  MLPCHK(scratch_address(&buf));
  if (n == 0) return TEFMM_OK;
  MLPCHK(m->net.forward_in(x, n, y, (hipStream_t)stream, buf, n * m->net.width, 2));
  return TEFMM_OK;
}

extern "C" int tefmm_mlp_loss_grad(tefmm_mlp_t m, const float* x, const float* t, int64_t n, double* loss,
                                   float* grad, void* stream) {
  if (!m || n < 1 || !x || !t) return TEFMM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  MLPCHK(m->net.reserve(n));
  MLPCHK(hipMemsetAsync(m->net.d_loss, 0, sizeof(double), s));
  MLPCHK(m->net.loss_grad(x, t, n, s));
  MLPCHK(hipStreamSynchronize(s));
  if (loss) MLPCHK(hipMemcpy(loss, m->net.d_loss, sizeof(double), hipMemcpyDeviceToHost));
  if (grad) MLPCHK(hipMemcpy(grad, m->net.grad, sizeof(float) * m->net.P, hipMemcpyDeviceToHost));
  return TEFMM_OK;
}

extern "C" int tefmm_mlp_adam_step(tefmm_mlp_t m, float lr, void* stream) {
  if (!m) return TEFMM_ERR_INVALID_ARG;
  MLPCHK(m->net.adam(lr, (hipStream_t)stream));
  MLPCHK(hipStreamSynchronize((hipStream_t)stream));
  return TEFMM_OK;
}

extern "C" int tefmm_mlp_train(tefmm_mlp_t m, const float* x, const float* t, int64_t n, int epochs, int batch,
                               float lr, uint64_t seed, double* epoch_loss, void* stream) {
  if (!m || n < 1 || !x || !t || epochs < 0 || batch < 1 || !(lr > 0)) return TEFMM_ERR_INVALID_ARG;
  std::vector<double> losses;
  MLPCHK(m->net.train(x, t, n, epochs, batch, lr, seed, losses, (hipStream_t)stream));
  if (epoch_loss)
    for (size_t i = 0; i < losses.size(); ++i) epoch_loss[i] = losses[i];
  return TEFMM_OK;
}
