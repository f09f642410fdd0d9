// M2L on the matrix cores (gfx950 MFMA 16x16x4, FP64 or FP32).
//
// Sec. 3.1 / Eq. tesourceboxtotargetbox: beta_k = sum_k' alpha_k' D^k D'^k' F / (k! k'!).
// With box-scaled moments and locals and G_g = h^{|g|} D^g F (the derivative
// table of the key) this becomes the Hankel contraction
//     b_k = sum_{k'} G_{k+k'} a_{k'},   a_{k'} = s (-1)^{|k'|} alpha^_{k'} / k'!,
//     beta^_k = b_k / k!,
// with s = (-1)^{k3'} for the Sigma family (whose kernel depends on z + z',
// so that source derivatives in z enter with a plus sign) and s = 1 otherwise.
// Both a and b are used in the Helmholtz-reduced form (k1 <= 1, (p+1)^2
// entries; see k_reduce / k_expand), so the operator is (p+1)^2 x (p+1)^2 and
// only table entries with g1 <= 2 are read.
//
// Work decomposition: a workgroup owns a tile of 16 target boxes that share
// z index and the parity of x and y (so all 16 have the same 6x6x6 window of
// candidate source offsets and the same table keys); it loops over the window
// and, per offset, stages the key's compact table (C(2p+3,3) complex values)
// and the 16 source moment vectors in LDS.  MFMA rows are output indices k,
// columns the 16 targets, K the source index k'; the A operand G_{k+k'} is
// gathered from the compact table in LDS.  Four waves split the row blocks.
#include <hip/hip_runtime.h>

#include "fmm_kernels.hpp"
#include "kernels.hpp"

namespace tefmm {

template <typename T>
struct M2LTypes;
template <>
struct M2LTypes<double> {
  typedef double2 T2;
  typedef d4 acc;
  __device__ static acc mfma(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static const T2* table(const M2LArgs& a, int pass) { return pass ? a.TS : a.Tfd; }
  __device__ static T2 cvt(double2 v) { return v; }
  // FP64 16x16x4 result: register i of lane l holds row (l >> 4) + 4 i, column l & 15
  __device__ static int row(int lane_hi, int i) { return lane_hi + 4 * i; }
};
template <>
struct M2LTypes<float> {
  typedef float2 T2;
  typedef f4 acc;
  __device__ static acc mfma(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static const T2* table(const M2LArgs& a, int pass) { return pass ? a.TS32 : a.Tfd32; }
  __device__ static T2 cvt(double2 v) { return make_float2((float)v.x, (float)v.y); }
  // FP32 16x16x4 result: register i of lane l holds row 4 (l >> 4) + i, column l & 15
  __device__ static int row(int lane_hi, int i) { return 4 * lane_hi + i; }
};

template <typename T, int RB>
__global__ __launch_bounds__(256) void k_m2l(M2LArgs a) {
  typedef M2LTypes<T> Ty;
  typedef typename Ty::T2 T2;
  typedef typename Ty::acc AC;
  extern __shared__ double lds_m2l[];
  T2* sG = (T2*)lds_m2l;
  T2* sA = sG + a.nG;
  int* sMi = (int*)(sA + 16 * a.nRs);

  // XCD-aware tile order: consecutive tiles (same z slab) stay on one XCD.
  const int per = (a.ntiles + 7) / 8;
  const int tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= a.ntiles) return;
  const int r = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int t = tile;
  const int X0 = t % a.tiles_x;
  t /= a.tiles_x;
  const int Y0 = t % a.tiles_x;
  t /= a.tiles_x;
  const int px = t & 1, py = (t >> 1) & 1, iz = t >> 2;
  const int N = a.n, pz = iz & 1;
  // target n (0..15): ix = px + 2(4 X0 + (n & 3)), iy = py + 2(4 Y0 + (n >> 2))
  unsigned tmask = 0;
  for (int n = 0; n < 16; ++n) {
    const int ix = px + 2 * (4 * X0 + (n & 3)), iy = py + 2 * (4 * Y0 + (n >> 2));
    if (ix < N && iy < N) tmask |= 1u << n;
  }

  const double2* alpha = a.a + (int64_t)r * a.rhs_stride;
  for (int e = tid; e < 16 * a.nRs; e += 256) {
    sA[e].x = 0;
    sA[e].y = 0;
  }
  for (int e = tid; e < 4 * a.nKB; e += 256) sMi[e] = e < a.nR ? a.rmi[e] : -1;

  const int col = lane & 15, krow = lane >> 4;
  int rowmi[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const int rb = w + 4 * j, k = 16 * rb + col;
    rowmi[j] = (rb < a.nRB && k < a.nR) ? a.rmi[k] : -1;
  }
  AC accR[RB], accI[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    accR[j] = AC{0, 0, 0, 0};
    accI[j] = AC{0, 0, 0, 0};
  }

  for (int pass = 0; pass < 2; ++pass) {
    const T2* table = Ty::table(a, pass);
    if (!table) continue;
    const bool mirror = pass == 1;
    const bool near_ok = pass ? a.near_s : a.near_fd;
    for (int oz = 0; oz < 6; ++oz) {
      const int dz = oz - 2 - pz;
      if (iz + dz < 0 || iz + dz >= N) continue;
      for (int oy = 0; oy < 6; ++oy) {
        const int dy = oy - 2 - py;
        for (int ox = 0; ox < 6; ++ox) {
          const int dx = ox - 2 - px;
          const bool nearb = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
          if (nearb && !(a.leaf && near_ok)) continue;
          unsigned smask = 0;
          for (int n = 0; n < 16; ++n) {
            const int ix = px + 2 * (4 * X0 + (n & 3)) + dx, iy = py + 2 * (4 * Y0 + (n >> 2)) + dy;
            if (((tmask >> n) & 1) && ix >= 0 && iy >= 0 && ix < N && iy < N) smask |= 1u << n;
          }
          if (!smask) continue;
          const int key = pass ? ((dx + 3) * 7 + (dy + 3)) * (2 * N - 1) + (2 * iz + dz)
                               : ((dx + 3) * 7 + (dy + 3)) * 7 + (dz + 3);
          __syncthreads();
          const T2* g = table + (int64_t)key * a.nG;
          for (int e = tid; e < a.nG; e += 256) sG[e] = g[e];
          for (int e = tid; e < 16 * a.nR; e += 256) {
            const int n = e / a.nR, kk = e - n * a.nR;
            T2 v;
            v.x = 0;
            v.y = 0;
            if ((smask >> n) & 1) {
              const int ix = px + 2 * (4 * X0 + (n & 3)) + dx, iy = py + 2 * (4 * Y0 + (n >> 2)) + dy;
              const int64_t sb = ((int64_t)ix * N + iy) * N + (iz + dz);
              const double s = (mirror && ((sMi[kk] >> 16) & 1)) ? -1.0 : 1.0;
              const double2 av = alpha[sb * a.nR + kk];
              v = Ty::cvt(make_double2(av.x * s, av.y * s));
            }
            sA[n * a.nRs + kk] = v;
          }
          __syncthreads();
          for (int kb = 0; kb < a.nKB; ++kb) {
            const int kp = 4 * kb + krow;
            const T2 bv = sA[col * a.nRs + kp];
            const int mp = sMi[kp];
#pragma unroll
            for (int j = 0; j < RB; ++j) {
              if (w + 4 * j < a.nRB) {
                T2 gv;
                gv.x = 0;
                gv.y = 0;
                if (rowmi[j] >= 0 && mp >= 0) {
                  const int gg = rowmi[j] + mp;
                  gv = sG[g_index(gg & 255, (gg >> 8) & 255, gg >> 16)];
                }
                accR[j] = Ty::mfma(gv.x, bv.x, accR[j]);
                accR[j] = Ty::mfma(-gv.y, bv.y, accR[j]);
                accI[j] = Ty::mfma(gv.x, bv.y, accI[j]);
                accI[j] = Ty::mfma(gv.y, bv.x, accI[j]);
              }
            }
          }
        }
      }
    }
  }
  // epilogue: result rows per the precision's MFMA layout, columns = targets
  double2* beta = a.b + (int64_t)r * a.rhs_stride;
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const int rb = w + 4 * j;
    if (rb >= a.nRB) continue;
    const int n = col;
    if (!((tmask >> n) & 1)) continue;
    const int ix = px + 2 * (4 * X0 + (n & 3)), iy = py + 2 * (4 * Y0 + (n >> 2));
    const int64_t tb = ((int64_t)ix * N + iy) * N + iz;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 16 * rb + Ty::row(krow, i);
      if (k < a.nR) beta[tb * a.nR + k] = make_double2((double)accR[j][i], (double)accI[j][i]);
    }
  }
}

template <typename T>
static hipError_t launch_t(const M2LArgs& a, int nrhs, hipStream_t s) {
  typedef typename M2LTypes<T>::T2 T2;
  size_t lds = (size_t)a.nG * sizeof(T2) + (size_t)16 * a.nRs * sizeof(T2) + (4 * (size_t)a.nKB + 4) * sizeof(int);
  const int RB = (a.nRB + 3) / 4;
  dim3 grid(8 * ((a.ntiles + 7) / 8), nrhs), block(256);
  void (*fn)(M2LArgs) = nullptr;
  switch (RB) {
    case 1: fn = k_m2l<T, 1>; break;
    case 2: fn = k_m2l<T, 2>; break;
    case 3: fn = k_m2l<T, 3>; break;
    case 4: fn = k_m2l<T, 4>; break;
    case 5: fn = k_m2l<T, 5>; break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, grid, block, lds, s, a);
  return hipGetLastError();
}

hipError_t launch_m2l(const M2LArgs& a, int nrhs, bool fp32, hipStream_t s) {
  return fp32 ? launch_t<float>(a, nrhs, s) : launch_t<double>(a, nrhs, s);
}

}  // namespace tefmm
