// HIP kernels of the layered-media Taylor-expansion FMM (gfx950).
//
// Notation (Sec. 3.1, Sec. 3.2): a box of side h at centre c carries scaled
// multipole moments  alpha^_k = sum_j q_j ((r_j - c)/h)^k  and scaled local
// coefficients beta^_k (the Taylor coefficients of the far field in
// (r - c)/h).  Multi-indices are stored in the graded order of mi_index().
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fmm_kernels.hpp"
#include "kernels.hpp"

namespace tefmm {

__constant__ double c_binom[24][24];

void upload_binomials() {
  double b[24][24] = {};
  for (int n = 0; n < 24; ++n) {
    b[n][0] = 1.0;
    for (int k = 1; k <= n; ++k) b[n][k] = b[n - 1][k - 1] + (k <= n - 1 ? b[n - 1][k] : 0.0);
  }
  (void)hipMemcpyToSymbol(HIP_SYMBOL(c_binom), b, sizeof(b));
}

// ---------------------------------------------------------------------------
// Derivative tables (Sec. 3.3, Eq. derivativeapp with the recurrence of
// Eq. recurrsion in corrected form).  For f = exp(i k R)/R and
// psi = exp(i k R), with a_g = D^g f / g!, b_g = D^g psi / g! at a point x
// (third coordinate possibly complex) and n = |g| >= 1:
//   n b_g = i k ( sum_i x_i a_{g-e_i} + sum_i a_{g-2e_i} )
//   n R^2 a_g = i k ( sum_i x_i b_{g-e_i} + sum_i b_{g-2e_i} )
//               - (2n-1) sum_i x_i a_{g-e_i} - (n-1) sum_i a_{g-2e_i}
// which follows from  R^2 d_i f + x_i f = i k x_i psi  and  d_i psi = i k x_i f
// by comparing Taylor coefficients.  Coordinates are in box units (x / h) and
// k is replaced by k h; the table entry is  G_g = h^{|g|} D^g F = g! a_g / h
// summed over the key's terms  F = sum coef * f(x, y, zeta)  (zeta -> -zeta
// direction flips contribute (-1)^{g3}).
// One workgroup of NW waves per key: wave w runs the recurrence for terms
// t0 + w, t0 + w + NW, ... in an LDS region of its own, and the waves' sums are
// added in wave order at the end.
// ---------------------------------------------------------------------------
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_table_gen(TableGenArgs a) {
  // Only entries with g1 <= 2 are generated (compact order of g_index); the
  // recurrence for such g needs g - e_i and g - 2 e_i, which stay in that set.
  extern __shared__ double2 lds_tab[];
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  double2* sa = lds_tab + (size_t)2 * a.nG * w;
  double2* sb = sa + a.nG;
  const int key = blockIdx.x;
  const int t0 = a.term_start[key], t1 = a.term_start[key + 1];
  constexpr int MAXJ = 25;  // nG <= 1600 (order <= 32)
  dc acc[MAXJ];
#pragma unroll
  for (int j = 0; j < MAXJ; ++j) acc[j] = {0.0, 0.0};
  const double kh = a.k * a.h[key];
  // rounds of NW terms, the same number of barriers in every wave; a wave without a
  // term in the last round repeats the round's first term and drops its result
  for (int tb = t0; tb < t1; tb += NW) {
    const bool on = tb + w < t1;
    const TableTerm tm = a.terms[on ? tb + w : tb];
    // swap13: the table is generated in the frame (zeta, y, x), i.e. restricted
    // to small orders in z instead of x (cross-layer translations)
    const dc xr = {tm.x, 0.0}, zc = {tm.zr, tm.zi};
    const dc x1 = a.swap13 ? zc : xr, x2 = {tm.y, 0.0}, x3 = a.swap13 ? xr : zc;
    const dc R2 = cadd(cadd(cmul(x1, x1), cmul(x2, x2)), cmul(x3, x3));
    const dc R = csqrt_pr(R2);
    const dc e = cexp_i(R, kh);
    const dc invR2 = cdiv({1.0, 0.0}, R2);
    if (lane == 0) {
      const dc f = cdiv(e, R);
      sa[0] = make_double2(f.x, f.y);
      sb[0] = make_double2(e.x, e.y);
    }
    __syncthreads();
    for (int n = 1; n <= a.order; ++n) {
      const int off = g_offset(n), cnt = g_offset(n + 1) - off;
      for (int i = lane; i < cnt; i += 64) {
        const int g = off + i;
        const short* nb = a.nbr + 6 * g;
        dc s1a = {0, 0}, s2a = {0, 0}, s1b = {0, 0}, s2b = {0, 0};
        const dc xs[3] = {x1, x2, x3};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int i1 = nb[d], i2 = nb[3 + d];
          if (i1 >= 0) {
            const dc av = {sa[i1].x, sa[i1].y}, bv = {sb[i1].x, sb[i1].y};
            s1a = cadd(s1a, cmul(xs[d], av));
            s1b = cadd(s1b, cmul(xs[d], bv));
          }
          if (i2 >= 0) {
            s2a = cadd(s2a, {sa[i2].x, sa[i2].y});
            s2b = cadd(s2b, {sb[i2].x, sb[i2].y});
          }
        }
        const dc ik = {0.0, kh};
        const dc bn = cscale(cmul(ik, cadd(s1a, s2a)), 1.0 / n);
        const dc num = csub(csub(cmul(ik, cadd(s1b, s2b)), cscale(s1a, 2.0 * n - 1.0)), cscale(s2a, n - 1.0));
        const dc an = cscale(cmul(num, invR2), 1.0 / n);
        sa[g] = make_double2(an.x, an.y);
        sb[g] = make_double2(bn.x, bn.y);
      }
      __syncthreads();
    }
    const dc cf = {tm.cr, tm.ci};
    if (on) {
#pragma unroll
      for (int j = 0; j < MAXJ; ++j) {
        const int g = lane + 64 * j;
        if (g < a.nG) {
          dc v = cmul(cf, {sa[g].x, sa[g].y});
          if (tm.flip && ((a.swap13 ? a.g1[g] : a.g3[g]) & 1)) v = {-v.x, -v.y};
          acc[j] = cadd(acc[j], v);
        }
      }
    }
    __syncthreads();
  }
  const double invh = 1.0 / a.h[key];
  if (NW == 1) {
#pragma unroll
    for (int j = 0; j < MAXJ; ++j) {
      const int g = lane + 64 * j;
      if (g < a.nG) {
        const double sc = a.fact[g] * invh;
        a.out[(size_t)key * a.nG + g] = make_double2(acc[j].x * sc, acc[j].y * sc);
      }
    }
    return;
  }
  // each wave's sums to its own region, then added in wave order
#pragma unroll
  for (int j = 0; j < MAXJ; ++j) {
    const int g = lane + 64 * j;
    if (g < a.nG) sa[g] = make_double2(acc[j].x, acc[j].y);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < a.nG; g += 64 * NW) {
    double2 v = lds_tab[g];
    for (int u = 1; u < NW; ++u) {
      const double2 o = lds_tab[(size_t)2 * a.nG * u + g];
      v.x += o.x, v.y += o.y;
    }
    const double sc = a.fact[g] * invh;
    a.out[(size_t)key * a.nG + g] = make_double2(v.x * sc, v.y * sc);
  }
}
template __global__ void k_table_gen<1>(TableGenArgs);
template __global__ void k_table_gen<2>(TableGenArgs);
template __global__ void k_table_gen<4>(TableGenArgs);
template __global__ void k_table_gen<8>(TableGenArgs);

__global__ void k_to_f32(const double2* in, size_t n, float2* out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

// Scaled Taylor coefficients at arbitrary points (introspection): same
// recurrence, one wave per point, output a_g * (order-independent) 1/h.
__global__ __launch_bounds__(64) void k_taylor_points(const double* px, const double* py,
                                                      const double* pz, double k, double h, int order,
                                                      int nT, const short* nbr, double2* out) {
  extern __shared__ double2 lds_tp[];
  double2* sa = lds_tp;
  double2* sb = lds_tp + nT;
  const int p = blockIdx.x, lane = threadIdx.x;
  const double kh = k * h;
  const dc x1 = {px[p] / h, 0}, x2 = {py[p] / h, 0}, x3 = {pz[2 * p] / h, pz[2 * p + 1] / h};
  const dc R2 = cadd(cadd(cmul(x1, x1), cmul(x2, x2)), cmul(x3, x3));
  const dc R = csqrt_pr(R2);
  const dc e = cexp_i(R, kh);
  const dc invR2 = cdiv({1.0, 0.0}, R2);
  if (lane == 0) {
    dc f = cdiv(e, R);
    sa[0] = make_double2(f.x, f.y);
    sb[0] = make_double2(e.x, e.y);
  }
  __syncthreads();
  for (int n = 1; n <= order; ++n) {
    const int off = (n * (n + 1) * (n + 2)) / 6, cnt = ((n + 1) * (n + 2)) / 2;
    for (int i = lane; i < cnt; i += 64) {
      const int g = off + i;
      const short* nb = nbr + 6 * g;
      dc s1a = {0, 0}, s2a = {0, 0}, s1b = {0, 0}, s2b = {0, 0};
      const dc xs[3] = {x1, x2, x3};
      for (int d = 0; d < 3; ++d) {
        int i1 = nb[d], i2 = nb[3 + d];
        if (i1 >= 0) {
          s1a = cadd(s1a, cmul(xs[d], {sa[i1].x, sa[i1].y}));
          s1b = cadd(s1b, cmul(xs[d], {sb[i1].x, sb[i1].y}));
        }
        if (i2 >= 0) {
          s2a = cadd(s2a, {sa[i2].x, sa[i2].y});
          s2b = cadd(s2b, {sb[i2].x, sb[i2].y});
        }
      }
      const dc ik = {0.0, kh};
      dc bn = cscale(cmul(ik, cadd(s1a, s2a)), 1.0 / n);
      dc num = csub(csub(cmul(ik, cadd(s1b, s2b)), cscale(s1a, 2.0 * n - 1.0)), cscale(s2a, n - 1.0));
      dc an = cscale(cmul(num, invR2), 1.0 / n);
      sa[g] = make_double2(an.x, an.y);
      sb[g] = make_double2(bn.x, bn.y);
    }
    __syncthreads();
  }
  for (int g = lane; g < nT; g += 64) out[(size_t)p * nT + g] = make_double2(sa[g].x / h, sa[g].y / h);
}

// ---------------------------------------------------------------------------
// MFMA lane layout self test (16x16x4, FP64 and FP32).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_selftest_mfma(double* out64, float* out32) {
  const int l = threadIdx.x;
  const int m = l & 15, kk = l >> 4;
  double a = 1.0 + m + 0.25 * kk, b = 2.0 - 0.5 * kk + 0.125 * m;
  d4 acc = {0, 0, 0, 0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  f4 accf = {0, 0, 0, 0};
  accf = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, accf, 0, 0, 0);
  // operands: lane l holds A[l & 15][l >> 4] and B[l >> 4][l & 15]; results differ by precision
  for (int i = 0; i < 4; ++i) {
    const int col = l & 15;
    out64[((l >> 4) + 4 * i) * 16 + col] = acc[i];
    out32[(4 * (l >> 4) + i) * 16 + col] = accf[i];
  }
}

// ---------------------------------------------------------------------------
// Tree construction.
// ---------------------------------------------------------------------------
__global__ void k_layer_stats(const double* xyz, int64_t n, int nif, const double* ifz, double eps,
                              double* part, int* bad) {
  // per block and layer (up to MAX_LAYERS): min/max of x, y, z and the count; each thread
  // keeps its own per layer (selects, no indexed registers), then one layer at a time is
  // reduced through LDS
  __shared__ double smin[3][256], smax[3][256];
  __shared__ int scnt[256];
  const int tid = threadIdx.x;
  double mn[MAX_LAYERS][3], mx[MAX_LAYERS][3];
  int cnt[MAX_LAYERS];
#pragma unroll
  for (int l = 0; l < MAX_LAYERS; ++l) {
#pragma unroll
    for (int c = 0; c < 3; ++c) mn[l][c] = 1e300, mx[l][c] = -1e300;
    cnt[l] = 0;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
    int ly = 0;
    for (int j = 0; j < nif; ++j) {
      ly += (z < ifz[j]);
      if (fabs(z - ifz[j]) < eps) atomicOr(bad, 1);
    }
    if (!(x == x) || !(y == y) || !(z == z)) atomicOr(bad, 2);
    const double v[3] = {x, y, z};
#pragma unroll
    for (int l = 0; l < MAX_LAYERS; ++l)
      if (l == ly) {
#pragma unroll
        for (int c = 0; c < 3; ++c) mn[l][c] = fmin(mn[l][c], v[c]), mx[l][c] = fmax(mx[l][c], v[c]);
        cnt[l] += 1;
      }
  }
#pragma unroll
  for (int l = 0; l < MAX_LAYERS; ++l) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) smin[c][tid] = mn[l][c], smax[c][tid] = mx[l][c];
    scnt[tid] = cnt[l];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if (tid < s) {
        for (int c = 0; c < 3; ++c) {
          smin[c][tid] = fmin(smin[c][tid], smin[c][tid + s]);
          smax[c][tid] = fmax(smax[c][tid], smax[c][tid + s]);
        }
        scnt[tid] += scnt[tid + s];
      }
      __syncthreads();
    }
    if (tid == 0) {
      double* o = part + ((size_t)blockIdx.x * MAX_LAYERS + l) * 7;
      for (int c = 0; c < 3; ++c) o[c] = smin[c][0], o[3 + c] = smax[c][0];
      o[6] = (double)scnt[0];
    }
  }
}

__global__ void k_leaf_keys(const double* xyz, int64_t n, int nif, const double* ifz, TreeGeom geo,
                            unsigned* keys, int* perm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = xyz[i], y = xyz[n + i], z = xyz[2 * n + i];
  int l = 0;
  for (int j = 0; j < nif; ++j) l += (z < ifz[j]);
  const int g = geo.group_of_layer[l];
  const int nb = 1 << geo.depth[g];
  const double inv = nb / geo.side[g];
  int ix = (int)floor((x - geo.lo[g][0]) * inv);
  int iy = (int)floor((y - geo.lo[g][1]) * inv);
  int iz = (int)floor((z - geo.lo[g][2]) * inv);
  ix = min(max(ix, 0), nb - 1);
  iy = min(max(iy, 0), nb - 1);
  iz = min(max(iz, 0), nb - 1);
  keys[i] = (unsigned)(geo.leaf_offset[g] + ((int64_t)ix * nb + iy) * nb + iz);
  perm[i] = (int)i;
}

__global__ void k_count_keys(const unsigned* keys, int64_t n, int* count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&count[keys[i]], 1);
}

__global__ void k_gather_pos(const double* xyz, const int* perm, int64_t n, double* xs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int j = perm[i];
  xs[i] = xyz[j];
  xs[n + i] = xyz[n + j];
  xs[2 * n + i] = xyz[2 * n + j];
}

// ---------------------------------------------------------------------------
// Charges in, potentials out.
// ---------------------------------------------------------------------------
__global__ void k_gather_q(const double2* q, const int* perm, int64_t n, double2* qs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (i < n) qs[(int64_t)r * n + i] = q[(int64_t)r * n + perm[i]];
}

__global__ void k_finalize(const double2* phi_s, const double2* phi_near, const int* perm, int64_t start, int64_t cnt,
                           int64_t n, double sr, double si, double2* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int r = blockIdx.y;
  if (i >= cnt) return;
  i += start;
  const double2 f = phi_s[(int64_t)r * n + i], c = phi_near[(int64_t)r * n + i];
  const double2 v = make_double2(f.x + c.x, f.y + c.y);
  out[(int64_t)r * n + perm[i]] = make_double2(v.x * sr - v.y * si, v.x * si + v.y * sr);
}

// ---------------------------------------------------------------------------
// Direct Sigma-family reaction interactions of listed leaf pairs (the local
// reaction interactions of Algorithm 1 evaluated directly, here only where the
// expansions would not converge).  One workgroup of 128 per listed target leaf and
// charge vector (blockIdx.y); targets in passes of 128, sources staged in LDS in
// chunks of 128; every target written by one lane (no atomics).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void k_sigma_direct(SigmaDirectArgs a) {
  __shared__ double sx[128], sy[128], sz[128];
  __shared__ double2 sq[128];
  __shared__ double2 simg[2 * SIGMA_DIRECT_MAX_IMAGES];
  const int tl = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int nimg = a.nup + a.ndn;
  for (int i = tid; i < 2 * nimg; i += 128) simg[i] = a.img[i];
  const int leaf = a.tgt[tl];
  const int ts = a.leaf_start[a.leaf_base + leaf], tc = a.leaf_count[a.leaf_base + leaf];
  const int s0 = a.src_start[tl], s1 = a.src_start[tl + 1];
  const double* X = a.xs;
  const double* Y = a.xs + a.n;
  const double* Z = a.xs + 2 * a.n;
  const double2* q = a.q + (int64_t)r * a.n;
  for (int t0 = 0; t0 < tc; t0 += 128) {
    const int i = t0 + tid;
    const bool act = i < tc;
    const double xt = act ? X[ts + i] : 0.0, yt = act ? Y[ts + i] : 0.0, zt = act ? Z[ts + i] : 0.0;
    dc acc = {0.0, 0.0};
    for (int e = s0; e < s1; ++e) {
      const int sl = a.src[e];
      const int ss = a.leaf_start[a.leaf_base + sl], sc = a.leaf_count[a.leaf_base + sl];
      for (int c0 = 0; c0 < sc; c0 += 128) {
        const int cn = min(128, sc - c0);
        __syncthreads();
        if (tid < cn) {
          const int j = ss + c0 + tid;
          sx[tid] = X[j], sy[tid] = Y[j], sz[tid] = Z[j], sq[tid] = q[j];
        }
        __syncthreads();
        if (!act) continue;
        for (int j = 0; j < cn; ++j) {
          const double dx = xt - sx[j], dy = yt - sy[j], S = zt + sz[j];
          const double rho2 = dx * dx + dy * dy;
          dc kv = {0.0, 0.0};
          for (int m = 0; m < nimg; ++m) {
            const double2 A = simg[2 * m], Zi = simg[2 * m + 1];
            const double e0 = m < a.nup ? S - a.two_dl : a.two_dt - S;
            const dc zeta = {e0 - Zi.x, -Zi.y};
            if (zeta.x <= 0.0) continue;
            const dc R2 = {rho2 + zeta.x * zeta.x - zeta.y * zeta.y, 2.0 * zeta.x * zeta.y};
            const dc R = csqrt_pr(R2);
            kv = cadd(kv, cmul({A.x, A.y}, cdiv(cexp_i(R, a.k), R)));
          }
          acc = cadd(acc, cmul(kv, {sq[j].x, sq[j].y}));
        }
      }
    }
    if (act) {
      double2* o = a.phi + (int64_t)r * a.n + ts + i;
      *o = make_double2(o->x + acc.x, o->y + acc.y);
    }
  }
}

// ---------------------------------------------------------------------------
// P2M (Sec. 3.1, Eq. taylorexpfarxcfree): alpha^_k = sum_j q_j u_j^k,
// u_j = (r_j - c)/h, one 64-lane block per leaf.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_p2m(PassArgs a) {
  extern __shared__ double lds_p2m[];
  const int P1 = a.p + 1;
  double* pw = lds_p2m;                              // [64][3][P1]
  double2* sq = (double2*)(lds_p2m + 64 * 3 * P1);   // [64]
  const int leaf = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int nb = a.nbox_dim;
  const int ix = leaf / (nb * nb), iy = (leaf / nb) % nb, iz = leaf % nb;
  const double h = a.h;
  const double cx = a.lo[0] + (ix + 0.5) * h, cy = a.lo[1] + (iy + 0.5) * h, cz = a.lo[2] + (iz + 0.5) * h;
  const int start = a.leaf_start[a.leaf_base + leaf], cnt = a.leaf_count[a.leaf_base + leaf];
  const double2* q = a.q + (int64_t)r * a.n;
  constexpr int MAXK = 16;  // nC <= 1024 (p <= 16)
  dc acc[MAXK];
#pragma unroll
  for (int j = 0; j < MAXK; ++j) acc[j] = {0, 0};
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    const int m = min(64, cnt - c0);
    if (tid < m) {
      const int64_t i = start + c0 + tid;
      const double u[3] = {(a.xs[i] - cx) / h, (a.xs[a.n + i] - cy) / h, (a.xs[2 * a.n + i] - cz) / h};
      for (int d = 0; d < 3; ++d) {
        double v = 1.0;
        for (int e = 0; e < P1; ++e) pw[(tid * 3 + d) * P1 + e] = v, v *= u[d];
      }
      sq[tid] = q[i];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MAXK; ++j) {
      const int k = tid + 64 * j;
      if (k < a.nC) {
        const int pk = a.mi[k];
        const int k1 = pk & 255, k2 = (pk >> 8) & 255, k3 = pk >> 16;
        dc s = acc[j];
        for (int t = 0; t < m; ++t) {
          const double w = pw[(t * 3 + 0) * P1 + k1] * pw[(t * 3 + 1) * P1 + k2] * pw[(t * 3 + 2) * P1 + k3];
          s.x += sq[t].x * w;
          s.y += sq[t].y * w;
        }
        acc[j] = s;
      }
    }
    __syncthreads();
  }
  double2* out = a.alpha + (int64_t)r * a.rhs_stride + (int64_t)leaf * a.nC;
#pragma unroll
  for (int j = 0; j < MAXK; ++j) {
    const int k = tid + 64 * j;
    if (k < a.nC) out[k] = make_double2(acc[j].x, acc[j].y);
  }
}

// ---------------------------------------------------------------------------
// Helmholtz reduction.  Every table satisfies the Helmholtz equation in the
// displacement: G_{g+2e1} = -G_{g+2e2} - G_{g+2e3} - (kh)^2 G_g.  In the M2L sum
// b_k = sum_{k'} G_{k+k'} a_{k'} the terms with k'1 >= 2 can therefore be moved
// onto k' - 2e1 + 2e2, k' - 2e1 + 2e3 and k' - 2e1 (same or lower order), which
// leaves moments with k'1 <= 1 only; likewise only b_k with k1 <= 1 need to be
// computed and the rest follow from the same identity.  Both steps are exact.
// k_reduce: a_k = (-1)^{|k|} alpha^_k / k!, folded down to k1 <= 1.
// One 64-lane block per box.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reduce(ReduceArgs a) {
  extern __shared__ double2 lds_red[];  // [nC]
  const int box = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const double2* in = a.in + (int64_t)r * a.in_stride + (int64_t)box * a.nC;
  for (int k = tid; k < a.nC; k += 64) {
    const double s = a.scale[k];
    const double2 v = in[k];
    lds_red[k] = make_double2(v.x * s, v.y * s);
  }
  __syncthreads();
  // gather form, targets at level k1 = t1 receive from level t1 + 2 (already final)
  for (int t1 = a.p - 2; t1 >= 0; --t1) {
    const int m = a.p - t1;  // k2 + k3 <= m
    const int cnt = ((m + 1) * (m + 2)) / 2;
    for (int e = tid; e < cnt; e += 64) {
      // enumerate (k2, k3) with k2 + k3 <= m
      int tt = 0;
      while ((tt + 1) * (tt + 2) / 2 <= e) ++tt;
      const int k3 = e - tt * (tt + 1) / 2, k2 = tt - k3;
      double2 acc = lds_red[mi_index(t1, k2, k3)];
      if (k2 >= 2) {
        const double2 v = lds_red[mi_index(t1 + 2, k2 - 2, k3)];
        acc.x -= v.x, acc.y -= v.y;
      }
      if (k3 >= 2) {
        const double2 v = lds_red[mi_index(t1 + 2, k2, k3 - 2)];
        acc.x -= v.x, acc.y -= v.y;
      }
      if (t1 + 2 + k2 + k3 <= a.p) {
        const double2 v = lds_red[mi_index(t1 + 2, k2, k3)];
        acc.x -= a.kh2 * v.x, acc.y -= a.kh2 * v.y;
      }
      lds_red[mi_index(t1, k2, k3)] = acc;
    }
    __syncthreads();
  }
  if (a.out32) {
    float2* out = a.out32 + (int64_t)r * a.out_stride + (int64_t)box * a.nR;
    for (int i = tid; i < a.nR; i += 64) {
      const double2 v = lds_red[a.rfull[i]];
      out[i] = make_float2((float)v.x, (float)v.y);
    }
    return;
  }
  double2* out = a.out + (int64_t)r * a.out_stride + (int64_t)box * a.nR;
  for (int i = tid; i < a.nR; i += 64) out[i] = lds_red[a.rfull[i]];
}

// Index of the multi-index whose component along `ax` is t and whose other two
// components (in increasing axis order) are u, v.
__device__ __forceinline__ int mi_axis(int ax, int t, int u, int v) {
  return ax == 0 ? mi_index(t, u, v) : (ax == 1 ? mi_index(u, t, v) : mi_index(u, v, t));
}

// The same reduction along z (moments with k3 <= 1), used by the cross-layer
// translation: a_k = (-1)^{|k|} alpha^_k / k!, folded with
// G_{g+2e3} = -G_{g+2e1} - G_{g+2e2} - (kh)^2 G_g.
__global__ __launch_bounds__(64) void k_reduce_z(ReduceArgs a) {
  extern __shared__ double2 lds_rz[];  // [nC]
  const int box = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const double2* in = a.in + (int64_t)r * a.in_stride + (int64_t)box * a.nC;
  for (int k = tid; k < a.nC; k += 64) {
    const double s = a.scale[k];
    const double2 v = in[k];
    lds_rz[k] = make_double2(v.x * s, v.y * s);
  }
  __syncthreads();
  for (int t3 = a.p - 2; t3 >= 0; --t3) {
    const int m = a.p - t3;
    const int cnt = ((m + 1) * (m + 2)) / 2;
    for (int e = tid; e < cnt; e += 64) {
      int tt = 0;
      while ((tt + 1) * (tt + 2) / 2 <= e) ++tt;
      const int k2 = e - tt * (tt + 1) / 2, k1 = tt - k2;
      double2 acc = lds_rz[mi_axis(2, t3, k1, k2)];
      if (k1 >= 2) {
        const double2 v = lds_rz[mi_axis(2, t3 + 2, k1 - 2, k2)];
        acc.x -= v.x, acc.y -= v.y;
      }
      if (k2 >= 2) {
        const double2 v = lds_rz[mi_axis(2, t3 + 2, k1, k2 - 2)];
        acc.x -= v.x, acc.y -= v.y;
      }
      if (t3 + 2 + k1 + k2 <= a.p) {
        const double2 v = lds_rz[mi_axis(2, t3 + 2, k1, k2)];
        acc.x -= a.kh2 * v.x, acc.y -= a.kh2 * v.y;
      }
      lds_rz[mi_axis(2, t3, k1, k2)] = acc;
    }
    __syncthreads();
  }
  double2* out = a.out + (int64_t)r * a.out_stride + (int64_t)box * a.nR;
  for (int i = tid; i < a.nR; i += 64) out[i] = lds_rz[a.rfull[i]];
}

// z-direction expansion of cross-layer locals (k3 <= 1 -> all |k| <= p), then
// beta^_k += b_k / k!  (adds to the locals already written).
__global__ __launch_bounds__(64) void k_expand_z_add(ReduceArgs a) {
  extern __shared__ double2 lds_ez[];  // [nC]
  const int box = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const double2* in = a.in + (int64_t)r * a.in_stride + (int64_t)box * a.nR;
  for (int i = tid; i < a.nR; i += 64) {
    double2 v = in[i];
    for (int sp = 1; sp < a.nsplit; ++sp) {  // partial sets of a split translation, fixed order
      const double2 u = in[(int64_t)sp * a.split_stride + i];
      v.x += u.x, v.y += u.y;
    }
    lds_ez[a.rfull[i]] = v;
  }
  __syncthreads();
  for (int k3 = 2; k3 <= a.p; ++k3) {
    const int m = a.p - k3;
    const int cnt = ((m + 1) * (m + 2)) / 2;
    for (int e = tid; e < cnt; e += 64) {
      int tt = 0;
      while ((tt + 1) * (tt + 2) / 2 <= e) ++tt;
      const int k2 = e - tt * (tt + 1) / 2, k1 = tt - k2;
      const double2 u = lds_ez[mi_axis(2, k3 - 2, k1 + 2, k2)];
      const double2 v = lds_ez[mi_axis(2, k3 - 2, k1, k2 + 2)];
      const double2 w = lds_ez[mi_axis(2, k3 - 2, k1, k2)];
      lds_ez[mi_axis(2, k3, k1, k2)] = make_double2(-u.x - v.x - a.kh2 * w.x, -u.y - v.y - a.kh2 * w.y);
    }
    __syncthreads();
  }
  double2* out = a.out + (int64_t)r * a.out_stride + (int64_t)box * a.nC;
  for (int k = tid; k < a.nC; k += 64) {
    const double f = a.invfact[k];
    const double2 v = lds_ez[k], o = out[k];
    out[k] = make_double2(o.x + v.x * f, o.y + v.y * f);
  }
}

// k_expand: b (k1 <= 1; the sum of nsplit partial sets) -> all |k| <= p by
// b_k = -b_{k-2e1+2e2} - b_{k-2e1+2e3} - (kh)^2 b_{k-2e1}, then beta^_k = b_k / k!.
// Overwrites beta^.
__global__ __launch_bounds__(64) void k_expand(ReduceArgs a) {
  extern __shared__ double2 lds_exp[];  // [nC]
  const int box = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const double2* in = a.in + (int64_t)r * a.in_stride + (int64_t)box * a.nR;
  for (int i = tid; i < a.nR; i += 64) {
    double2 v = in[i];
    for (int sp = 1; sp < a.nsplit; ++sp) {  // partial sets of a split M2L, fixed order
      const double2 u = in[(int64_t)sp * a.split_stride + i];
      v.x += u.x, v.y += u.y;
    }
    lds_exp[a.rfull[i]] = v;
  }
  __syncthreads();
  for (int k1 = 2; k1 <= a.p; ++k1) {
    const int m = a.p - k1;
    const int cnt = ((m + 1) * (m + 2)) / 2;
    for (int e = tid; e < cnt; e += 64) {
      int tt = 0;
      while ((tt + 1) * (tt + 2) / 2 <= e) ++tt;
      const int k3 = e - tt * (tt + 1) / 2, k2 = tt - k3;
      const double2 u = lds_exp[mi_index(k1 - 2, k2 + 2, k3)];
      const double2 v = lds_exp[mi_index(k1 - 2, k2, k3 + 2)];
      const double2 w = lds_exp[mi_index(k1 - 2, k2, k3)];
      lds_exp[mi_index(k1, k2, k3)] = make_double2(-u.x - v.x - a.kh2 * w.x, -u.y - v.y - a.kh2 * w.y);
    }
    __syncthreads();
  }
  double2* out = a.out + (int64_t)r * a.out_stride + (int64_t)box * a.nC;
  for (int k = tid; k < a.nC; k += 64) {
    const double f = a.invfact[k];
    const double2 v = lds_exp[k];
    out[k] = make_double2(v.x * f, v.y * f);
  }
}

// ---------------------------------------------------------------------------
// M2M (Sec. 3.1, Eq. TETartoTETar) and L2L (Eq. freeletole).  Both shifts are
// products of one-dimensional binomial shifts, applied here as three passes
// (x, then y, then z) over the coefficient set |k| <= p; every intermediate
// that the final result needs also has total order <= p, so the passes are
// exact.  Child centre relative to the parent, in parent units:
// delta_i = (c_i - 1/2)/2 = +-1/4.
//   M2M: alpha^P_k = sum_{k' <= k} prod_i C(k_i, k'_i) delta_i^{k_i-k'_i} 2^{-k'_i} alpha^C_{k'}
//   L2L: beta^C_k = sum_{k' >= k} prod_i C(k'_i, k_i) delta_i^{k'_i-k_i} 2^{-k_i} beta^P_{k'}
// ---------------------------------------------------------------------------
__device__ __forceinline__ double quarter_pow(int neg, int e) {
  // (+-1/4)^e
  const double v = ldexp(1.0, -2 * e);
  return (neg && (e & 1)) ? -v : v;
}

// One coefficient of a pass along axis `ax` of the upward shift: for the packed
// multi-index pk = k, sum_{j <= k_ax} C(k_ax, j) delta^{k_ax - j} 2^{-j} src[k with k_ax -> j]
__device__ __forceinline__ double2 m2m_coef(const double2* src, int pk, int ax, int neg) {
  int c[3] = {pk & 255, (pk >> 8) & 255, pk >> 16};
  const int ka = c[ax];
  double sx = 0, sy = 0;
  for (int j = 0; j <= ka; ++j) {
    c[ax] = j;
    const double f = c_binom[ka][j] * quarter_pow(neg, ka - j) * ldexp(1.0, -j);
    const double2 v = src[mi_index(c[0], c[1], c[2])];
    sx += f * v.x;
    sy += f * v.y;
  }
  return make_double2(sx, sy);
}

// Within a wave, data written to LDS by some lanes and read by others: the
// wave's LDS operations complete in order, so only the compiler must keep them
// in order.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// One workgroup per parent box; its W waves (W = blockDim.x / 64, a divisor of 8)
// take the children c = w, w + W, ...  Each wave stages its child in its own two
// LDS buffers, applies the x and y passes there and the z pass straight into its
// registers (coefficient lane + 64 i in slot i), so the waves need no barrier until
// their sums of shifted children are added, in wave order.
constexpr int M2M_SLOTS = 16;  // coefficients per lane: nC <= 1024 (p <= 16)
__global__ __launch_bounds__(512) void k_m2m(PassArgs a) {
  extern __shared__ double2 lds_m2m[];  // per wave 2 x nC, then the multi-indices (nC ints)
  const int W = blockDim.x >> 6, nC = a.nC;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double2* b0 = lds_m2m + (size_t)w * 2 * nC;
  double2* b1 = b0 + nC;
  int* smi = (int*)(lds_m2m + (size_t)W * 2 * nC);
  const int pb = blockIdx.x, r = blockIdx.y;
  const int np = a.nbox_dim;  // parent grid size
  const int nc = 2 * np;
  const int ix = pb / (np * np), iy = (pb / np) % np, iz = pb % np;
  const double2* ch = a.alpha_child + (int64_t)r * a.rhs_stride_child;
  for (int k = tid; k < nC; k += blockDim.x) smi[k] = a.mi[k];
  __syncthreads();
  double sx[M2M_SLOTS], sy[M2M_SLOTS];
#pragma unroll
  for (int i = 0; i < M2M_SLOTS; ++i) sx[i] = 0.0, sy[i] = 0.0;
  for (int c = w; c < 8; c += W) {
    const int cx = (c >> 2) & 1, cy = (c >> 1) & 1, cz = c & 1;
    const int64_t cb = ((int64_t)(2 * ix + cx) * nc + (2 * iy + cy)) * nc + (2 * iz + cz);
    for (int k = lane; k < nC; k += 64) b0[k] = ch[cb * nC + k];
    wave_lds_sync();
    for (int k = lane; k < nC; k += 64) b1[k] = m2m_coef(b0, smi[k], 0, !cx);
    wave_lds_sync();
    for (int k = lane; k < nC; k += 64) b0[k] = m2m_coef(b1, smi[k], 1, !cy);
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < M2M_SLOTS; ++i) {
      const int k = lane + 64 * i;
      if (k < nC) {
        const double2 v = m2m_coef(b0, smi[k], 2, !cz);
        sx[i] += v.x, sy[i] += v.y;
      }
    }
    wave_lds_sync();  // the next child overwrites b0
  }
#pragma unroll
  for (int i = 0; i < M2M_SLOTS; ++i) {
    const int k = lane + 64 * i;
    if (k < nC) b1[k] = make_double2(sx[i], sy[i]);
  }
  __syncthreads();
  double2* out = a.alpha + (int64_t)r * a.rhs_stride + (int64_t)pb * nC;
  for (int k = tid; k < nC; k += blockDim.x) {
    double2 v = lds_m2m[nC + k];
    for (int ww = 1; ww < W; ++ww) {
      const double2 u = lds_m2m[(size_t)ww * 2 * nC + nC + k];
      v.x += u.x, v.y += u.y;
    }
    out[k] = v;
  }
}

// One pass of the downward shift: dst[k] = 2^{-k_ax} sum_{j >= k_ax} C(j, k_ax) delta^{j - k_ax}
// src[k with k_ax -> j], j up to p minus the other two components.
__device__ __forceinline__ void l2l_pass(const double2* src, double2* dst, const int* mi, int nC, int p, int ax,
                                         int neg, int tid) {
  for (int k = tid; k < nC; k += 64) {
    const int pk = mi[k];
    int c[3] = {pk & 255, (pk >> 8) & 255, pk >> 16};
    const int ka = c[ax];
    const int top = p - (c[0] + c[1] + c[2] - ka);
    double sx = 0, sy = 0;
    for (int j = ka; j <= top; ++j) {
      c[ax] = j;
      const double f = c_binom[j][ka] * quarter_pow(neg, j - ka);
      const double2 v = src[mi_index(c[0], c[1], c[2])];
      sx += f * v.x;
      sy += f * v.y;
    }
    const double s = ldexp(1.0, -ka);
    dst[k] = make_double2(s * sx, s * sy);
  }
}

__global__ __launch_bounds__(64) void k_l2l(PassArgs a) {
  extern __shared__ double2 lds_l2l[];  // b0, b1: 2 x nC
  double2* b0 = lds_l2l;
  double2* b1 = b0 + a.nC;
  int* smi = (int*)(b1 + a.nC);
  const int cb = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int nc = a.nbox_dim, np = nc / 2;
  const int ix = cb / (nc * nc), iy = (cb / nc) % nc, iz = cb % nc;
  const int64_t pb = ((int64_t)(ix >> 1) * np + (iy >> 1)) * np + (iz >> 1);
  const double2* par = a.beta_parent + (int64_t)r * a.rhs_stride_parent + pb * a.nC;
  for (int k = tid; k < a.nC; k += 64) b0[k] = par[k], smi[k] = a.mi[k];
  __syncthreads();
  l2l_pass(b0, b1, smi, a.nC, a.p, 0, !(ix & 1), tid);
  __syncthreads();
  l2l_pass(b1, b0, smi, a.nC, a.p, 1, !(iy & 1), tid);
  __syncthreads();
  l2l_pass(b0, b1, smi, a.nC, a.p, 2, !(iz & 1), tid);
  __syncthreads();
  double2* out = a.beta + (int64_t)r * a.rhs_stride + (int64_t)cb * a.nC;
  for (int k = tid; k < a.nC; k += 64) {
    const double2 o = out[k];
    out[k] = make_double2(o.x + b1[k].x, o.y + b1[k].y);
  }
}

// ---------------------------------------------------------------------------
// L2P (Sec. 3.1, Eq. taylorexplocxclfree): phi_i = sum_k beta^_k u_i^k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_l2p(PassArgs a) {
  // the leaf's local coefficients in nested order (k1, then k2, then k3 ascending), so
  // that each particle walks them with running products of its scaled offsets
  extern __shared__ double lds_l2p[];
  double2* sb = (double2*)lds_l2p;  // [nC]
  const int p = a.p;
  const int leaf = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
  const int nb = a.nbox_dim;
  const int ix = leaf / (nb * nb), iy = (leaf / nb) % nb, iz = leaf % nb;
  const double h = a.h;
  const double cx = a.lo[0] + (ix + 0.5) * h, cy = a.lo[1] + (iy + 0.5) * h, cz = a.lo[2] + (iz + 0.5) * h;
  const int start = a.leaf_start[a.leaf_base + leaf], cnt = a.leaf_count[a.leaf_base + leaf];
  if (cnt == 0) return;
  const double2* bt = a.beta + (int64_t)r * a.rhs_stride + (int64_t)leaf * a.nC;
  for (int k = tid; k < a.nC; k += 64) {
    const int pk = a.mi[k];
    const int k1 = pk & 255, k2 = (pk >> 8) & 255, k3 = pk >> 16;
    int pos = 0;  // tuples before (k1, k2, k3) in nested order
    for (int t = 0; t < k1; ++t) pos += ((p - t + 1) * (p - t + 2)) / 2;
    for (int t = 0; t < k2; ++t) pos += p - k1 - t + 1;
    sb[pos + k3] = bt[k];
  }
  __syncthreads();
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    if (c0 + tid >= cnt) break;
    const int64_t i = start + c0 + tid;
    const double ux = (a.xs[i] - cx) / h, uy = (a.xs[a.n + i] - cy) / h, uz = (a.xs[2 * a.n + i] - cz) / h;
    double sx = 0.0, sy = 0.0, wx = 1.0;
    int e = 0;
    for (int k1 = 0; k1 <= p; ++k1) {
      double wxy = wx;
      for (int k2 = 0; k2 <= p - k1; ++k2) {
        double w = wxy;
        for (int k3 = 0; k3 <= p - k1 - k2; ++k3, ++e) {
          sx = fma(sb[e].x, w, sx);
          sy = fma(sb[e].y, w, sy);
          w *= uz;
        }
        wxy *= uy;
      }
      wx *= ux;
    }
    a.phi[(int64_t)r * a.n + i] = make_double2(sx, sy);
  }
}

// ---------------------------------------------------------------------------
// P2P, free space (Eq. totalinteraction, free part): for every target in a
// leaf, sum over the 27 neighbour leaves (itself included, j = i excluded) of
// q_j exp(i k r)/r.  One block of BS lanes (64 or 256, by mean leaf occupancy)
// per target leaf.  Leaves are stored in
// (x, y, z) order, so the three z-neighbours of one (x, y) column are one
// contiguous particle range: nine ranges per leaf, staged through LDS.
// Writes the near-field sum (its own buffer: it runs beside the far field).
// ---------------------------------------------------------------------------

// sin and cos of 0 <= x < 1e4 in FP64: x = q pi/2 + y with pi/2 split in two
// parts (Cody and Waite), |y| <= pi/4, then the Taylor series of sin y (to
// y^15) and cos y (to y^16); the first omitted terms are below 5e-17 and 2e-18.
__device__ __forceinline__ void sincos_f64(double x, double* s, double* c) {
  const double q = rint(x * 0.63661977236758134308);
  double y = fma(-q, 1.5707963267948965580e+00, x);
  y = fma(-q, 6.1232339957367658e-17, y);
  const double y2 = y * y;
  double ps = -7.6471637318198164759e-13;         // -1/15!
  ps = fma(ps, y2, 1.6059043836821614599e-10);    //  1/13!
  ps = fma(ps, y2, -2.5052108385441718775e-08);   // -1/11!
  ps = fma(ps, y2, 2.7557319223985890653e-06);    //  1/9!
  ps = fma(ps, y2, -1.9841269841269841270e-04);   // -1/7!
  ps = fma(ps, y2, 8.3333333333333333333e-03);    //  1/5!
  ps = fma(ps, y2, -1.6666666666666666667e-01);   // -1/3!
  const double sy = fma(y * y2, ps, y);
  double pc = 4.7794773323873852974e-14;          //  1/16!
  pc = fma(pc, y2, -1.1470745597729724714e-11);   // -1/14!
  pc = fma(pc, y2, 2.0876756987868098979e-09);    //  1/12!
  pc = fma(pc, y2, -2.7557319223985890653e-07);   // -1/10!
  pc = fma(pc, y2, 2.4801587301587301587e-05);    //  1/8!
  pc = fma(pc, y2, -1.3888888888888888889e-03);   // -1/6!
  pc = fma(pc, y2, 4.1666666666666666667e-02);    //  1/4!
  pc = fma(pc, y2, -0.5);
  const double cy = fma(y2, pc, 1.0);
  const int qi = ((int)q) & 3;
  const double s0 = (qi & 1) ? cy : sy, c0 = (qi & 1) ? sy : cy;
  *s = (qi & 2) ? -s0 : s0;
  *c = ((qi + 1) & 2) ? -c0 : c0;
}

// 1/sqrt(r2) in FP64: FP32 estimate (relative error ~1e-7) refined by one
// Newton step (error squared: ~2e-14, far below the FP64 mode's 1e-6 target).
__device__ __forceinline__ double rsqrt_f64(double r2) {
  // the hardware estimate directly (pair distances are far above the FP32 denormal range)
  const double y = (double)__builtin_amdgcn_rsqf((float)r2);
  return y * fma(-0.5 * r2, y * y, 1.5);
}

// The same sine and cosine for 0 <= x <= pi/4 (no reduction needed).
__device__ __forceinline__ void sincos_f64_small(double y, double* s, double* c) {
  const double y2 = y * y;
  double ps = -7.6471637318198164759e-13;
  ps = fma(ps, y2, 1.6059043836821614599e-10);
  ps = fma(ps, y2, -2.5052108385441718775e-08);
  ps = fma(ps, y2, 2.7557319223985890653e-06);
  ps = fma(ps, y2, -1.9841269841269841270e-04);
  ps = fma(ps, y2, 8.3333333333333333333e-03);
  ps = fma(ps, y2, -1.6666666666666666667e-01);
  *s = fma(y * y2, ps, y);
  double pc = 4.7794773323873852974e-14;
  pc = fma(pc, y2, -1.1470745597729724714e-11);
  pc = fma(pc, y2, 2.0876756987868098979e-09);
  pc = fma(pc, y2, -2.7557319223985890653e-07);
  pc = fma(pc, y2, 2.4801587301587301587e-05);
  pc = fma(pc, y2, -1.3888888888888888889e-03);
  pc = fma(pc, y2, 4.1666666666666666667e-02);
  pc = fma(pc, y2, -0.5);
  *c = fma(y2, pc, 1.0);
}

__device__ __forceinline__ void pair_kernel(double r2, double k, double* er, double* ei) {
  const double ri = rsqrt_f64(r2);
  double sn, cs;
  sincos_f64(k * (r2 * ri), &sn, &cs);
  *er = cs * ri, *ei = sn * ri;
}
// FP32 pair on coordinates pre-scaled by k / (2 pi): r2 is (k r / 2 pi)^2, the
// hardware sine and cosine take revolutions, and the common factor k / (2 pi)
// of 1/r is applied once to the sum.
__device__ __forceinline__ void pair_kernel(float r2, float, float* er, float* ei) {
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float rv = r2 * ri;
  *er = __builtin_amdgcn_cosf(rv) * ri, *ei = __builtin_amdgcn_sinf(rv) * ri;
}
// The same value with cos(2 pi r) and sin(2 pi r) / r from quadratics in r2 fitted
// over the distances at hand (POLY): one transcendental (the reciprocal square root)
// and five multiply-adds in place of three transcendentals and three products.
template <bool POLY>
__device__ __forceinline__ void pair_value(float r2, const NearPoly& np, float* er, float* ei) {
  if (POLY) {
    const float ri = __builtin_amdgcn_rsqf(r2);
    *er = fmaf(fmaf(np.c2, r2, np.c1), r2, np.c0) * ri;
    *ei = fmaf(fmaf(np.s2, r2, np.s1), r2, np.s0);
  } else {
    pair_kernel(r2, 0.0f, er, ei);
  }
}

// FP64 pair loop over m staged sources (see k_p2p).
template <int RB, bool SMALL, bool SELF, typename T>
__device__ __forceinline__ void p2p_f64_rows(int m, T tx, T ty, T tz, const T* sx, const T* sy, const T* sz,
                                             const T (*sq)[2 * RB], double k, T* accr, T* acci) {
#pragma unroll 4
  for (int t = 0; t < m; ++t) {
    const double dx = tx - sx[t], dy = ty - sy[t], dz = tz - sz[t];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const bool self = SELF && !(r2 > 0);
    const double ri = rsqrt_f64(self ? 1.0 : r2);
    double sn, cs;
    if (SMALL)
      sincos_f64_small(k * (r2 * ri), &sn, &cs);
    else
      sincos_f64(k * (r2 * ri), &sn, &cs);
    const double er = cs * ri, ei = sn * ri;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const double wr = self ? 0.0 : (double)sq[t][2 * b], wi = self ? 0.0 : (double)sq[t][2 * b + 1];
      accr[b] += wr * er - wi * ei;
      acci[b] += wr * ei + wi * er;
      // several vectors: keep the sums with this source (else the compiler defers them and
      // holds every pair value: 256 registers and spills at 8 vectors).  One vector: left
      // alone, its 122 registers leave room for the far field running beside it.
      if (RB > 1) asm volatile("" : "+v"(accr[b]), "+v"(acci[b]));
    }
  }
}

// FP32 pair loop over m staged sources (see k_p2p). Every pair is evaluated in
// FP32 with its squared distance raised to at least rns2, so the pair with
// itself and near-singular pairs (closer than 5% of the leaf side, where the
// FP32 difference has lost digits) give a finite, known term. Sources are taken
// four at a time and one wave-wide test per four decides whether any lane met
// such a pair; only then (rare) the known FP32 term is taken back in FP64 and
// the pair redone in FP64 from the stored coordinates (the pair with itself: 0).
template <int RB, bool POLY, bool OWN>
__device__ __forceinline__ void p2p_f32_rows(int m, float tx, float ty, float tz, const float4* s4,
                                             const float (*sq)[2 * RB], const int* sidx, float rns2, float ecr,
                                             float eci, double kap, const PassArgs& a, int64_t i, double txd,
                                             double tyd, double tzd, int r0, int nrhs, float* accr, float* acci,
                                             double* ns, const NearPoly& np) {
  // OWN (the column holding the target itself): the pair of a particle with itself,
  // found by its index, gets weight 0 in the FP32 sum and is moved out of the near test;
  // pairs with r2 < rns2 (a distinct particle at FP32 distance 0 included) are taken
  // back and redone in FP64, their sums kept in ns[2 b], ns[2 b + 1] (FP64, in LDS: rare)
  const unsigned near_lim = (unsigned)__float_as_int(rns2);
  auto nearp = [&](float r2) { return (unsigned)__float_as_int(r2) < near_lim; };
  auto fixup = [&](int t, float r2) {
    if (!nearp(r2)) return;
    const int64_t j = sidx[t];
    double er = 0.0, ei = 0.0;
    if (j != i) {
      const double ex = txd - a.xs[j], ey = tyd - a.xs[a.n + j], ez = tzd - a.xs[2 * a.n + j];
      pair_kernel(ex * ex + ey * ey + ez * ez, a.k, &er, &ei);
    }
#pragma unroll
    for (int b = 0; b < RB; ++b)
      if (r0 + b < nrhs) {
        const double2 qv = a.q[(int64_t)(r0 + b) * a.n + j];
        const double qr = sq[t][2 * b], qi = sq[t][2 * b + 1];
        ns[2 * b] += qv.x * er - qv.y * ei - kap * (qr * ecr - qi * eci);
        ns[2 * b + 1] += qv.x * ei + qv.y * er - kap * (qr * eci + qi * ecr);
      }
  };
  // a source's charges in registers: RB complex values, loaded four floats at a time
  // (two at RB = 1), so that the next source's are in flight while this one's sums form
  constexpr int Q4 = (2 * RB + 3) / 4;
  struct QV {
    float4 v[Q4];
  };
  auto qload = [&](int t, QV& q) {
    if constexpr (RB == 1) {
      const float2 c = *(const float2*)sq[t];
      q.v[0] = make_float4(c.x, c.y, 0.0f, 0.0f);
    } else {
#pragma unroll
      for (int k = 0; k < Q4; ++k) q.v[k] = ((const float4*)sq[t])[k];
    }
  };
  auto pair = [&](float r2, const QV& q, bool self) {
    // max of two non-negative floats as the max of their bit patterns (no canonicalising)
    float er, ei;
    pair_value<POLY>(__int_as_float(max(__float_as_int(r2), __float_as_int(rns2))), np, &er, &ei);
    if (self) er = 0.0f, ei = 0.0f;
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      const float4 w = q.v[b >> 1];
      const float qr = (b & 1) ? w.z : w.x, qi = (b & 1) ? w.w : w.y;
      accr[b] = fmaf(qr, er, fmaf(-qi, ei, accr[b]));
      acci[b] = fmaf(qr, ei, fmaf(qi, er, acci[b]));
      // keep the sums with this source (else the compiler defers them and holds every pair value)
      asm volatile("" : "+v"(accr[b]), "+v"(acci[b]));
    }
  };
  m = __builtin_amdgcn_readfirstlane(m);
  int t = 0;
  QV qa, qb;
  if (m >= 4) qload(0, qa);
  for (; t + 4 <= m; t += 4) {
    float r2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float4 s = s4[t + u];
      const float dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
      r2[u] = dx * dx + dy * dy + dz * dz;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // source t + u's charges are in qa (u even) or qb (u odd); the next source's go
      // into the other set before this one's sums
      QV& cur = (u & 1) ? qb : qa;
      QV& nxt = (u & 1) ? qa : qb;
      if (u < 3 || t + 4 < m) qload(t + u + 1, nxt);
      pair(r2[u], cur, OWN && sidx[t + u] == i);
    }
    // the self pair's stand-in distance: beyond the near test (after its use above,
    // where only its weight mattered)
    if (OWN)
#pragma unroll
      for (int u = 0; u < 4; ++u) r2[u] = sidx[t + u] == i ? 3.0e38f : r2[u];
    const unsigned mn = min(min((unsigned)__float_as_int(r2[0]), (unsigned)__float_as_int(r2[1])),
                            min((unsigned)__float_as_int(r2[2]), (unsigned)__float_as_int(r2[3])));
    if (__any(mn < near_lim)) {
#pragma unroll
      for (int u = 0; u < 4; ++u) fixup(t + u, r2[u]);
    }
  }
  for (; t < m; ++t) {
    const float4 s = s4[t];
    const float dx = tx - s.x, dy = ty - s.y, dz = tz - s.z;
    float r2 = dx * dx + dy * dy + dz * dz;
    QV q;
    qload(t, q);
    pair(r2, q, OWN && sidx[t] == i);
    if (OWN && sidx[t] == i) r2 = 3.0e38f;
    fixup(t, r2);
  }
}

// RB charge vectors per block (blockIdx.y = group of RB): the pair kernel is
// computed once and applied to all of them, in the same order as for one vector.
template <typename T, int BS, int RB, bool POLY>
__global__ __launch_bounds__(BS) void k_p2p(PassArgs a, int nrhs, NearPoly np, const unsigned* items, XcdSegs seg) {
  constexpr bool F32 = sizeof(T) == 4;
  // FP64 sources as three coordinate arrays; FP32 sources as (x, y, z, unused)
  __shared__ T sx[F32 ? 1 : BS], sy[F32 ? 1 : BS], sz[F32 ? 1 : BS];
  __shared__ float4 s4[F32 ? BS : 1];
  __shared__ __align__(16) T sq[BS][2 * RB];
  __shared__ int sidx[BS];
  // FP32: each target's FP64 sums of its near-singular pairs (rare), per charge vector
  __shared__ double sns[F32 ? BS : 1][2 * RB];
  // the leaf: item blockIdx.x / 8 of XCD segment blockIdx.x % 8 (occupied leaves, the
  // longest first within a segment)
  const int xs_ = blockIdx.x % 8, j_ = seg.start[xs_] + (int)(blockIdx.x / 8);
  if (j_ >= seg.start[xs_ + 1]) return;
  const int leaf = (int)items[j_], r0 = blockIdx.y * RB, tid = threadIdx.x;
  const int nb = a.nbox_dim;
  const int ix = leaf / (nb * nb), iy = (leaf / nb) % nb, iz = leaf % nb;
  const int start = a.leaf_start[a.leaf_base + leaf], cnt = a.leaf_count[a.leaf_base + leaf];
  // FP32: coordinates in units of 2 pi / k (see pair_kernel); FP64: physical
  const double kap = F32 ? a.k / 6.283185307179586477 : 1.0;
  // pairs closer than 5% of the leaf side are evaluated in FP64 in the FP32 path
  const float rns2 = (float)(0.0025 * a.h * a.h * kap * kap);
  // the FP32 pair term at squared distance rns2, as every lane computes it
  float ecr = 0.0f, eci = 0.0f;
  if (F32) pair_value<POLY>(rns2, np, &ecr, &eci);
  const int z0 = max(iz - 1, 0), z1 = min(iz + 1, nb - 1);
  // largest k r in the 3 x 3 x 3 leaf block: the corners of a 2 x 2 x 2 span, sqrt(3) 2 h
  const bool small = a.k * 3.4641016151377546 * a.h <= 0.78539816339744831;
  for (int c0 = 0; c0 < cnt; c0 += BS) {
    const bool act = c0 + tid < cnt;
    const int64_t i = start + c0 + tid;
    const double txd = act ? a.xs[i] : 0.0, tyd = act ? a.xs[a.n + i] : 0.0, tzd = act ? a.xs[2 * a.n + i] : 0.0;
    // coordinates relative to the root corner keep FP32 differences accurate
    const T tx = (T)((txd - a.lo[0]) * kap), ty = (T)((tyd - a.lo[1]) * kap), tz = (T)((tzd - a.lo[2]) * kap);
    T accr[RB], acci[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) accr[b] = 0, acci[b] = 0;
    if constexpr (F32)
#pragma unroll
      for (int b = 0; b < 2 * RB; ++b) sns[tid][b] = 0.0;
    for (int col = 0; col < 9; ++col) {
      const int jx = ix + col / 3 - 1, jy = iy + col % 3 - 1;
      if (jx < 0 || jy < 0 || jx >= nb || jy >= nb) continue;
      const int64_t kl = a.leaf_base + ((int64_t)jx * nb + jy) * nb;
      const int ss = a.leaf_start[kl + z0], se = a.leaf_start[kl + z1] + a.leaf_count[kl + z1];
      for (int s0 = ss; s0 < se; s0 += BS) {
        const int m = min(BS, se - s0);
        __syncthreads();
        if (tid < m) {
          const int64_t j = s0 + tid;
          const T x = (T)((a.xs[j] - a.lo[0]) * kap), y = (T)((a.xs[a.n + j] - a.lo[1]) * kap),
                  z = (T)((a.xs[2 * a.n + j] - a.lo[2]) * kap);
          if constexpr (F32)
            s4[tid] = make_float4(x, y, z, 0.0f);
          else
            sx[tid] = x, sy[tid] = y, sz[tid] = z;
#pragma unroll
          for (int b = 0; b < RB; ++b) {
            const double2 qv = r0 + b < nrhs ? a.q[(int64_t)(r0 + b) * a.n + j] : make_double2(0.0, 0.0);
            sq[tid][2 * b] = (T)qv.x;
            sq[tid][2 * b + 1] = (T)qv.y;
          }
          sidx[tid] = (int)j;
        }
        __syncthreads();
        if (!act) continue;
        if constexpr (F32) {
          if (col == 4)
            p2p_f32_rows<RB, POLY, true>(m, tx, ty, tz, s4, sq, sidx, rns2, ecr, eci, kap, a, i, txd, tyd, tzd, r0,
                                         nrhs, accr, acci, sns[tid], np);
          else
            p2p_f32_rows<RB, POLY, false>(m, tx, ty, tz, s4, sq, sidx, rns2, ecr, eci, kap, a, i, txd, tyd, tzd, r0,
                                          nrhs, accr, acci, sns[tid], np);
        } else {
          // Only the centre column holds the target itself; there the pair with
          // r2 = 0 (same coordinates, same arithmetic) gets weight 0, branch free.
          // When k r stays below pi/4 for every pair of the leaf's neighbourhood the
          // sine and cosine need no argument reduction.
          if (col == 4) {
            if (small)
              p2p_f64_rows<RB, true, true>(m, tx, ty, tz, sx, sy, sz, sq, a.k, accr, acci);
            else
              p2p_f64_rows<RB, false, true>(m, tx, ty, tz, sx, sy, sz, sq, a.k, accr, acci);
          } else {
            if (small)
              p2p_f64_rows<RB, true, false>(m, tx, ty, tz, sx, sy, sz, sq, a.k, accr, acci);
            else
              p2p_f64_rows<RB, false, false>(m, tx, ty, tz, sx, sy, sz, sq, a.k, accr, acci);
          }
        }
      }
    }
    if (act)
#pragma unroll
      for (int b = 0; b < RB; ++b)
        if (r0 + b < nrhs)
          a.phi[(int64_t)(r0 + b) * a.n + i] =
              make_double2((double)accr[b] * kap + (F32 ? sns[tid][2 * b] : 0.0),
                           (double)acci[b] * kap + (F32 ? sns[tid][2 * b + 1] : 0.0));
  }
}

// ---------------------------------------------------------------------------
// Near field with each pair of particles in different leaves evaluated once
// (one charge vector, FP32 or FP64).  The free-space kernel e^{ikr}/r is
// symmetric in its two points, so the pair (i, j) adds q_j G to phi_i and q_i G
// to phi_j.  Of the 26 neighbour leaves of a leaf A only the forward half is
// visited: the columns (dx, dy) = (0, 1), (1, -1), (1, 0), (1, 1) with
// dz = -1, 0, 1 (slots 3 c + dz + 1, c the column) and the leaf (0, 0, 1)
// (slot 12); A's own leaf is done in full.  A workgroup of A adds the q_j G terms
// to its targets in registers; the q_i G terms for a source j of a forward
// neighbour B are summed over the pass's targets (per wave, a transposing
// butterfly over the 64 lanes, eight sources at a time) and written to
// part[G slot + h][j] (h the workgroup's index among A's G).  k_p2p_sym_gather
// then adds to each particle of B the slots of its existing, non-empty backward
// neighbours, in slot order: the result is deterministic.
// FP32: near-singular pairs (closer than 5% of the leaf side) get G from FP64
// coordinate differences; in both precisions the pair with itself gets 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fwd_column(int c, int* dx, int* dy) {
  *dx = c == 0 ? 0 : 1;
  *dy = c == 0 ? 1 : c - 2;
}

// Squared distance of an FP32 near-field pair as used for its value, one
// rounding order wherever it is formed.  SYM (sources in other leaves): plus
// eps2, a 1e-8 fraction of the near-singular threshold, which only keeps two
// particles that coincide in FP32 finite.  Otherwise (the leaf itself, which
// holds the pair of each particle with itself): raised to at least rns2, so that
// this pair's stand-in value is small.
template <bool SYM>
__device__ __forceinline__ float sym_r2(float tx, float ty, float tz, const float4& sp, float eps2, float rns2) {
  const float dx = tx - sp.x, dy = ty - sp.y, dz = tz - sp.z;
  if (SYM) return fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
  // max of two non-negative floats as the max of their bit patterns
  return __int_as_float(max(__float_as_int(fmaf(dz, dz, fmaf(dy, dy, dx * dx))), __float_as_int(rns2)));
}

// Lane exchanges inside rows of 16 lanes through the DPP crossbar (no LDS round
// trip, usually folded into the add that uses them): MIRROR16 takes lane 15 - l of
// the row, MIRROR8 lane 7 - l of the eight, XOR2 and XOR1 the quad permutations
// (2, 3, 0, 1) and (1, 0, 3, 2).  Each pairs every lane with one whose bit 3, 2, 1
// or 0 respectively differs and whose higher bits agree, which is all a
// butterfly reduction needs.
enum : int { DPP_MIRROR16 = 0x140, DPP_MIRROR8 = 0x141, DPP_XOR2 = 0x4E, DPP_XOR1 = 0xB1 };
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// The last four stages of the transposing butterfly over 64 lanes (masks 8, 4,
// 2, 1) for the four values left, c0 .. c3: after the stages with masks 8 and 4
// lane l keeps value ((l >> 2) & 3), summed over its group of 16 lanes, and the
// two quad stages complete the sum.  The values come in as separate registers
// (pinned), so that the selects stay selects of values and do not turn into an
// indexed read of a vector.
template <typename R>
__device__ __forceinline__ R butterfly_tail(R c0, R c1, R c2, R c3, int lane) {
  asm volatile("" : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3));
  const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0;
  R s0 = h8 ? c0 : c2, s1 = h8 ? c1 : c3;
  R k0 = h8 ? c2 : c0, k1 = h8 ? c3 : c1;
  if constexpr (sizeof(R) == 4) {
    k0 += dpp_f32<DPP_MIRROR16>(s0), k1 += dpp_f32<DPP_MIRROR16>(s1);
  } else {
    k0 += dpp_f64<DPP_MIRROR16>(s0), k1 += dpp_f64<DPP_MIRROR16>(s1);
  }
  const R send = h4 ? k0 : k1, keep = h4 ? k1 : k0;
  R tot;
  if constexpr (sizeof(R) == 4) {
    tot = keep + dpp_f32<DPP_MIRROR8>(send);
    tot += dpp_f32<DPP_XOR2>(tot);
    tot += dpp_f32<DPP_XOR1>(tot);
  } else {
    tot = keep + dpp_f64<DPP_MIRROR8>(send);
    tot += dpp_f64<DPP_XOR2>(tot);
    tot += dpp_f64<DPP_XOR1>(tot);
  }
  return tot;
}

// Eight staged sources [t, t + 8) against this lane's T targets.  SYM: also the
// eight source-side sums over the wave's 64 T targets, written to
// psw[2 (t + u) + c] (c = 0 real, 1 imaginary part).  Every pair is applied
// with the FP32 value at the squared distance from sym_r2, except the pair of a
// particle with itself in the leaf's own pass (found by its index), which gets
// weight 0: its clamped value would be of the order of the inverse threshold, and
// taking it back later would cancel against everything else in the FP32 sum.
// Pairs closer than the threshold rns2 (rare: two particles closer than 5% of
// the leaf side, whose FP32 coordinate differences have lost digits) are found
// by one wave-wide test of the least squared distance over the eight sources;
// only then the lanes that met one redo their tests and take those pairs one by
// one: the value used is replaced by the one from FP64 differences, its
// source-side part added to dps[2 (t + u) + c].
// S = 2 or 4 (with T = 1): the wave holds 64 / S targets, lane l = (64 / S) g + j
// taking target j and the 8 / S sources t + (8 / S) g, ...; the source-side sums are
// then summed over the 64 / S lanes of the subgroup only (the butterfly without its
// first one or two stages), and the caller adds the S subgroups' target sums.
template <int T, bool SYM, bool POLY, int S = 1>
__device__ __forceinline__ void p2p_sym8(int t, int tbase, const float (&tx)[T], const float (&ty)[T],
                                         const float (&tz)[T], const float (&qri)[T], const float (&qii)[T],
                                         const bool (&act)[T], const float4* s4, const float* sqi,
                                         const int* sidx, float rns2, float eps2, double kap2,
                                         const PassArgs& a, float (&accr)[T], float (&acci)[T], float* psw,
                                         float* dps, const NearPoly& np) {
  static_assert(S == 1 || (T == 1 && (S == 2 || S == 4)), "source subgroups need one target per lane");
  constexpr int NS = 8 / S;  // sources per lane and step
  const int lane = threadIdx.x & 63;
  const int sb = S == 1 ? t : t + NS * (lane / (64 / S));  // this lane's first source
  // a vector value, not an array: the butterfly's selects stay selects of values
  typedef float f16v __attribute__((ext_vector_type(2 * NS)));
  f16v c;
  // the squared distance a pair is tested with: SYM, the one used; the own pass, the
  // plain one (the clamp only ever raises it to the threshold itself), with the pair
  // of a particle with itself moved out of the test's range
  auto tested = [&](int k, const float4& sp, int sj) -> float {
    if (SYM) return sym_r2<true>(tx[k], ty[k], tz[k], sp, eps2, rns2);
    const float dx = tx[k] - sp.x, dy = ty[k] - sp.y, dz = tz[k] - sp.z;
    // a distinct particle at FP32 distance 0 is a near pair like any other
    return sj == tbase + 64 * k ? 3.0e38f : fmaf(dz, dz, fmaf(dy, dy, dx * dx));
  };
  float mn = 3.0e38f;
#pragma unroll
  for (int v = 0; v < NS / 2; ++v) {  // two sources at a time
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float4 sp = s4[sb + 2 * v + u];
      const float qr = sp.w, qi = sqi[sb + 2 * v + u];
      const int sj = SYM ? 0 : sidx[sb + 2 * v + u];
      float cr = 0.0f, ci = 0.0f;
#pragma unroll
      for (int k = 0; k < T; ++k) {
        const float r2 = tested(k, sp, sj);
        mn = fminf(mn, r2);
        const bool self = !SYM && sj == tbase + 64 * k;
        const float used = SYM ? r2 : __int_as_float(max(__float_as_int(r2), __float_as_int(rns2)));
        float er, ei;
        pair_value<POLY>(used, np, &er, &ei);
        if (self) er = 0.0f, ei = 0.0f;
        accr[k] = fmaf(qr, er, fmaf(-qi, ei, accr[k]));
        acci[k] = fmaf(qr, ei, fmaf(qi, er, acci[k]));
        if (SYM) {
          cr = fmaf(qri[k], er, fmaf(-qii[k], ei, cr));
          ci = fmaf(qri[k], ei, fmaf(qii[k], er, ci));
        }
      }
      // pin the sums to this source (left to itself the compiler sinks the
      // accumulations towards their use and keeps every pair value alive)
      if (SYM) {
        asm volatile("" : "+v"(cr), "+v"(ci));
        c[2 * (2 * v + u)] = cr, c[2 * (2 * v + u) + 1] = ci;
      }
#pragma unroll
      for (int k = 0; k < T; ++k) asm volatile("" : "+v"(accr[k]), "+v"(acci[k]));
    }
    // the least distance taken at each step (else every distance stays alive to the end)
    asm volatile("" : "+v"(mn));
    // one step at a time: interleaving the steps would only raise register pressure
    __builtin_amdgcn_sched_barrier(0);
  }
  if (SYM) {
    // transposing butterfly over the 16 values: after the stage with mask m a
    // lane holds the half of its values selected by (lane & m), summed with the
    // partner's same half.  Masks 32 and 16 by the lane-swap instructions (value
    // k to the low half of the lanes, k + H to the high half), the rest through
    // the DPP crossbar; lane l ends with value (l >> 2) summed over the 64 lanes.
    // With S subgroups the first log2 S stages are left out: each subgroup's lanes
    // form whole halves (S = 2) or rows (S = 4), and lane l still ends with value
    // (l >> 2) of the step's 16, source t + (l >> 3), summed over its subgroup.
    if constexpr (S == 1) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[k]), __float_as_uint(c[k + 8]), false, false);
        c[k] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
      }
    }
    if constexpr (S <= 2) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(c[k]), __float_as_uint(c[k + 4]), false, false);
        c[k] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
      }
    }
    const float tot = butterfly_tail<float>(c[0], c[1], c[2], c[3], lane);
    if (!(lane & 3)) psw[2 * t + (lane >> 2)] = tot;
  }
  if (!__any(mn < rns2)) return;
  // the near pairs, lane by lane, pair by pair (a fixed order)
  unsigned mine = 0;  // bit uu T + k: pair (source uu, target slot k)
#pragma unroll 1
  for (int uu = 0; uu < 8; ++uu)
#pragma unroll
    for (int k = 0; k < T; ++k)
      mine |= (act[k] && t + uu >= sb && t + uu < sb + NS && tested(k, s4[t + uu], SYM ? 0 : sidx[t + uu]) < rns2)
                  ? 1u << (uu * T + k)
                  : 0u;
  unsigned long long bal = __ballot(mine != 0);
  while (bal) {
    const int l = __builtin_ctzll(bal);
    bal &= bal - 1;
    if (lane != l) continue;
#pragma unroll 1
    for (int uu = 0; uu < 8; ++uu)
#pragma unroll
      for (int k = 0; k < T; ++k) {
        if (!((mine >> (uu * T + k)) & 1)) continue;
        const int64_t j = sidx[t + uu], i = tbase + 64 * k;
        // the digits lost are those of the coordinate differences: those in FP64,
        // the rest of the pair in FP32 as above
        float er = 0.0f, ei = 0.0f;
        if (j >= 0 && j != i) {
          const double ex = a.xs[i] - a.xs[j], ey = a.xs[a.n + i] - a.xs[a.n + j],
                       ez = a.xs[2 * a.n + i] - a.xs[2 * a.n + j];
          pair_value<POLY>((float)((ex * ex + ey * ey + ez * ez) * kap2), np, &er, &ei);
        }
        float ur, ui;  // the value used above
        pair_value<POLY>(sym_r2<SYM>(tx[k], ty[k], tz[k], s4[t + uu], eps2, rns2), np, &ur, &ui);
        const float der = er - ur, dei = ei - ui;
        const float qr = s4[t + uu].w, qi = sqi[t + uu];
        accr[k] = fmaf(qr, der, fmaf(-qi, dei, accr[k]));
        acci[k] = fmaf(qr, dei, fmaf(qi, der, acci[k]));
        if (SYM) {
          dps[2 * (t + uu)] += fmaf(qri[k], der, -qii[k] * dei);
          dps[2 * (t + uu) + 1] += fmaf(qri[k], dei, qii[k] * der);
        }
      }
  }
}

// FP64 form of p2p_sym8 on physical coordinates.  FP64 differences keep their
// digits, so no near-pair fix-up is needed; in the leaf's own pass (not SYM) a
// pair at distance 0 (a particle with itself) gets weight 0.  SMALL: k r <= pi/4
// for every pair of the 3 x 3 x 3 leaf block, so sin and cos need no reduction.
// The two 32-bit halves of a double go through the lane swaps one after the other.
__device__ __forceinline__ void swap32_f64(double& x, double& y) {
  const unsigned long long xb = (unsigned long long)__double_as_longlong(x);
  const unsigned long long yb = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)xb, (unsigned)yb, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(xb >> 32), (unsigned)(yb >> 32), false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void swap16_f64(double& x, double& y) {
  const unsigned long long xb = (unsigned long long)__double_as_longlong(x);
  const unsigned long long yb = (unsigned long long)__double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)xb, (unsigned)yb, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(xb >> 32), (unsigned)(yb >> 32), false, false);
  x = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  y = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// S = 2, 4 (T = 1): source subgroups as in p2p_sym8.
template <int T, bool SYM, bool SMALL, int S = 1>
__device__ __forceinline__ void p2p_sym8_f64(int t, const double (&tx)[T], const double (&ty)[T],
                                             const double (&tz)[T], const double (&qri)[T], const double (&qii)[T],
                                             const double4* s4, const double* sqi, double k, double (&accr)[T],
                                             double (&acci)[T], double* psw) {
  static_assert(S == 1 || (T == 1 && (S == 2 || S == 4)), "source subgroups need one target per lane");
  constexpr int NS = 8 / S;
  const int lane = threadIdx.x & 63;
  const int sb = S == 1 ? t : t + NS * (lane / (64 / S));
  typedef double d16v __attribute__((ext_vector_type(2 * NS)));
  d16v c;
#pragma unroll
  for (int v = 0; v < NS; ++v) {
    const double4 sp = s4[sb + v];
    const double qr = sp.w, qi = sqi[sb + v];
    double cr = 0.0, ci = 0.0;
#pragma unroll
    for (int kk = 0; kk < T; ++kk) {
      const double dx = tx[kk] - sp.x, dy = ty[kk] - sp.y, dz = tz[kk] - sp.z;
      const double r2 = dx * dx + dy * dy + dz * dz;
      const bool self = !SYM && !(r2 > 0);
      const double ri = rsqrt_f64(self ? 1.0 : r2);
      double sn, cs;
      if (SMALL)
        sincos_f64_small(k * (r2 * ri), &sn, &cs);
      else
        sincos_f64(k * (r2 * ri), &sn, &cs);
      const double er = cs * ri, ei = sn * ri;
      const double wr = self ? 0.0 : qr, wi = self ? 0.0 : qi;
      accr[kk] = fma(wr, er, fma(-wi, ei, accr[kk]));
      acci[kk] = fma(wr, ei, fma(wi, er, acci[kk]));
      if (SYM) {
        cr = fma(qri[kk], er, fma(-qii[kk], ei, cr));
        ci = fma(qri[kk], ei, fma(qii[kk], er, ci));
      }
    }
    // the sums are kept with this source (else the compiler defers them and holds
    // every pair value)
    if (SYM) {
      asm volatile("" : "+v"(cr), "+v"(ci));
      c[2 * v] = cr, c[2 * v + 1] = ci;
    }
#pragma unroll
    for (int kk = 0; kk < T; ++kk) asm volatile("" : "+v"(accr[kk]), "+v"(acci[kk]));
  }
  if (SYM) {
    // the transposing butterfly of p2p_sym8: lane 4 u ends with the wave's (subgroup's)
    // sum of value u
    if constexpr (S == 1) {
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        double x = c[kk], y = c[kk + 8];
        swap32_f64(x, y);
        c[kk] = x + y;
      }
    }
    if constexpr (S <= 2) {
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        double x = c[kk], y = c[kk + 4];
        swap16_f64(x, y);
        c[kk] = x + y;
      }
    }
    const double tot = butterfly_tail<double>(c[0], c[1], c[2], c[3], lane);
    if (!(lane & 3)) psw[2 * t + (lane >> 2)] = tot;
  }
}

// The symmetric near field's LDS: NW waves, up to TMAX targets per lane.
template <typename R, int TMAX, int NW>
struct SymShared {
  typedef typename SymTypes<R>::R4 R4;
  typedef typename SymTypes<R>::R2 R2;
  static constexpr bool F32 = std::is_same<R, float>::value;
  static constexpr int SC = 128;
  R4 s4[NW][SC];  // x, y, z (FP32: scaled) and the real part of the charge
  R sqi[NW][SC];
  R psw[NW][2 * SC];
  // FP32 only: source indices and near-singular corrections of the source-side sums
  int sidx[F32 ? NW : 1][F32 ? SC : 1];
  float dps[F32 ? NW : 1][F32 ? 2 * SC : 1];
  R2 tacc[NW > 1 ? NW : 1][NW > 1 ? 64 * TMAX : 1];
};

// One work item of the symmetric near field, wi = leaf G + half: workgroup `half` of
// the G of leaf A takes A's target passes half, half + G, ... (T targets per lane;
// the 64 T targets of a pass are the same for the NW waves, which share out the
// staged source chunks of SC sources: chunk c of the pass, counted over the ranges,
// goes to wave c mod NW).  Each wave stages, evaluates and writes its chunks'
// source-side sums on its own (part[G slot + half]); at the end of a pass the waves'
// target sums are added in wave order.  Charge vector r of nrhs.  A last pass of at most
// 32 or 16 targets has 2 or 4 lanes per target sharing out the sources.
template <typename R, int T, int NW, bool POLY, typename SH>
__device__ __forceinline__ void p2p_sym_item(const PassArgs& a, int nrhs, int r, int G,
                                             typename SymTypes<R>::R2* part, const NearPoly& np, int wi, SH& sh) {
  typedef typename SymTypes<R>::R4 R4;
  typedef typename SymTypes<R>::R2 R2;
  constexpr bool F32 = std::is_same<R, float>::value;
  constexpr int SC = 128, TP = 64 * T;  // sources per chunk, targets per pass
  auto& s4 = sh.s4;
  auto& sqi = sh.sqi;
  auto& psw = sh.psw;
  auto& sidx = sh.sidx;
  auto& dps = sh.dps;
  auto& tacc = sh.tacc;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int nb = a.nbox_dim;
  // FP32: coordinates in units of 2 pi / k (see pair_kernel); FP64: physical
  const double kap = F32 ? a.k / 6.283185307179586477 : 1.0;
  const float rns2 = (float)(0.0025 * a.h * a.h * kap * kap);
  const float eps2 = 1e-8f * rns2;
  // FP64: k r <= pi/4 over the 3 x 3 x 3 leaf block (its longest pair: 2 sqrt(3) h)
  const bool small = a.k * 3.4641016151377546 * a.h <= 0.78539816339744831;
  const double2* q = a.q + (int64_t)r * a.n;
  // the quadratics' middle coefficients in vector registers: a multiply-add takes at
  // most one scalar operand, and left in scalar registers they are copied over for
  // every pair
  NearPoly npv = np;
  if constexpr (F32 && POLY) asm volatile("" : "+v"(npv.c1), "+v"(npv.s1));
  {
    const int leaf = wi / G, half = wi - leaf * G;
    const int ix = leaf / (nb * nb), iy = (leaf / nb) % nb, iz = leaf % nb;
    const int start = a.leaf_start[a.leaf_base + leaf], cnt = a.leaf_count[a.leaf_base + leaf];
    if (half * TP >= cnt) return;
    // one pass over the neighbourhood for 64 TT targets from c0 on; SS = 2, 4 (TT = 1):
    // 64 / SS targets, each on SS lanes that share out the sources
    auto pass = [&](auto tt, auto ss, int c0) {
      constexpr int TT = decltype(tt)::value;
      constexpr int SS = decltype(ss)::value;
      R tx[TT], ty[TT], tz[TT], qri[TT], qii[TT], accr[TT], acci[TT];
      bool act[TT];
      const int tl = SS == 1 ? lane : lane % (64 / SS);
      const int tbase = start + c0 + tl;  // target index of slot k: tbase + 64 k
#pragma unroll
      for (int k = 0; k < TT; ++k) {
        const int c = c0 + 64 * k + tl;
        act[k] = c < cnt;
        const int64_t i = start + (act[k] ? c : 0);
        tx[k] = (R)((a.xs[i] - a.lo[0]) * kap);
        ty[k] = (R)((a.xs[a.n + i] - a.lo[1]) * kap);
        tz[k] = (R)((a.xs[2 * a.n + i] - a.lo[2]) * kap);
        const double2 qv = act[k] ? q[i] : make_double2(0.0, 0.0);
        qri[k] = (R)qv.x, qii[k] = (R)qv.y;
        accr[k] = 0, acci[k] = 0;
      }
      int chunk = 0;
      // ranges: 0 = the leaf itself, 1..4 = forward columns, 5 = the leaf above
      for (int rg = 0; rg < 6; ++rg) {
        int ss, se, z1 = iz;
        int64_t kl = 0;
        if (rg == 0) {
          ss = start, se = start + cnt;
        } else if (rg == 5) {
          if (iz + 1 >= nb) continue;
          kl = a.leaf_base + ((int64_t)ix * nb + iy) * nb;
          ss = a.leaf_start[kl + iz + 1], se = ss + a.leaf_count[kl + iz + 1];
        } else {
          int dx, dy;
          fwd_column(rg - 1, &dx, &dy);
          const int jx = ix + dx, jy = iy + dy;
          if (jx >= nb || jy < 0 || jy >= nb) continue;
          kl = a.leaf_base + ((int64_t)jx * nb + jy) * nb;
          const int z0 = max(iz - 1, 0);
          z1 = min(iz + 1, nb - 1);
          ss = a.leaf_start[kl + z0], se = a.leaf_start[kl + z1] + a.leaf_count[kl + z1];
        }
        for (int s0 = ss; s0 < se; s0 += SC, ++chunk) {
          if (chunk % NW != w) continue;
          const int m = min(SC, se - s0), m8 = (m + 7) & ~7;
          wave_lds_sync();
          for (int e = lane; e < m8; e += 64) {
            // eight-aligned tail: copies of the first source with charge 0 and no index
            const int64_t j = s0 + (e < m ? e : 0);
            const double2 qj = q[j];
            R4 sv;
            sv.x = (R)((a.xs[j] - a.lo[0]) * kap), sv.y = (R)((a.xs[a.n + j] - a.lo[1]) * kap);
            sv.z = (R)((a.xs[2 * a.n + j] - a.lo[2]) * kap), sv.w = e < m ? (R)qj.x : (R)0;
            s4[w][e] = sv;
            sqi[w][e] = e < m ? (R)qj.y : (R)0;
            if constexpr (F32) {
              sidx[w][e] = e < m ? (int)j : -1;
              dps[w][2 * e] = 0.0f, dps[w][2 * e + 1] = 0.0f;
            }
          }
          wave_lds_sync();
          const int mu = __builtin_amdgcn_readfirstlane(m8);
          if constexpr (F32) {
            if (rg == 0) {
              for (int t = 0; t < mu; t += 8)
                p2p_sym8<TT, false, POLY, SS>(t, tbase, tx, ty, tz, qri, qii, act, s4[w], sqi[w], sidx[w], rns2,
                                              eps2, kap * kap, a, accr, acci, psw[w], dps[w], npv);
              continue;
            }
            for (int t = 0; t < mu; t += 8)
              p2p_sym8<TT, true, POLY, SS>(t, tbase, tx, ty, tz, qri, qii, act, s4[w], sqi[w], sidx[w], rns2, eps2,
                                           kap * kap, a, accr, acci, psw[w], dps[w], npv);
          } else {
            if (rg == 0) {
              for (int t = 0; t < mu; t += 8) {
                if (small)
                  p2p_sym8_f64<TT, false, true, SS>(t, tx, ty, tz, qri, qii, s4[w], sqi[w], a.k, accr, acci, psw[w]);
                else
                  p2p_sym8_f64<TT, false, false, SS>(t, tx, ty, tz, qri, qii, s4[w], sqi[w], a.k, accr, acci, psw[w]);
              }
              continue;
            }
            for (int t = 0; t < mu; t += 8) {
              if (small)
                p2p_sym8_f64<TT, true, true, SS>(t, tx, ty, tz, qri, qii, s4[w], sqi[w], a.k, accr, acci, psw[w]);
              else
                p2p_sym8_f64<TT, true, false, SS>(t, tx, ty, tz, qri, qii, s4[w], sqi[w], a.k, accr, acci, psw[w]);
            }
          }
          wave_lds_sync();
          for (int e = lane; e < m; e += 64) {
            const int64_t j = s0 + e;
            R pr = psw[w][2 * e], pi = psw[w][2 * e + 1];
            if constexpr (F32) pr += dps[w][2 * e], pi += dps[w][2 * e + 1];
            int slot = 12;
            if (rg < 5) {
              const int zj = (z1 > iz && j >= a.leaf_start[kl + iz + 1]) ? iz + 1
                             : (j >= a.leaf_start[kl + iz])               ? iz
                                                                           : iz - 1;
              slot = 3 * (rg - 1) + (zj - iz + 1);
            }
            R2* dst = part + ((int64_t)(G * slot + half) * nrhs + r) * a.n + j;
            const bool first = c0 == half * TP;
            R2 v;
            v.x = first ? pr : dst->x + pr, v.y = first ? pi : dst->y + pi;
            *dst = v;
          }
        }
      }
      if constexpr (SS > 1) {
        // the subgroups' target sums: halves, then (SS = 4) rows, added alike in every lane
#pragma unroll
        for (int k = 0; k < TT; ++k) {
          if constexpr (F32) {
            auto sr = __builtin_amdgcn_permlane32_swap(__float_as_uint(accr[k]), __float_as_uint(accr[k]), false, false);
            auto si = __builtin_amdgcn_permlane32_swap(__float_as_uint(acci[k]), __float_as_uint(acci[k]), false, false);
            accr[k] = __uint_as_float(sr[0]) + __uint_as_float(sr[1]);
            acci[k] = __uint_as_float(si[0]) + __uint_as_float(si[1]);
            if constexpr (SS == 4) {
              sr = __builtin_amdgcn_permlane16_swap(__float_as_uint(accr[k]), __float_as_uint(accr[k]), false, false);
              si = __builtin_amdgcn_permlane16_swap(__float_as_uint(acci[k]), __float_as_uint(acci[k]), false, false);
              accr[k] = __uint_as_float(sr[0]) + __uint_as_float(sr[1]);
              acci[k] = __uint_as_float(si[0]) + __uint_as_float(si[1]);
            }
          } else {
            double xr = accr[k], yr = accr[k], xi = acci[k], yi = acci[k];
            swap32_f64(xr, yr), swap32_f64(xi, yi);
            accr[k] = xr + yr, acci[k] = xi + yi;
            if constexpr (SS == 4) {
              xr = yr = accr[k], xi = yi = acci[k];
              swap16_f64(xr, yr), swap16_f64(xi, yi);
              accr[k] = xr + yr, acci[k] = xi + yi;
            }
          }
        }
      }
      if (NW > 1) {
        // the waves' target sums, added in wave order
#pragma unroll
        for (int k = 0; k < TT; ++k) tacc[w][64 * k + lane].x = accr[k], tacc[w][64 * k + lane].y = acci[k];
        __syncthreads();
        if (w == 0) {
#pragma unroll
          for (int k = 0; k < TT; ++k) {
            accr[k] = tacc[0][64 * k + lane].x, acci[k] = tacc[0][64 * k + lane].y;
            for (int ww = 1; ww < NW; ++ww) accr[k] += tacc[ww][64 * k + lane].x, acci[k] += tacc[ww][64 * k + lane].y;
          }
        }
        __syncthreads();
      }
      if (w == 0 && tl == lane)
#pragma unroll
        for (int k = 0; k < TT; ++k)
          if (act[k])
            a.phi[(int64_t)r * a.n + tbase + 64 * k] = make_double2((double)accr[k] * kap, (double)acci[k] * kap);
    };
    // passes of 64 T targets (this workgroup's: every G-th one); a last one of at most 64
    // with one target per lane, and of at most 32 or 16 on 2 or 4 lanes each
    for (int c0 = half * TP; c0 < cnt; c0 += G * TP) {
      const int left = cnt - c0;
      if (left <= 16)
        pass(std::integral_constant<int, 1>(), std::integral_constant<int, 4>(), c0);
      else if (left <= 32)
        pass(std::integral_constant<int, 1>(), std::integral_constant<int, 2>(), c0);
      else if (T > 1 && left <= 64)
        pass(std::integral_constant<int, 1>(), std::integral_constant<int, 1>(), c0);
      else
        pass(std::integral_constant<int, T>(), std::integral_constant<int, 1>(), c0);
    }
  }
}

// One work item per workgroup (see p2p_sym_item), charge vector blockIdx.y.  Workgroups
// are dealt round-robin over the 8 XCDs; XCD x takes its segment of the work list in
// order (neighbouring leaves, whose source leaves overlap in that XCD's L2), the
// segments holding about equal pair work.  The grid is 8 times the longest segment.
template <typename R, int T, int NW, bool POLY>
__global__ __launch_bounds__(64 * NW) void k_p2p_sym(PassArgs a, int nrhs, int G, typename SymTypes<R>::R2* part,
                                                     NearPoly np, const unsigned* items, XcdSegs seg) {
  __shared__ SymShared<R, T, NW> sh;
  const int x = blockIdx.x % 8, j = seg.start[x] + (int)(blockIdx.x / 8);
  if (j >= seg.start[x + 1]) return;
  p2p_sym_item<R, T, NW, POLY>(a, nrhs, blockIdx.y, G, part, np, (int)items[j], sh);
}

// Adds to each particle of leaf B the source-side sums that its backward
// neighbours A = B - o (o in the forward half, A inside the grid and not empty)
// left in part, in slot order (see k_p2p_sym).
template <typename R2>
__device__ __forceinline__ void p2p_sym_gather_leaf(const PassArgs& a, int nrhs, int tp, int G, const R2* part,
                                                    int leaf, int r) {
  typedef decltype(R2::x) R;
  const int nb = a.nbox_dim;
  const int ix = leaf / (nb * nb), iy = (leaf / nb) % nb, iz = leaf % nb;
  const int start = a.leaf_start[a.leaf_base + leaf], cnt = a.leaf_count[a.leaf_base + leaf];
  if (cnt == 0) return;
  // have: A exists and holds particles (and wrote slot sums from its workgroups with
  // index below ceil(count / tp), at most G); count per slot in ca
  unsigned have = 0;
  int ca_s[13];
  for (int slot = 0; slot < 13; ++slot) {
    int dx = 0, dy = 0, dz = 1;
    if (slot < 12) fwd_column(slot / 3, &dx, &dy), dz = slot % 3 - 1;
    const int ax = ix - dx, ay = iy - dy, az = iz - dz;
    if (ax < 0 || ay < 0 || az < 0 || ax >= nb || ay >= nb || az >= nb) continue;
    const int ca = a.leaf_count[a.leaf_base + ((int64_t)ax * nb + ay) * nb + az];
    if (ca > 0) have |= 1u << slot;
    ca_s[slot] = ca;
  }
  // FP32 sums are in the scaled units of k_p2p_sym
  const double kap = sizeof(R) == 4 ? a.k / 6.283185307179586477 : 1.0;
  for (int c = threadIdx.x; c < cnt; c += blockDim.x) {
    const int64_t j = start + c;
    R sr = 0, si = 0;
    for (int slot = 0; slot < 13; ++slot)
      if ((have >> slot) & 1)
        for (int hf = 0; hf < G && hf * tp < ca_s[slot]; ++hf) {
          const R2 v = part[((int64_t)(G * slot + hf) * nrhs + r) * a.n + j];
          sr += v.x, si += v.y;
        }
    double2* o = a.phi + (int64_t)r * a.n + j;
    *o = make_double2(o->x + (double)sr * kap, o->y + (double)si * kap);
  }
}

template <typename R2>
__global__ void k_p2p_sym_gather(PassArgs a, int nrhs, int tp, int G, const R2* part) {
  p2p_sym_gather_leaf<R2>(a, nrhs, tp, G, part, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// The batched near field as one persistent launch (see NFQueueGeom).  Items are
// taken in ticket order, so a gather item only ever waits for pair items that
// workgroups already hold and finish without waiting: the wait ends.  It is still
// bounded (spin_limit polls, then err is set and the item goes on).  A pair item's
// stores reach the other workgroups through a release at agent scope after the
// workgroup barrier; a gather item acquires before its reads.
// ---------------------------------------------------------------------------
__global__ void k_nf_queue_reset(unsigned* ticket, unsigned* done, int ngeo, int* err) {
  const int t = threadIdx.x;
  if (t == 0) *ticket = 0u, *err = 0;
  for (int g = t; g < ngeo; g += blockDim.x) done[g] = 0u;
}

template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_nf_queue(NFQueueArgs q) {
  typedef typename SymTypes<R>::R2 R2;
  constexpr bool F32 = std::is_same<R, float>::value;
  __shared__ SymShared<R, 2, 4> sh;
  __shared__ unsigned s_it;
  const unsigned P = (unsigned)q.n_p2p, Q = P + (unsigned)q.n_gather;
  for (;;) {
    __syncthreads();  // the previous item no longer needs s_it or the LDS
    if (threadIdx.x == 0) s_it = atomicAdd(q.ticket, 1u);
    __syncthreads();
    const unsigned it = s_it;
    if (it >= Q) return;
    if (it < P) {
      const unsigned itm = q.items[it];
      const int g = (int)(itm >> 24), wi = (int)(itm & 0xFFFFFFu);
      const NFQueueGeom& ge = q.geo[g];
      R2* part = (R2*)ge.part;
      if constexpr (F32) {
        if (ge.tpl == 2) {
          if (ge.poly)
            p2p_sym_item<float, 2, 4, true>(ge.a, 1, 0, ge.G, part, ge.np, wi, sh);
          else
            p2p_sym_item<float, 2, 4, false>(ge.a, 1, 0, ge.G, part, ge.np, wi, sh);
        } else {
          if (ge.poly)
            p2p_sym_item<float, 1, 4, true>(ge.a, 1, 0, ge.G, part, ge.np, wi, sh);
          else
            p2p_sym_item<float, 1, 4, false>(ge.a, 1, 0, ge.G, part, ge.np, wi, sh);
        }
      } else {
        if (ge.tpl == 2)
          p2p_sym_item<double, 2, 4, false>(ge.a, 1, 0, ge.G, part, ge.np, wi, sh);
        else
          p2p_sym_item<double, 1, 4, false>(ge.a, 1, 0, ge.G, part, ge.np, wi, sh);
      }
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_fetch_add(&q.done[g], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const unsigned itm = q.items[it];
      const int g = (int)(itm >> 24), leaf = (int)(itm & 0xFFFFFFu);
      const NFQueueGeom& ge = q.geo[g];
      if (threadIdx.x == 0) {
        int spins = 0;
        while (__hip_atomic_load(&q.done[g], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)ge.p2p_items) {
          if (++spins > q.spin_limit) {
            atomicExch(q.err, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      p2p_sym_gather_leaf<R2>(ge.a, 1, 64 * ge.tpl, ge.G, (const R2*)ge.part, leaf, 0);
    }
  }
}
template __global__ void k_nf_queue<float>(NFQueueArgs);
template __global__ void k_nf_queue<double>(NFQueueArgs);

template __global__ void k_p2p_sym<float, 1, 4, false>(PassArgs, int, int, float2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym<float, 2, 4, false>(PassArgs, int, int, float2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym<float, 4, 4, false>(PassArgs, int, int, float2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym<float, 1, 4, true>(PassArgs, int, int, float2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym<float, 2, 4, true>(PassArgs, int, int, float2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym<float, 4, 4, true>(PassArgs, int, int, float2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym<double, 1, 4, false>(PassArgs, int, int, double2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym<double, 2, 4, false>(PassArgs, int, int, double2*, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p_sym_gather<float2>(PassArgs, int, int, int, const float2*);
template __global__ void k_p2p_sym_gather<double2>(PassArgs, int, int, int, const double2*);

template __global__ void k_p2p<double, 64, 1, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 64, 1, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 64, 1, true>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<double, 256, 1, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 256, 1, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 256, 1, true>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<double, 64, 8, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 64, 8, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 64, 8, true>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<double, 256, 8, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 256, 8, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 256, 8, true>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<double, 128, 1, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 128, 1, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 128, 1, true>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<double, 128, 8, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 128, 8, false>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);
template __global__ void k_p2p<float, 128, 8, true>(PassArgs, int, NearPoly, const unsigned*, XcdSegs);

// ---------------------------------------------------------------------------
// Surrogate tables.  Entry g of a reaction table at (x, y, S) is scaled by the
// Cauchy-type envelope of a source at distance R_e (the distance to the nearer
// mirror point):  W_g = D^g K R_e^{|g|+1} / |g|!.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Rotation-free derivatives of the Sigma-family kernel (the same-layer reaction
// term that depends on x - x', y - y' and S = z + z', Sec. 3.2).  The kernel is
// axisymmetric, K = sum_img A f(w, zeta) with w = rho^2 and
// f = e^{ik sqrt(w + zeta^2)} / sqrt(w + zeta^2); with u = x + i y,
//   (d_x + i d_y)^m d_S^c K = u^m H_{m,c},  (d_x - i d_y)^m d_S^c K = conj(u)^m H_{m,c},
//   H_{m,c}(w, S) = (2 d_w)^m d_S^c K,   m + c <= P2,
// stored at index (m + c)(m + c + 1)/2 + m.  f = g(s), s = w + zeta^2, and the Taylor
// coefficients g_n = g^(n)(s) / n! of g(s) = e^{ik sqrt s} / sqrt s follow from the
// spherical Hankel functions of the first kind, (r^-1 d_r)^n h_0(kr) = (-k^2)^n h_n(kr) / (kr)^n:
//   g_n = (-1)^n i k^(2n+1) q_n / (2^n n!),  q_n = h_n(kr) / (kr)^n,  r = sqrt(s),
//   q_0 = -i e^{ikr} / (kr),  q_1 = -e^{ikr} (kr + i) / (kr)^3,  q_{n+1} = ((2n+1) q_n - q_{n-1}) / (kr)^2.
// Composing with s - s0 = dw + 2 zeta dzeta + dzeta^2:
//   d_w^m d_zeta^c f / (m! c!) = sum_q g_{m+c-q} (m+c-q)! / (m! (c-2q)! q!) (2 zeta)^(c-2q).
// zeta = S - 2 d_l - Z for the up-going family and 2 d_{l-1} - S - Z for the down-going
// one (there d_S = -d_zeta); images with Re zeta <= 0 are left out, as in the tables.
// One block of 64 per point; thread m owns the entries (m, c) in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_sigma_h(const double* w, const double* S, int n, const double2* img, int nup,
                                                int ndn, double two_dl, double two_dt, double k, int P2, double2* H) {
  __shared__ double2 sh[SIGMA_H_MAX];
  __shared__ double2 sg[SIGMA_P2_MAX + 1], sz2[SIGMA_P2_MAX + 1];
  __shared__ double fct[SIGMA_P2_MAX + 1];
  const int pt = blockIdx.x, m = threadIdx.x;
  if (pt >= n) return;
  const int nH = (P2 + 1) * (P2 + 2) / 2;
  for (int e = m; e < nH; e += 64) sh[e] = make_double2(0.0, 0.0);
  if (m == 0) {
    fct[0] = 1.0;
    for (int i = 1; i <= P2; ++i) fct[i] = fct[i - 1] * i;
  }
  const double wv = w[pt], Sv = S[pt];
  for (int j = 0; j < nup + ndn; ++j) {
    const bool dn = j >= nup;
    const double2 A = img[2 * j], Z = img[2 * j + 1];
    const dc zeta = {(dn ? two_dt - Sv : Sv - two_dl) - Z.x, -Z.y};
    if (zeta.x <= 0.0) continue;  // uniform over the block
    __syncthreads();
    if (m == 0) {
      const dc s0 = {wv + zeta.x * zeta.x - zeta.y * zeta.y, 2.0 * zeta.x * zeta.y};
      const dc z = cscale(csqrt_pr(s0), k);
      const dc e = cexp_i(z, 1.0);
      const dc iz = cdiv({1.0, 0.0}, z), iz2 = cmul(iz, iz);
      dc q0 = cmul({0.0, -1.0}, cmul(e, iz));
      dc q1 = cscale(cmul(cmul(e, cadd(z, {0.0, 1.0})), cmul(iz2, iz)), -1.0);
      double kp = k, tw = 1.0;  // k^(2n+1), 2^n n!
      for (int nn = 0; nn <= P2; ++nn) {
        const dc q = nn == 0 ? q0 : q1;
        const dc gn = cscale(cmul({0.0, (nn & 1) ? -kp : kp}, q), 1.0 / tw);
        sg[nn] = make_double2(gn.x, gn.y);
        if (nn >= 1) {
          const dc q2 = cmul(csub(cscale(q1, 2.0 * nn + 1.0), q0), iz2);
          q0 = q1, q1 = q2;
        }
        kp *= k * k, tw *= 2.0 * (nn + 1);
      }
      dc t = {1.0, 0.0};
      const dc z2 = cscale(zeta, 2.0);
      for (int i = 0; i <= P2; ++i) sz2[i] = make_double2(t.x, t.y), t = cmul(t, z2);
    }
    __syncthreads();
    if (m <= P2) {
      const dc a = {A.x, A.y};
      double pm = 1.0;
      for (int i = 0; i < m; ++i) pm *= 2.0;
      for (int c = 0; c <= P2 - m; ++c) {
        dc coef = {0.0, 0.0};
        for (int q = 0; 2 * q <= c; ++q) {
          const int nn = m + c - q;
          const double b = fct[nn] / (fct[m] * fct[c - 2 * q] * fct[q]);
          coef = cadd(coef, cscale(cmul({sg[nn].x, sg[nn].y}, {sz2[c - 2 * q].x, sz2[c - 2 * q].y}), b));
        }
        const double sc = pm * fct[m] * fct[c] * ((dn && (c & 1)) ? -1.0 : 1.0);
        const dc v = cscale(cmul(a, coef), sc);
        double2& o = sh[(m + c) * (m + c + 1) / 2 + m];
        o = make_double2(o.x + v.x, o.y + v.y);
      }
    }
  }
  __syncthreads();
  for (int e = m; e < nH; e += 64) H[(size_t)pt * nH + e] = sh[e];
}

// Envelope of H_{m,c}: the size of the term of a source at each mirror point, distances
// R2[0] and R2[1] (1e300: family absent), (2m-1)!! c! sum_f R_f^-(2m+c+1).
__device__ __forceinline__ double sigma_h_envelope(int m, int c, const double* R2) {
  double tot = 0.0;
  for (int f = 0; f < 2; ++f) {
    const double R = R2[f];
    if (!(R < 1e299)) continue;
    double e = 1.0 / R;
    for (int i = 1; i <= m; ++i) e *= (2.0 * i - 1.0) / (R * R);
    for (int i = 1; i <= c; ++i) e *= i / R;
    tot += e;
  }
  return tot;
}

// W = H - Hq (the quasi-static part taken out), divided by the envelope if env (Re: the
// two mirror distances per point), and the sums of |W|^2 per entry
__global__ void k_sur_normalize(const double2* H, const double2* Hq, const double* Re, int n, int P2, int env,
                                double2* W, double* sumsq) {
  const int pt = blockIdx.x;
  if (pt >= n) return;
  const int nH = (P2 + 1) * (P2 + 2) / 2;
  for (int e = threadIdx.x; e < nH; e += blockDim.x) {
    int nn = 0;
    while ((nn + 1) * (nn + 2) / 2 <= e) ++nn;
    const int m = e - nn * (nn + 1) / 2, c = nn - m;
    const double f = env ? 1.0 / sigma_h_envelope(m, c, Re + 2 * pt) : 1.0;
    const double2 v = H[(size_t)pt * nH + e], q = Hq[(size_t)pt * nH + e];
    const double2 wv = make_double2((v.x - q.x) * f, (v.y - q.y) * f);
    W[(size_t)pt * nH + e] = wv;
    if (sumsq) atomicAdd(&sumsq[e], wv.x * wv.x + wv.y * wv.y);
  }
}

// network targets: (Re W / sigma, Im W / sigma) per entry
__global__ void k_sur_targets(const double2* W, int n, int nH, const float* sigma, float* T) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * nH) return;
  const int g = (int)(e % nH);
  const double2 w = W[e];
  T[2 * e] = (float)(w.x / sigma[g]);
  T[2 * e + 1] = (float)(w.y / sigma[g]);
}

// H from the network's outputs, added to the quasi-static part already in H:
// H += sigma y (times the envelope if env)
__global__ void k_sur_h_from_net(const float* y, const double* Re, int n, int P2, const float* sigma, int env,
                                 double2* H) {
  const int pt = blockIdx.x;
  if (pt >= n) return;
  const int nH = (P2 + 1) * (P2 + 2) / 2;
  for (int e = threadIdx.x; e < nH; e += blockDim.x) {
    int nn = 0;
    while ((nn + 1) * (nn + 2) / 2 <= e) ++nn;
    const int m = e - nn * (nn + 1) / 2, c = nn - m;
    const double f = sigma[e] * (env ? sigma_h_envelope(m, c, Re + 2 * pt) : 1.0);
    double2& o = H[(size_t)pt * nH + e];
    o = make_double2(o.x + y[((size_t)pt * nH + e) * 2] * f, o.y + y[((size_t)pt * nH + e) * 2 + 1] * f);
  }
}

// Compact Cartesian table rows from H (exact algebra).  With D = d_x +- i d_y,
//   d_x^a d_y^b = 2^-(a+b) (-i)^b sum_{al, be} C(a, al) C(b, be) (-1)^(b-be) D+^(al+be) D-^(a+b-al-be),
// and, K solving the Helmholtz equation in (x, y, S) (every image does),
// D+ D- = d_x^2 + d_y^2 = -(d_S^2 + k^2), so for p >= q
//   D+^p D-^q d_S^c K = (-1)^q sum_t C(q, t) k^(2(q-t)) u^(p-q) H_{p-q, c+2t}
// (conj(u) and p, q swapped when q > p).  Row of key i: out[row[i]][g] = h^|g| d^g K at
// (X_i, Y_i) and the point's S, for the compact entries g (g1 <= 2), or added to the row
// already there (accumulate).  The third variable can be any one the kernel depends on
// through the target's z alone (S = z + z' for the Sigma families, w = z - z' for Delta).
// One block per key; key i reads H row hrow[i] (row i when hrow is null).
__global__ __launch_bounds__(64) void k_sigma_restore(const double2* H, const double* X, const double* Y, int nk,
                                                      const int* row, double h, double k, int P2, int nG,
                                                      const unsigned char* g1s, const unsigned char* g3s,
                                                      const unsigned char* gord, double2* out,
                                                      const int* hrow, int accumulate) {
  __shared__ double2 sh[SIGMA_H_MAX];
  __shared__ double2 up[SIGMA_P2_MAX + 1], dp[SIGMA_P2_MAX + 1];
  __shared__ double fct[SIGMA_P2_MAX + 1];
  const int i = blockIdx.x, tid = threadIdx.x;
  if (i >= nk) return;
  const int nH = (P2 + 1) * (P2 + 2) / 2;
  const size_t hr = hrow ? (size_t)hrow[i] : (size_t)i;
  for (int e = tid; e < nH; e += 64) sh[e] = H[hr * nH + e];
  if (tid == 0) {
    fct[0] = 1.0;
    for (int j = 1; j <= P2; ++j) fct[j] = fct[j - 1] * j;
    dc a = {1.0, 0.0}, b = {1.0, 0.0};
    const dc u = {X[i], Y[i]}, ub = {X[i], -Y[i]};
    for (int j = 0; j <= P2; ++j) up[j] = make_double2(a.x, a.y), dp[j] = make_double2(b.x, b.y), a = cmul(a, u),
                                  b = cmul(b, ub);
  }
  __syncthreads();
  auto binom = [&](int nn, int r) { return fct[nn] / (fct[r] * fct[nn - r]); };
  const double k2 = k * k;
  for (int g = tid; g < nG; g += 64) {
    const int a1 = g1s[g], c3 = g3s[g], nn = gord[g], b2 = nn - a1 - c3;
    dc acc = {0.0, 0.0};
    for (int al = 0; al <= a1; ++al)
      for (int be = 0; be <= b2; ++be) {
        const int pp = al + be, qq = a1 + b2 - pp;
        const int sm = min(pp, qq), md = pp >= qq ? pp - qq : qq - pp;
        const double2 vm = pp >= qq ? up[md] : dp[md];
        dc dsum = {0.0, 0.0};
        double kpow = 1.0;  // k^(2(sm - t)), t from sm down
        for (int t = sm; t >= 0; --t) {
          const double2 hv = sh[(md + c3 + 2 * t) * (md + c3 + 2 * t + 1) / 2 + md];
          dsum = cadd(dsum, cscale({hv.x, hv.y}, binom(sm, t) * kpow));
          kpow *= k2;
        }
        dsum = cmul(dsum, {vm.x, vm.y});
        const double sgn = ((sm & 1) ? -1.0 : 1.0) * (((b2 - be) & 1) ? -1.0 : 1.0);
        acc = cadd(acc, cscale(dsum, sgn * binom(a1, al) * binom(b2, be)));
      }
    // 2^-(a1+b2) (-i)^b2 h^|g|
    double sc = 1.0;
    for (int j = 0; j < a1 + b2; ++j) sc *= 0.5;
    for (int j = 0; j < nn; ++j) sc *= h;
    dc ph = {1.0, 0.0};
    for (int j = 0; j < b2; ++j) ph = cmul(ph, {0.0, -1.0});
    acc = cscale(cmul(acc, ph), sc);
    double2& o = out[(size_t)row[i] * nG + g];
    o = accumulate ? make_double2(o.x + acc.x, o.y + acc.y) : make_double2(acc.x, acc.y);
  }
}

// ---------------------------------------------------------------------------
// Sigma-family derivatives from the Sommerfeld integrals (Sec. 4.2: the
// integrals of Eq. symmetricdetable in rotation-free form, no image fit).
// Each family has the spectral form
//   K = i int k_rho J0(k_rho rho) e^{i k_z zeta} sigma(k_rho) / k_z dk_rho,
//   zeta = S - 2 d_l (up-going), 2 d_{l-1} - S (down-going, where d_S = -d_zeta),
// and (rho^-1 d_rho)^m J0(k_rho rho) = (-k_rho^2)^m J_m(x) / x^m, x = k_rho rho, so that
// on the nodes t (weights w) of the deformed contour
//   H_{m,c}(rho, S) = sum_t A_m(rho, t) B_c(S, t),
//   A_m = k_rho (-k_rho^2)^m J_m(x) / x^m,
//   B_c = (i k_z)^c e^{i k_z zeta_u} cu_t + (-i k_z)^c e^{i k_z zeta_d} cd_t,
//   cu, cd = w i (sigma - sigma_inf) / k_z.
// The limits sigma_inf (k_rho -> infinity) are one image at each mirror point,
// added exactly by k_sigma_h.  A and B are stored [row][index][node].
// ---------------------------------------------------------------------------
// J_m(x) / x^m for m = 0 .. M at complex x, times k_rho (-k_rho^2)^m, into
// out[m * ld] (one thread per node; ld = node count).  Power series for |x| <= 4;
// otherwise normalised backward recurrence (Miller's method: J_{n-1} = (2n/x) J_n - J_{n+1}
// from zero far above max(M, |x|), scaled by J_0 + 2 sum_k J_{2k} = 1).
__device__ void bessel_ratio_row(dc x, dc krho, int M, double2* out, int64_t ld) {
  const double ax = hypot(x.x, x.y);
  const dc mk2 = {-(krho.x * krho.x - krho.y * krho.y), -2.0 * krho.x * krho.y};  // -k_rho^2
  if (ax <= 4.0) {
    const dc q = cscale(cmul(x, x), -0.25);
    double inv = 1.0;  // 1 / (2^m m!)
    dc pk = krho;      // k_rho (-k_rho^2)^m
    for (int m = 0; m <= M; ++m) {
      dc term = {inv, 0.0}, sum = term;
      for (int kk = 1; kk < 200; ++kk) {
        term = cscale(cmul(term, q), 1.0 / ((double)kk * (m + kk)));
        sum = cadd(sum, term);
        if (hypot(term.x, term.y) <= 1e-17 * hypot(sum.x, sum.y)) break;
      }
      const dc v = cmul(sum, pk);
      out[(int64_t)m * ld] = make_double2(v.x, v.y);
      inv /= 2.0 * (m + 1);
      pk = cmul(pk, mk2);
    }
    return;
  }
  const dc ix = cdiv({1.0, 0.0}, x);
  int N = (int)(ax + 30.0) + M;
  N += N & 1;
  dc f1 = {0.0, 0.0}, f0 = {1e-250, 0.0};  // f_{n+1}, f_n
  dc norm = {0.0, 0.0};
  for (int n = N; n >= 1; --n) {
    if (n <= M) out[(int64_t)n * ld] = make_double2(f0.x, f0.y);
    if (!(n & 1)) norm = cadd(norm, cscale(f0, 2.0));
    const dc fm = csub(cmul(cscale(ix, 2.0 * n), f0), f1);
    f1 = f0, f0 = fm;
    if (fabs(f0.x) + fabs(f0.y) > 1e250) {  // rescale everything kept so far
      const double s = 1e-250;
      f0 = cscale(f0, s), f1 = cscale(f1, s), norm = cscale(norm, s);
      for (int j = n; j <= M; ++j) {
        const double2 v = out[(int64_t)j * ld];
        out[(int64_t)j * ld] = make_double2(v.x * s, v.y * s);
      }
    }
  }
  out[0] = make_double2(f0.x, f0.y);
  norm = cadd(norm, f0);
  // J_m = f_m / norm first (values of order one), then the factor k_rho (-k_rho^2 / x)^m:
  // the two scales apart can each exceed the double range
  const dc inorm = cdiv({1.0, 0.0}, norm);
  dc fac = krho;
  const dc step = cmul(mk2, ix);
  for (int m = 0; m <= M; ++m) {
    const double2 v = out[(int64_t)m * ld];
    const dc r = cmul(cmul({v.x, v.y}, inorm), fac);
    out[(int64_t)m * ld] = make_double2(r.x, r.y);
    fac = cmul(fac, step);
  }
}

// A[(ir (M+1) + m) nn + t] for the radial distances rho[ir] (grid: ceil(nn / 64) x nrho)
__global__ __launch_bounds__(64) void k_som_radial(const double2* krho, int nn, const double* rho, int M,
                                                   double2* A) {
  const int t = blockIdx.x * 64 + threadIdx.x, ir = blockIdx.y;
  if (t >= nn) return;
  const dc kr = {krho[t].x, krho[t].y};
  const dc x = cscale(kr, rho[ir]);
  bessel_ratio_row(x, kr, M, A + (int64_t)ir * (M + 1) * nn + t, nn);
}

// B[(is (M+1) + c) nn + t] for the heights S[is] (grid: ceil(nn / 64) x nS); a family
// takes part where zeta > zeta_eps (the image tables' validity rule) and cu / cd exist
__global__ __launch_bounds__(64) void k_som_vertical(const double2* kz, const double2* cu, const double2* cd, int nn,
                                                     const double* S, double two_dl, double two_dt, int has_up,
                                                     int has_dn, double zeta_eps, int M, double2* B) {
  const int t = blockIdx.x * 64 + threadIdx.x, is = blockIdx.y;
  if (t >= nn) return;
  const dc kzv = {kz[t].x, kz[t].y};
  const dc ikz = {-kzv.y, kzv.x};
  const double zu = S[is] - two_dl, zd = two_dt - S[is];
  dc eu = {0.0, 0.0}, ed = {0.0, 0.0};
  if (has_up && zu > zeta_eps) eu = cmul(cexp_i(kzv, zu), {cu[t].x, cu[t].y});
  if (has_dn && zd > zeta_eps) ed = cmul(cexp_i(kzv, zd), {cd[t].x, cd[t].y});
  double2* o = B + (int64_t)is * (M + 1) * nn + t;
  for (int c = 0; c <= M; ++c) {
    const dc v = cadd(eu, ed);
    o[(int64_t)c * nn] = make_double2(v.x, v.y);
    eu = cmul(eu, ikz), ed = cmul(ed, {-ikz.x, -ikz.y});
  }
}

// H[pair][(m + c)(m + c + 1)/2 + m] += sum_t A[ir][m][t] B[is][c][t] for m + c <= M, one
// block of 256 per pair (ir, is) = (pr[pair], ps[pair]); node chunks of 64 staged in LDS
// (rows padded to 65 so that the lanes' rows fall on different banks)
__global__ __launch_bounds__(256) void k_som_contract(const double2* A, const double2* B, int nn, int M,
                                                      const int* pr, const int* ps, double2* H) {
  extern __shared__ double2 lds_som[];
  constexpr int CH = 64, LD = CH + 1;
  double2* sa = lds_som;
  double2* sb = lds_som + (M + 1) * LD;
  const int pair = blockIdx.x, tid = threadIdx.x;
  const int nH = (M + 1) * (M + 2) / 2;
  const double2* Ar = A + (int64_t)pr[pair] * (M + 1) * nn;
  const double2* Bs = B + (int64_t)ps[pair] * (M + 1) * nn;
  constexpr int EPT = (SIGMA_H_MAX + 255) / 256;  // entries per thread at most
  dc acc[EPT];
  int em[EPT], ec[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    acc[j] = {0.0, 0.0};
    const int e = tid + 256 * j;
    int nn2 = 0;
    while ((nn2 + 1) * (nn2 + 2) / 2 <= e) ++nn2;
    em[j] = e - nn2 * (nn2 + 1) / 2, ec[j] = nn2 - em[j];
  }
  for (int t0 = 0; t0 < nn; t0 += CH) {
    const int cnt = min(CH, nn - t0);
    __syncthreads();
    for (int i = tid; i < (M + 1) * CH; i += 256) {
      const int r = i / CH, t = i - r * CH;
      sa[r * LD + t] = t < cnt ? Ar[(int64_t)r * nn + t0 + t] : make_double2(0.0, 0.0);
      sb[r * LD + t] = t < cnt ? Bs[(int64_t)r * nn + t0 + t] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      if (tid + 256 * j >= nH) break;
      const double2* a = sa + em[j] * LD;
      const double2* b = sb + ec[j] * LD;
      dc s = acc[j];
      for (int t = 0; t < CH; ++t) {
        const double2 av = a[t], bv = b[t];
        s.x = fma(av.x, bv.x, fma(-av.y, bv.y, s.x));
        s.y = fma(av.x, bv.y, fma(av.y, bv.x, s.y));
      }
      acc[j] = s;
    }
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = tid + 256 * j;
    if (e >= nH) break;
    double2& o = H[(int64_t)pair * nH + e];
    o = make_double2(o.x + acc[j].x, o.y + acc[j].y);
  }
}

// ---------------------------------------------------------------------------
// Vector kernels of the GMRES driver (complex128 vectors of length n; the Krylov
// basis V column-major with leading dimension ld).
// ---------------------------------------------------------------------------
// partial[c][blk] = sum over this block's rows of conj(V[c][r]) w[r], c < ncol
// (blockDim 256, grid GM_BLOCKS; the partials are summed by k_gm_reduce)
__global__ __launch_bounds__(256) void k_gm_multidot(const double2* V, int64_t ld, int ncol, const double2* w,
                                                     int64_t n, double2* partial) {
  __shared__ double2 red[256];
  const int tid = threadIdx.x;
  for (int c = 0; c < ncol; ++c) {
    const double2* v = V + (int64_t)c * ld;
    dc acc = {0.0, 0.0};
    for (int64_t r = (int64_t)blockIdx.x * 256 + tid; r < n; r += (int64_t)gridDim.x * 256) {
      const double2 a = v[r], b = w[r];
      acc = cadd(acc, {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x});
    }
    red[tid] = make_double2(acc.x, acc.y);
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] = make_double2(red[tid].x + red[tid + st].x, red[tid].y + red[tid + st].y);
      __syncthreads();
    }
    if (tid == 0) partial[(int64_t)c * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// out[c] = sum_b partial[c][b], one block of 256 per column (fixed order: deterministic)
__global__ __launch_bounds__(256) void k_gm_reduce(const double2* partial, int nblk, double2* out) {
  __shared__ double2 red[256];
  const int c = blockIdx.x, tid = threadIdx.x;
  double2 a = make_double2(0.0, 0.0);
  for (int b = tid; b < nblk; b += 256) a = make_double2(a.x + partial[(int64_t)c * nblk + b].x,
                                                         a.y + partial[(int64_t)c * nblk + b].y);
  red[tid] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] = make_double2(red[tid].x + red[tid + st].x, red[tid].y + red[tid + st].y);
    __syncthreads();
  }
  if (tid == 0) out[c] = red[0];
}

// w[r] += sgn * sum_c V[c][r] coef[c]
__global__ void k_gm_update(const double2* V, int64_t ld, int ncol, const double2* coef, double sgn, double2* w,
                            int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  dc acc = {0.0, 0.0};
  for (int c = 0; c < ncol; ++c) {
    const double2 v = V[(int64_t)c * ld + r], h = coef[c];
    acc = cadd(acc, cmul({v.x, v.y}, {h.x, h.y}));
  }
  w[r] = make_double2(w[r].x + sgn * acc.x, w[r].y + sgn * acc.y);
}

// y[r] = a x[r] + b y[r] (complex a, b)
__global__ void k_gm_axpby(double2 a, const double2* x, double2 b, double2* y, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const dc v = cadd(cmul({a.x, a.y}, {x[r].x, x[r].y}), cmul({b.x, b.y}, {y[r].x, y[r].y}));
  y[r] = make_double2(v.x, v.y);
}

}  // namespace tefmm
