// TEFMM-II translation in the symmetric basis (Sec. 4.1), free space.
//
// Index set (n, m, s), 0 <= s <= m <= n, ordered by n, then m, then s.  With
// D+- = (d_x +- i d_y)/k, D0 = -d_z/k and Omega^m_n = h_n(k r) Y^m_n (complex spherical
// harmonics with the Condon-Shortley phase, Y^{-m}_n = (-1)^m conj(Y^m_n)), Theorem 4.2
// moves each operator one step along the ladder:
//   D+ Omega^m_n = A+ Omega^{m+1}_{n+1} + B+ Omega^{m+1}_{n-1}, and likewise D-, D0,
// with A0 = +sqrt(((n+1)^2 - m^2)/((2n+1)(2n+3))), B0 = -sqrt((n^2 - m^2)/(4n^2 - 1)) (the
// signs that agree with the theorem's own special case D0 Omega^{+-n}_n =
// Omega^{+-n}_{n+1}/sqrt(2n+3)).  Hence, with h0 = sqrt(4 pi) Omega^0_0,
//   D^s_{nm} h0 = sqrt(4 pi) k^n (-1)^(n-m) (D-)^s (D+)^(m-s) (D0)^(n-m) Omega^0_0
//              = sqrt(4 pi) k^n (-1)^(n-m) sum_nu c^{nms}_nu Omega^{m-2s}_nu,
// nu = n, n-2, ... >= |m - 2s|.  The host expands the ladder once into the c's; a
// kernel evaluates the Omega's at each displacement and contracts.  The M2L
// (Eq. M2Ltransop) then reads, for target (n, m, s) and source (n', m', s'),
//   L = (-1)^n' D^{s+s'}_{n+n', m+m'} h0(R) / (F(n,m,s) F(n',m',s')),
//   F(n,m,s) = 2^m (n-m)! s! (m-s)!.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/tefmm.h"
#include "kernels.hpp"

namespace tefmm {

namespace {

constexpr int SYM_NMAX = 32;  // derivative order 2p, p <= 16

inline int sym_count(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
inline int sym_index(int n, int m, int s) { return n * (n + 1) * (n + 2) / 6 + m * (m + 1) / 2 + s; }

// the ladder coefficients (A, B) of op on Omega^m_n
void ladder(char op, int n, int m, double& A, double& B) {
  const double dn = n, dm = m;
  if (op == '+') {
    A = std::sqrt((dn + dm + 2) * (dn + dm + 1) / ((2 * dn + 1) * (2 * dn + 3)));
    const double b2 = n > 0 ? (dn - dm) * (dn - dm - 1) / (4 * dn * dn - 1) : 0.0;
    B = std::sqrt(std::max(b2, 0.0));
  } else if (op == '-') {
    A = -std::sqrt((dn - dm + 2) * (dn - dm + 1) / ((2 * dn + 1) * (2 * dn + 3)));
    const double b2 = n > 0 ? (dn + dm) * (dn + dm - 1) / (4 * dn * dn - 1) : 0.0;
    B = -std::sqrt(std::max(b2, 0.0));
  } else {
    A = std::sqrt(((dn + 1) * (dn + 1) - dm * dm) / ((2 * dn + 1) * (2 * dn + 3)));
    const double b2 = n > 0 ? (dn * dn - dm * dm) / (4 * dn * dn - 1) : 0.0;
    B = -std::sqrt(std::max(b2, 0.0));
  }
}

// an expansion sum c Omega^m_nu, stored over (nu, m + NMAX)
struct OmegaSum {
  std::map<std::pair<int, int>, double> c;
};

OmegaSum apply(const OmegaSum& E, char op) {
  const int dm = op == '+' ? 1 : op == '-' ? -1 : 0;
  OmegaSum out;
  for (const auto& kv : E.c) {
    const int n = kv.first.first, m = kv.first.second;
    double A, B;
    ladder(op, n, m, A, B);
    if (std::abs(m + dm) <= n + 1) out.c[{n + 1, m + dm}] += A * kv.second;
    if (n >= 1 && std::abs(m + dm) <= n - 1 && B != 0.0) out.c[{n - 1, m + dm}] += B * kv.second;
  }
  return out;
}

// coefficient tables of one derivative order N: for triple i = sym_index(n, m, s),
// c[i * (N + 1) + nu] (nu = 0 .. N; zero where nu has the wrong parity or is below |m - 2s|)
struct SymTables {
  int N = -1;
  std::vector<double> coef;
};
SymTables g_tables[SYM_NMAX + 1];  // host copies, built once per order

// the coefficients of order N, copied to a device buffer the caller frees
hipError_t sym_tables(int N, double** d_coef, hipStream_t s) {
  SymTables& T = g_tables[N];
  if (T.N != N) {
    const int cnt = sym_count(N);
    T.coef.assign((size_t)cnt * (N + 1), 0.0);
    OmegaSum E;
    E.c[{0, 0}] = 1.0;
    for (int c = 0; c <= N; ++c) {  // c = n - m applications of D0
      // (a, b) = applications of D+ and D-: all a + b <= N - c, built from (a - 1, b) or (0, b - 1)
      std::vector<std::vector<OmegaSum>> Tab(N - c + 1, std::vector<OmegaSum>(N - c + 1));
      Tab[0][0] = E;
      for (int tot = 1; tot <= N - c; ++tot)
        for (int b = 0; b <= tot; ++b) {
          const int a = tot - b;
          Tab[a][b] = a > 0 ? apply(Tab[a - 1][b], '+') : apply(Tab[a][b - 1], '-');
        }
      for (int a = 0; a + c <= N; ++a)
        for (int b = 0; a + b + c <= N; ++b) {
          const int m = a + b, n = c + m;  // s = b
          for (const auto& kv : Tab[a][b].c) T.coef[(size_t)sym_index(n, m, b) * (N + 1) + kv.first.first] += kv.second;
        }
      if (c < N) E = apply(E, '0');
    }
    T.N = N;
  }
  hipError_t e = hipMalloc(d_coef, sizeof(double) * T.coef.size());
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(*d_coef, T.coef.data(), sizeof(double) * T.coef.size(), hipMemcpyHostToDevice, s);
}

// Omega^mu_nu at R for nu <= N, |mu| <= nu, into om[nu (2 N + 1) + mu + N] (LDS), then
// D[i] = sqrt(4 pi) k^n (-1)^(n-m) sum_nu coef[i][nu] Omega^{m-2s}_nu for every triple i.
// One block of 64 per displacement.
__global__ __launch_bounds__(64) void k_sym_derivs(const double* R, int64_t nR, double k, int N, const double* coef,
                                                   double2* out) {
  __shared__ double2 om[(SYM_NMAX + 1) * (2 * SYM_NMAX + 1)];
  __shared__ double2 hn[SYM_NMAX + 1];
  const int64_t i = blockIdx.x;
  const int t = threadIdx.x;
  if (i >= nR) return;
  const double x = R[3 * i], y = R[3 * i + 1], z = R[3 * i + 2];
  const double rho = hypot(x, y), r = hypot(rho, z);
  const double ct = z / r, st = rho / r;
  const double cphi = rho > 0 ? x / rho : 1.0, sphi = rho > 0 ? y / rho : 0.0;
  const int W = 2 * N + 1;
  if (t == 0) {
    // spherical Hankel functions of the first kind by the upward recurrence
    const double kr = k * r;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const dc e = {cs, sn};
    dc h0v = cmul({0.0, -1.0 / kr}, e);                         // -i e^{ix}/x
    dc h1v = cscale(cmul(e, {kr, 1.0}), -1.0 / (kr * kr));     // -e^{ix}(x + i)/x^2
    hn[0] = make_double2(h0v.x, h0v.y);
    if (N >= 1) hn[1] = make_double2(h1v.x, h1v.y);
    for (int n = 1; n < N; ++n) {
      const dc h2 = csub(cscale(h1v, (2.0 * n + 1.0) / kr), h0v);
      hn[n + 1] = make_double2(h2.x, h2.y);
      h0v = h1v, h1v = h2;
    }
  }
  // normalised associated Legendre functions with the Condon-Shortley phase, one thread per m:
  // Yb_m^m = (-1)^m sqrt((2m+1)/(4 pi) (2m-1)!!^2/(2m)!) st^m, then the three-term recurrence in l
  for (int m = t; m <= N; m += 64) {
    double ymm = 1.0 / std::sqrt(4.0 * 3.14159265358979323846);
    for (int j = 1; j <= m; ++j) ymm *= -std::sqrt((2.0 * j + 1.0) / (2.0 * j)) * st;
    double cm, sm;  // e^{i m phi} by the double-angle powers of (cphi, sphi)
    {
      dc ph = {1.0, 0.0};
      for (int j = 0; j < m; ++j) ph = cmul(ph, {cphi, sphi});
      cm = ph.x, sm = ph.y;
    }
    double ylm2 = 0.0, ylm1 = ymm;
    for (int l = m; l <= N; ++l) {
      double yl;
      if (l == m)
        yl = ymm;
      else if (l == m + 1)
        yl = std::sqrt(2.0 * m + 3.0) * ct * ymm;
      else {
        const double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double b = std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
        yl = a * (ct * ylm1 - b * ylm2);
      }
      if (l > m) ylm2 = ylm1, ylm1 = yl;
      om[l * W + m + N] = make_double2(yl * cm, yl * sm);  // Y only; times h_l below
      if (m) om[l * W - m + N] = make_double2(((m & 1) ? -1.0 : 1.0) * yl * cm, ((m & 1) ? 1.0 : -1.0) * yl * sm);
    }
  }
  __syncthreads();
  for (int e = t; e < (N + 1) * W; e += 64) {
    const int l = e / W, mu = e - l * W - N;
    if (mu < -l || mu > l) continue;
    const dc v = cmul({om[e].x, om[e].y}, {hn[l].x, hn[l].y});
    om[e] = make_double2(v.x, v.y);
  }
  __syncthreads();
  const int cnt = (N + 1) * (N + 2) * (N + 3) / 6;
  for (int tr = t; tr < cnt; tr += 64) {
    int n = 0;
    while ((n + 1) * (n + 2) * (n + 3) / 6 <= tr) ++n;
    int rem = tr - n * (n + 1) * (n + 2) / 6, m = 0;
    while ((m + 1) * (m + 2) / 2 <= rem) ++m;
    const int s = rem - m * (m + 1) / 2, mu = m - 2 * s;
    dc acc = {0.0, 0.0};
    for (int nu = n; nu >= 0 && nu >= (mu < 0 ? -mu : mu); nu -= 2) {
      const double c = coef[(size_t)tr * (N + 1) + nu];
      const double2 o = om[nu * W + mu + N];
      acc = cadd(acc, cscale({o.x, o.y}, c));
    }
    double pre = std::sqrt(4.0 * 3.14159265358979323846) * (((n - m) & 1) ? -1.0 : 1.0);
    for (int j = 0; j < n; ++j) pre *= k;
    acc = cscale(acc, pre);
    out[(size_t)i * cnt + tr] = make_double2(acc.x, acc.y);
  }
}

// beta_i[(n, m, s)] = sum over (n', m', s') of alpha_i[(n', m', s')] (-1)^n' D_i[(n+n', m+m', s+s')]
//                     / (F(n,m,s) F(n',m',s')),  one block of 128 per displacement,
// the moments in LDS; ifac[t] = 1 / F of triple t
__global__ __launch_bounds__(128) void k_sym_m2l(const double2* D, int64_t nR, int p, const double* ifac,
                                                 const double2* alpha, double2* beta) {
  __shared__ double2 sa[(16 + 1) * (16 + 2) * (16 + 3) / 6];
  const int64_t i = blockIdx.x;
  const int t = threadIdx.x;
  if (i >= nR) return;
  const int C = (p + 1) * (p + 2) * (p + 3) / 6, CD = (2 * p + 1) * (2 * p + 2) * (2 * p + 3) / 6;
  for (int e = t; e < C; e += 128) {
    const double2 a = alpha[(size_t)i * C + e];
    const int n = [&] { int nn = 0; while ((nn + 1) * (nn + 2) * (nn + 3) / 6 <= e) ++nn; return nn; }();
    const double f = ((n & 1) ? -1.0 : 1.0) * ifac[e];
    sa[e] = make_double2(a.x * f, a.y * f);
  }
  __syncthreads();
  const double2* Di = D + (size_t)i * CD;
  for (int o = t; o < C; o += 128) {
    int n = 0;
    while ((n + 1) * (n + 2) * (n + 3) / 6 <= o) ++n;
    int rem = o - n * (n + 1) * (n + 2) / 6, m = 0;
    while ((m + 1) * (m + 2) / 2 <= rem) ++m;
    const int s = rem - m * (m + 1) / 2;
    dc acc = {0.0, 0.0};
    int j = 0;
    for (int n2 = 0; n2 <= p; ++n2)
      for (int m2 = 0; m2 <= n2; ++m2)
        for (int s2 = 0; s2 <= m2; ++s2, ++j) {
          const int N = n + n2, M = m + m2, S = s + s2;
          const double2 d = Di[N * (N + 1) * (N + 2) / 6 + M * (M + 1) / 2 + S];
          acc = cadd(acc, cmul({d.x, d.y}, {sa[j].x, sa[j].y}));
        }
    acc = cscale(acc, ifac[o]);
    beta[(size_t)i * C + o] = make_double2(acc.x, acc.y);
  }
}

}  // namespace

extern "C" int tefmm_sym_derivatives(double k, int order, int64_t n, const double* R, double* out, void* stream) {
  if (!(k > 0) || order < 0 || order > SYM_NMAX || n < 1 || n > (1 << 24) || !R || !out)
    return TEFMM_ERR_INVALID_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (!(R[3 * i] * R[3 * i] + R[3 * i + 1] * R[3 * i + 1] + R[3 * i + 2] * R[3 * i + 2] > 0))
      return TEFMM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  double* d_coef = nullptr;
  if (sym_tables(order, &d_coef, s) != hipSuccess) {
    if (d_coef) (void)hipFree(d_coef);
    return TEFMM_ERR_HIP;
  }
  const int cnt = sym_count(order);
  double* d_R = nullptr;
  double2* d_out = nullptr;
  int rc = TEFMM_OK;
  if (hipMalloc(&d_R, sizeof(double) * 3 * n) != hipSuccess ||
      hipMalloc(&d_out, sizeof(double2) * (size_t)n * cnt) != hipSuccess ||
      hipMemcpyAsync(d_R, R, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s) != hipSuccess)
    rc = TEFMM_ERR_HIP;
  if (rc == TEFMM_OK) {
    hipLaunchKernelGGL(k_sym_derivs, dim3((unsigned)n), dim3(64), 0, s, d_R, n, k, order, d_coef, d_out);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(out, d_out, sizeof(double2) * (size_t)n * cnt, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = TEFMM_ERR_HIP;
  }
  if (d_R) (void)hipFree(d_R);
  if (d_out) (void)hipFree(d_out);
  (void)hipFree(d_coef);
  return rc;
}

extern "C" int tefmm_sym_m2l(double k, int p, int64_t n, const double* R, const double* alpha, double* beta,
                             void* stream) {
  if (!(k > 0) || p < 0 || p > SYM_NMAX / 2 || n < 1 || n > (1 << 24) || !R || !alpha || !beta)
    return TEFMM_ERR_INVALID_ARG;
  for (int64_t i = 0; i < n; ++i)
    if (!(R[3 * i] * R[3 * i] + R[3 * i + 1] * R[3 * i + 1] + R[3 * i + 2] * R[3 * i + 2] > 0))
      return TEFMM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const int N = 2 * p, C = sym_count(p), CD = sym_count(N);
  double* d_coef = nullptr;
  if (sym_tables(N, &d_coef, s) != hipSuccess) {
    if (d_coef) (void)hipFree(d_coef);
    return TEFMM_ERR_HIP;
  }
  std::vector<double> ifac(C);
  for (int nn = 0; nn <= p; ++nn)
    for (int m = 0; m <= nn; ++m)
      for (int s2 = 0; s2 <= m; ++s2) {
        double f = std::ldexp(1.0, m);
        for (int j = 2; j <= nn - m; ++j) f *= j;
        for (int j = 2; j <= s2; ++j) f *= j;
        for (int j = 2; j <= m - s2; ++j) f *= j;
        ifac[sym_index(nn, m, s2)] = 1.0 / f;
      }
  double *d_R = nullptr, *d_if = nullptr;
  double2* d_D = nullptr;
  int rc = TEFMM_OK;
  if (hipMalloc(&d_R, sizeof(double) * 3 * n) != hipSuccess || hipMalloc(&d_if, sizeof(double) * C) != hipSuccess ||
      hipMalloc(&d_D, sizeof(double2) * (size_t)n * CD) != hipSuccess ||
      hipMemcpyAsync(d_R, R, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(d_if, ifac.data(), sizeof(double) * C, hipMemcpyHostToDevice, s) != hipSuccess)
    rc = TEFMM_ERR_HIP;
  if (rc == TEFMM_OK) {
    hipLaunchKernelGGL(k_sym_derivs, dim3((unsigned)n), dim3(64), 0, s, d_R, n, k, N, d_coef, d_D);
    hipLaunchKernelGGL(k_sym_m2l, dim3((unsigned)n), dim3(128), 0, s, (const double2*)d_D, n, p, (const double*)d_if,
                       (const double2*)alpha, (double2*)beta);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) rc = TEFMM_ERR_HIP;
  }
  if (d_R) (void)hipFree(d_R);
  if (d_if) (void)hipFree(d_if);
  if (d_D) (void)hipFree(d_D);
  (void)hipFree(d_coef);
  return rc;
}

}  // namespace tefmm
