// Host FP64: reaction densities (interface solve, Sec. 2.1) and two-level
// discrete complex images (Sec. 3.3) with a hand-written generalized
// pencil-of-function fit (complex one-sided Jacobi SVD, Hessenberg QR
// eigenvalues, Householder least squares).
#include "host_math.hpp"

#include <algorithm>
#include <cmath>

namespace tefmm {

static const double EPS = 2.220446049250313e-16;

cplx vertical_wavenumber(double k, cplx krho) {
  cplx v = std::sqrt(cplx(k * k, 0.0) - krho * krho);
  if (v.imag() < 0) v = -v;
  return v;
}

// ---------------------------------------------------------------------------
// Dense complex helpers (row-major storage, leading dimension = columns).
// ---------------------------------------------------------------------------
struct CMat {
  int r = 0, c = 0;
  std::vector<cplx> a;
  CMat() = default;
  CMat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, cplx(0, 0)) {}
  cplx& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  const cplx& operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

// Gaussian elimination with partial pivoting; solves A X = B in place (B: n x m).
static bool gauss_solve(CMat& A, CMat& B) {
  int n = A.r;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::abs(A(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A(i, k)) > best) best = std::abs(A(i, k)), piv = i;
    if (best == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(piv, j));
      for (int j = 0; j < B.c; ++j) std::swap(B(k, j), B(piv, j));
    }
    for (int i = k + 1; i < n; ++i) {
      cplx f = A(i, k) / A(k, k);
      if (f == cplx(0, 0)) continue;
      for (int j = k; j < n; ++j) A(i, j) -= f * A(k, j);
      for (int j = 0; j < B.c; ++j) B(i, j) -= f * B(k, j);
    }
  }
  for (int k = n - 1; k >= 0; --k)
    for (int j = 0; j < B.c; ++j) {
      cplx s = B(k, j);
      for (int i = k + 1; i < n; ++i) s -= A(k, i) * B(i, j);
      B(k, j) = s / A(k, k);
    }
  return true;
}

// ---------------------------------------------------------------------------
// Reaction densities: unknowns per layer m are the up-going amplitude b_m
// (m < L, wave exp(i kz (z - d_m))) and the down-going amplitude a_m (m > 0,
// wave exp(i kz (d_{m-1} - z))); the field of layer m is (1/k_mz)(...).  Two
// conditions per interface: the value and k * d/dz are continuous.  The
// right-hand sides are the two incident waves of the source layer.
// ---------------------------------------------------------------------------
void reaction_densities(const MediumDesc& med, int lp, cplx krho, std::vector<cplx>& sig) {
  const int L = med.L;
  sig.assign((size_t)(L + 1) * 4, cplx(0, 0));
  if (L == 0) return;
  std::vector<int> col_b(L + 1, -1), col_a(L + 1, -1);
  int n = 0;
  for (int m = 0; m <= L; ++m) {
    if (m < L) col_b[m] = n++;
    if (m > 0) col_a[m] = n++;
  }
  std::vector<cplx> KZ(L + 1);
  for (int m = 0; m <= L; ++m) KZ[m] = vertical_wavenumber(med.k[m], krho);
  const cplx I(0, 1);
  CMat A(n, n), B(n, 2);
  const bool has_up = lp < L, has_dn = lp > 0;
  for (int j = 0; j < L; ++j) {
    const int rv = 2 * j, rf = 2 * j + 1, up = j, lo = j + 1;
    const double ku = med.k[up], kl = med.k[lo];
    A(rv, col_b[up]) += 1.0 / KZ[up];
    A(rf, col_b[up]) += ku * I;
    if (up > 0) {
      cplx e = std::exp(I * KZ[up] * med.thickness(up));
      A(rv, col_a[up]) += e / KZ[up];
      A(rf, col_a[up]) += -ku * I * e;
    }
    A(rv, col_a[lo]) -= 1.0 / KZ[lo];
    A(rf, col_a[lo]) -= -kl * I;
    if (lo < L) {
      cplx e = std::exp(I * KZ[lo] * med.thickness(lo));
      A(rv, col_b[lo]) -= e / KZ[lo];
      A(rf, col_b[lo]) -= kl * I * e;
    }
    if (has_up && lp == up) {  // incident wave travelling down onto z = d_j
      B(rv, 0) -= 1.0 / KZ[lp];
      B(rf, 0) -= ku * (-I);
    }
    if (has_dn && lp == lo) {  // incident wave travelling up onto z = d_j
      B(rv, 1) += 1.0 / KZ[lp];
      B(rf, 1) += kl * I;
    }
  }
  if (!gauss_solve(A, B)) return;
  for (int m = 0; m <= L; ++m) {
    if (m < L) {
      if (has_up) sig[m * 4 + 0] = B(col_b[m], 0);  // uu
      if (has_dn) sig[m * 4 + 1] = B(col_b[m], 1);  // ud
    }
    if (m > 0) {
      if (has_up) sig[m * 4 + 2] = B(col_a[m], 0);  // du
      if (has_dn) sig[m * 4 + 3] = B(col_a[m], 1);  // dd
    }
  }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of A (m x n): returns singular values (descending) and
// the right singular vectors V (n x n, columns).
// ---------------------------------------------------------------------------
static void jacobi_svd(CMat A, std::vector<double>& sv, CMat& V) {
  const int m = A.r, n = A.c;
  // working copies by columns (contiguous), real and imaginary parts apart
  std::vector<double> xr((size_t)m * n), xi((size_t)m * n), vr((size_t)n * n, 0.0), vi((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < m; ++i) xr[(size_t)j * m + i] = A(i, j).real(), xi[(size_t)j * m + i] = A(i, j).imag();
    vr[(size_t)j * n + j] = 1.0;
  }
  // rotate columns p and q: with ph = <p, q> / |<p, q>| and w = q conj(ph),
  // p <- c p - s w,  q <- (s p + c w) ph
  auto rotate = [](double* pr, double* pi, double* qr, double* qi, int len, double c, double s, double phr,
                   double phi) {
    for (int i = 0; i < len; ++i) {
      const double apr = pr[i], api = pi[i];
      const double wr = qr[i] * phr + qi[i] * phi, wi = qi[i] * phr - qr[i] * phi;
      pr[i] = c * apr - s * wr, pi[i] = c * api - s * wi;
      const double tr = s * apr + c * wr, ti = s * api + c * wi;
      qr[i] = tr * phr - ti * phi, qi[i] = tr * phi + ti * phr;
    }
  };
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double* pr = &xr[(size_t)p * m];
        double* pi = &xi[(size_t)p * m];
        double* qr = &xr[(size_t)q * m];
        double* qi = &xi[(size_t)q * m];
        double al = 0, be = 0, gr = 0, gi = 0;  // |p|^2, |q|^2, <p, q> = sum conj(p) q
        for (int i = 0; i < m; ++i) {
          al += pr[i] * pr[i] + pi[i] * pi[i];
          be += qr[i] * qr[i] + qi[i] * qi[i];
          gr += pr[i] * qr[i] + pi[i] * qi[i];
          gi += pr[i] * qi[i] - pi[i] * qr[i];
        }
        const double g = std::hypot(gr, gi);
        if (g == 0.0 || g <= 1e-15 * std::sqrt(al * be)) continue;
        off = std::max(off, g / std::sqrt(al * be));
        const double phr = gr / g, phi = gi / g;
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        rotate(pr, pi, qr, qi, m, c, s, phr, phi);
        rotate(&vr[(size_t)p * n], &vi[(size_t)p * n], &vr[(size_t)q * n], &vi[(size_t)q * n], n, c, s, phr, phi);
      }
    if (off < 1e-15) break;
  }
  std::vector<double> nrm(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += xr[(size_t)j * m + i] * xr[(size_t)j * m + i] + xi[(size_t)j * m + i] * xi[(size_t)j * m + i];
    nrm[j] = std::sqrt(s);
  }
  std::vector<int> ord(n);
  for (int j = 0; j < n; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  V = CMat(n, n);
  sv.resize(n);
  for (int j = 0; j < n; ++j) {
    sv[j] = nrm[ord[j]];
    for (int i = 0; i < n; ++i) V(i, j) = cplx(vr[(size_t)ord[j] * n + i], vi[(size_t)ord[j] * n + i]);
  }
}

// Householder QR least squares: minimise ||A X - B|| (A: m x n, m >= n; B: m x k).
static bool householder_lstsq(CMat A, CMat B, CMat& X) {
  const int m = A.r, n = A.c, k = B.c;
  for (int j = 0; j < n; ++j) {
    double nx = 0;
    for (int i = j; i < m; ++i) nx += std::norm(A(i, j));
    nx = std::sqrt(nx);
    if (nx == 0.0) return false;
    cplx x0 = A(j, j);
    cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1, 0);
    cplx alpha = -ph * nx;
    std::vector<cplx> v(m - j);
    for (int i = j; i < m; ++i) v[i - j] = A(i, j);
    v[0] -= alpha;
    double nv = 0;
    for (auto& e : v) nv += std::norm(e);
    nv = std::sqrt(nv);
    if (nv == 0.0) continue;
    for (auto& e : v) e /= nv;
    for (int c = j; c < n; ++c) {
      cplx s(0, 0);
      for (int i = j; i < m; ++i) s += std::conj(v[i - j]) * A(i, c);
      for (int i = j; i < m; ++i) A(i, c) -= 2.0 * v[i - j] * s;
    }
    for (int c = 0; c < k; ++c) {
      cplx s(0, 0);
      for (int i = j; i < m; ++i) s += std::conj(v[i - j]) * B(i, c);
      for (int i = j; i < m; ++i) B(i, c) -= 2.0 * v[i - j] * s;
    }
  }
  X = CMat(n, k);
  for (int c = 0; c < k; ++c)
    for (int i = n - 1; i >= 0; --i) {
      cplx s = B(i, c);
      for (int t = i + 1; t < n; ++t) s -= A(i, t) * X(t, c);
      if (A(i, i) == cplx(0, 0)) return false;
      X(i, c) = s / A(i, i);
    }
  return true;
}

// Eigenvalues of a general complex matrix: Householder reduction to Hessenberg
// form, then single-shift QR with Wilkinson shifts and deflation.
static bool eigenvalues(CMat H, std::vector<cplx>& ev) {
  const int n = H.r;
  ev.assign(n, cplx(0, 0));
  for (int k = 0; k < n - 2; ++k) {
    double nx = 0;
    for (int i = k + 1; i < n; ++i) nx += std::norm(H(i, k));
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    cplx x0 = H(k + 1, k);
    cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1, 0);
    std::vector<cplx> v(n - k - 1);
    for (int i = k + 1; i < n; ++i) v[i - k - 1] = H(i, k);
    v[0] += ph * nx;
    double nv = 0;
    for (auto& e : v) nv += std::norm(e);
    nv = std::sqrt(nv);
    for (auto& e : v) e /= nv;
    for (int c = 0; c < n; ++c) {  // H <- (I - 2vv^H) H
      cplx s(0, 0);
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i - k - 1]) * H(i, c);
      for (int i = k + 1; i < n; ++i) H(i, c) -= 2.0 * v[i - k - 1] * s;
    }
    for (int r = 0; r < n; ++r) {  // H <- H (I - 2vv^H)
      cplx s(0, 0);
      for (int i = k + 1; i < n; ++i) s += H(r, i) * v[i - k - 1];
      for (int i = k + 1; i < n; ++i) H(r, i) -= 2.0 * s * std::conj(v[i - k - 1]);
    }
  }
  int hi = n - 1, iter = 0;
  while (hi >= 0) {
    if (hi == 0) {
      ev[0] = H(0, 0);
      break;
    }
    int l = hi;
    while (l > 0 && std::abs(H(l, l - 1)) > EPS * (std::abs(H(l, l)) + std::abs(H(l - 1, l - 1)))) --l;
    if (l > 0) H(l, l - 1) = 0.0;
    if (l == hi) {
      ev[hi] = H(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 300 * n) return false;
    cplx a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    cplx tr2 = 0.5 * (a + d), disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
    cplx mu1 = tr2 + disc, mu2 = tr2 - disc;
    cplx mu = std::abs(mu1 - d) < std::abs(mu2 - d) ? mu1 : mu2;
    if (iter % 17 == 0) mu = d + std::abs(c);  // exceptional shift
    for (int i = l; i <= hi; ++i) H(i, i) -= mu;
    std::vector<double> cs(hi - l);
    std::vector<cplx> sn(hi - l);
    for (int k = l; k < hi; ++k) {
      cplx x = H(k, k), y = H(k + 1, k);
      double r = std::sqrt(std::norm(x) + std::norm(y));
      double cc;
      cplx ss;
      if (r == 0.0) {
        cc = 1.0, ss = 0.0;
      } else if (std::abs(x) == 0.0) {
        cc = 0.0, ss = std::conj(y) / std::abs(y);
      } else {
        cc = std::abs(x) / r;
        ss = (x / std::abs(x)) * std::conj(y) / r;
      }
      cs[k - l] = cc, sn[k - l] = ss;
      for (int j = k; j <= hi; ++j) {
        cplx h1 = H(k, j), h2 = H(k + 1, j);
        H(k, j) = cc * h1 + ss * h2;
        H(k + 1, j) = -std::conj(ss) * h1 + cc * h2;
      }
    }
    for (int k = l; k < hi; ++k) {
      double cc = cs[k - l];
      cplx ss = sn[k - l];
      int rmax = std::min(k + 2, hi);
      for (int i = l; i <= rmax; ++i) {
        cplx h1 = H(i, k), h2 = H(i, k + 1);
        H(i, k) = cc * h1 + std::conj(ss) * h2;
        H(i, k + 1) = -ss * h1 + cc * h2;
      }
    }
    for (int i = l; i <= hi; ++i) H(i, i) += mu;
  }
  return true;
}

bool residues_ls(const std::vector<cplx>& y, const std::vector<cplx>& w, std::vector<cplx>& r, std::string& err) {
  const int N = (int)y.size(), M = (int)w.size();
  r.assign(M, cplx(0, 0));
  if (M == 0) return true;
  CMat Vd(N, M), rhs(N, 1), res;
  for (int n = 0; n < N; ++n) {
    rhs(n, 0) = y[n];
    for (int i = 0; i < M; ++i) Vd(n, i) = std::pow(w[i], (double)n);
  }
  if (!householder_lstsq(Vd, rhs, res)) {
    err = "pencil: singular Vandermonde";
    return false;
  }
  for (int i = 0; i < M; ++i) r[i] = res(i, 0);
  return true;
}

bool pencil_fit(const std::vector<cplx>& y, double svd_tol, int max_terms, PencilFit& out,
                std::string& err) {
  const int N = (int)y.size();
  const int Lp = N / 2;  // pencil parameter
  CMat Y(N - Lp, Lp + 1);
  for (int i = 0; i < N - Lp; ++i)
    for (int j = 0; j <= Lp; ++j) Y(i, j) = y[i + j];
  std::vector<double> sv;
  CMat V;
  jacobi_svd(Y, sv, V);
  if (sv.empty() || sv[0] == 0.0) {
    out.w.clear(), out.r.clear();
    return true;  // identically zero data: no terms
  }
  int M = 0;
  while (M < (int)sv.size() && sv[M] > svd_tol * sv[0]) ++M;
  M = std::min(M, std::min(max_terms, Lp));
  if (M == 0) {
    out.w.clear(), out.r.clear();
    return true;
  }
  CMat V1(Lp, M), V2(Lp, M);
  for (int i = 0; i < Lp; ++i)
    for (int j = 0; j < M; ++j) V1(i, j) = V(i, j), V2(i, j) = V(i + 1, j);
  CMat Zm;
  if (!householder_lstsq(V1, V2, Zm)) {
    err = "pencil: singular V1";
    return false;
  }
  std::vector<cplx> lam;
  if (!eigenvalues(Zm, lam)) {
    err = "pencil: QR iteration did not converge";
    return false;
  }
  out.w.resize(M);
  for (int i = 0; i < M; ++i) out.w[i] = std::conj(lam[i]);
  CMat Vd(N, M), rhs(N, 1), res;
  for (int n = 0; n < N; ++n) {
    rhs(n, 0) = y[n];
    cplx p(1, 0);
    for (int i = 0; i < M; ++i) Vd(n, i) = std::pow(out.w[i], (double)n);
  }
  if (!householder_lstsq(Vd, rhs, res)) {
    err = "pencil: singular Vandermonde";
    return false;
  }
  out.r.resize(M);
  for (int i = 0; i < M; ++i) out.r[i] = res(i, 0);
  return true;
}

template <class F>
bool two_level_dcim(F theta, double k, double T0, double T1, int samples, double svd_tol,
                    ImageSet& out, std::string& err) {
  const cplx I(0, 1);
  out.A.clear(), out.Z.clear();
  double ymax = 0.0;
  // level 1: k_z = i k (T0 + t), 0 <= t <= T1
  const double dt1 = T1 / (samples - 1);
  std::vector<cplx> y1(samples), kz1(samples);
  for (int n = 0; n < samples; ++n) {
    kz1[n] = I * k * (T0 + n * dt1);
    y1[n] = theta(kz1[n]);
    ymax = std::max(ymax, std::abs(y1[n]));
  }
  const double dt2 = T0 / (samples - 1);
  std::vector<cplx> y2(samples), kz2(samples), full2(samples);
  for (int n = 0; n < samples; ++n) {
    const double t = n * dt2;
    kz2[n] = k * cplx(1.0 - t / T0, t);
    full2[n] = theta(kz2[n]);
    ymax = std::max(ymax, std::abs(full2[n]));
  }
  // a spectral function that vanishes to rounding (e.g. a wave that a uniform
  // medium does not produce) has no images
  if (!(ymax > 1e-13)) {
    out.fit_err = 0.0;
    return true;
  }
  PencilFit f1;
  if (!pencil_fit(y1, svd_tol, samples / 2, f1, err)) return false;
  // An image is usable only if its depth has Re Z < 0 (then Re(zeta) > 0 wherever
  // the kernel is evaluated, as the Sommerfeld identity requires); other poles are
  // dropped and the residues re-solved on the same samples.
  auto keep_valid = [&](PencilFit& f, const std::vector<cplx>& y, auto zmap) {
    std::vector<cplx> w;
    for (size_t i = 0; i < f.w.size(); ++i) {
      const cplx Z = zmap(f.w[i]);
      if (std::isfinite(Z.real()) && std::isfinite(Z.imag()) && Z.real() < -1e-12) w.push_back(f.w[i]);
    }
    if (w.size() == f.w.size()) return true;
    f.w = w;
    return residues_ls(y, f.w, f.r, err);
  };
  if (!keep_valid(f1, y1, [&](cplx w) { return std::log(w) / (k * dt1); })) return false;
  for (size_t i = 0; i < f1.w.size(); ++i) {
    cplx Z = std::log(f1.w[i]) / (k * dt1);
    out.Z.push_back(Z);
    out.A.push_back(f1.r[i] * std::exp(-k * T0 * Z));
  }
  const size_t n1 = out.A.size();
  // level 2: k_z = k (1 - t/T0 + i t), 0 <= t <= T0, after removing level 1
  for (int n = 0; n < samples; ++n) {
    cplx s(0, 0);
    for (size_t i = 0; i < n1; ++i) s += out.A[i] * std::exp(-I * kz2[n] * out.Z[i]);
    y2[n] = full2[n] - s;
  }
  PencilFit f2;
  if (!pencil_fit(y2, svd_tol, samples / 2, f2, err)) return false;
  const cplx g = -I * k * cplx(-1.0 / T0, 1.0) * dt2;  // w = exp(g Z)
  if (!keep_valid(f2, y2, [&](cplx w) { return std::log(w) / g; })) return false;
  for (size_t i = 0; i < f2.w.size(); ++i) {
    cplx Z = std::log(f2.w[i]) / g;
    out.Z.push_back(Z);
    out.A.push_back(f2.r[i] * std::exp(I * k * Z));
  }
  // misfit over both paths
  double e = 0.0;
  for (int n = 0; n < samples; ++n) {
    cplx s1(0, 0), s2(0, 0);
    for (size_t i = 0; i < out.A.size(); ++i) {
      s1 += out.A[i] * std::exp(-I * kz1[n] * out.Z[i]);
      s2 += out.A[i] * std::exp(-I * kz2[n] * out.Z[i]);
    }
    e = std::max(e, std::abs(s1 - y1[n]));
    e = std::max(e, std::abs(s2 - full2[n]));
  }
  out.fit_err = ymax > 0 ? e / ymax : 0.0;
  for (size_t i = 0; i < out.A.size(); ++i)
    if (!std::isfinite(out.A[i].real()) || !std::isfinite(out.Z[i].real())) {
      err = "dcim: non-finite image";
      return false;
    }
  return true;
}

// Cancellation among the image terms in space: the largest ratio of sum |term| to
// |sum of terms| of K(rho, Z) = sum_j A_j e^{ikR_j}/R_j, R_j^2 = rho^2 + (Z - Z_j)^2,
// over heights Z = 0, span/2, span above the decay shift and rho = 0, 0.5, 2.  A fit whose
// singular values just pass the cut can pair nearly equal poles with huge opposite
// residues: the spectral samples are matched, but in space the terms cancel to few
// digits.
static double image_cancellation(const ImageSet& im, double k, double span) {
  double worst = 1.0;
  const cplx I(0, 1);
  for (double Zr : {0.0, 0.5 * span, span})
    for (double rho : {0.0, 0.5, 2.0}) {
      cplx s(0, 0);
      double a = 0.0;
      for (size_t j = 0; j < im.A.size(); ++j) {
        const cplx zeta = Zr - im.Z[j];
        const cplx R = std::sqrt(rho * rho + zeta * zeta);
        const cplx t = im.A[j] * std::exp(I * k * R) / R;
        s += t, a += std::abs(t);
      }
      if (a > 0) worst = std::max(worst, std::abs(s) > 0 ? a / std::abs(s) : 1e300);
    }
  return worst;
}

// two_level_dcim with the singular-value cut raised tenfold (up to four times) while the
// image terms cancel in space by more than twelve digits (a degenerate pole pair; usual
// fits, whose deep images carry large amplitudes, stay well below); the least
// cancelling fit is kept.
template <class F>
static bool robust_dcim(F theta, double k, double T0, double T1, int samples, double svd_tol, double span,
                        ImageSet& out, std::string& err) {
  double best = 0.0;
  bool have = false;
  double tol = svd_tol;
  for (int attempt = 0; attempt < 5; ++attempt, tol *= 10.0) {
    ImageSet im;
    std::string e2;
    if (!two_level_dcim(theta, k, T0, T1, samples, tol, im, e2)) {
      if (!have) err = e2;
      continue;
    }
    const double c = image_cancellation(im, k, span);
    if (!have || c < best) out = im, best = c, have = true;
    if (c <= 1e12) break;
  }
  return have;
}

bool same_layer_family(const MediumDesc& med, int l, int family, double z_lo, double z_hi,
                       double T1, int samples, double svd_tol, std::vector<cplx>& amp,
                       std::vector<cplx>& depth, double& fit_err, std::string& err) {
  amp.clear(), depth.clear();
  fit_err = 0.0;
  const int L = med.L;
  if (family == 0 && l >= L) return true;             // no up-going reaction in the bottom layer
  if (family == 1 && l == 0) return true;             // no down-going reaction in the top layer
  if (family == 2 && (l == 0 || l == L)) return true; // Delta needs both waves
  double zmin;
  int ab;
  if (family == 0) {
    zmin = 2.0 * (z_lo - med.d[l]);
    ab = 0;
  } else if (family == 1) {
    zmin = 2.0 * (med.d[l - 1] - z_hi);
    ab = 3;
  } else {
    zmin = med.thickness(l) - (z_hi - z_lo);
    ab = 1;
  }
  zmin = std::max(zmin, 0.0);
  const double kl = med.k[l];
  double kmax = 0;
  for (double kk : med.k) kmax = std::max(kmax, kk);
  const double T0 = std::sqrt(((kmax + 0.8) / kl) * ((kmax + 0.8) / kl) - 1.0);
  const cplx I(0, 1);
  std::vector<cplx> sig;
  // Quasi-static image of the Sigma families: the density tends to a constant sigma_inf
  // as k_rho grows (the reflection coefficient of the interface for evanescent waves),
  // which in space is one image at the mirror point, sigma_inf e^{ikR}/R with R the
  // mirror distance.  It is taken out exactly and only the remainder (falling like
  // k_rho^-2) is fitted: the sampling paths reach |k_z| ~ k (T0 + T1) only, too short
  // to pin the constant for pairs much closer than 1/(k T1) to the mirror point.
  cplx sig_inf(0, 0);
  if (family != 2) {
    reaction_densities(med, l, cplx(1e8 * kl, 0), sig);
    sig_inf = sig[l * 4 + ab];
  }
  auto theta = [&](cplx kzl) {
    cplx krho = std::sqrt(cplx(kl * kl, 0) - kzl * kzl);
    reaction_densities(med, l, krho, sig);
    return (sig[l * 4 + ab] - sig_inf) * std::exp(I * kzl * zmin);
  };
  // Pairs closer to the mirror point than ~1/(k T1) need the density beyond the first
  // path's end |k_z| = k (T0 + T1): for the Sigma families the path is lengthened to
  // T1 = 1.2 / (k z_min) when that is longer (at most 40), with the sample spacing kept.
  double T1e = T1;
  int ns = samples;
  if (family != 2) {
    const double want = 1.2 / (kl * std::max(zmin, 1e-12));
    if (want > T1) {
      T1e = std::min(want, std::max(T1, 40.0));
      ns = std::min(std::max(samples, 401), (int)std::ceil(samples * T1e / T1)) | 1;
    }
  }
  ImageSet im;
  if (!robust_dcim(theta, kl, T0, T1e, ns, svd_tol, 2.0 * (z_hi - z_lo), im, err)) return false;
  fit_err = im.fit_err;
  for (size_t i = 0; i < im.A.size(); ++i) {
    amp.push_back(im.A[i]);
    depth.push_back(zmin + im.Z[i]);
  }
  if (std::abs(sig_inf) > 0) {
    amp.push_back(sig_inf);
    depth.push_back(cplx(0, 0));
  }
  return true;
}

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  // roots of P_n by Newton's method from the Chebyshev-like first guesses, then mapped to [0, 1]
  x.assign(n, 0.0), w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double t = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1, p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (std::abs(dt) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1, p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
    }
    const double wt = 2.0 / ((1.0 - t * t) * dp * dp);
    x[i] = 0.5 * (1.0 - t), x[n - 1 - i] = 0.5 * (1.0 + t);
    w[i] = w[n - 1 - i] = 0.5 * wt;
  }
}

bool cross_layer_fit(const MediumDesc& med, int l, int lp, int a, double zs, int k3p, double z_lo, double z_hi,
                     double T1, int samples, double svd_tol, std::vector<cplx>& amp, std::vector<cplx>& depth,
                     double& fit_err, std::string& err) {
  amp.clear(), depth.clear();
  fit_err = 0.0;
  const int L = med.L;
  if (l == lp || (a == 0 && l >= L) || (a == 1 && l == 0)) return true;
  double zmin = a == 0 ? z_lo - med.d[l] : med.d[l - 1] - z_hi;
  zmin = std::max(zmin, 0.0);
  const double kl = med.k[l];
  double kmax = 0;
  for (double kk : med.k) kmax = std::max(kmax, kk);
  const double T0 = std::sqrt(((kmax + 0.8) / kl) * ((kmax + 0.8) / kl) - 1.0);
  const cplx I(0, 1);
  double kf = 1.0;
  for (int i = 2; i <= k3p; ++i) kf *= i;
  std::vector<cplx> sig;
  auto theta = [&](cplx kzl) {
    const cplx krho = std::sqrt(cplx(kl * kl, 0) - kzl * kzl);
    reaction_densities(med, lp, krho, sig);
    const cplx kzp = vertical_wavenumber(med.k[lp], krho);
    cplx s(0, 0);
    const int ai = a == 0 ? 0 : 2;  // uu/ud or du/dd
    if (lp < L) s += sig[l * 4 + ai + 0] * std::pow(I * kzp, (double)k3p) * std::exp(I * kzp * (zs - med.d[lp]));
    if (lp > 0) s += sig[l * 4 + ai + 1] * std::pow(-I * kzp, (double)k3p) * std::exp(I * kzp * (med.d[lp - 1] - zs));
    return s / kf * std::exp(I * kzl * zmin);
  };
  ImageSet im;
  if (!robust_dcim(theta, kl, T0, T1, samples, svd_tol, z_hi - z_lo, im, err)) return false;
  fit_err = im.fit_err;
  for (size_t i = 0; i < im.A.size(); ++i) {
    amp.push_back(im.A[i]);
    depth.push_back(zmin + im.Z[i]);
  }
  return true;
}

}  // namespace tefmm
