// Host-side FP64 mathematics of the layered medium: reaction densities by the
// interface solve (Sec. 2.1) and discrete complex images by a two-level
// generalized pencil-of-function fit (Sec. 3.3).
#pragma once
#include <complex>
#include <string>
#include <vector>

namespace tefmm {

using cplx = std::complex<double>;

struct MediumDesc {
  int L = 0;                 // number of interfaces (layers 0..L)
  std::vector<double> k;     // L+1 wave numbers
  std::vector<double> d;     // L interfaces, decreasing
  double top(int m) const { return m == 0 ? 1e300 : d[m - 1]; }
  double bottom(int m) const { return m == L ? -1e300 : d[m]; }
  double thickness(int m) const { return top(m) - bottom(m); }
  int layer_of(double z) const {
    int c = 0;
    for (int j = 0; j < L; ++j) c += (z < d[j]);
    return c;
  }
};

// sqrt(k^2 - krho^2) with Im >= 0.
cplx vertical_wavenumber(double k, cplx krho);

// Densities for a source in layer lp at one k_rho:
// sig[m][ab], ab = 0:uu 1:ud 2:du 3:dd; absent entries are zero.
void reaction_densities(const MediumDesc& med, int lp, cplx krho, std::vector<cplx>& sig);

// A complex-exponential fit  y_n ~ sum_i r_i w_i^n  (matrix pencil from the SVD of
// the Hankel data matrix, residues by least squares).
struct PencilFit {
  std::vector<cplx> w, r;
};
bool pencil_fit(const std::vector<cplx>& y, double svd_tol, int max_terms, PencilFit& out,
                std::string& err);
// Least-squares residues r for fixed poles w:  y_n ~ sum_i r_i w_i^n.
bool residues_ls(const std::vector<cplx>& y, const std::vector<cplx>& w, std::vector<cplx>& r, std::string& err);

// Complex images of a spectral function  Theta(k_z) ~ sum_j A_j exp(-i k_z Z_j)
// (Eq. compleximageapp) by the paper's two-level sampling (paths C_ap1, C_ap2).
struct ImageSet {
  std::vector<cplx> A, Z;
  double fit_err = 0;  // max relative misfit over both sampling paths
};
template <class F>
bool two_level_dcim(F theta, double k, double T0, double T1, int samples, double svd_tol,
                    ImageSet& out, std::string& err);

// The three same-layer families of layer l (see tefmm.h, tefmm_dcim_family).
// Fills amp/depth in the kernel form sum_j A_j e^{ikR_j}/(4 pi R_j),
// R_j = sqrt(rho^2 + (Z - depth_j)^2).
bool same_layer_family(const MediumDesc& med, int l, int family, double z_lo, double z_hi,
                       double T1, int samples, double svd_tol, std::vector<cplx>& amp,
                       std::vector<cplx>& depth, double& fit_err, std::string& err);

// n-point Gauss-Legendre rule on [0, 1] (nodes ascending).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);

// Cross-layer complex images (Sec. 3.3, the paper's per source height and per
// z' derivative fits): target layer l, source layer lp != l, target-side wave
// a (0 = up-going, needs l < L; 1 = down-going, needs l > 0), source height zs,
// z' derivative order k3p.  The kernel  d^{k3p}/dz'^{k3p} G^{(a)}_{l,lp}(r, r') / k3p!
// at z' = zs is  sum_j A_j e^{i k_l R_j} / (4 pi R_j),
// R_j = sqrt(rho^2 + (Z_a(z) - depth_j)^2),  Z_up(z) = z - d_l,  Z_dn(z) = d_{l-1} - z.
bool cross_layer_fit(const MediumDesc& med, int l, int lp, int a, double zs, int k3p, double z_lo, double z_hi,
                     double T1, int samples, double svd_tol, std::vector<cplx>& amp, std::vector<cplx>& depth,
                     double& fit_err, std::string& err);

}  // namespace tefmm
