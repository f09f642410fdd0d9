// Host-only entry points of the C ABI (no GPU work): option defaults,
// densities and complex-image fits.
#include <cstring>

#include "../../include/tefmm.h"
#include "host_math.hpp"

using tefmm::cplx;

namespace tefmm {
bool medium_from_desc(const tefmm_medium* m, MediumDesc& out, std::string& err) {
  if (!m || m->n_layers < 1 || m->n_layers > TEFMM_MAX_LAYERS || !m->k || (m->n_layers > 1 && !m->interfaces)) {
    err = "invalid medium";
    return false;
  }
  out.L = m->n_layers - 1;
  out.k.assign(m->k, m->k + m->n_layers);
  out.d.assign(m->interfaces, m->interfaces + out.L);
  for (double kk : out.k)
    if (!(kk > 0)) {
      err = "wave numbers must be positive";
      return false;
    }
  for (int j = 1; j < out.L; ++j)
    if (!(out.d[j] < out.d[j - 1])) {
      err = "interfaces must be strictly decreasing";
      return false;
    }
  return true;
}
}  // namespace tefmm

extern "C" void tefmm_default_options(tefmm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->p = 8;
  o->depth = 0;
  o->max_leaf = 64;
  o->precision = TEFMM_FP64;
  o->normalization = TEFMM_NORM_PHYSICAL;
  o->dcim_T1 = 10.0;
  o->dcim_samples = 101;
  o->dcim_svd_tol = 1e-12;
  o->interface_eps = 1e-9;
  o->n_rhs_max = 64;
  o->dcim_T1_cross = 30.0;
}

extern "C" int tefmm_densities(const tefmm_medium* medium, int lp, int n, const double* krho,
                               double* out) {
  tefmm::MediumDesc med;
  std::string err;
  if (!tefmm::medium_from_desc(medium, med, err)) return TEFMM_ERR_INVALID_ARG;
  if (lp < 0 || lp > med.L || n < 0 || (n > 0 && (!krho || !out))) return TEFMM_ERR_INVALID_ARG;
  std::vector<cplx> sig;
  const int nl = med.L + 1;
  for (int i = 0; i < n; ++i) {
    tefmm::reaction_densities(med, lp, cplx(krho[2 * i], krho[2 * i + 1]), sig);
    for (int m = 0; m < nl; ++m)
      for (int ab = 0; ab < 4; ++ab) {
        size_t o = ((size_t)(m * 4 + ab) * n + i) * 2;
        out[o] = sig[m * 4 + ab].real();
        out[o + 1] = sig[m * 4 + ab].imag();
      }
  }
  return TEFMM_OK;
}

extern "C" int tefmm_dcim_family(const tefmm_medium* medium, const tefmm_options* opt, int l,
                                 int family, double z_lo, double z_hi, int cap, int* m,
                                 double* amp, double* depth, double* fit_err) {
  tefmm::MediumDesc med;
  std::string err;
  if (!tefmm::medium_from_desc(medium, med, err)) return TEFMM_ERR_INVALID_ARG;
  tefmm_options o;
  if (opt)
    o = *opt;
  else
    tefmm_default_options(&o);
  if (l < 0 || l > med.L || family < 0 || family > 2 || !m) return TEFMM_ERR_INVALID_ARG;
  std::vector<cplx> A, Z;
  double fe = 0;
  if (!tefmm::same_layer_family(med, l, family, z_lo, z_hi, o.dcim_T1, o.dcim_samples,
                                o.dcim_svd_tol, A, Z, fe, err))
    return TEFMM_ERR_DCIM_FIT;
  *m = (int)A.size();
  if (fit_err) *fit_err = fe;
  if ((int)A.size() > cap) return TEFMM_ERR_INVALID_ARG;
  for (size_t i = 0; i < A.size(); ++i) {
    amp[2 * i] = A[i].real(), amp[2 * i + 1] = A[i].imag();
    depth[2 * i] = Z[i].real(), depth[2 * i + 1] = Z[i].imag();
  }
  return TEFMM_OK;
}

extern "C" int tefmm_dcim_cross(const tefmm_medium* medium, const tefmm_options* opt, int l, int lp, int a,
                                double zs, int k3p, double z_lo, double z_hi, int cap, int* m, double* amp,
                                double* depth, double* fit_err) {
  tefmm::MediumDesc med;
  std::string err;
  if (!tefmm::medium_from_desc(medium, med, err)) return TEFMM_ERR_INVALID_ARG;
  tefmm_options o;
  if (opt)
    o = *opt;
  else
    tefmm_default_options(&o);
  if (l < 0 || l > med.L || lp < 0 || lp > med.L || l == lp || a < 0 || a > 1 || k3p < 0 || k3p > 32 || !m)
    return TEFMM_ERR_INVALID_ARG;
  std::vector<cplx> A, Z;
  double fe = 0;
  if (!tefmm::cross_layer_fit(med, l, lp, a, zs, k3p, z_lo, z_hi, o.dcim_T1_cross, o.dcim_samples, o.dcim_svd_tol, A, Z,
                              fe, err))
    return TEFMM_ERR_DCIM_FIT;
  *m = (int)A.size();
  if (fit_err) *fit_err = fe;
  if ((int)A.size() > cap) return TEFMM_ERR_INVALID_ARG;
  for (size_t i = 0; i < A.size(); ++i) {
    amp[2 * i] = A[i].real(), amp[2 * i + 1] = A[i].imag();
    depth[2 * i] = Z[i].real(), depth[2 * i + 1] = Z[i].imag();
  }
  return TEFMM_OK;
}
