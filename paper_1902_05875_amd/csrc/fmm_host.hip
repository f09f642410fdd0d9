// Host orchestration and the C ABI of the layered-media TE-FMM.
//
// set_particles: per-layer uniform octrees (GPU radix sort by leaf), complex
// image fits of the same-layer reaction families (host FP64), derivative
// tables for every translation key (GPU FP64).  evaluate: P2M, M2M, M2L
// (free + Delta family and Sigma family, MFMA), L2L, L2P, P2P, scale and
// un-permute, all stream ordered on the caller's stream (Algorithm 1 for the
// reaction components, fused with the free-space FMM of Algorithm 2 for the
// same layer).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/tefmm.h"
#include "fmm_kernels.hpp"
static_assert(tefmm::MAX_LAYERS == TEFMM_MAX_LAYERS, "layer limit of the kernels and of the C ABI");
#include "host_math.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "sort_scan.hpp"

namespace tefmm {
bool medium_from_desc(const tefmm_medium* m, MediumDesc& out, std::string& err);
}

using namespace tefmm;

namespace {

const double PI = 3.14159265358979323846;

// Solve the 3 x 3 system A x = b (Cramer's rule; A symmetric positive definite here).
void solve3(const double (&A)[3][3], const double (&b)[3], double (&x)[3]) {
  auto det = [](const double (&M)[3][3]) {
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  };
  const double d = det(A);
  for (int c = 0; c < 3; ++c) {
    double M[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[i][j] = j == c ? b[i] : A[i][j];
    x[c] = det(M) / d;
  }
}

// The FP32 near field's pair value in scaled units (r = k |x - y| / (2 pi)) is
// cos(2 pi r) / r + i sin(2 pi r) / r.  Over a leaf's 3 x 3 x 3 block r stays below
// rmax = 2 sqrt(3) h k / (2 pi), where both cos(2 pi r) and sin(2 pi r) / r are smooth
// functions of s = r^2 with rapidly falling Taylor terms; fit each by a quadratic in s
// (least squares at 64 Chebyshev points of [0, rmax^2], in t = s / rmax^2), then take
// the largest error of the FP32-rounded coefficients over 4097 points, as a fraction of
// the pair value's size 1/r: |cos error| and r |sine error|.  Returns whether it is
// within tol (never for a leaf of zero size, where all particles coincide).
bool fit_near_poly(double k, double h, double tol, NearPoly* np, double* err) {
  const double rmax = 2.0 * std::sqrt(3.0) * h * k / (2.0 * PI) * (1.0 + 1e-6);
  const double S = rmax * rmax;
  *err = 0;
  if (!(S > 0) || !std::isfinite(S)) return false;
  auto fc = [](double s) { return std::cos(2.0 * PI * std::sqrt(s)); };
  auto fs = [](double s) {
    const double r = std::sqrt(s);
    return r > 0 ? std::sin(2.0 * PI * r) / r : 2.0 * PI;
  };
  double A[3][3] = {}, bc[3] = {}, bs[3] = {};
  const int m = 64;
  for (int i = 0; i < m; ++i) {
    const double t = 0.5 - 0.5 * std::cos(PI * (i + 0.5) / m);
    const double ph[3] = {1.0, t, t * t};
    for (int u = 0; u < 3; ++u) {
      for (int v = 0; v < 3; ++v) A[u][v] += ph[u] * ph[v];
      bc[u] += ph[u] * fc(t * S), bs[u] += ph[u] * fs(t * S);
    }
  }
  double xc[3], xs[3];
  solve3(A, bc, xc);
  solve3(A, bs, xs);
  np->c0 = (float)xc[0], np->c1 = (float)(xc[1] / S), np->c2 = (float)(xc[2] / (S * S));
  np->s0 = (float)xs[0], np->s1 = (float)(xs[1] / S), np->s2 = (float)(xs[2] / (S * S));
  double e = 0;
  bool finite = true;
  for (int i = 0; i <= 4096; ++i) {
    const double s = S * i / 4096.0, r = std::sqrt(s);
    const double pc = ((double)np->c2 * s + np->c1) * s + np->c0;
    const double ps = ((double)np->s2 * s + np->s1) * s + np->s0;
    const double d = std::max(std::fabs(pc - fc(s)), r * std::fabs(ps - fs(s)));
    finite = finite && std::isfinite(d);  // std::max passes over a NaN
    e = std::max(e, d);
  }
  *err = finite ? e : 0;
  return finite && e <= tol;
}

struct Group {
  int layer = 0, depth = 2;
  double lo[3] = {0, 0, 0}, side = 1;
  int64_t start = 0, count = 0, leaf_base = 0;
  double zlo = 0, zhi = 0;
  std::vector<cplx> famA[3], famZ[3];
  double fam_err[3] = {0, 0, 0};
  bool has[3] = {false, false, false};
  std::vector<double2*> alpha, beta;  // by level, full Taylor sets [rhs][box][nC]
  std::vector<double2*> ared, bred;   // by level, Helmholtz-reduced sets [rhs][box][nR]
  std::vector<float2*> ared32;        // reduced moments in FP32 (mixed precision; ared unused then)
  std::vector<double2*> Tfd, TS;
  std::vector<float2*> Tfd32, TS32;
  std::vector<int64_t> nbox;          // boxes at level
  std::vector<int64_t> far_pairs, near_pairs;  // per level from 2: interaction-list / neighbour pairs
                                               // between occupied boxes
  std::vector<std::vector<unsigned char>> occ;  // per level: 1 where the box holds particles
  std::vector<unsigned char*> d_occ;            // device copies (read by the M2L)
  double fit_zlo = 0, fit_zhi = 0;              // height range of the complex-image fits
  // cross-layer (this group as target): z-reduced moments/locals and per-level lists and tables
  std::vector<double2*> azred, bzred;
  std::vector<int*> xlist_start;
  std::vector<CrossEntry*> xlist;
  std::vector<int> xkeys;                       // keys per level
  std::vector<double2*> XT0, XT1;
  std::vector<float2*> XT032, XT132;
  double cross_flops_per_rhs = 0;
  int64_t cross_pairs = 0, cross_forced = 0;  // forced: leaf pairs translated below the acceptance test
  // symmetric near field: targets per lane and workgroups per leaf (each taking every
  // p2p_split-th pass of 64 p2p_tpl targets), from the leaf occupancy
  int p2p_tpl = 1, p2p_split = 1;
  double mean_occ = 0;  // mean particles per occupied leaf
  // work items of the symmetric near field (leaves with particles, halves with a pass), in
  // leaf order, and their cut into 8 segments of about equal pair work (one per XCD)
  std::vector<unsigned> nf_items;
  XcdSegs nf_seg{};
  int nf_seg_max = 0;
  unsigned* d_nf_items = nullptr;
  // the same for the one-sided near field: occupied leaves, work = targets x the particles of
  // the 27-leaf block
  std::vector<unsigned> p2p_items;
  XcdSegs p2p_seg{};
  int p2p_seg_max = 0;
  unsigned* d_p2p_items = nullptr;
  // FP32 near-field pair value from quadratics in r^2 (np_on) and the fit's error
  NearPoly np{};
  bool np_on = false;
  double np_err = 0;
  int n_cross_fits = 0;
  double cross_fit_err = 0;
  bool has_cross = false;
  // Sigma-family keys of the leaf level whose expansion would not converge (boxes next
  // to an interface): their table rows are zero and their leaf pairs are evaluated
  // directly from the complex images (k_sigma_direct) on the lists below
  std::vector<char> sig_flag;               // [49 (2 nb - 1)] at the leaf level
  int* d_sd_tgt = nullptr;                  // listed target leaves
  int* d_sd_start = nullptr;                // [ntgt + 1] into d_sd_src
  int* d_sd_src = nullptr;                  // their source leaves
  double2* d_sd_img = nullptr;              // images: A, Z of Sigma-up, then of Sigma-down
  int sd_ntgt = 0, sd_nup = 0, sd_ndn = 0;
  int64_t sd_pairs = 0;                     // particle pairs evaluated directly (per charge vector)
  int64_t keys_forced = 0;                  // reaction keys translated with a poor separation ratio
};

template <class T>
void dfree_raw(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

}  // namespace

struct tefmm_ctx {
  MediumDesc med;
  tefmm_options opt;
  std::string err;
  int nC = 0, nR = 0, nG = 0, nKB = 0, nRB = 0, nRs = 0;
  // constant tables
  int* d_mi = nullptr;      // [nC] graded multi-indices (packed)
  int* d_rmi = nullptr;     // [nR] reduced multi-indices (packed)
  int* d_rfull = nullptr;   // [nR] graded index of each reduced entry
  int* d_gpad = nullptr;    // [nG] padded LDS position of each compact table entry
  int* d_rzmi = nullptr;    // [nR] z-reduced multi-indices (packed)
  int* d_rzfull = nullptr;  // [nR] graded index of each z-reduced entry
  int* d_gpadz = nullptr;   // [nG] padded LDS position for the cross tables (-1: unused)
  unsigned char* d_g1 = nullptr;
  short* d_nbr = nullptr;   // [nG][6] compact-table recurrence neighbours
  unsigned char* d_g3 = nullptr;
  unsigned char* d_gord = nullptr;  // [nG] order |g| of each compact table entry
  double *d_fact = nullptr, *d_scale = nullptr, *d_invfact = nullptr;
  // geometry
  int64_t n = 0;
  double* d_xs = nullptr;   // sorted SoA
  int* d_perm = nullptr;
  int* d_leaf_start = nullptr;
  int* d_leaf_count = nullptr;
  int64_t total_leaves = 0;
  std::vector<int> leaf_count_host;  // copy of d_leaf_count (work lists of the batched near field)
  std::vector<Group> groups;
  // evaluate buffers
  double2 *d_q = nullptr, *d_phi = nullptr, *d_phi_near = nullptr;
  // source-side sums of the symmetric near field: [13 slots x G][n] float2 (FP32) or double2 (FP64)
  void* d_part = nullptr;
  // the near field runs on a second stream beside the far field (fork/join by events)
  hipStream_t s2 = nullptr;
  hipEvent_t e_fork = nullptr, e_join = nullptr;
  // with several layer groups their M2L launches run on streams of their own
  hipStream_t sg[MAX_LAYERS] = {};
  hipEvent_t e_gfork = nullptr, e_gjoin[MAX_LAYERS] = {};
  int nrhs_alloc = 0;
  bool ready = false;
  // stats
  tefmm_stats st;
  std::vector<hipEvent_t> ev;  // EV_RING sets of 8 phase events
  int ev_next = 0, ev_count = 0;
  int64_t p2p_pairs = 0, m2l_pairs = 0, p2p_same = 0;
  int64_t sigma_keys = 0, sur_keys = 0;  // Sigma table rows of the geometry / answered by the surrogate
  int64_t som_nodes = 0, som_keys = 0;   // Sigma quadrature: largest node count / rows produced
  // copy of the caller's positions (SoA), kept for re-building the tree (autotuner)
  double* d_xyz_user = nullptr;
  int m2l_ncb = 0;  // M2L tile width override (0 = automatic)
  // where the near field forks from the far field: -1 by precision (FP32 at once, FP64
  // after the upward pass), 0 at once, 1 after the upward pass, 2 not at all (the near
  // field first, then the far field, on the caller's stream); set by the autotuner
  int fork_late = -1;
  tefmm_surrogate* sur = nullptr;  // surrogate for the Sigma tables (borrowed)
  // caller's device allocator (tefmm_set_allocator); null: hipMalloc / hipFree
  tefmm_alloc_fn alloc_fn = nullptr;
  tefmm_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  uint64_t gen = 0; // changes whenever device buffers are (re)allocated
  // graph of the last batched evaluation
  struct Batch {
    std::vector<tefmm_ctx*> hs;
    std::vector<uint64_t> gens;
    std::vector<const double*> q;
    std::vector<double*> phi;
    std::vector<int> nrhs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t origin = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;  // EV_RING sets of 8 phase events
  int ev_next = 0, ev_count = 0;
    // the persistent near-field queue (tefmm_evaluate_batch_queue)
    bool queue = false;
    hipStream_t nf = nullptr;
    hipEvent_t ev_nf = nullptr;   // the queue's near fields done
    hipEvent_t ev_q = nullptr;    // every geometry's charges in tree order
    hipEvent_t ev_ff = nullptr;   // the far-field graph done
    NFQueueGeom* d_geo = nullptr;
    unsigned* d_start = nullptr;  // the work list: pair items, then gather items
    int n_p2p = 0, n_gather = 0;
    unsigned* d_ctr = nullptr;    // ticket, then done[ngeo]
    int* d_err = nullptr;
    int ngeo = 0, qgrid = 0;
    bool f32q = false;
  } batch;
};

static void batch_destroy(tefmm_t h, tefmm_ctx::Batch& b);

// Device memory owned by a handle: from the caller's allocator when one is set
// (tefmm_set_allocator), else hipMalloc / hipFree.  A failed allocation reads as
// hipErrorOutOfMemory (TEFMM_ERR_OOM at the ABI).
template <class T>
static hipError_t dmalloc(tefmm_t h, T** p, size_t bytes) {
  *p = nullptr;
  if (h->alloc_fn) {
    void* v = bytes ? h->alloc_fn(bytes, h->alloc_user) : nullptr;
    if (bytes && !v) return hipErrorOutOfMemory;
    *p = (T*)v;
    return hipSuccess;
  }
  return hipMalloc((void**)p, bytes);
}
template <class T>
static void dfree(tefmm_t h, T*& p) {
  if (p) {
    if (h->free_fn)
      h->free_fn((void*)p, h->alloc_user);
    else
      (void)hipFree((void*)p);
  }
  p = nullptr;
}
static constexpr int EV_RING = 64;  // evaluations whose phase times are kept
static std::atomic<uint64_t> g_generation{1};

static int fail(tefmm_t h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}
#define HIPCHK(h, x)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (x);                                                                        \
    if (e_ != hipSuccess)                                                                       \
      return fail(h, e_ == hipErrorOutOfMemory ? TEFMM_ERR_OOM : TEFMM_ERR_HIP,                 \
                  std::string(#x) + ": " + hipGetErrorString(e_));                              \
  } while (0)

static void free_geometry(tefmm_t h) {
  dfree(h, h->d_xs);
  dfree(h, h->d_perm);
  dfree(h, h->d_leaf_start);
  dfree(h, h->d_leaf_count);
  for (auto& g : h->groups) {
    for (auto& p : g.alpha) dfree(h, p);
    for (auto& p : g.beta) dfree(h, p);
    for (auto& p : g.ared) dfree(h, p);
    for (auto& p : g.ared32) dfree(h, p);
    for (auto& p : g.bred) dfree(h, p);
    for (auto& p : g.azred) dfree(h, p);
    for (auto& p : g.bzred) dfree(h, p);
    for (auto& p : g.xlist_start) dfree(h, p);
    for (auto& p : g.xlist) dfree(h, p);
    for (auto& p : g.XT0) dfree(h, p);
    for (auto& p : g.XT1) dfree(h, p);
    for (auto& p : g.XT032) dfree(h, p);
    for (auto& p : g.XT132) dfree(h, p);
    for (auto& p : g.Tfd) dfree(h, p);
    for (auto& p : g.TS) dfree(h, p);
    for (auto& p : g.Tfd32) dfree(h, p);
    for (auto& p : g.TS32) dfree(h, p);
    dfree(h, g.d_sd_tgt);
    dfree(h, g.d_sd_start);
    dfree(h, g.d_sd_src);
    dfree(h, g.d_sd_img);
    for (auto& p : g.d_occ) dfree(h, p);
    dfree(h, g.d_nf_items);
    dfree(h, g.d_p2p_items);
  }
  h->groups.clear();
  dfree(h, h->d_q);
  dfree(h, h->d_phi);
  dfree(h, h->d_phi_near);
  dfree(h, h->d_part);
  h->nrhs_alloc = 0;
  h->ready = false;
}

// Whether the near field with one charge vector takes the symmetric kernel.
static bool sym_near(const tefmm_options& o) { return o.p2p_targets >= 0; }

static int build_constant_tables(tefmm_t h) {
  const int p = h->opt.p;
  h->nC = mi_count(p);
  h->nR = (p + 1) * (p + 1);
  h->nG = g_count(2 * p);
  h->nKB = (h->nR + 3) / 4;
  h->nRB = (h->nR + 15) / 16;
  int rs = 4 * h->nKB;
  while (rs % 16 != 1) ++rs;
  h->nRs = rs;
  const int nC = h->nC, nR = h->nR, nG = h->nG;
  auto f = [](int n) {
    double r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
  };
  std::vector<int> mi(nC), rmi, rfull;
  std::vector<double> scale(nC), invfact(nC);
  for (int m = 0; m <= p; ++m)
    for (int a = m; a >= 0; --a)
      for (int b = m - a; b >= 0; --b) {
        const int c = m - a - b, i = mi_index(a, b, c);
        mi[i] = a | (b << 8) | (c << 16);
        const double fa = f(a) * f(b) * f(c);
        scale[i] = ((m & 1) ? -1.0 : 1.0) / fa;
        invfact[i] = 1.0 / fa;
      }
  for (int k1 = 0; k1 <= std::min(1, p); ++k1)
    for (int t = 0; t <= p - k1; ++t)
      for (int k3 = 0; k3 <= t; ++k3) {
        const int k2 = t - k3;
        rmi.push_back(k1 | (k2 << 8) | (k3 << 16));
        rfull.push_back(mi_index(k1, k2, k3));
      }
  if ((int)rmi.size() != nR) return fail(h, TEFMM_ERR_STATE, "reduced index set size");
  std::vector<int> rzmi, rzfull;
  for (int k3 = 0; k3 <= std::min(1, p); ++k3)
    for (int t = 0; t <= p - k3; ++t)
      for (int k1 = t; k1 >= 0; --k1) {
        const int k2 = t - k1;
        rzmi.push_back(k1 | (k2 << 8) | (k3 << 16));
        rzfull.push_back(mi_index(k1, k2, k3));
      }
  if ((int)rzmi.size() != nR) return fail(h, TEFMM_ERR_STATE, "z-reduced index set size");
  std::vector<short> nbr(6 * nG, -1);
  std::vector<int> gpad(nG), gpadz(nG, -1);
  std::vector<unsigned char> g3(nG), g1v(nG);
  std::vector<double> fact(nG);
  int cnt = 0;
  for (int n = 0; n <= 2 * p; ++n)
    for (int g1 = 0; g1 <= std::min(2, n); ++g1)
      for (int c = 0; c <= n - g1; ++c) {
        const int b = n - g1 - c, i = g_index(g1, b, c);
        if (i != cnt++) return fail(h, TEFMM_ERR_STATE, "compact table order");
        g3[i] = (unsigned char)c;
        gpad[i] = (g1 * (2 * p + 1) + (b + c)) * (2 * p + 1) + c;
        g1v[i] = (unsigned char)g1;
        if (g1 <= 1) gpadz[i] = (g1 * (2 * p + 1) + (b + c)) * (2 * p + 1) + c;
        fact[i] = f(g1) * f(b) * f(c);
        if (g1 >= 1) nbr[6 * i + 0] = (short)g_index(g1 - 1, b, c);
        if (b >= 1) nbr[6 * i + 1] = (short)g_index(g1, b - 1, c);
        if (c >= 1) nbr[6 * i + 2] = (short)g_index(g1, b, c - 1);
        if (g1 >= 2) nbr[6 * i + 3] = (short)g_index(g1 - 2, b, c);
        if (b >= 2) nbr[6 * i + 4] = (short)g_index(g1, b - 2, c);
        if (c >= 2) nbr[6 * i + 5] = (short)g_index(g1, b, c - 2);
      }
  if (cnt != nG) return fail(h, TEFMM_ERR_STATE, "compact table size");
  HIPCHK(h, dmalloc(h, &h->d_mi, sizeof(int) * nC));
  HIPCHK(h, dmalloc(h, &h->d_rmi, sizeof(int) * nR));
  HIPCHK(h, dmalloc(h, &h->d_rfull, sizeof(int) * nR));
  HIPCHK(h, dmalloc(h, &h->d_nbr, sizeof(short) * 6 * nG));
  HIPCHK(h, dmalloc(h, &h->d_gpad, sizeof(int) * nG));
  HIPCHK(h, dmalloc(h, &h->d_gpadz, sizeof(int) * nG));
  HIPCHK(h, hipMemcpy(h->d_gpadz, gpadz.data(), sizeof(int) * nG, hipMemcpyHostToDevice));
  HIPCHK(h, dmalloc(h, &h->d_g1, nG));
  HIPCHK(h, hipMemcpy(h->d_g1, g1v.data(), nG, hipMemcpyHostToDevice));
  HIPCHK(h, dmalloc(h, &h->d_rzmi, sizeof(int) * nR));
  HIPCHK(h, hipMemcpy(h->d_rzmi, rzmi.data(), sizeof(int) * nR, hipMemcpyHostToDevice));
  HIPCHK(h, dmalloc(h, &h->d_rzfull, sizeof(int) * nR));
  HIPCHK(h, hipMemcpy(h->d_rzfull, rzfull.data(), sizeof(int) * nR, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->d_gpad, gpad.data(), sizeof(int) * nG, hipMemcpyHostToDevice));
  HIPCHK(h, dmalloc(h, &h->d_g3, nG));
  HIPCHK(h, dmalloc(h, &h->d_fact, sizeof(double) * nG));
  HIPCHK(h, dmalloc(h, &h->d_scale, sizeof(double) * nC));
  HIPCHK(h, dmalloc(h, &h->d_invfact, sizeof(double) * nC));
  HIPCHK(h, hipMemcpy(h->d_mi, mi.data(), sizeof(int) * nC, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->d_rmi, rmi.data(), sizeof(int) * nR, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->d_rfull, rfull.data(), sizeof(int) * nR, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->d_nbr, nbr.data(), sizeof(short) * 6 * nG, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->d_g3, g3.data(), nG, hipMemcpyHostToDevice));
  {
    std::vector<unsigned char> gord(nG);
    for (int n = 0; n <= 2 * h->opt.p; ++n)
      for (int i = g_offset(n); i < g_offset(n + 1) && i < nG; ++i) gord[i] = (unsigned char)n;
    HIPCHK(h, dmalloc(h, &h->d_gord, nG));
    HIPCHK(h, hipMemcpy(h->d_gord, gord.data(), nG, hipMemcpyHostToDevice));
  }
  HIPCHK(h, hipMemcpy(h->d_fact, fact.data(), sizeof(double) * nG, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->d_scale, scale.data(), sizeof(double) * nC, hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->d_invfact, invfact.data(), sizeof(double) * nC, hipMemcpyHostToDevice));
  upload_binomials();
  return TEFMM_OK;
}

extern "C" int tefmm_create(tefmm_t* out, const tefmm_medium* medium, const tefmm_options* opt) {
  if (!out) return TEFMM_ERR_INVALID_ARG;
  *out = nullptr;
  tefmm_ctx* h = new tefmm_ctx();
  std::string err;
  if (!medium_from_desc(medium, h->med, err)) {
    delete h;
    return TEFMM_ERR_INVALID_ARG;
  }
  if (opt)
    h->opt = *opt;
  else
    tefmm_default_options(&h->opt);
  const tefmm_options& o = h->opt;
  if (o.p < 1 || o.p > 16 || o.depth < 0 || o.depth > 7 || o.max_leaf < 1 ||
      (o.precision != TEFMM_FP64 && o.precision != TEFMM_MIXED_FP32) ||
      (o.normalization != TEFMM_NORM_PHYSICAL && o.normalization != TEFMM_NORM_PAPER) || o.dcim_samples < 8 ||
      !(o.dcim_T1 > 0) || !(o.dcim_T1_cross > 0) || !(o.dcim_svd_tol > 0) || o.m2l_tile < 0 || o.m2l_tile > 2 ||
      !(o.interface_eps >= 0) || o.n_rhs_max < 1 ||
      !(o.p2p_targets == -1 || o.p2p_targets == 0 || o.p2p_targets == 1 || o.p2p_targets == 2 ||
        o.p2p_targets == 4) ||
      (o.precision == TEFMM_FP64 && o.p2p_targets == 4) || !(o.p2p_poly == 0 || o.p2p_poly == -1) ||
      !(o.sigma_tables == TEFMM_SIGMA_IMAGES || o.sigma_tables == TEFMM_SIGMA_SOMMERFELD)) {
    delete h;
    return TEFMM_ERR_INVALID_ARG;
  }
  std::memset(&h->st, 0, sizeof(h->st));
  int rc = build_constant_tables(h);
  if (rc != TEFMM_OK) {
    tefmm_destroy(h);
    return rc;
  }
  *out = h;
  return TEFMM_OK;
}

static void free_constant_tables(tefmm_t h) {
  dfree(h, h->d_mi);
  dfree(h, h->d_rmi);
  dfree(h, h->d_rfull);
  dfree(h, h->d_gpad);
  dfree(h, h->d_gpadz);
  dfree(h, h->d_g1);
  dfree(h, h->d_rzmi);
  dfree(h, h->d_rzfull);
  dfree(h, h->d_nbr);
  dfree(h, h->d_g3);
  dfree(h, h->d_gord);
  dfree(h, h->d_fact);
  dfree(h, h->d_scale);
  dfree(h, h->d_invfact);
}

extern "C" int tefmm_set_allocator(tefmm_t h, tefmm_alloc_fn alloc, tefmm_free_fn free_fn, void* user) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(h, TEFMM_ERR_INVALID_ARG, "tefmm_set_allocator: give both functions or neither");
  // everything the handle holds is released with the allocator that gave it, then the
  // constant tables are uploaded again into memory from the new one
  batch_destroy(h, h->batch);
  free_geometry(h);
  dfree(h, h->d_xyz_user);
  free_constant_tables(h);
  h->alloc_fn = alloc, h->free_fn = free_fn, h->alloc_user = user;
  h->gen = g_generation++;
  return build_constant_tables(h);
}

extern "C" void tefmm_destroy(tefmm_t h) {
  if (!h) return;
  free_geometry(h);
  free_constant_tables(h);
  for (auto& e : h->ev) (void)hipEventDestroy(e);
  if (h->e_fork) (void)hipEventDestroy(h->e_fork);
  if (h->e_join) (void)hipEventDestroy(h->e_join);
  if (h->s2) (void)hipStreamDestroy(h->s2);
  if (h->e_gfork) (void)hipEventDestroy(h->e_gfork);
  for (int i = 0; i < MAX_LAYERS; ++i) {
    if (h->e_gjoin[i]) (void)hipEventDestroy(h->e_gjoin[i]);
    if (h->sg[i]) (void)hipStreamDestroy(h->sg[i]);
  }
  batch_destroy(h, h->batch);
  dfree(h, h->d_xyz_user);
  delete h;
}

extern "C" const char* tefmm_last_error(tefmm_t h) { return h ? h->err.c_str() : "null handle"; }

struct SigmaKeys {
  std::vector<int> key;                // table row
  std::vector<double> X, Y, S, Re;     // key geometry and envelope distance
};
static int surrogate_tables(tefmm_t h, const SigmaKeys& sk, double hb, double2* d_out, hipStream_t s);
static bool surrogate_accepts(const tefmm_surrogate* su, double X, double Y, double S);
static bool surrogate_applies(const tefmm_surrogate* su, int layer, bool up, bool dn);
static bool surrogate_serves_leaves(const tefmm_surrogate* su);
static void sigma_mirror_dist(const MediumDesc& med, int l, bool up, bool dn, double X, double Y, double S,
                              std::vector<double>& out);

// ---------------------------------------------------------------------------
// Sigma-family tables from the Sommerfeld integrals (Sec. 4.2).  The path is the
// paper's: Gamma1 from 0 to -ib, Gamma2 from -ib to t_max - ib (b = 1), with
// composite 16-point Gauss-Legendre panels.  Along Gamma2 the integrand of H_{m,c}
// is at most of size t^(2 P2 + 1) e^{-t zeta_min} (zeta_min: the least mirror
// distance of the keys served), so the path ends where that bound falls to 1e-18 of
// its peak (at most t = 8000); Gamma2 panels are at most min(2, pi / rho_max) wide
// (J_m(k_rho rho) oscillates with period 2 pi / rho).  Per node the host solves the
// interface system for the densities and keeps cu, cd = w i (sigma - sigma_inf) / k_z
// of the up- and down-going families; sigma_inf (the density at k_rho = 1e8 k) is the
// weight of the image at each mirror point, which k_sigma_h adds exactly.
// ---------------------------------------------------------------------------
static const double SOM_B = 1.0;
static const double SOM_T_CAP = 8000.0;
struct SomPath {
  std::vector<cplx> krho, kz, cu, cd;
  cplx sinf_u = 0.0, sinf_d = 0.0;
};

// delta: the Delta family of the layer instead, sigma^{ud} e^{i k_z (D + w)} + sigma^{du}
// e^{i k_z (D - w)} (w = z - z', D the layer's thickness), whose densities vanish as
// k_rho grows (no mirror-point image); cu, cd then hold sigma^{ud} and sigma^{du}.
// The nodes and weights of the contour (see above) for derivative orders up to P2 and the
// least vertical distance zeta_min of the keys served.
static void som_nodes(const MediumDesc& med, double zeta_min, double rho_max, int P2, std::vector<cplx>& krho,
                      std::vector<cplx>& wts) {
  const int ORD = 16;
  std::vector<double> gx, gw;
  gauss_legendre01(ORD, gx, gw);
  const double q = 2.0 * P2 + 1.0, Z = std::max(zeta_min, 1e-3);
  const double tpk = std::max(q / Z, 1.0);
  double t_max = tpk;
  while (t_max < SOM_T_CAP && q * std::log(t_max / tpk) - Z * (t_max - tpk) > -41.5) t_max *= 1.05;
  double kmax = 0;
  for (double kk : med.k) kmax = std::max(kmax, kk);
  t_max = std::max(std::min(t_max, SOM_T_CAP), kmax + 4.0);
  const double wmax = std::min(2.0, 3.14159265358979324 / std::max(rho_max, 1e-12));
  const int npan = (int)std::ceil(t_max / wmax);
  const double wp = t_max / npan;
  krho.clear(), wts.clear();
  for (int j = 0; j < ORD; ++j) krho.push_back(cplx(0.0, -SOM_B * gx[j])), wts.push_back(cplx(0.0, -SOM_B * gw[j]));
  for (int pn = 0; pn < npan; ++pn)
    for (int j = 0; j < ORD; ++j) krho.push_back(cplx((pn + gx[j]) * wp, -SOM_B)), wts.push_back(wp * gw[j]);
}

static void sommerfeld_path(const MediumDesc& med, int l, bool up, bool dn, double zeta_min, double rho_max, int P2,
                            SomPath& P, bool delta = false) {
  std::vector<cplx> wts;
  som_nodes(med, zeta_min, rho_max, P2, P.krho, wts);
  P.kz.clear(), P.cu.clear(), P.cd.clear();
  std::vector<cplx> sig;
  const int iu = delta ? 1 : 0, id = delta ? 2 : 3;  // densities: uu, ud, du, dd
  reaction_densities(med, l, cplx(1e8 * med.k[l], 0.0), sig);
  P.sinf_u = up && !delta ? sig[l * 4 + iu] : cplx(0.0);
  P.sinf_d = dn && !delta ? sig[l * 4 + id] : cplx(0.0);
  const cplx I(0.0, 1.0);
  for (size_t t = 0; t < P.krho.size(); ++t) {
    reaction_densities(med, l, P.krho[t], sig);
    const cplx kz = vertical_wavenumber(med.k[l], P.krho[t]);
    P.kz.push_back(kz);
    P.cu.push_back(up ? wts[t] * I * (sig[l * 4 + iu] - P.sinf_u) / kz : cplx(0.0));
    P.cd.push_back(dn ? wts[t] * I * (sig[l * 4 + id] - P.sinf_d) / kz : cplx(0.0));
  }
}

// Offsets of the two vertical distances: zeta_u = S - two_dl, zeta_d = two_dt - S.  The
// Sigma families: S = z + z' against the mirror planes 2 d_l and 2 d_{l-1}; the Delta
// family: S = w = z - z', zeta = D + w and D - w.
static void som_offsets(const MediumDesc& med, int l, bool delta, double* two_dl, double* two_dt) {
  if (delta) {
    const double D = med.thickness(l);
    *two_dl = -D, *two_dt = D;
    return;
  }
  *two_dl = l < med.L ? 2 * med.d[l] : 0.0;
  *two_dt = l > 0 ? 2 * med.d[l - 1] : 0.0;
}

// H (one row per pair) of the Sigma families (or, delta, the Delta family) of layer l at
// the pairs (rho[pr[i]], S[ps[i]]): the mirror-point images by k_sigma_h (none for Delta),
// then the node contraction added to them.
static int sommerfeld_h(tefmm_t h, int l, bool up, bool dn, const SomPath& P, int P2, const std::vector<double>& rho,
                        const std::vector<double>& S, const std::vector<int>& pr, const std::vector<int>& ps,
                        double2* d_H, hipStream_t s, bool delta = false, const double* offs = nullptr) {
  const MediumDesc& med = h->med;
  const int nn = (int)P.krho.size(), np = (int)pr.size(), nr = (int)rho.size(), nsv = (int)S.size(), M = P2;
  if (!np) return TEFMM_OK;
  double two_dl, two_dt;
  som_offsets(med, l, delta, &two_dl, &two_dt);
  if (offs) two_dl = offs[0], two_dt = offs[1];  // explicit vertical offsets (cross-layer terms)
  auto pack = [](const std::vector<cplx>& v) {
    std::vector<double2> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = make_double2(v[i].real(), v[i].imag());
    return o;
  };
  const std::vector<double2> hk = pack(P.krho), hz = pack(P.kz), hu = pack(P.cu), hd = pack(P.cd);
  std::vector<double2> qs;
  int nup = 0, ndn = 0;
  if (up && P.sinf_u != 0.0) qs.push_back(make_double2(P.sinf_u.real(), P.sinf_u.imag())), qs.push_back({0, 0}), nup = 1;
  if (dn && P.sinf_d != 0.0) qs.push_back(make_double2(P.sinf_d.real(), P.sinf_d.imag())), qs.push_back({0, 0}), ndn = 1;
  std::vector<double> w(np), Sp(np);
  for (int i = 0; i < np; ++i) w[i] = rho[pr[i]] * rho[pr[i]], Sp[i] = S[ps[i]];
  double2 *d_k = nullptr, *d_z = nullptr, *d_u = nullptr, *d_d = nullptr, *d_qs = nullptr, *d_A = nullptr, *d_B = nullptr;
  double *d_rho = nullptr, *d_S = nullptr, *d_w = nullptr, *d_Sp = nullptr;
  int *d_pr = nullptr, *d_ps = nullptr;
  int rc = TEFMM_OK;
  auto run = [&]() -> int {
    HIPCHK(h, dmalloc(h, &d_k, sizeof(double2) * nn));
    HIPCHK(h, dmalloc(h, &d_z, sizeof(double2) * nn));
    HIPCHK(h, dmalloc(h, &d_u, sizeof(double2) * nn));
    HIPCHK(h, dmalloc(h, &d_d, sizeof(double2) * nn));
    HIPCHK(h, dmalloc(h, &d_qs, sizeof(double2) * std::max<size_t>(qs.size(), 1)));
    HIPCHK(h, dmalloc(h, &d_A, sizeof(double2) * (size_t)nr * (M + 1) * nn));
    HIPCHK(h, dmalloc(h, &d_B, sizeof(double2) * (size_t)nsv * (M + 1) * nn));
    HIPCHK(h, dmalloc(h, &d_rho, sizeof(double) * nr));
    HIPCHK(h, dmalloc(h, &d_S, sizeof(double) * nsv));
    HIPCHK(h, dmalloc(h, &d_w, sizeof(double) * np));
    HIPCHK(h, dmalloc(h, &d_Sp, sizeof(double) * np));
    HIPCHK(h, dmalloc(h, &d_pr, sizeof(int) * np));
    HIPCHK(h, dmalloc(h, &d_ps, sizeof(int) * np));
    HIPCHK(h, hipMemcpyAsync(d_k, hk.data(), sizeof(double2) * nn, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_z, hz.data(), sizeof(double2) * nn, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_u, hu.data(), sizeof(double2) * nn, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_d, hd.data(), sizeof(double2) * nn, hipMemcpyHostToDevice, s));
    if (!qs.empty())
      HIPCHK(h, hipMemcpyAsync(d_qs, qs.data(), sizeof(double2) * qs.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_rho, rho.data(), sizeof(double) * nr, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_S, S.data(), sizeof(double) * nsv, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_w, w.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_Sp, Sp.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_pr, pr.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_ps, ps.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sigma_h, dim3(np), dim3(64), 0, s, d_w, d_Sp, np, d_qs, nup, ndn, two_dl, two_dt, med.k[l],
                       P2, d_H);
    HIPCHK(h, hipGetLastError());
    hipLaunchKernelGGL(k_som_radial, dim3((nn + 63) / 64, nr), dim3(64), 0, s, d_k, nn, d_rho, M, d_A);
    HIPCHK(h, hipGetLastError());
    hipLaunchKernelGGL(k_som_vertical, dim3((nn + 63) / 64, nsv), dim3(64), 0, s, d_z, d_u, d_d, nn, d_S, two_dl,
                       two_dt, up ? 1 : 0, dn ? 1 : 0, 0.0, M, d_B);
    HIPCHK(h, hipGetLastError());
    const size_t lds = 2 * sizeof(double2) * (M + 1) * 65;
    HIPCHK(h, hipFuncSetAttribute((const void*)k_som_contract, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_som_contract, dim3(np), dim3(256), lds, s, d_A, d_B, nn, M, d_pr, d_ps, d_H);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(s));
    return TEFMM_OK;
  };
  rc = run();
  dfree(h, d_k), dfree(h, d_z), dfree(h, d_u), dfree(h, d_d), dfree(h, d_qs), dfree(h, d_A), dfree(h, d_B);
  dfree(h, d_rho), dfree(h, d_S), dfree(h, d_w), dfree(h, d_Sp), dfree(h, d_pr), dfree(h, d_ps);
  return rc;
}

// Rows sk.key of d_out (level box size hb) from the Sommerfeld H, computed once per
// distinct (rho, S) of the keys and rebuilt into the compact Cartesian layout.  delta:
// the Delta family at (rho, w = sk.S), added to the rows (which hold the free-space part).
static int sommerfeld_tables(tefmm_t h, const Group& g, const SomPath& P, const SigmaKeys& sk, double hb,
                             double2* d_out, hipStream_t s, bool delta = false) {
  const int nk = (int)sk.key.size(), P2 = 2 * h->opt.p, nH = (P2 + 1) * (P2 + 2) / 2;
  std::map<double, int> rmap, smap;
  std::map<std::pair<int, int>, int> pmap;
  std::vector<double> rho, S;
  std::vector<int> pr, ps, hrow(nk);
  for (int i = 0; i < nk; ++i) {
    const double r2 = sk.X[i] * sk.X[i] + sk.Y[i] * sk.Y[i];
    auto ri = rmap.emplace(r2, (int)rho.size());
    if (ri.second) rho.push_back(std::sqrt(r2));
    auto si = smap.emplace(sk.S[i], (int)S.size());
    if (si.second) S.push_back(sk.S[i]);
    auto pi = pmap.emplace(std::make_pair(ri.first->second, si.first->second), (int)pr.size());
    if (pi.second) pr.push_back(ri.first->second), ps.push_back(si.first->second);
    hrow[i] = pi.first->second;
  }
  double2* d_H = nullptr;
  double *d_x = nullptr, *d_y = nullptr;
  int *d_key = nullptr, *d_hrow = nullptr;
  auto run = [&]() -> int {
    HIPCHK(h, dmalloc(h, &d_H, sizeof(double2) * pr.size() * nH));
    const int rc = delta ? sommerfeld_h(h, g.layer, true, true, P, P2, rho, S, pr, ps, d_H, s, true)
                         : sommerfeld_h(h, g.layer, g.has[0], g.has[1], P, P2, rho, S, pr, ps, d_H, s);
    if (rc != TEFMM_OK) return rc;
    HIPCHK(h, dmalloc(h, &d_x, sizeof(double) * nk));
    HIPCHK(h, dmalloc(h, &d_y, sizeof(double) * nk));
    HIPCHK(h, dmalloc(h, &d_key, sizeof(int) * nk));
    HIPCHK(h, dmalloc(h, &d_hrow, sizeof(int) * nk));
    HIPCHK(h, hipMemcpyAsync(d_x, sk.X.data(), sizeof(double) * nk, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_y, sk.Y.data(), sizeof(double) * nk, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_key, sk.key.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_hrow, hrow.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sigma_restore, dim3(nk), dim3(64), 0, s, d_H, d_x, d_y, nk, d_key, hb, h->med.k[g.layer], P2,
                       h->nG, h->d_g1, h->d_g3, h->d_gord, d_out, d_hrow, delta ? 1 : 0);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(s));
    return TEFMM_OK;
  };
  const int rc = run();
  dfree(h, d_H), dfree(h, d_x), dfree(h, d_y), dfree(h, d_key), dfree(h, d_hrow);
  return rc;
}

// ---------------------------------------------------------------------------
// Derivative tables of one group (all levels).
// ---------------------------------------------------------------------------
// k_table_gen with as many waves per key (1, 2, 4 or 8) as fit 150 KiB of LDS
// (two arrays of nG complex values per wave)
static hipError_t launch_table_gen(const TableGenArgs& ta, int nkeys, hipStream_t s) {
  const size_t per = 2 * sizeof(double2) * (size_t)ta.nG;
  int nw = 8;
  while (nw > 1 && nw * per > 150 * 1024) nw /= 2;
  void (*fn)(TableGenArgs) = nw == 8 ? k_table_gen<8> : nw == 4 ? k_table_gen<4> : nw == 2 ? k_table_gen<2> : k_table_gen<1>;
  const size_t lds = nw * per;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(nkeys), dim3(64 * nw), lds, s, ta);
  return hipGetLastError();
}

// FP32 copy (the mixed mode's tables) of cnt complex values, from the handle's allocator
static int tables_to_f32(tefmm_t h, const double2* d, size_t cnt, float2** out, hipStream_t s) {
  HIPCHK(h, dmalloc(h, out, sizeof(float2) * std::max<size_t>(cnt, 1)));
  if (cnt) {
    const int blocks = (int)std::min<size_t>((cnt + 255) / 256, 4096);
    hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, s, d, cnt, *out);
    HIPCHK(h, hipGetLastError());
  }
  return TEFMM_OK;
}

static int build_tables(tefmm_t h, Group& g, hipStream_t s) {
  const MediumDesc& med = h->med;
  const int l_ = g.layer;
  const double D = (l_ > 0 && l_ < med.L) ? med.thickness(l_) : 0.0;
  const double k = med.k[l_];
  g.Tfd.assign(g.depth + 1, nullptr);
  g.TS.assign(g.depth + 1, nullptr);
  g.Tfd32.assign(g.depth + 1, nullptr);
  g.TS32.assign(g.depth + 1, nullptr);
  const bool has_sigma = g.has[0] || g.has[1];
  // Sigma rows from the Sommerfeld integrals: one contour for all levels, ending where
  // the least mirror distance of the keys served needs it
  SomPath som;
  const bool som_on = has_sigma && h->opt.sigma_tables == TEFMM_SIGMA_SOMMERFELD;
  if (som_on) {
    if (2 * h->opt.p > SIGMA_P2_MAX)
      return fail(h, TEFMM_ERR_UNSUPPORTED, "Sommerfeld Sigma tables need 2p <= " + std::to_string(SIGMA_P2_MAX));
    double zmin = 1e300;
    for (int lev = 2; lev <= g.depth; ++lev) {
      const int nb = 1 << lev, nm = 2 * nb - 1;
      const double hb = g.side / nb;
      for (int m = 0; m < nm; ++m) {
        if (lev == g.depth && !g.sig_flag.empty()) {
          bool all = true;  // every key of this S evaluated directly
          for (int c = 0; c < 49 && all; ++c) all = g.sig_flag[(size_t)c * nm + m] != 0;
          if (all) continue;
        }
        const double S = 2 * g.lo[2] + (m + 1) * hb;
        if (g.has[0] && S - 2 * med.d[l_] > 0) zmin = std::min(zmin, S - 2 * med.d[l_]);
        if (g.has[1] && 2 * med.d[l_ - 1] - S > 0) zmin = std::min(zmin, 2 * med.d[l_ - 1] - S);
      }
    }
    sommerfeld_path(med, l_, g.has[0], g.has[1], zmin, 3.0 * std::sqrt(2.0) * g.side / 4, 2 * h->opt.p, som);
    h->som_nodes = std::max<int64_t>(h->som_nodes, (int64_t)som.krho.size());
  }
  // Delta rows from the Sommerfeld integrals too (functions of rho and w = z - z'); keys
  // whose centres are a layer's thickness apart or more join a box outside the layer and
  // are left out, as in the image route
  SomPath somd;
  const bool som_delta = g.has[2] && h->opt.sigma_tables == TEFMM_SIGMA_SOMMERFELD;
  if (som_delta) {
    if (2 * h->opt.p > SIGMA_P2_MAX)
      return fail(h, TEFMM_ERR_UNSUPPORTED, "Sommerfeld Delta tables need 2p <= " + std::to_string(SIGMA_P2_MAX));
    double zmin = 1e300;
    for (int lev = 2; lev <= g.depth; ++lev)
      for (int dz = 0; dz <= 3; ++dz) {
        const double zd = D - dz * g.side / (1 << lev);
        if (zd > 1e-9) zmin = std::min(zmin, zd);
      }
    sommerfeld_path(med, l_, true, true, zmin, 3.0 * std::sqrt(2.0) * g.side / 4, 2 * h->opt.p, somd, true);
    h->som_nodes = std::max<int64_t>(h->som_nodes, (int64_t)somd.krho.size());
  }
  for (int lev = 2; lev <= g.depth; ++lev) {
    const int nb = 1 << lev;
    const double hb = g.side / nb;
    const bool leaf = lev == g.depth;
    for (int which = 0; which < 2; ++which) {
      if (which == 1 && !has_sigma) continue;
      std::vector<TableTerm> terms;
      std::vector<int> start;
      std::vector<double> hk;
      SigmaKeys sk, sq;  // rows answered by the surrogate / by the Sommerfeld integrals
      int nkeys;
      auto push = [&](double x, double y, cplx zeta, cplx coef, int flip, bool image) {
        // an image term is valid only for Re(zeta) > 0; keys failing this join
        // boxes outside the layer (empty, zero moments) and are left out
        if (image && zeta.real() <= 1e-9) return;
        TableTerm t;
        t.x = x, t.y = y, t.zr = zeta.real(), t.zi = zeta.imag(), t.cr = coef.real(), t.ci = coef.imag();
        t.flip = flip, t.pad = 0;
        terms.push_back(t);
      };
      if (which == 0) {
        nkeys = 343;
        for (int dx = -3; dx <= 3; ++dx)
          for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz) {
              start.push_back((int)terms.size());
              hk.push_back(hb);
              const bool nearb = std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) <= 1;
              // the key (dx, dy, dz) is the source offset; the kernel is evaluated at the
              // centre displacement target - source = -(dx, dy, dz) h
              if (!nearb) push(-dx, -dy, cplx(-dz, 0), cplx(1, 0), 0, false);
              if (g.has[2] && (!nearb || leaf) && som_delta) {
                const double w = -dz * hb;
                if (D - std::fabs(w) > 1e-9) {
                  sq.key.push_back((int)start.size() - 1);
                  sq.X.push_back(-dx * hb), sq.Y.push_back(-dy * hb), sq.S.push_back(w);
                }
              } else if (g.has[2] && (!nearb || leaf)) {
                // w = z_t - z_s = -dz h enters as D + w (flip 0) and D - w (flip 1)
                for (size_t j = 0; j < g.famA[2].size(); ++j) {
                  const cplx A = g.famA[2][j], Z = g.famZ[2][j];
                  push(-dx, -dy, (D - dz * hb - Z) / hb, A, 0, true);
                  push(-dx, -dy, (D + dz * hb - Z) / hb, A, 1, true);
                }
              }
            }
      } else {
        nkeys = 49 * (2 * nb - 1);
        const bool use_sur = h->sur && surrogate_applies(h->sur, l_, g.has[0], g.has[1]) &&
                             (!leaf || surrogate_serves_leaves(h->sur));
        for (int dx = -3; dx <= 3; ++dx)
          for (int dy = -3; dy <= 3; ++dy)
            for (int m = 0; m <= 2 * nb - 2; ++m) {
              start.push_back((int)terms.size());
              hk.push_back(hb);
              const double S = 2 * g.lo[2] + (m + 1) * hb;
              // evaluated directly (k_sigma_direct): the row stays zero
              if (leaf && !g.sig_flag.empty() && g.sig_flag[start.size() - 1]) continue;
              if (use_sur && surrogate_accepts(h->sur, -dx * hb, -dy * hb, S)) {
                // answered by the network after the image tables are generated
                sk.key.push_back((int)start.size() - 1);
                sk.X.push_back(-dx * hb), sk.Y.push_back(-dy * hb), sk.S.push_back(S);
                sigma_mirror_dist(med, l_, g.has[0], g.has[1], -dx * hb, -dy * hb, S, sk.Re);
                continue;
              }
              if (som_on) {
                sq.key.push_back((int)start.size() - 1);
                sq.X.push_back(-dx * hb), sq.Y.push_back(-dy * hb), sq.S.push_back(S);
                continue;
              }
              if (g.has[0])
                for (size_t j = 0; j < g.famA[0].size(); ++j)
                  push(-dx, -dy, (S - 2 * med.d[l_] - g.famZ[0][j]) / hb, g.famA[0][j], 0, true);
              if (g.has[1])
                for (size_t j = 0; j < g.famA[1].size(); ++j)
                  push(-dx, -dy, (2 * med.d[l_ - 1] - S - g.famZ[1][j]) / hb, g.famA[1][j], 1, true);
            }
      }
      start.push_back((int)terms.size());
      TableTerm* d_terms = nullptr;
      int* d_start = nullptr;
      double* d_h = nullptr;
      double2* d_out = nullptr;
      HIPCHK(h, dmalloc(h, &d_terms, sizeof(TableTerm) * std::max<size_t>(terms.size(), 1)));
      HIPCHK(h, dmalloc(h, &d_start, sizeof(int) * start.size()));
      HIPCHK(h, dmalloc(h, &d_h, sizeof(double) * hk.size()));
      HIPCHK(h, dmalloc(h, &d_out, sizeof(double2) * (size_t)nkeys * h->nG));
      if (!terms.empty())
        HIPCHK(h, hipMemcpyAsync(d_terms, terms.data(), sizeof(TableTerm) * terms.size(), hipMemcpyHostToDevice, s));
      HIPCHK(h, hipMemcpyAsync(d_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice, s));
      HIPCHK(h, hipMemcpyAsync(d_h, hk.data(), sizeof(double) * hk.size(), hipMemcpyHostToDevice, s));
      TableGenArgs ta;
      ta.terms = d_terms, ta.term_start = d_start, ta.h = d_h, ta.k = k, ta.order = 2 * h->opt.p, ta.nG = h->nG;
      ta.nbr = h->d_nbr, ta.g3 = h->d_g3, ta.g1 = h->d_g1, ta.swap13 = 0, ta.fact = h->d_fact, ta.out = d_out;
      HIPCHK(h, launch_table_gen(ta, nkeys, s));
      HIPCHK(h, hipStreamSynchronize(s));
      dfree(h, d_terms);
      dfree(h, d_start);
      dfree(h, d_h);
      if (!sk.key.empty()) {
        int rc = surrogate_tables(h, sk, hb, d_out, s);
        if (rc != TEFMM_OK) {
          dfree(h, d_out);
          return rc;
        }
        h->sur_keys += (int64_t)sk.key.size();
      }
      if (!sq.key.empty()) {
        int rc = sommerfeld_tables(h, g, which == 0 ? somd : som, sq, hb, d_out, s, which == 0);
        if (rc != TEFMM_OK) {
          dfree(h, d_out);
          return rc;
        }
        h->som_keys += (int64_t)sq.key.size();
      }
      if (which == 1) h->sigma_keys += nkeys;
      if (which == 0)
        g.Tfd[lev] = d_out;
      else
        g.TS[lev] = d_out;
      if (h->opt.precision == TEFMM_MIXED_FP32) {
        float2* d32 = nullptr;
        const int rc = tables_to_f32(h, d_out, (size_t)nkeys * h->nG, &d32, s);
        if (rc != TEFMM_OK) return rc;
        if (which == 0)
          g.Tfd32[lev] = d32;
        else
          g.TS32[lev] = d32;
      }
    }
  }
  return TEFMM_OK;
}

// Near-field work list (items in leaf order, work per item) cut into 8 contiguous
// segments of about equal work, one per XCD, the longest items first within a segment
// (stable), so that the last workgroups dealt out are short.
static void cut_xcd_segments(std::vector<unsigned>& items, const std::vector<double>& work, XcdSegs& seg,
                             int& seg_max) {
  double tot = 0;
  for (double w : work) tot += w;
  int x = 0;
  double run = 0;
  seg.start[0] = 0;
  for (size_t i = 0; i < work.size() && x < 7; ++i) {
    run += work[i];
    while (x < 7 && run >= tot * (x + 1) / 8.0) seg.start[++x] = (int)i + 1;
  }
  while (x < 8) seg.start[++x] = (int)work.size();
  seg_max = 0;
  for (int s8 = 0; s8 < 8; ++s8) seg_max = std::max(seg_max, seg.start[s8 + 1] - seg.start[s8]);
  for (int s8 = 0; s8 < 8; ++s8) {
    const int b = seg.start[s8], e = seg.start[s8 + 1];
    std::vector<int> ord(e - b);
    for (int i = 0; i < e - b; ++i) ord[i] = b + i;
    std::stable_sort(ord.begin(), ord.end(), [&](int u, int v) { return work[u] > work[v]; });
    std::vector<unsigned> sg(e - b);
    for (int i = 0; i < e - b; ++i) sg[i] = items[ord[i]];
    std::copy(sg.begin(), sg.end(), items.begin() + b);
  }
}

// ---------------------------------------------------------------------------
// Cross-layer interaction lists, complex images and tables of target group gt.
// A pair of boxes (target in gt, source in another group) at level l is
// translated at l if it passes the acceptance test sqrt(3) h <= theta |c_t - c_s|
// and its parent pair failed it (or l = 2), or if l is the leaf level.  The
// test is monotone under refinement for theta <= 1, so every leaf pair is
// translated exactly once.  Lists depend only on the target's x/y parity and
// z index (common x-y grid), keys on (source group, dx, dy, iz_t, iz_s).
// ---------------------------------------------------------------------------
static const double CROSS_THETA = 0.6;

// ---------------------------------------------------------------------------
// Cross-layer rows from the Sommerfeld integrals (Sec. 4.2).  For a target in layer l and
// a source in layer l' the kernel is
//   K = i int k_rho J0(k_rho rho) / k_z sum_{a,b} P_a(z) sigma^{ab}_{l l'} E_b(z') dk_rho
// (k_z of the target layer; P_u = e^{i k_z (z - d_l)}, P_d = e^{i k_z (d_{l-1} - z)}; E_u,
// E_d the source layer's waves at z').  For one source height it is the Sigma form in the
// target's z, with the vertical distances z - d_l and d_{l-1} - z and the node coefficients
//   cu, cd = w i / k_z sum_b sigma^{ab} (+-i k'_z)^{k3} E_b(z') (-h)^{k3}   (a = u, d),
// so that the rows hold (-1)^{k3} h^{k3} h^{|g|} D^g d_{z'}^{k3} K as the image rows do.
// Both waves fall off with k_rho (no mirror-point image).  The rows are written in the
// frame (z, y, x) of the cross tables (the restore's x and z orders swapped).  Keys whose
// target or source centre lies outside its layer join boxes without particles and stay zero.
// ---------------------------------------------------------------------------
struct CrossKey {
  int sg, dx, dy, izt, izs;
};

static int sommerfeld_cross_rows(tefmm_t h, const Group& G, int lev, int k3, const std::vector<CrossKey>& keys,
                                 double2* d_out, hipStream_t s) {
  const MediumDesc& med = h->med;
  const int lt = G.layer, L = med.L, P2 = 2 * h->opt.p, nH = (P2 + 1) * (P2 + 2) / 2;
  const double hb = G.side / (1 << lev);
  const bool up = lt < L, dn = lt > 0;
  const double offs[2] = {up ? med.d[lt] : 0.0, dn ? med.d[lt - 1] : 0.0};
  const cplx I(0.0, 1.0);
  auto inside = [&](int l, double z) { return z > med.bottom(l) && z < med.top(l); };
  std::map<int, std::map<int, std::vector<int>>> by;  // source group -> source slab -> keys
  for (int i = 0; i < (int)keys.size(); ++i) {
    const CrossKey& k = keys[i];
    const Group& S = h->groups[k.sg];
    const double zt = G.lo[2] + (k.izt + 0.5) * hb, zs = S.lo[2] + (k.izs + 0.5) * hb;
    if (inside(lt, zt) && inside(S.layer, zs)) by[k.sg][k.izs].push_back(i);
  }
  for (auto& sgv : by) {
    const Group& S = h->groups[sgv.first];
    const int ls = S.layer;
    // the least decay length (target to its interface plus source to its interface) and
    // the largest horizontal distance of the keys served
    double zmin = 1e300, rmax = 0.0;
    for (auto& zv : sgv.second)
      for (int i : zv.second) {
        const CrossKey& k = keys[i];
        const double zt = G.lo[2] + (k.izt + 0.5) * hb, zs = S.lo[2] + (k.izs + 0.5) * hb;
        const double za = std::min(up ? zt - med.d[lt] : 1e300, dn ? med.d[lt - 1] - zt : 1e300);
        const double zb = std::min(ls < L ? zs - med.d[ls] : 1e300, ls > 0 ? med.d[ls - 1] - zs : 1e300);
        zmin = std::min(zmin, za + zb);
        rmax = std::max(rmax, hb * std::hypot((double)k.dx, (double)k.dy));
      }
    std::vector<cplx> krho, wts;
    som_nodes(med, zmin, rmax, P2 + 1, krho, wts);
    const size_t nn = krho.size();
    std::vector<cplx> kz(nn), kzp(nn), sg4(4 * nn);
    std::vector<cplx> sig;
    for (size_t t = 0; t < nn; ++t) {
      reaction_densities(med, ls, krho[t], sig);
      kz[t] = vertical_wavenumber(med.k[lt], krho[t]);
      kzp[t] = vertical_wavenumber(med.k[ls], krho[t]);
      for (int j = 0; j < 4; ++j) sg4[4 * t + j] = sig[lt * 4 + j];
    }
    h->som_nodes = std::max<int64_t>(h->som_nodes, (int64_t)nn);
    for (auto& zv : sgv.second) {
      const double zs = S.lo[2] + (zv.first + 0.5) * hb;
      SomPath P;
      P.krho = krho, P.kz = kz;
      P.cu.resize(nn), P.cd.resize(nn);
      const double sc = k3 ? -hb : 1.0;
      for (size_t t = 0; t < nn; ++t) {
        cplx eu = 0.0, ed = 0.0;
        if (ls < L) eu = std::pow(I * kzp[t], (double)k3) * std::exp(I * kzp[t] * (zs - med.d[ls]));
        if (ls > 0) ed = std::pow(-I * kzp[t], (double)k3) * std::exp(I * kzp[t] * (med.d[ls - 1] - zs));
        const cplx f = wts[t] * I / kz[t] * sc;
        P.cu[t] = up ? f * (sg4[4 * t + 0] * eu + sg4[4 * t + 1] * ed) : cplx(0.0);
        P.cd[t] = dn ? f * (sg4[4 * t + 2] * eu + sg4[4 * t + 3] * ed) : cplx(0.0);
      }
      // distinct horizontal distances and target heights of these keys, and their pairs
      std::map<long long, int> rmap, zmap;
      std::map<std::pair<int, int>, int> pmap;
      std::vector<double> rho, zt;
      std::vector<int> pr, ps, hrow, rows;
      std::vector<double> X, Y;
      for (int i : zv.second) {
        const CrossKey& k = keys[i];
        const long long r2 = (long long)k.dx * k.dx + (long long)k.dy * k.dy;
        auto ri = rmap.emplace(r2, (int)rho.size());
        if (ri.second) rho.push_back(hb * std::sqrt((double)r2));
        auto zi = zmap.emplace(k.izt, (int)zt.size());
        if (zi.second) zt.push_back(G.lo[2] + (k.izt + 0.5) * hb);
        auto pi = pmap.emplace(std::make_pair(ri.first->second, zi.first->second), (int)pr.size());
        if (pi.second) pr.push_back(ri.first->second), ps.push_back(zi.first->second);
        hrow.push_back(pi.first->second), rows.push_back(i);
        X.push_back(-k.dx * hb), Y.push_back(-k.dy * hb);
      }
      const int nk = (int)rows.size();
      double2* d_H = nullptr;
      double *d_x = nullptr, *d_y = nullptr;
      int *d_row = nullptr, *d_hrow = nullptr;
      auto run = [&]() -> int {
        HIPCHK(h, dmalloc(h, &d_H, sizeof(double2) * pr.size() * nH));
        const int rc = sommerfeld_h(h, lt, up, dn, P, P2, rho, zt, pr, ps, d_H, s, false, offs);
        if (rc != TEFMM_OK) return rc;
        HIPCHK(h, dmalloc(h, &d_x, sizeof(double) * nk));
        HIPCHK(h, dmalloc(h, &d_y, sizeof(double) * nk));
        HIPCHK(h, dmalloc(h, &d_row, sizeof(int) * nk));
        HIPCHK(h, dmalloc(h, &d_hrow, sizeof(int) * nk));
        HIPCHK(h, hipMemcpyAsync(d_x, X.data(), sizeof(double) * nk, hipMemcpyHostToDevice, s));
        HIPCHK(h, hipMemcpyAsync(d_y, Y.data(), sizeof(double) * nk, hipMemcpyHostToDevice, s));
        HIPCHK(h, hipMemcpyAsync(d_row, rows.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
        HIPCHK(h, hipMemcpyAsync(d_hrow, hrow.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
        // frame (z, y, x): the compact entry's first order is the z order, its third the x order
        hipLaunchKernelGGL(k_sigma_restore, dim3(nk), dim3(64), 0, s, d_H, d_x, d_y, nk, d_row, hb, med.k[lt], P2,
                           h->nG, h->d_g3, h->d_g1, h->d_gord, d_out, d_hrow, 0);
        HIPCHK(h, hipGetLastError());
        HIPCHK(h, hipStreamSynchronize(s));
        return TEFMM_OK;
      };
      const int rc = run();
      dfree(h, d_H), dfree(h, d_x), dfree(h, d_y), dfree(h, d_row), dfree(h, d_hrow);
      if (rc != TEFMM_OK) return rc;
      h->som_keys += nk;
    }
  }
  return TEFMM_OK;
}

static int build_cross(tefmm_t h, int gt, hipStream_t s) {
  Group& G = h->groups[gt];
  const MediumDesc& med = h->med;
  const int H = G.depth, p = h->opt.p;
  const int lt = G.layer;
  const int ng = (int)h->groups.size();
  G.xlist_start.assign(H + 1, nullptr);
  G.xlist.assign(H + 1, nullptr);
  G.xkeys.assign(H + 1, 0);
  G.XT0.assign(H + 1, nullptr), G.XT1.assign(H + 1, nullptr);
  G.XT032.assign(H + 1, nullptr), G.XT132.assign(H + 1, nullptr);
  G.cross_flops_per_rhs = 0;
  G.cross_pairs = 0, G.cross_forced = 0, G.n_cross_fits = 0, G.cross_fit_err = 0;
  G.has_cross = ng > 1;
  if (!G.has_cross) return TEFMM_OK;
  std::vector<int> waves;
  if (lt < med.L) waves.push_back(0);
  if (lt > 0) waves.push_back(1);
  const double sq3 = std::sqrt(3.0);
  auto mac = [&](int sg, int l, int dx, int dy, int izt, int izs) {
    const double hh = G.side / (1 << l);
    const double zt = G.lo[2] + (izt + 0.5) * hh, zs = h->groups[sg].lo[2] + (izs + 0.5) * hh;
    const double D = std::sqrt((dx * hh) * (dx * hh) + (dy * hh) * (dy * hh) + (zt - zs) * (zt - zs));
    return sq3 * hh <= CROSS_THETA * D;
  };
  auto nvalid = [](int d, int par, int n) {
    int c = 0;
    for (int i = par; i < n; i += 2)
      if (i + d >= 0 && i + d < n) ++c;
    return c;
  };
  typedef CrossKey KeyRec;
  std::vector<std::vector<KeyRec>> keys(H + 1);
  std::vector<std::vector<std::vector<CrossEntry>>> lists(H + 1);
  // fits needed: (sg, level, izs)
  std::map<std::tuple<int, int, int>, int> fitmap;
  for (int lev = 2; lev <= H; ++lev) {
    const int n = 1 << lev;
    lists[lev].assign(4 * n, {});
    std::map<std::tuple<int, int, int, int, int>, int> kmap;
    for (int sg = 0; sg < ng; ++sg) {
      if (sg == gt) continue;
      for (int izt = 0; izt < n; ++izt)
        for (int pc = 0; pc < 4; ++pc) {
          const int px = pc & 1, py = pc >> 1;
          std::vector<std::array<int, 3>> cand;
          if (lev == 2) {
            for (int dx = -(n - 1); dx <= n - 1; ++dx)
              for (int dy = -(n - 1); dy <= n - 1; ++dy)
                for (int izs = 0; izs < n; ++izs) cand.push_back({dx, dy, izs});
          } else {
            const int W = 3;
            for (int Pdx = -W; Pdx <= W; ++Pdx)
              for (int Pdy = -W; Pdy <= W; ++Pdy)
                for (int Pz = 0; Pz < n / 2; ++Pz) {
                  if (mac(sg, lev - 1, Pdx, Pdy, izt >> 1, Pz)) continue;
                  for (int c = 0; c < 8; ++c)
                    cand.push_back({2 * Pdx + ((c >> 2) & 1) - px, 2 * Pdy + ((c >> 1) & 1) - py, 2 * Pz + (c & 1)});
                }
          }
          for (auto& cd : cand) {
            const int dx = cd[0], dy = cd[1], izs = cd[2];
            const bool pass = mac(sg, lev, dx, dy, izt, izs);
            if (!(pass || lev == H)) continue;
            const int vx = nvalid(dx, px, n), vy = nvalid(dy, py, n);
            if (!vx || !vy) continue;
            auto kt = std::make_tuple(sg, dx, dy, izt, izs);
            auto it = kmap.find(kt);
            int key;
            if (it == kmap.end()) {
              key = (int)keys[lev].size();
              kmap[kt] = key;
              keys[lev].push_back({sg, dx, dy, izt, izs});
              fitmap.emplace(std::make_tuple(sg, lev, izs), 0);
            } else {
              key = it->second;
            }
            lists[lev][4 * izt + pc].push_back({sg, dx, dy, izs, key});
            G.cross_flops_per_rhs += 8.0 * h->nR * h->nR * vx * vy;
            G.cross_pairs += (int64_t)vx * vy;
            if (!pass) G.cross_forced += (int64_t)vx * vy;
          }
        }
    }
  }
  // complex images: (sg, level, izs) x k3' in {0, 1} x target waves, fitted in parallel
  struct Job {
    int sg, lev, izs, k3, a;
    std::vector<cplx> A, Z;
    double fe = 0;
    bool ok = true;
    std::string err;
  };
  std::vector<Job> jobs;
  // from the Sommerfeld integrals instead: no fits (sommerfeld_cross_rows)
  const bool som_x = h->opt.sigma_tables == TEFMM_SIGMA_SOMMERFELD;
  for (auto& kv : fitmap) {
    if (som_x) break;
    int idx = (int)jobs.size();
    kv.second = idx;
    for (int k3 = 0; k3 < 2; ++k3)
      for (int a : waves) {
        Job j;
        j.sg = std::get<0>(kv.first), j.lev = std::get<1>(kv.first), j.izs = std::get<2>(kv.first);
        j.k3 = k3, j.a = a;
        jobs.push_back(j);
      }
  }
  {
    const int nthr = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    for (int t = 0; t < nthr; ++t)
      th.emplace_back([&]() {
        for (;;) {
          const int i = next++;
          if (i >= (int)jobs.size()) break;
          Job& j = jobs[i];
          const Group& S = h->groups[j.sg];
          const double hh = G.side / (1 << j.lev);
          const double zs = S.lo[2] + (j.izs + 0.5) * hh;
          j.ok = cross_layer_fit(med, lt, S.layer, j.a, zs, j.k3, G.fit_zlo, G.fit_zhi, h->opt.dcim_T1_cross,
                                 h->opt.dcim_samples, h->opt.dcim_svd_tol, j.A, j.Z, j.fe, j.err);
        }
      });
    for (auto& t : th) t.join();
  }
  for (auto& j : jobs)
    if (!j.ok) return fail(h, TEFMM_ERR_DCIM_FIT, "cross-layer complex-image fit failed: " + j.err);
  G.n_cross_fits = (int)jobs.size();
  G.cross_fit_err = 0;
  for (auto& j : jobs) G.cross_fit_err = std::max(G.cross_fit_err, j.fe);
  // the images represent the kernel only for heights inside the layers; a box that
  // may hold particles must have its centre there (target and source side)
  for (int lev = 2; lev <= H; ++lev)
    for (const KeyRec& kr : keys[lev]) {
      const double hb = G.side / (1 << lev);
      const Group& S = h->groups[kr.sg];
      const double zt = G.lo[2] + (kr.izt + 0.5) * hb, zs = S.lo[2] + (kr.izs + 0.5) * hb;
      const bool t_occ = zt - 0.5 * hb < G.zhi && zt + 0.5 * hb > G.zlo;
      const bool s_occ = zs - 0.5 * hb < S.zhi && zs + 0.5 * hb > S.zlo;
      if ((t_occ && (zt <= med.bottom(lt) || zt >= med.top(lt))) ||
          (s_occ && (zs <= med.bottom(S.layer) || zs >= med.top(S.layer))))
        return fail(h, TEFMM_ERR_UNSUPPORTED,
                    "cross-layer geometry: a box holding particles has its centre outside its layer "
                    "(layer thinner than the common box side)");
    }
  // tables per level and k3'
  for (int lev = 2; lev <= H; ++lev) {
    const int n = 1 << lev;
    const double hb = G.side / n;
    const int nkeys = (int)keys[lev].size();
    G.xkeys[lev] = nkeys;
    std::vector<int> starts(4 * n + 1, 0);
    std::vector<CrossEntry> flat;
    for (int c = 0; c < 4 * n; ++c) {
      starts[c] = (int)flat.size();
      flat.insert(flat.end(), lists[lev][c].begin(), lists[lev][c].end());
    }
    starts[4 * n] = (int)flat.size();
    HIPCHK(h, dmalloc(h, &G.xlist_start[lev], sizeof(int) * (4 * n + 1)));
    HIPCHK(h, hipMemcpy(G.xlist_start[lev], starts.data(), sizeof(int) * (4 * n + 1), hipMemcpyHostToDevice));
    HIPCHK(h, dmalloc(h, &G.xlist[lev], sizeof(CrossEntry) * std::max<size_t>(1, flat.size())));
    if (!flat.empty())
      HIPCHK(h, hipMemcpy(G.xlist[lev], flat.data(), sizeof(CrossEntry) * flat.size(), hipMemcpyHostToDevice));
    for (int k3 = 0; k3 < 2; ++k3) {
      std::vector<TableTerm> terms;
      std::vector<int> start;
      std::vector<double> hk;
      for (const KeyRec& kr : keys[lev]) {
        start.push_back((int)terms.size());
        hk.push_back(hb);
        if (som_x) continue;  // rows written below
        const double zt = G.lo[2] + (kr.izt + 0.5) * hb;
        const int fi = fitmap.at(std::make_tuple(kr.sg, lev, kr.izs));
        for (int wi = 0; wi < (int)waves.size(); ++wi) {
          const int a = waves[wi];
          const Job& j = jobs[fi + k3 * (int)waves.size() + wi];
          const double Za = a == 0 ? zt - med.d[lt] : med.d[lt - 1] - zt;
          const cplx sc = k3 ? cplx(-hb, 0) : cplx(1, 0);
          for (size_t q = 0; q < j.A.size(); ++q) {
            const cplx zeta = (Za - j.Z[q]) / hb;
            if (zeta.real() <= 1e-9) continue;
            TableTerm t;
            t.x = -kr.dx, t.y = -kr.dy, t.zr = zeta.real(), t.zi = zeta.imag();
            const cplx cf = j.A[q] * sc;
            t.cr = cf.real(), t.ci = cf.imag(), t.flip = a == 1, t.pad = 0;
            terms.push_back(t);
          }
        }
      }
      start.push_back((int)terms.size());
      double2* d_out = nullptr;
      HIPCHK(h, dmalloc(h, &d_out, sizeof(double2) * std::max<size_t>(1, (size_t)nkeys * h->nG)));
      if (nkeys > 0) {
        TableTerm* d_terms = nullptr;
        int* d_start = nullptr;
        double* d_h = nullptr;
        HIPCHK(h, dmalloc(h, &d_terms, sizeof(TableTerm) * std::max<size_t>(terms.size(), 1)));
        HIPCHK(h, dmalloc(h, &d_start, sizeof(int) * start.size()));
        HIPCHK(h, dmalloc(h, &d_h, sizeof(double) * hk.size()));
        if (!terms.empty())
          HIPCHK(h, hipMemcpyAsync(d_terms, terms.data(), sizeof(TableTerm) * terms.size(), hipMemcpyHostToDevice, s));
        HIPCHK(h, hipMemcpyAsync(d_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice, s));
        HIPCHK(h, hipMemcpyAsync(d_h, hk.data(), sizeof(double) * hk.size(), hipMemcpyHostToDevice, s));
        TableGenArgs ta;
        ta.terms = d_terms, ta.term_start = d_start, ta.h = d_h, ta.k = med.k[lt], ta.order = 2 * p, ta.nG = h->nG;
        ta.nbr = h->d_nbr, ta.g3 = h->d_g3, ta.g1 = h->d_g1, ta.swap13 = 1, ta.fact = h->d_fact, ta.out = d_out;
        HIPCHK(h, launch_table_gen(ta, nkeys, s));
        HIPCHK(h, hipStreamSynchronize(s));
        dfree(h, d_terms);
        dfree(h, d_start);
        dfree(h, d_h);
        if (som_x) {
          const int rc = sommerfeld_cross_rows(h, G, lev, k3, keys[lev], d_out, s);
          if (rc != TEFMM_OK) {
            dfree(h, d_out);
            return rc;
          }
        }
      }
      (k3 ? G.XT1[lev] : G.XT0[lev]) = d_out;
      if (h->opt.precision == TEFMM_MIXED_FP32) {
        float2* d32 = nullptr;
        const int rc = tables_to_f32(h, d_out, (size_t)nkeys * h->nG, &d32, s);
        if (rc != TEFMM_OK) return rc;
        (k3 ? G.XT132[lev] : G.XT032[lev]) = d32;
      }
    }
  }
  return TEFMM_OK;
}

// ---------------------------------------------------------------------------
// Convergence of the reaction expansions.  A translation between boxes of side h
// converges when the kernel's nearest singularity is farther from the key's centre
// displacement than the two boxes reach, sqrt(3) h; the free-space far field works
// at a ratio sqrt(3) h / distance of at most sqrt(3)/2 (boxes two sides apart), and
// the reaction keys are held to the same.  For the Sigma family the singularity is
// the mirror point z + z' = 2 d (distance sqrt(dx^2 + dy^2 + (S - 2d)^2) for a key
// with centre height sum S); for the Delta family it is |z - z'| = D (distance
// D - |w| at w = z - z').  Leaf-level Sigma keys above SIGMA_LEAF_THETA are evaluated
// directly (their rows stay zero); other keys above REACTION_THETA are counted.
// ---------------------------------------------------------------------------
static const double REACTION_THETA = 0.87;  // just above sqrt(3)/2
// Leaf-level Sigma keys are evaluated directly already above this ratio: next to an
// interface many pairs sit near the worst corner, and a ratio close to sqrt(3)/2 then
// converges too slowly for the FP64 mode (particles 0.01 from an interface: 1.6e-6 at
// 0.87, p = 12)
static const double SIGMA_LEAF_THETA = 0.75;

static int reaction_convergence(tefmm_t h, Group& g, const std::vector<int>& lc, hipStream_t s) {
  const MediumDesc& med = h->med;
  const int l = g.layer, H = g.depth, nbH = 1 << H;
  const double sq3 = std::sqrt(3.0);
  const bool sig = g.has[0] || g.has[1];
  // occupied z slabs per level
  std::vector<std::vector<char>> occ(H + 1);
  for (int lev = 2; lev <= H; ++lev) occ[lev].assign(1 << lev, 0);
  for (int ix = 0; ix < nbH; ++ix)
    for (int iy = 0; iy < nbH; ++iy)
      for (int iz = 0; iz < nbH; ++iz)
        if (lc[g.leaf_base + ((int64_t)ix * nbH + iy) * nbH + iz] > 0)
          for (int lev = 2; lev <= H; ++lev) occ[lev][iz >> (H - lev)] = 1;
  auto sigma_dist = [&](double rho2, double S) {
    double d = 1e300;
    if (g.has[0]) d = std::min(d, std::sqrt(rho2 + (S - 2 * med.d[l]) * (S - 2 * med.d[l])));
    if (g.has[1]) d = std::min(d, std::sqrt(rho2 + (2 * med.d[l - 1] - S) * (2 * med.d[l - 1] - S)));
    return d;
  };
  g.keys_forced = 0;
  for (int lev = 2; lev <= H; ++lev) {
    const int nb = 1 << lev;
    const double hb = g.side / nb;
    const bool leaf = lev == H;
    for (int it = 0; it < nb; ++it) {
      if (!occ[lev][it]) continue;
      for (int dz = -2 - (it & 1); dz <= 3 - (it & 1); ++dz) {
        const int is = it + dz;
        if (is < 0 || is >= nb || !occ[lev][is]) continue;
        const bool nearz = std::abs(dz) <= 1;
        // Delta family (with the free-space kernel): translated far pairs, and at the
        // leaf level the neighbours too; worst case dx = dy = 0
        if (g.has[2] && (leaf || !nearz)) {
          const double dist = med.thickness(l) - std::abs(dz) * hb;
          if (!(dist > 0) || sq3 * hb > REACTION_THETA * dist) ++g.keys_forced;
        }
        // Sigma family above the leaf level (far in z; pairs far only in x or y are two
        // sides apart horizontally, within the ratio)
        if (sig && !leaf && !nearz) {
          const double S = 2 * g.lo[2] + (it + is + 1) * hb;
          if (sq3 * hb > REACTION_THETA * sigma_dist(0.0, S)) ++g.keys_forced;
        }
      }
    }
  }
  // Sigma family at the leaf level: flag keys, list the occupied leaf pairs using them
  g.sig_flag.clear();
  g.sd_ntgt = 0, g.sd_pairs = 0;
  if (!sig) return TEFMM_OK;
  const double hb = g.side / nbH;
  const int nm = 2 * nbH - 1;
  g.sig_flag.assign((size_t)49 * nm, 0);
  bool any = false;
  for (int dx = -3; dx <= 3; ++dx)
    for (int dy = -3; dy <= 3; ++dy)
      for (int m = 0; m < nm; ++m) {
        const double S = 2 * g.lo[2] + (m + 1) * hb;
        if (sq3 * hb > SIGMA_LEAF_THETA * sigma_dist((dx * dx + dy * dy) * hb * hb, S)) {
          g.sig_flag[((size_t)(dx + 3) * 7 + (dy + 3)) * nm + m] = 1;
          any = true;
        }
      }
  if (!any) return TEFMM_OK;
  std::vector<int> tgt, start, src;
  for (int ix = 0; ix < nbH; ++ix)
    for (int iy = 0; iy < nbH; ++iy)
      for (int iz = 0; iz < nbH; ++iz) {
        const int tleaf = (ix * nbH + iy) * nbH + iz;
        const int tc = lc[g.leaf_base + tleaf];
        if (tc == 0) continue;
        const size_t before = src.size();
        for (int dx = -2 - (ix & 1); dx <= 3 - (ix & 1); ++dx) {
          const int jx = ix + dx;
          if (jx < 0 || jx >= nbH) continue;
          for (int dy = -2 - (iy & 1); dy <= 3 - (iy & 1); ++dy) {
            const int jy = iy + dy;
            if (jy < 0 || jy >= nbH) continue;
            for (int dz = -2 - (iz & 1); dz <= 3 - (iz & 1); ++dz) {
              const int jz = iz + dz;
              if (jz < 0 || jz >= nbH) continue;
              if (!g.sig_flag[((size_t)(dx + 3) * 7 + (dy + 3)) * nm + (iz + jz)]) continue;
              const int sleaf = (jx * nbH + jy) * nbH + jz;
              const int sc = lc[g.leaf_base + sleaf];
              if (sc == 0) continue;
              src.push_back(sleaf);
              g.sd_pairs += (int64_t)tc * sc;
            }
          }
        }
        if (src.size() > before) {
          tgt.push_back(tleaf);
          start.push_back((int)before);
        }
      }
  if (tgt.empty()) return TEFMM_OK;
  start.push_back((int)src.size());
  std::vector<double2> img;
  for (int fam = 0; fam < 2; ++fam)
    if (g.has[fam])
      for (size_t j = 0; j < g.famA[fam].size(); ++j) {
        img.push_back(make_double2(g.famA[fam][j].real(), g.famA[fam][j].imag()));
        img.push_back(make_double2(g.famZ[fam][j].real(), g.famZ[fam][j].imag()));
      }
  g.sd_nup = g.has[0] ? (int)g.famA[0].size() : 0;
  g.sd_ndn = g.has[1] ? (int)g.famA[1].size() : 0;
  if (g.sd_nup + g.sd_ndn > SIGMA_DIRECT_MAX_IMAGES)
    return fail(h, TEFMM_ERR_UNSUPPORTED, "too many complex images for the direct near-interface evaluation");
  g.sd_ntgt = (int)tgt.size();
  HIPCHK(h, dmalloc(h, &g.d_sd_tgt, sizeof(int) * tgt.size()));
  HIPCHK(h, dmalloc(h, &g.d_sd_start, sizeof(int) * start.size()));
  HIPCHK(h, dmalloc(h, &g.d_sd_src, sizeof(int) * src.size()));
  HIPCHK(h, dmalloc(h, &g.d_sd_img, sizeof(double2) * std::max<size_t>(img.size(), 1)));
  HIPCHK(h, hipMemcpyAsync(g.d_sd_tgt, tgt.data(), sizeof(int) * tgt.size(), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(g.d_sd_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(g.d_sd_src, src.data(), sizeof(int) * src.size(), hipMemcpyHostToDevice, s));
  if (!img.empty())
    HIPCHK(h, hipMemcpyAsync(g.d_sd_img, img.data(), sizeof(double2) * img.size(), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return TEFMM_OK;
}

extern "C" int tefmm_set_particles(tefmm_t h, int64_t n, const double* xyz, int on_device, void* stream) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  if (n < 1 || !xyz) return fail(h, TEFMM_ERR_INVALID_ARG, "need n >= 1 particles");
  if (n > (int64_t)2000000000) return fail(h, TEFMM_ERR_INVALID_ARG, "too many particles");
  hipStream_t s = (hipStream_t)stream;
  free_geometry(h);
  const MediumDesc& med = h->med;
  const int L = med.L;
  hipEvent_t e0, e1, e2;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  HIPCHK(h, hipEventCreate(&e2));
  HIPCHK(h, hipEventRecord(e0, s));
  double* d_in = nullptr;
  const double* src = xyz;
  if (!on_device) {
    HIPCHK(h, dmalloc(h, &d_in, sizeof(double) * 3 * n));
    HIPCHK(h, hipMemcpyAsync(d_in, xyz, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    src = d_in;
  }
  if (src != h->d_xyz_user) {
    dfree(h, h->d_xyz_user);
    HIPCHK(h, dmalloc(h, &h->d_xyz_user, sizeof(double) * 3 * n));
    HIPCHK(h, hipMemcpyAsync(h->d_xyz_user, src, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, s));
  }
  double* d_if = nullptr;
  HIPCHK(h, dmalloc(h, &d_if, sizeof(double) * std::max(L, 1)));
  if (L) HIPCHK(h, hipMemcpyAsync(d_if, med.d.data(), sizeof(double) * L, hipMemcpyHostToDevice, s));
  // layer statistics
  const int nblk = (int)std::min<int64_t>(1024, (n + 255) / 256);
  double* d_part = nullptr;
  int* d_bad = nullptr;
  HIPCHK(h, dmalloc(h, &d_part, sizeof(double) * nblk * MAX_LAYERS * 7));
  HIPCHK(h, dmalloc(h, &d_bad, sizeof(int)));
  HIPCHK(h, hipMemsetAsync(d_bad, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_layer_stats, dim3(nblk), dim3(256), 0, s, src, n, L, d_if, h->opt.interface_eps, d_part, d_bad);
  HIPCHK(h, hipGetLastError());
  std::vector<double> part((size_t)nblk * MAX_LAYERS * 7);
  int bad = 0;
  HIPCHK(h, hipMemcpyAsync(part.data(), d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  dfree(h, d_part);
  dfree(h, d_bad);
  if (bad & 2) {
    dfree(h, d_in), dfree(h, d_if);
    return fail(h, TEFMM_ERR_INVALID_ARG, "non-finite particle coordinate");
  }
  if (bad & 1) {
    dfree(h, d_in), dfree(h, d_if);
    return fail(h, TEFMM_ERR_PARTICLE_ON_INTERFACE, "a particle lies within interface_eps of an interface");
  }
  double mn[MAX_LAYERS][3], mx[MAX_LAYERS][3];
  int64_t cnt[MAX_LAYERS] = {};
  for (int l = 0; l < MAX_LAYERS; ++l)
    for (int c = 0; c < 3; ++c) mn[l][c] = 1e300, mx[l][c] = -1e300;
  for (int b = 0; b < nblk; ++b)
    for (int l = 0; l < MAX_LAYERS; ++l) {
      const double* o = &part[((size_t)b * MAX_LAYERS + l) * 7];
      for (int c = 0; c < 3; ++c) mn[l][c] = std::min(mn[l][c], o[c]), mx[l][c] = std::max(mx[l][c], o[3 + c]);
      cnt[l] += (int64_t)o[6];
    }
  int ngroups = 0;
  for (int l = 0; l <= L; ++l) ngroups += cnt[l] > 0;
  // Several layers: one common x-y box grid (so that cross-layer offsets are whole
  // boxes), one common cube side and one depth; each layer's cube is centred on
  // its particles in z.
  double cx0 = 1e300, cx1 = -1e300, cy0 = 1e300, cy1 = -1e300, zext = 0;
  int depth_common = 2;
  for (int l = 0; l <= L; ++l) {
    if (!cnt[l]) continue;
    cx0 = std::min(cx0, mn[l][0]), cx1 = std::max(cx1, mx[l][0]);
    cy0 = std::min(cy0, mn[l][1]), cy1 = std::max(cy1, mx[l][1]);
    zext = std::max(zext, mx[l][2] - mn[l][2]);
    int dl = 2;
    while (dl < 7 && (double)cnt[l] / std::pow(8.0, dl) > h->opt.max_leaf) ++dl;
    depth_common = std::max(depth_common, dl);
  }
  const double side_common = std::max(std::max(cx1 - cx0, cy1 - cy0), zext) * (1 + 1e-9) + 1e-12;
  // z origin of each layer's cube: centred on the layer's particles, then moved
  // (keeping them inside) so that the cube stays within the layer when the layer
  // is thick enough
  double lo_z[MAX_LAYERS] = {};
  for (int l = 0; l <= L; ++l) {
    if (!cnt[l]) continue;
    double z0 = 0.5 * (mn[l][2] + mx[l][2]) - 0.5 * side_common;
    const double a0 = std::max(mx[l][2] - side_common, med.bottom(l)), a1 = std::min(mn[l][2], med.top(l) - side_common);
    if (a0 <= a1) z0 = std::min(std::max(z0, a0), a1);
    lo_z[l] = z0;
  }
  // Automatic depth with several layers: deep enough that the closest occupied
  // leaf slabs of two layers pass the cross-layer acceptance test (so no
  // cross-layer pair is translated below it), up to the depth limit.
  if (ngroups > 1 && h->opt.depth == 0) {
    auto slab_gap_ok = [&](int dep) {
      const double hb = side_common / (1 << dep);
      for (int a = 0; a <= L; ++a)
        for (int b = a + 1; b <= L; ++b) {
          if (!cnt[a] || !cnt[b]) continue;
          // occupied slab centres of a and b closest to each other
          const int ia0 = (int)std::floor((mn[a][2] - lo_z[a]) / hb), ib1 = (int)std::floor((mx[b][2] - lo_z[b]) / hb);
          const double za = lo_z[a] + (std::max(ia0, 0) + 0.5) * hb;
          const double zb = lo_z[b] + (std::min(ib1, (1 << dep) - 1) + 0.5) * hb;
          if (std::sqrt(3.0) * hb > CROSS_THETA * std::fabs(za - zb)) return false;
        }
      return true;
    };
    while (depth_common < 7 && !slab_gap_ok(depth_common)) ++depth_common;
  }
  TreeGeom geo;
  std::memset(&geo, 0, sizeof(geo));
  for (int l = 0; l < MAX_LAYERS; ++l) geo.group_of_layer[l] = 0;
  int64_t leaf_off = 0, pos = 0;
  for (int l = 0; l <= L; ++l) {
    if (!cnt[l]) continue;
    Group g;
    g.layer = l;
    g.count = cnt[l];
    g.start = pos;
    pos += cnt[l];
    double side = 0;
    for (int c = 0; c < 3; ++c) side = std::max(side, mx[l][c] - mn[l][c]);
    side = side * (1 + 1e-9) + 1e-12;
    for (int c = 0; c < 3; ++c) g.lo[c] = 0.5 * (mn[l][c] + mx[l][c]) - 0.5 * side;
    // a cube taller than its particles' extent is moved (keeping them inside) to lie
    // within the layer when the layer is thick enough: no box of it then reaches across
    // an interface, where the reaction expansions of its lowest or highest slab would not
    // converge above the leaf level
    {
      const double a0 = std::max(mx[l][2] - side, med.bottom(l)), a1 = std::min(mn[l][2], med.top(l) - side);
      if (a0 <= a1) g.lo[2] = std::min(std::max(g.lo[2], a0), a1);
    }
    if (ngroups > 1) {
      side = side_common;
      g.lo[0] = 0.5 * (cx0 + cx1) - 0.5 * side;
      g.lo[1] = 0.5 * (cy0 + cy1) - 0.5 * side;
      g.lo[2] = lo_z[l];
    }
    g.side = side;
    int depth = h->opt.depth;
    if (depth == 0) {
      depth = 2;
      while (depth < 7 && (double)cnt[l] / std::pow(8.0, depth) > h->opt.max_leaf) ++depth;
      if (ngroups > 1) depth = depth_common;
    }
    g.depth = std::max(2, std::min(7, depth));
    g.leaf_base = leaf_off;
    leaf_off += (int64_t)1 << (3 * g.depth);
    g.zlo = mn[l][2], g.zhi = mx[l][2];
    const int gi = (int)h->groups.size();
    geo.group_of_layer[l] = gi;
    geo.depth[gi] = g.depth;
    for (int c = 0; c < 3; ++c) geo.lo[gi][c] = g.lo[c];
    geo.side[gi] = g.side;
    geo.leaf_offset[gi] = g.leaf_base;
    h->groups.push_back(g);
  }
  h->total_leaves = leaf_off;
  h->n = n;
  // sort particles by leaf
  unsigned *d_keys = nullptr, *d_keys2 = nullptr;
  int* d_perm_in = nullptr;
  HIPCHK(h, dmalloc(h, &d_keys, sizeof(unsigned) * n));
  HIPCHK(h, dmalloc(h, &d_keys2, sizeof(unsigned) * n));
  HIPCHK(h, dmalloc(h, &d_perm_in, sizeof(int) * n));
  HIPCHK(h, dmalloc(h, &h->d_perm, sizeof(int) * n));
  const int nb256 = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_leaf_keys, dim3(nb256), dim3(256), 0, s, src, n, L, d_if, geo, d_keys, d_perm_in);
  HIPCHK(h, hipGetLastError());
  int end_bit = 1;
  while (((int64_t)1 << end_bit) < leaf_off) ++end_bit;
  // stable radix sort by leaf key and the leaf starts by an exclusive scan of the counts
  // (sort_scan.hip), with scratch from the handle's allocator
  void* d_tmp = nullptr;
  HIPCHK(h, dmalloc(h, &d_tmp, std::max(sort_scratch_bytes(n), scan_scratch_bytes(leaf_off))));
  HIPCHK(h, radix_sort_pairs(d_keys, d_keys2, d_perm_in, h->d_perm, n, end_bit, d_tmp, s));
  HIPCHK(h, dmalloc(h, &h->d_leaf_count, sizeof(int) * leaf_off));
  HIPCHK(h, dmalloc(h, &h->d_leaf_start, sizeof(int) * leaf_off));
  HIPCHK(h, hipMemsetAsync(h->d_leaf_count, 0, sizeof(int) * leaf_off, s));
  hipLaunchKernelGGL(k_count_keys, dim3(nb256), dim3(256), 0, s, d_keys2, n, h->d_leaf_count);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, exclusive_scan((const unsigned*)h->d_leaf_count, (unsigned*)h->d_leaf_start, leaf_off, d_tmp, s));
  HIPCHK(h, dmalloc(h, &h->d_xs, sizeof(double) * 3 * n));
  hipLaunchKernelGGL(k_gather_pos, dim3(nb256), dim3(256), 0, s, src, h->d_perm, n, h->d_xs);
  HIPCHK(h, hipGetLastError());
  std::vector<int>& lc = h->leaf_count_host;
  lc.assign(leaf_off, 0);
  HIPCHK(h, hipMemcpyAsync(lc.data(), h->d_leaf_count, sizeof(int) * leaf_off, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  dfree(h, d_tmp);
  dfree(h, d_keys);
  dfree(h, d_keys2);
  dfree(h, d_perm_in);
  dfree(h, d_in);
  dfree(h, d_if);
  HIPCHK(h, hipEventRecord(e1, s));
  // leaf occupancy and interaction counts (statistics)
  int64_t occ_leaves = 0, max_leaf = 0;
  for (int64_t b = 0; b < leaf_off; ++b) occ_leaves += lc[b] > 0, max_leaf = std::max<int64_t>(max_leaf, lc[b]);
  h->p2p_pairs = 0;
  h->p2p_same = 0;
  h->m2l_pairs = 0;
  for (auto& g : h->groups) {
    const int nb = 1 << g.depth;
    for (int ix = 0; ix < nb; ++ix)
      for (int iy = 0; iy < nb; ++iy)
        for (int iz = 0; iz < nb; ++iz) {
          int64_t c = lc[g.leaf_base + ((int64_t)ix * nb + iy) * nb + iz], nbsum = 0;
          for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dz = -1; dz <= 1; ++dz) {
                int jx = ix + dx, jy = iy + dy, jz = iz + dz;
                if (jx < 0 || jy < 0 || jz < 0 || jx >= nb || jy >= nb || jz >= nb) continue;
                nbsum += lc[g.leaf_base + ((int64_t)jx * nb + jy) * nb + jz];
              }
          h->p2p_pairs += c * nbsum - c;
          h->p2p_same += c * c - c;
        }
    // targets per lane: 2 above a mean occupancy of 96 over the occupied leaves, else 1
    // (unless set); workgroups per leaf: the passes a leaf of mean occupied size needs (at
    // most 8)
    // (the per-level box counts are set up later, with the buffers: the leaf count directly)
    const int64_t nleaf = (int64_t)1 << (3 * g.depth);
    int64_t occ = 0;
    for (int64_t b = 0; b < nleaf; ++b) occ += lc[g.leaf_base + b] > 0;
    const double mean_occ = occ ? (double)g.count / (double)occ : 0.0;
    g.mean_occ = mean_occ;
    g.p2p_tpl = h->opt.p2p_targets > 0 ? h->opt.p2p_targets : (mean_occ > 96 ? 2 : 1);
    g.p2p_split = std::max(1, std::min(8, (int)std::ceil(mean_occ / (64.0 * g.p2p_tpl))));
    {
      // the near field's work list: item leaf G + half for each half with a pass, its work
      // the targets of its passes times the sources of the leaf's forward neighbourhood
      const int nb = 1 << g.depth, G = g.p2p_split, TP = 64 * g.p2p_tpl;
      auto cnt = [&](int x, int y, int z) -> int64_t {
        if (x < 0 || y < 0 || z < 0 || x >= nb || y >= nb || z >= nb) return 0;
        return lc[g.leaf_base + ((int64_t)x * nb + y) * nb + z];
      };
      g.nf_items.clear();
      std::vector<double> work;
      for (int ix = 0; ix < nb; ++ix)
        for (int iy = 0; iy < nb; ++iy)
          for (int iz = 0; iz < nb; ++iz) {
            const int64_t c = cnt(ix, iy, iz);
            if (!c) continue;
            int64_t src = c + cnt(ix, iy, iz + 1);
            const int cols[4][2] = {{0, 1}, {1, -1}, {1, 0}, {1, 1}};
            for (auto& cc : cols)
              for (int dz = -1; dz <= 1; ++dz) src += cnt(ix + cc[0], iy + cc[1], iz + dz);
            const unsigned leaf = (unsigned)(((int64_t)ix * nb + iy) * nb + iz);
            for (int half = 0; half < G && (int64_t)half * TP < c; ++half) {
              int64_t tg = 0;
              for (int64_t c0 = (int64_t)half * TP; c0 < c; c0 += (int64_t)G * TP) tg += std::min<int64_t>(TP, c - c0);
              g.nf_items.push_back(leaf * (unsigned)G + (unsigned)half);
              work.push_back((double)tg * (double)src);
            }
          }
      cut_xcd_segments(g.nf_items, work, g.nf_seg, g.nf_seg_max);
      if (!g.nf_items.empty()) {
        HIPCHK(h, dmalloc(h, &g.d_nf_items, sizeof(unsigned) * g.nf_items.size()));
        HIPCHK(h, hipMemcpyAsync(g.d_nf_items, g.nf_items.data(), sizeof(unsigned) * g.nf_items.size(),
                                 hipMemcpyHostToDevice, s));
      }
      // the one-sided kernel's list: occupied leaves, work = targets x the 27-leaf block
      g.p2p_items.clear();
      work.clear();
      for (int ix = 0; ix < nb; ++ix)
        for (int iy = 0; iy < nb; ++iy)
          for (int iz = 0; iz < nb; ++iz) {
            const int64_t c = cnt(ix, iy, iz);
            if (!c) continue;
            int64_t src = 0;
            for (int dx = -1; dx <= 1; ++dx)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) src += cnt(ix + dx, iy + dy, iz + dz);
            g.p2p_items.push_back((unsigned)(((int64_t)ix * nb + iy) * nb + iz));
            work.push_back((double)c * (double)src);
          }
      cut_xcd_segments(g.p2p_items, work, g.p2p_seg, g.p2p_seg_max);
      if (!g.p2p_items.empty()) {
        HIPCHK(h, dmalloc(h, &g.d_p2p_items, sizeof(unsigned) * g.p2p_items.size()));
        HIPCHK(h, hipMemcpyAsync(g.d_p2p_items, g.p2p_items.data(), sizeof(unsigned) * g.p2p_items.size(),
                                 hipMemcpyHostToDevice, s));
      }
    }
    g.np_err = 0;
    g.np_on = h->opt.p2p_poly == 0 &&
              fit_near_poly(h->med.k[g.layer], g.side / (double)(1 << g.depth), 3e-7, &g.np, &g.np_err);
    // box occupancy per level (leaf counts, then the parents of occupied boxes), on the
    // device for the M2L, which skips empty targets and sources
    g.occ.assign(g.depth + 1, {});
    g.d_occ.assign(g.depth + 1, nullptr);
    {
      auto& o = g.occ[g.depth];
      o.resize((size_t)nleaf);
      for (int64_t b = 0; b < nleaf; ++b) o[b] = lc[g.leaf_base + b] > 0;
      for (int lev = g.depth - 1; lev >= 2; --lev) {
        const int nc = 1 << (lev + 1), np = 1 << lev;
        auto& po = g.occ[lev];
        const auto& co = g.occ[lev + 1];
        po.assign((size_t)np * np * np, 0);
        for (int ix = 0; ix < nc; ++ix)
          for (int iy = 0; iy < nc; ++iy)
            for (int iz = 0; iz < nc; ++iz)
              if (co[((size_t)ix * nc + iy) * nc + iz]) po[((size_t)(ix >> 1) * np + (iy >> 1)) * np + (iz >> 1)] = 1;
      }
      // a level with every box occupied keeps no map (the M2L then has nothing to skip)
      for (int lev = 2; lev <= g.depth; ++lev) {
        const auto& o = g.occ[lev];
        if (std::find(o.begin(), o.end(), (unsigned char)0) == o.end()) continue;
        HIPCHK(h, dmalloc(h, &g.d_occ[lev], o.size()));
        HIPCHK(h, hipMemcpyAsync(g.d_occ[lev], o.data(), o.size(), hipMemcpyHostToDevice, s));
      }
    }
    for (int lev = 2; lev <= g.depth; ++lev) {
      const int nb2 = 1 << lev;
      const auto& ol = g.occ[lev];
      int64_t nocc = 0;
      for (unsigned char v : ol) nocc += v;
      // (target, source) pairs of the parity class windows between occupied boxes, split
      // into far and near
      int64_t far1 = 0, near1 = 0;
      if (nocc < (int64_t)ol.size()) {
        for (int ix = 0; ix < nb2; ++ix)
          for (int iy = 0; iy < nb2; ++iy)
            for (int iz = 0; iz < nb2; ++iz) {
              if (!ol[((size_t)ix * nb2 + iy) * nb2 + iz]) continue;
              for (int dx = -2 - (ix & 1); dx <= 3 - (ix & 1); ++dx)
                for (int dy = -2 - (iy & 1); dy <= 3 - (iy & 1); ++dy)
                  for (int dz = -2 - (iz & 1); dz <= 3 - (iz & 1); ++dz) {
                    const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
                    if (jx < 0 || jy < 0 || jz < 0 || jx >= nb2 || jy >= nb2 || jz >= nb2) continue;
                    if (!ol[((size_t)jx * nb2 + jy) * nb2 + jz]) continue;
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1)
                      ++near1;
                    else
                      ++far1;
                  }
            }
      } else {
        for (int ix = 0; ix < nb2; ++ix)
          for (int dx = -2 - (ix & 1); dx <= 3 - (ix & 1); ++dx) {
            if (ix + dx < 0 || ix + dx >= nb2) continue;
            for (int iy = 0; iy < nb2; ++iy)
              for (int dy = -2 - (iy & 1); dy <= 3 - (iy & 1); ++dy) {
                if (iy + dy < 0 || iy + dy >= nb2) continue;
                for (int iz = 0; iz < nb2; ++iz)
                  for (int dz = -2 - (iz & 1); dz <= 3 - (iz & 1); ++dz) {
                    if (iz + dz < 0 || iz + dz >= nb2) continue;
                    if (std::abs(dx) <= 1 && std::abs(dy) <= 1 && std::abs(dz) <= 1)
                      ++near1;
                    else
                      ++far1;
                  }
              }
          }
      }
      g.far_pairs.push_back(far1);
      g.near_pairs.push_back(near1);
      h->m2l_pairs += far1;
    }
  }
  // complex images (host FP64): every (group, family) fit is independent, one host thread each
  for (auto& g : h->groups) {
    const int l = g.layer;
    const double hleaf = g.side / (1 << g.depth);
    double zlo = std::min(g.zlo, g.lo[2] + 0.5 * hleaf), zhi = std::max(g.zhi, g.lo[2] + g.side - 0.5 * hleaf);
    const double top = med.top(l), bot = med.bottom(l);
    zlo = std::max(zlo, bot + 1e-6);
    zhi = std::min(zhi, top - 1e-6);
    g.fit_zlo = zlo, g.fit_zhi = zhi;
  }
  const auto t_fit0 = std::chrono::steady_clock::now();
  {
    const int nfit = 3 * (int)h->groups.size();
    std::vector<std::string> ferr(nfit);
    std::vector<char> fok(nfit, 0);
    const int nthr = std::max(1, std::min(nfit, std::min(16, (int)std::thread::hardware_concurrency())));
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    for (int t = 0; t < nthr; ++t)
      th.emplace_back([&]() {
        for (;;) {
          const int i = next++;
          if (i >= nfit) break;
          Group& g = h->groups[i / 3];
          const int fam = i % 3;
          fok[i] = same_layer_family(med, g.layer, fam, g.fit_zlo, g.fit_zhi, h->opt.dcim_T1, h->opt.dcim_samples,
                                     h->opt.dcim_svd_tol, g.famA[fam], g.famZ[fam], g.fam_err[fam], ferr[i]);
        }
      });
    for (auto& t : th) t.join();
    for (int i = 0; i < nfit; ++i)
      if (!fok[i]) return fail(h, TEFMM_ERR_DCIM_FIT, "complex-image fit failed: " + ferr[i]);
    for (auto& g : h->groups)
      for (int fam = 0; fam < 3; ++fam) g.has[fam] = !g.famA[fam].empty();
  }
  const double fit_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_fit0).count();
  // reaction keys that would not converge: direct lists and counts
  for (auto& g : h->groups) {
    int rc = reaction_convergence(h, g, lc, s);
    if (rc != TEFMM_OK) return rc;
  }
  // derivative tables
  h->sigma_keys = 0, h->sur_keys = 0, h->som_nodes = 0, h->som_keys = 0;
  for (auto& g : h->groups) {
    int rc = build_tables(h, g, s);
    if (rc != TEFMM_OK) return rc;
  }
  for (int gi = 0; gi < (int)h->groups.size(); ++gi) {
    int rc = build_cross(h, gi, s);
    if (rc != TEFMM_OK) return rc;
  }
  HIPCHK(h, hipEventRecord(e2, s));
  HIPCHK(h, hipEventSynchronize(e2));
  float ms1 = 0, ms2 = 0;
  (void)hipEventElapsedTime(&ms1, e0, e1);
  (void)hipEventElapsedTime(&ms2, e1, e2);
  std::memset(&h->st, 0, sizeof(h->st));
  h->st.t_setup_tree_ms = ms1;
  h->st.t_setup_tables_ms = ms2;
  h->st.t_setup_dcim_ms = fit_ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  int fi = 0;
  for (size_t gi = 0; gi < h->groups.size() && gi < (size_t)MAX_LAYERS; ++gi) {
    auto& g = h->groups[gi];
    h->st.depth[gi] = g.depth;
    for (int fam = 0; fam < 3 && fi < 3 * MAX_LAYERS; ++fam)
      if (g.has[fam]) {
        h->st.n_images[fi] = (int)g.famA[fam].size();
        h->st.dcim_fit_err[fi] = g.fam_err[fam];
        ++fi;
      }
  }
  h->st.n_families = fi;
  h->st.sigma_keys = h->sigma_keys;
  h->st.surrogate_keys = h->sur_keys;
  h->st.sigma_quad_nodes = h->som_nodes;
  h->st.sigma_quad_keys = h->som_keys;
  for (auto& g : h->groups) {
    h->st.sigma_direct_pairs += g.sd_pairs;
    h->st.reaction_keys_forced += g.keys_forced;
    h->st.cross_pairs += g.cross_pairs;
    h->st.cross_pairs_forced += g.cross_forced;
    h->st.n_cross_fits += g.n_cross_fits;
    h->st.cross_fit_err = std::max(h->st.cross_fit_err, g.cross_fit_err);
  }
  h->st.p2p_pairs = h->p2p_pairs;
  h->st.p2p_pairs_same_leaf = h->p2p_same;
  h->st.occupied_leaves = occ_leaves;
  h->st.max_leaf_count = max_leaf;
  h->st.p2p_poly_err = 0;
  if (h->opt.precision == TEFMM_MIXED_FP32)
    for (auto& g : h->groups)
      if (g.np_on) h->st.p2p_poly_err = std::max(h->st.p2p_poly_err, g.np_err);
  h->st.m2l_pairs = h->m2l_pairs;
  h->ready = true;
  h->gen = g_generation++;
  return TEFMM_OK;
}

// Offset splits of the same-layer M2L: shallow trees have few tiles (304 work-
// groups at depth 4), so each tile's offsets are shared by several workgroups.
static int m2l_split(int depth) { return depth <= 4 ? 4 : (depth == 5 ? 2 : 1); }
// The cross-layer lists of the coarse levels hold up to 2 x 196 entries per tile
// on few tiles; their entries are split over this many workgroups.
static constexpr int CROSS_SPLIT = 8;

static int ensure_rhs(tefmm_t h, int nrhs) {
  if (nrhs <= h->nrhs_alloc) return TEFMM_OK;
  dfree(h, h->d_q);
  dfree(h, h->d_phi);
  dfree(h, h->d_phi_near);
  for (auto& g : h->groups) {
    for (auto& p : g.alpha) dfree(h, p);
    for (auto& p : g.beta) dfree(h, p);
    for (auto& p : g.ared) dfree(h, p);
    for (auto& p : g.ared32) dfree(h, p);
    for (auto& p : g.bred) dfree(h, p);
    for (auto& p : g.azred) dfree(h, p);
    for (auto& p : g.bzred) dfree(h, p);
  }
  HIPCHK(h, dmalloc(h, &h->d_q, sizeof(double2) * h->n * nrhs));
  HIPCHK(h, dmalloc(h, &h->d_phi, sizeof(double2) * h->n * nrhs));
  HIPCHK(h, dmalloc(h, &h->d_phi_near, sizeof(double2) * h->n * nrhs));
  dfree(h, h->d_part);
  if (sym_near(h->opt)) {
    int gmax = 1;
    for (auto& g : h->groups) gmax = std::max(gmax, g.p2p_split);
    HIPCHK(h, dmalloc(h, &h->d_part,
                        (h->opt.precision == TEFMM_FP64 ? sizeof(double2) : sizeof(float2)) * 13 * gmax * h->n));
  }
  for (auto& g : h->groups) {
    g.alpha.assign(g.depth + 1, nullptr);
    g.beta.assign(g.depth + 1, nullptr);
    g.ared.assign(g.depth + 1, nullptr);
    g.ared32.assign(g.depth + 1, nullptr);
    g.bred.assign(g.depth + 1, nullptr);
    g.azred.assign(g.depth + 1, nullptr);
    g.bzred.assign(g.depth + 1, nullptr);
    g.nbox.assign(g.depth + 1, 0);
    for (int lev = 2; lev <= g.depth; ++lev) {
      const int64_t nbx = (int64_t)1 << (3 * lev);
      g.nbox[lev] = nbx;
      HIPCHK(h, dmalloc(h, &g.alpha[lev], sizeof(double2) * nbx * h->nC * nrhs));
      HIPCHK(h, dmalloc(h, &g.beta[lev], sizeof(double2) * nbx * h->nC * nrhs));
      if (h->opt.precision == TEFMM_MIXED_FP32)
        HIPCHK(h, dmalloc(h, &g.ared32[lev], sizeof(float2) * nbx * h->nR * nrhs));
      else
        HIPCHK(h, dmalloc(h, &g.ared[lev], sizeof(double2) * nbx * h->nR * nrhs));
      HIPCHK(h, dmalloc(h, &g.bred[lev], sizeof(double2) * nbx * h->nR * nrhs * m2l_split(g.depth)));
      if (h->groups.size() > 1) {
        HIPCHK(h, dmalloc(h, &g.azred[lev], sizeof(double2) * nbx * h->nR * nrhs));
        HIPCHK(h, dmalloc(h, &g.bzred[lev], sizeof(double2) * nbx * h->nR * nrhs * CROSS_SPLIT));
      }
    }
  }
  h->nrhs_alloc = nrhs;
  h->gen = g_generation++;
  return TEFMM_OK;
}

static int check_eval_args(tefmm_t h, const double* q, int nrhs, double* phi) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  if (!h->ready) return fail(h, TEFMM_ERR_STATE, "set_particles has not succeeded");
  if (!q || !phi || nrhs < 1 || nrhs > h->opt.n_rhs_max) return fail(h, TEFMM_ERR_INVALID_ARG, "bad q/phi/n_rhs");
  return TEFMM_OK;
}

// Enqueue one evaluation on stream s (buffers must already be sized for nrhs).
// With timed = false no events are recorded (graph capture).
// The final scaling of the far- and near-field sums into the caller's order (k_finalize).
static int enqueue_finalize(tefmm_t h, int nrhs, double* phi, hipStream_t s) {
  for (auto& g : h->groups) {
    double sr = 1.0 / (4 * PI), si = 0.0;
    if (h->opt.normalization == TEFMM_NORM_PAPER) {  // divide by i k of the target layer
      const double kk = h->med.k[g.layer];
      sr = 0.0, si = -1.0 / kk;
    }
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((g.count + 255) / 256), nrhs), dim3(256), 0, s, h->d_phi,
                       h->d_phi_near, h->d_perm, g.start, g.count, h->n, sr, si, (double2*)phi);
    HIPCHK(h, hipGetLastError());
  }
  return TEFMM_OK;
}

// The charges in tree order (k_gather_q).
static int enqueue_gather_q(tefmm_t h, const double* q, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_q, dim3((unsigned)((h->n + 255) / 256), nrhs), dim3(256), 0, s, (const double2*)q,
                     h->d_perm, h->n, h->d_q);
  HIPCHK(h, hipGetLastError());
  return TEFMM_OK;
}

// far_only: the far field alone (the batched queue of tefmm_evaluate_batch_queue puts the
// charges in tree order before, runs the near fields in one launch and the final scaling
// after): no k_gather_q, no near field, no enqueue_finalize.
static int enqueue_evaluate(tefmm_t h, const double* q, int nrhs, double* phi, hipStream_t s, bool timed,
                            bool far_only = false) {
  if (timed && h->ev.empty()) {
    h->ev.resize(9 * EV_RING);
    for (auto& e : h->ev) HIPCHK(h, hipEventCreate(&e));
  }
  if (!h->s2) {
    HIPCHK(h, hipStreamCreateWithFlags(&h->s2, hipStreamNonBlocking));
    HIPCHK(h, hipEventCreateWithFlags(&h->e_fork, hipEventDisableTiming));
    HIPCHK(h, hipEventCreateWithFlags(&h->e_join, hipEventDisableTiming));
    HIPCHK(h, hipEventCreateWithFlags(&h->e_gfork, hipEventDisableTiming));
    for (int i = 1; i < MAX_LAYERS; ++i) {
      HIPCHK(h, hipStreamCreateWithFlags(&h->sg[i], hipStreamNonBlocking));
      HIPCHK(h, hipEventCreateWithFlags(&h->e_gjoin[i], hipEventDisableTiming));
    }
  }
  // phase events of this evaluation: set ev_next of the ring
  const int evset = h->ev_next;
  if (timed) {
    h->ev_next = (h->ev_next + 1) % EV_RING;
    h->ev_count = std::min(h->ev_count + 1, EV_RING);
  }
#define EVREC(i)                                                 \
  do {                                                           \
    if (timed) HIPCHK(h, hipEventRecord(h->ev[9 * evset + (i)], s)); \
  } while (0)
  const int64_t n = h->n;
  const int p = h->opt.p;
  const bool fp32 = h->opt.precision == TEFMM_MIXED_FP32;
  const bool cross = h->groups.size() > 1;
  double m2l_flops = 0;
  int m2l_launches = 0;
  auto pass_args = [&](const Group& g) {
    PassArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.p = p, pa.nC = h->nC, pa.k = h->med.k[g.layer], pa.n = n, pa.xs = h->d_xs, pa.q = h->d_q, pa.phi = h->d_phi;
    pa.leaf_start = h->d_leaf_start, pa.leaf_count = h->d_leaf_count, pa.leaf_base = g.leaf_base, pa.mi = h->d_mi;
    for (int c = 0; c < 3; ++c) pa.lo[c] = g.lo[c];
    return pa;
  };
  auto reduce_args = [&](const Group& g, int lev, bool z) {
    ReduceArgs ra;
    const double hl = g.side / (1 << lev), kh = h->med.k[g.layer] * hl;
    ra.p = p, ra.nC = h->nC, ra.nR = h->nR, ra.kh2 = kh * kh, ra.mi = h->d_mi, ra.rfull = z ? h->d_rzfull : h->d_rfull;
    ra.scale = h->d_scale, ra.invfact = h->d_invfact;
    ra.nsplit = 1, ra.split_stride = 0, ra.out32 = nullptr;
    return ra;
  };
  EVREC(0);
  if (!far_only) {
    const int rc = enqueue_gather_q(h, q, nrhs, s);
    if (rc != TEFMM_OK) return rc;
  }
  // near field (P2P, Eq. totalinteraction free part) on the second stream: it reads only
  // particles and charges and writes its own sum, so it overlaps the far field.  Under
  // graph capture (the batch, whose geometries are already concurrent branches) it
  // stays on the captured stream.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPCHK(h, hipStreamIsCapturing(s, &cap));
  const bool fork = cap == hipStreamCaptureStatusNone && h->fork_late != 2;
  hipStream_t sn = fork ? h->s2 : s;
  // When the far field is the longer branch (FP64 by default) the upward pass (P2M,
  // M2M and the reduced moments; short, narrow kernels) runs alone and the near field
  // starts beside the M2L; when the near field is the longer one (FP32 by default) it
  // starts at once.  The autotuner measures both.
  const bool late = fork && (h->fork_late < 0 ? !fp32 : h->fork_late == 1);
  auto near_field = [&]() -> int {
    if (fork) {
      HIPCHK(h, hipEventRecord(h->e_fork, s));
      HIPCHK(h, hipStreamWaitEvent(h->s2, h->e_fork, 0));
    }
    if (timed) HIPCHK(h, hipEventRecord(h->ev[9 * evset + 8], sn));
    for (auto& g : h->groups) {
      PassArgs a = pass_args(g);
      a.phi = h->d_phi_near;
      a.nbox_dim = 1 << g.depth, a.h = g.side / (1 << g.depth);
      // one-sided kernel: one target per thread, a block of 64, 128 or 256 threads by the
      // mean occupancy of the occupied leaves (a leaf's targets in as few passes as fill them)
      const int bs = g.mean_occ > 192 ? 256 : g.mean_occ > 64 ? 128 : 64;
      // several charge vectors share each pair kernel, 8 per block
      const bool multi = nrhs > 1;
      if (!multi && h->d_part) {
        // each pair of particles in different leaves once (k_p2p_sym): 1 or 2 targets per
        // lane (4 holds more registers than it saves work), up to G workgroups per leaf over
        // the balanced work list, then one per leaf to gather the source-side sums
        const int tpl = g.p2p_tpl, G = g.p2p_split;
        const dim3 grid2((unsigned)(8 * g.nf_seg_max), 1), grid((unsigned)g.nbox[g.depth], 1);
        const int tp = 64 * tpl;
        if (fp32) {
          void (*fs)(PassArgs, int, int, float2*, NearPoly, const unsigned*, XcdSegs) =
              g.np_on ? (tpl == 1 ? k_p2p_sym<float, 1, 4, true> : tpl == 2 ? k_p2p_sym<float, 2, 4, true>
                                                                           : k_p2p_sym<float, 4, 4, true>)
                      : (tpl == 1 ? k_p2p_sym<float, 1, 4, false> : tpl == 2 ? k_p2p_sym<float, 2, 4, false>
                                                                            : k_p2p_sym<float, 4, 4, false>);
          if (g.nf_seg_max > 0)
            hipLaunchKernelGGL(fs, grid2, dim3(256), 0, sn, a, 1, G, (float2*)h->d_part, g.np,
                               (const unsigned*)g.d_nf_items, g.nf_seg);
          HIPCHK(h, hipGetLastError());
          hipLaunchKernelGGL(k_p2p_sym_gather<float2>, grid, dim3(128), 0, sn, a, 1, tp, G, (const float2*)h->d_part);
        } else {
          void (*fs)(PassArgs, int, int, double2*, NearPoly, const unsigned*, XcdSegs) =
              tpl == 1 ? k_p2p_sym<double, 1, 4, false> : k_p2p_sym<double, 2, 4, false>;
          if (g.nf_seg_max > 0)
            hipLaunchKernelGGL(fs, grid2, dim3(256), 0, sn, a, 1, G, (double2*)h->d_part, g.np,
                               (const unsigned*)g.d_nf_items, g.nf_seg);
          HIPCHK(h, hipGetLastError());
          hipLaunchKernelGGL(k_p2p_sym_gather<double2>, grid, dim3(128), 0, sn, a, 1, tp, G, (const double2*)h->d_part);
        }
        HIPCHK(h, hipGetLastError());
        continue;
      }
      const dim3 grid((unsigned)(8 * g.p2p_seg_max), multi ? (nrhs + 7) / 8 : 1);
      void (*fn)(PassArgs, int, NearPoly, const unsigned*, XcdSegs) = nullptr;
      if (fp32 && g.np_on)
        fn = bs == 256   ? (multi ? k_p2p<float, 256, 8, true> : k_p2p<float, 256, 1, true>)
             : bs == 128 ? (multi ? k_p2p<float, 128, 8, true> : k_p2p<float, 128, 1, true>)
                         : (multi ? k_p2p<float, 64, 8, true> : k_p2p<float, 64, 1, true>);
      else if (fp32)
        fn = bs == 256   ? (multi ? k_p2p<float, 256, 8, false> : k_p2p<float, 256, 1, false>)
             : bs == 128 ? (multi ? k_p2p<float, 128, 8, false> : k_p2p<float, 128, 1, false>)
                         : (multi ? k_p2p<float, 64, 8, false> : k_p2p<float, 64, 1, false>);
      else
        fn = bs == 256   ? (multi ? k_p2p<double, 256, 8, false> : k_p2p<double, 256, 1, false>)
             : bs == 128 ? (multi ? k_p2p<double, 128, 8, false> : k_p2p<double, 128, 1, false>)
                         : (multi ? k_p2p<double, 64, 8, false> : k_p2p<double, 64, 1, false>);
      if (g.p2p_seg_max > 0)
        hipLaunchKernelGGL(fn, grid, dim3(bs), 0, sn, a, nrhs, g.np, (const unsigned*)g.d_p2p_items, g.p2p_seg);
      HIPCHK(h, hipGetLastError());
    }
    if (timed) HIPCHK(h, hipEventRecord(h->ev[9 * evset + 6], sn));
    if (fork) HIPCHK(h, hipEventRecord(h->e_join, h->s2));
    return TEFMM_OK;
  };
  if (!late && !far_only) {
    const int rc = near_field();
    if (rc != TEFMM_OK) return rc;
  }
  // P2M at the leaves (Sec. 3.1)
  for (auto& g : h->groups) {
    const int H = g.depth;
    PassArgs a = pass_args(g);
    a.nbox_dim = 1 << H, a.h = g.side / (1 << H), a.alpha = g.alpha[H], a.rhs_stride = g.nbox[H] * h->nC;
    const size_t lds = sizeof(double) * 64 * 3 * (p + 1) + sizeof(double2) * 64;
    hipLaunchKernelGGL(k_p2m, dim3((unsigned)g.nbox[H], nrhs), dim3(64), lds, s, a);
    HIPCHK(h, hipGetLastError());
  }
  EVREC(1);
  // M2M, then the reduced moments of every level (x-reduced for the same-layer
  // translations, z-reduced for the cross-layer ones)
  for (auto& g : h->groups) {
    const int H = g.depth;
    for (int lev = H - 1; lev >= 2; --lev) {
      PassArgs a = pass_args(g);
      a.nbox_dim = 1 << lev, a.alpha = g.alpha[lev], a.rhs_stride = g.nbox[lev] * h->nC;
      a.alpha_child = g.alpha[lev + 1], a.rhs_stride_child = g.nbox[lev + 1] * h->nC;
      // waves per parent (each takes 8 / W children).  Beside the near field, one: a
      // wider workgroup waits for a CU with that many free wave slots, which the near
      // field's workgroups hold until they end.  Otherwise the most whose two buffers
      // fit 96 KiB.
      int W = fork && !late ? 1 : 8;
      while (W > 1 && (size_t)W * 2 * sizeof(double2) * h->nC + sizeof(int) * h->nC > 96 * 1024) W /= 2;
      const size_t lds = (size_t)W * 2 * sizeof(double2) * h->nC + sizeof(int) * h->nC;
      HIPCHK(h, hipFuncSetAttribute((const void*)k_m2m, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(k_m2m, dim3((unsigned)g.nbox[lev], nrhs), dim3(64 * W), lds, s, a);
      HIPCHK(h, hipGetLastError());
    }
    for (int lev = 2; lev <= H; ++lev) {
      ReduceArgs ra = reduce_args(g, lev, false);
      ra.in = g.alpha[lev], ra.out = g.ared[lev], ra.out32 = g.ared32[lev];
      ra.in_stride = g.nbox[lev] * h->nC, ra.out_stride = g.nbox[lev] * h->nR;
      hipLaunchKernelGGL(k_reduce, dim3((unsigned)g.nbox[lev], nrhs), dim3(64), sizeof(double2) * h->nC, s, ra);
      HIPCHK(h, hipGetLastError());
      if (cross) {
        ReduceArgs rz = reduce_args(g, lev, true);
        rz.in = g.alpha[lev], rz.out = g.azred[lev];
        rz.in_stride = g.nbox[lev] * h->nC, rz.out_stride = g.nbox[lev] * h->nR;
        hipLaunchKernelGGL(k_reduce_z, dim3((unsigned)g.nbox[lev], nrhs), dim3(64), sizeof(double2) * h->nC, s, rz);
        HIPCHK(h, hipGetLastError());
      }
    }
  }
  EVREC(2);
  if (late && !far_only) {
    const int rc = near_field();
    if (rc != TEFMM_OK) return rc;
  }
  // M2L: same-layer families, then cross-layer components (Algorithm 2).  The groups'
  // launches are independent (each writes only its own locals): with several groups
  // and no graph capture, group gi > 0 runs on stream sg[gi], joined before the locals.
  const int ngr = (int)h->groups.size();
  const bool gfork = cap == hipStreamCaptureStatusNone && ngr > 1;
  if (gfork) {
    HIPCHK(h, hipEventRecord(h->e_gfork, s));
    for (int gi = 1; gi < ngr; ++gi) HIPCHK(h, hipStreamWaitEvent(h->sg[gi], h->e_gfork, 0));
  }
  for (int gi = 0; gi < ngr; ++gi) {
    Group& g = h->groups[gi];
    const hipStream_t sm = (gfork && gi > 0) ? h->sg[gi] : s;
    const int H = g.depth;
    M2LArgs m;
    std::memset(&m, 0, sizeof(m));
    m.nR = h->nR, m.nRs = h->nRs, m.nKB = h->nKB, m.nRB = h->nRB, m.nG = h->nG, m.p = p, m.P2 = 2 * p + 1;
    m.rmi = h->d_rmi, m.gpad = h->d_gpad;
    m.nlev = H - 1;
    for (int lev = 2; lev <= H; ++lev) {
      M2LLevel& L = m.lev[lev - 2];
      L.n = 1 << lev, L.leaf = lev == H;
      L.near_fd = g.has[2], L.near_s = g.has[0] || g.has[1];
      L.a = g.ared[lev], L.a32 = g.ared32[lev], L.b = g.bred[lev], L.rhs_stride = g.nbox[lev] * h->nR;
      L.split_stride = g.nbox[lev] * h->nR * h->nrhs_alloc;
      L.Tfd = g.Tfd[lev], L.TS = g.TS[lev], L.Tfd32 = g.Tfd32[lev], L.TS32 = g.TS32[lev];
      L.occ = g.d_occ[lev];
    }
    m.ncb = h->m2l_ncb ? h->m2l_ncb : h->opt.m2l_tile;
    m.nsplit = m2l_split(H);
    m.ksplit = 1;
    HIPCHK(h, launch_m2l(m, nrhs, fp32, sm));
    const double per = 8.0 * (double)h->nR * (double)h->nR;
    for (int lev = 2; lev <= H; ++lev) {
      const int64_t far = g.far_pairs[lev - 2], nr = g.near_pairs[lev - 2];
      const bool sig = g.has[0] || g.has[1];
      double pairs = (double)far + (sig ? (double)far : 0.0);
      if (lev == H) pairs += (g.has[2] ? (double)nr : 0.0) + (sig ? (double)nr : 0.0);
      m2l_flops += per * pairs * nrhs;
    }
    ++m2l_launches;
    if (g.has_cross) {
      M2LCrossArgs c;
      std::memset(&c, 0, sizeof(c));
      c.nR = h->nR, c.nRs = h->nRs, c.nKB = h->nKB, c.nRB = h->nRB, c.nG = h->nG, c.p = p, c.P2 = 2 * p + 1;
      c.rzmi = h->d_rzmi, c.gpadz = h->d_gpadz;
      c.nlev = H - 1;
      c.nsplit = CROSS_SPLIT;
      for (int lev = 2; lev <= H; ++lev) {
        M2LCrossLevel& L = c.lev[lev - 2];
        L.n = 1 << lev;
        L.list_start = g.xlist_start[lev], L.list = g.xlist[lev];
        L.b = g.bzred[lev], L.rhs_stride = g.nbox[lev] * h->nR;
        L.split_stride = g.nbox[lev] * h->nR * h->nrhs_alloc;
        L.T[0] = g.XT0[lev], L.T[1] = g.XT1[lev], L.T32[0] = g.XT032[lev], L.T32[1] = g.XT132[lev];
        for (size_t sg = 0; sg < h->groups.size() && sg < (size_t)MAX_LAYERS; ++sg) {
          L.asrc[sg] = h->groups[sg].azred[lev];
          L.src_stride[sg] = h->groups[sg].nbox[lev] * h->nR;
        }
      }
      HIPCHK(h, launch_m2l_cross(c, nrhs, fp32, sm));
      m2l_flops += g.cross_flops_per_rhs * nrhs;
      ++m2l_launches;
    }
    if (gfork && gi > 0) HIPCHK(h, hipEventRecord(h->e_gjoin[gi], sm));
  }
  if (gfork)
    for (int gi = 1; gi < ngr; ++gi) HIPCHK(h, hipStreamWaitEvent(s, h->e_gjoin[gi], 0));
  EVREC(3);
  // locals: expansion of the reduced sets, cross-layer part added, then L2L
  for (auto& g : h->groups) {
    const int H = g.depth;
    for (int lev = 2; lev <= H; ++lev) {
      ReduceArgs ra = reduce_args(g, lev, false);
      ra.in = g.bred[lev], ra.out = g.beta[lev];
      ra.in_stride = g.nbox[lev] * h->nR, ra.out_stride = g.nbox[lev] * h->nC;
      ra.nsplit = m2l_split(H), ra.split_stride = g.nbox[lev] * h->nR * h->nrhs_alloc;
      hipLaunchKernelGGL(k_expand, dim3((unsigned)g.nbox[lev], nrhs), dim3(64), sizeof(double2) * h->nC, s, ra);
      HIPCHK(h, hipGetLastError());
      if (g.has_cross) {
        ReduceArgs rz = reduce_args(g, lev, true);
        rz.in = g.bzred[lev], rz.out = g.beta[lev];
        rz.in_stride = g.nbox[lev] * h->nR, rz.out_stride = g.nbox[lev] * h->nC;
        rz.nsplit = CROSS_SPLIT, rz.split_stride = g.nbox[lev] * h->nR * h->nrhs_alloc;
        hipLaunchKernelGGL(k_expand_z_add, dim3((unsigned)g.nbox[lev], nrhs), dim3(64), sizeof(double2) * h->nC, s,
                           rz);
        HIPCHK(h, hipGetLastError());
      }
      if (lev >= 3) {
        PassArgs a = pass_args(g);
        a.nbox_dim = 1 << lev, a.beta = g.beta[lev], a.rhs_stride = g.nbox[lev] * h->nC;
        a.beta_parent = g.beta[lev - 1], a.rhs_stride_parent = g.nbox[lev - 1] * h->nC;
        hipLaunchKernelGGL(k_l2l, dim3((unsigned)g.nbox[lev], nrhs), dim3(64), (2 * sizeof(double2) + sizeof(int)) * h->nC,
                           s, a);
        HIPCHK(h, hipGetLastError());
      }
    }
  }
  EVREC(4);
  for (auto& g : h->groups) {
    const int H = g.depth;
    PassArgs a = pass_args(g);
    a.nbox_dim = 1 << H, a.h = g.side / (1 << H), a.beta = g.beta[H], a.rhs_stride = g.nbox[H] * h->nC;
    const size_t lds = sizeof(double2) * h->nC;
    hipLaunchKernelGGL(k_l2p, dim3((unsigned)g.nbox[H], nrhs), dim3(64), lds, s, a);
    HIPCHK(h, hipGetLastError());
  }
  // near-interface Sigma pairs evaluated directly (added to the far-field sums)
  for (auto& g : h->groups) {
    if (!g.sd_ntgt) continue;
    SigmaDirectArgs sd;
    sd.xs = h->d_xs, sd.n = n, sd.q = h->d_q, sd.phi = h->d_phi;
    sd.leaf_start = h->d_leaf_start, sd.leaf_count = h->d_leaf_count, sd.leaf_base = g.leaf_base;
    sd.tgt = g.d_sd_tgt, sd.src_start = g.d_sd_start, sd.src = g.d_sd_src, sd.img = g.d_sd_img;
    sd.nup = g.sd_nup, sd.ndn = g.sd_ndn;
    sd.two_dl = g.layer < h->med.L ? 2 * h->med.d[g.layer] : 0.0;
    sd.two_dt = g.layer > 0 ? 2 * h->med.d[g.layer - 1] : 0.0;
    sd.k = h->med.k[g.layer];
    hipLaunchKernelGGL(k_sigma_direct, dim3((unsigned)g.sd_ntgt, nrhs), dim3(128), 0, s, sd);
    HIPCHK(h, hipGetLastError());
  }
  EVREC(5);
  h->st.m2l_flops = m2l_flops;
  h->st.m2l_launches = m2l_launches;
  h->st.n_rhs = nrhs;
  if (far_only) return TEFMM_OK;
  if (fork) HIPCHK(h, hipStreamWaitEvent(s, h->e_join, 0));
  const int rc = enqueue_finalize(h, nrhs, phi, s);
  if (rc != TEFMM_OK) return rc;
  EVREC(7);
#undef EVREC
  return TEFMM_OK;
}

extern "C" int tefmm_evaluate(tefmm_t h, const double* q, int nrhs, double* phi, void* stream) {
  int rc = check_eval_args(h, q, nrhs, phi);
  if (rc != TEFMM_OK) return rc;
  rc = ensure_rhs(h, nrhs);
  if (rc != TEFMM_OK) return rc;
  return enqueue_evaluate(h, q, nrhs, phi, (hipStream_t)stream, true);
}

// ---------------------------------------------------------------------------
// GMRES(m) on the handle's operator: (I - tau G) x = b, G the evaluation of (1) with
// one charge vector (the Foldy-Lax system of point scatterers of strength tau in the
// layered medium, a second-kind integral equation discretised at the particles).
// Classical Gram-Schmidt applied twice per step (two multi-column dot products and
// updates per step), Givens rotations on the host, restart after m steps with the
// true residual recomputed.  Every vector operation is a HIP kernel on `stream`;
// the host only handles the (m+1) x m Hessenberg matrix.
// ---------------------------------------------------------------------------
extern "C" int tefmm_gmres(tefmm_t h, double tau_re, double tau_im, const double* b, double* x, int x0_given,
                           int restart, int max_iter, double tol, void* stream, tefmm_gmres_info* info) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  if (!h->ready) return fail(h, TEFMM_ERR_STATE, "set_particles has not succeeded");
  if (!b || !x || restart < 1 || restart > 200 || max_iter < 1 || !(tol > 0))
    return fail(h, TEFMM_ERR_INVALID_ARG, "tefmm_gmres: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_rhs(h, 1);
  if (rc != TEFMM_OK) return rc;
  const int64_t n = h->n;
  const int m = restart;
  const unsigned nb = (unsigned)((n + 255) / 256);
  double2 *V = nullptr, *w = nullptr, *gv = nullptr, *part = nullptr, *dh = nullptr;
  HIPCHK(h, dmalloc(h, &V, sizeof(double2) * (size_t)n * (m + 1)));
  HIPCHK(h, dmalloc(h, &w, sizeof(double2) * (size_t)n));
  HIPCHK(h, dmalloc(h, &gv, sizeof(double2) * (size_t)n));
  HIPCHK(h, dmalloc(h, &part, sizeof(double2) * (size_t)GM_BLOCKS * (m + 1)));
  HIPCHK(h, dmalloc(h, &dh, sizeof(double2) * (size_t)(m + 1)));
  auto cleanup = [&]() {
    dfree(h, V), dfree(h, w), dfree(h, gv), dfree(h, part), dfree(h, dh);
  };
  const cplx tau(tau_re, tau_im);
  auto d2 = [](cplx c) { return make_double2(c.real(), c.imag()); };
  // y = conj(V[0..ncol))^T v on the host
  auto dots = [&](const double2* Vb, int ncol, const double2* v, std::vector<cplx>& out) -> int {
    hipLaunchKernelGGL(k_gm_multidot, dim3(GM_BLOCKS), dim3(256), 0, s, Vb, (int64_t)n, ncol, v, n, part);
    HIPCHK(h, hipGetLastError());
    hipLaunchKernelGGL(k_gm_reduce, dim3(ncol), dim3(256), 0, s, part, GM_BLOCKS, dh);
    HIPCHK(h, hipGetLastError());
    std::vector<double2> tmp(ncol);
    HIPCHK(h, hipMemcpyAsync(tmp.data(), dh, sizeof(double2) * ncol, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    out.resize(ncol);
    for (int c = 0; c < ncol; ++c) out[c] = cplx(tmp[c].x, tmp[c].y);
    return TEFMM_OK;
  };
  // out = v - tau G v
  int matvecs = 0;
  auto apply = [&](const double2* v, double2* out) -> int {
    int r2 = enqueue_evaluate(h, (const double*)v, 1, (double*)gv, s, false);
    if (r2 != TEFMM_OK) return r2;
    HIPCHK(h, hipMemcpyAsync(out, v, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_gm_axpby, dim3(nb), dim3(256), 0, s, d2(-tau), gv, make_double2(1.0, 0.0), out, n);
    HIPCHK(h, hipGetLastError());
    ++matvecs;
    return TEFMM_OK;
  };
  auto norm = [&](const double2* v, double* out) -> int {
    std::vector<cplx> d;
    int r2 = dots(v, 1, v, d);
    *out = std::sqrt(std::max(0.0, d[0].real()));
    return r2;
  };
  auto run = [&]() -> int {
    const double2* bb = (const double2*)b;
    double2* xx = (double2*)x;
    double bnorm = 0;
    int r2 = norm(bb, &bnorm);
    if (r2 != TEFMM_OK) return r2;
    if (!(bnorm > 0)) bnorm = 1.0;
    // r = b - A x (x = 0 unless given); r kept in column 0 of V
    if (x0_given) {
      if ((r2 = apply(xx, w)) != TEFMM_OK) return r2;
      HIPCHK(h, hipMemcpyAsync(V, bb, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(k_gm_axpby, dim3(nb), dim3(256), 0, s, make_double2(-1.0, 0.0), w, make_double2(1.0, 0.0),
                         V, n);
      HIPCHK(h, hipGetLastError());
    } else {
      HIPCHK(h, hipMemsetAsync(xx, 0, sizeof(double2) * n, s));
      HIPCHK(h, hipMemcpyAsync(V, bb, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
    }
    double beta = 0;
    if ((r2 = norm(V, &beta)) != TEFMM_OK) return r2;
    int it = 0;
    double est = beta / bnorm;
    std::vector<cplx> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hc, hc2;
    while (est > tol && it < max_iter) {
      hipLaunchKernelGGL(k_gm_axpby, dim3(nb), dim3(256), 0, s, make_double2(1.0 / beta, 0.0), V,
                         make_double2(0.0, 0.0), V, n);
      HIPCHK(h, hipGetLastError());
      std::fill(g.begin(), g.end(), cplx(0, 0));
      std::fill(H.begin(), H.end(), cplx(0, 0));
      g[0] = beta;
      int j = 0;
      for (; j < m && it < max_iter; ++j, ++it) {
        if ((r2 = apply(V + (size_t)j * n, w)) != TEFMM_OK) return r2;
        // classical Gram-Schmidt, twice
        for (int pass = 0; pass < 2; ++pass) {
          if ((r2 = dots(V, j + 1, w, hc)) != TEFMM_OK) return r2;
          std::vector<double2> hd(j + 1);
          for (int i = 0; i <= j; ++i) hd[i] = d2(hc[i]), H[(size_t)i * m + j] += hc[i];
          HIPCHK(h, hipMemcpyAsync(dh, hd.data(), sizeof(double2) * (j + 1), hipMemcpyHostToDevice, s));
          hipLaunchKernelGGL(k_gm_update, dim3(nb), dim3(256), 0, s, V, (int64_t)n, j + 1, dh, -1.0, w, n);
          HIPCHK(h, hipGetLastError());
        }
        double hn = 0;
        if ((r2 = norm(w, &hn)) != TEFMM_OK) return r2;
        H[(size_t)(j + 1) * m + j] = hn;
        if (hn > 0) {
          hipLaunchKernelGGL(k_gm_axpby, dim3(nb), dim3(256), 0, s, make_double2(1.0 / hn, 0.0), w,
                             make_double2(0.0, 0.0), V + (size_t)(j + 1) * n, n);
          HIPCHK(h, hipGetLastError());
        }
        // previous rotations on column j, then this step's
        for (int i = 0; i < j; ++i) {
          const cplx a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
          H[(size_t)i * m + j] = std::conj(cs[i]) * a + std::conj(sn[i]) * c;
          H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
        }
        const cplx a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
        const double r = std::sqrt(std::norm(a) + std::norm(c));
        cs[j] = r > 0 ? a / r : cplx(1, 0);
        sn[j] = r > 0 ? c / r : cplx(0, 0);
        H[(size_t)j * m + j] = r;
        H[(size_t)(j + 1) * m + j] = 0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = std::conj(cs[j]) * g[j];
        est = std::abs(g[j + 1]) / bnorm;
        if (est <= tol || !(hn > 0)) {
          ++j, ++it;
          break;
        }
      }
      // y = H^-1 g (upper triangular j x j), x += V y
      std::vector<cplx> y(j);
      for (int i = j - 1; i >= 0; --i) {
        cplx acc = g[i];
        for (int k2 = i + 1; k2 < j; ++k2) acc -= H[(size_t)i * m + k2] * y[k2];
        y[i] = acc / H[(size_t)i * m + i];
      }
      std::vector<double2> yd(j);
      for (int i = 0; i < j; ++i) yd[i] = d2(y[i]);
      HIPCHK(h, hipMemcpyAsync(dh, yd.data(), sizeof(double2) * j, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_gm_update, dim3(nb), dim3(256), 0, s, V, (int64_t)n, j, dh, 1.0, xx, n);
      HIPCHK(h, hipGetLastError());
      // true residual for the restart (and the report)
      if ((r2 = apply(xx, w)) != TEFMM_OK) return r2;
      HIPCHK(h, hipMemcpyAsync(V, bb, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(k_gm_axpby, dim3(nb), dim3(256), 0, s, make_double2(-1.0, 0.0), w, make_double2(1.0, 0.0),
                         V, n);
      HIPCHK(h, hipGetLastError());
      if ((r2 = norm(V, &beta)) != TEFMM_OK) return r2;
      est = beta / bnorm;
    }
    if (info) {
      info->iterations = it;
      info->matvecs = matvecs;
      info->rel_residual = est;
      info->converged = est <= tol;
    }
    return TEFMM_OK;
  };
  rc = run();
  HIPCHK(h, hipStreamSynchronize(s));
  cleanup();
  return rc;
}

static void batch_clear(tefmm_t h, tefmm_ctx::Batch& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr, b.graph = nullptr;
  b.hs.clear(), b.gens.clear(), b.q.clear(), b.phi.clear(), b.nrhs.clear();
  dfree(h, b.d_geo), dfree(h, b.d_start), dfree(h, b.d_ctr), dfree(h, b.d_err);
  b.queue = false;
}

static void batch_destroy(tefmm_t h, tefmm_ctx::Batch& b) {
  batch_clear(h, b);
  for (auto& e : b.ev) (void)hipEventDestroy(e);
  if (b.ev_nf) (void)hipEventDestroy(b.ev_nf);
  if (b.ev_q) (void)hipEventDestroy(b.ev_q);
  if (b.ev_ff) (void)hipEventDestroy(b.ev_ff);
  for (auto& st : b.side) (void)hipStreamDestroy(st);
  if (b.origin) (void)hipStreamDestroy(b.origin);
  if (b.nf) (void)hipStreamDestroy(b.nf);
  b.ev.clear(), b.side.clear(), b.origin = nullptr, b.nf = nullptr, b.ev_nf = nullptr;
  b.ev_q = nullptr, b.ev_ff = nullptr;
}

// Whether the geometries' near fields can run as one queue: one charge vector each, one
// precision, the symmetric near field with at most 2 targets per lane.
static bool queue_eligible(tefmm_t* hs, int n_geom, const int* nrhs, std::string& why) {
  for (int g = 0; g < n_geom; ++g) {
    tefmm_t h = hs[g];
    if (nrhs[g] != 1) return why = "several charge vectors", false;
    if (h->opt.precision != hs[0]->opt.precision) return why = "mixed precisions", false;
    if (!h->d_part) return why = "the one-sided near field (p2p_targets = -1)", false;
    for (auto& gr : h->groups)
      if (gr.p2p_tpl > 2) return why = "4 targets per lane", false;
  }
  return true;
}

// Batched evaluation (E2): the geometries' evaluation sequences are captured once
// into a HIP graph, each on its own stream branch so that independent geometries
// run concurrently, and the graph is replayed while the argument lists match.
extern "C" int tefmm_evaluate_batch(tefmm_t* hs, int n_geom, const double* const* q, const int* nrhs,
                                    double* const* phi, void* stream) {
  if (!hs || n_geom < 1 || !q || !nrhs || !phi || !hs[0]) return TEFMM_ERR_INVALID_ARG;
  tefmm_t h0 = hs[0];
  for (int g = 0; g < n_geom; ++g) {
    if (!hs[g]) return fail(h0, TEFMM_ERR_INVALID_ARG, "null handle in batch");
    for (int g2 = 0; g2 < g; ++g2)
      if (hs[g2] == hs[g]) return fail(h0, TEFMM_ERR_INVALID_ARG, "a handle appears twice in the batch");
    int rc = check_eval_args(hs[g], q[g], nrhs[g], phi[g]);
    if (rc != TEFMM_OK) return fail(h0, rc, "geometry " + std::to_string(g) + ": " + hs[g]->err);
    rc = ensure_rhs(hs[g], nrhs[g]);
    if (rc != TEFMM_OK) return fail(h0, rc, "geometry " + std::to_string(g) + ": " + hs[g]->err);
  }
  tefmm_ctx::Batch& b = h0->batch;
  bool same = b.exec && (int)b.hs.size() == n_geom && !b.queue;
  for (int g = 0; same && g < n_geom; ++g)
    same = b.hs[g] == hs[g] && b.gens[g] == hs[g]->gen && b.q[g] == q[g] && b.phi[g] == phi[g] &&
           b.nrhs[g] == nrhs[g];
  if (!same) {
    batch_clear(h0, b);
    if (!b.origin) HIPCHK(h0, hipStreamCreateWithFlags(&b.origin, hipStreamNonBlocking));
    while ((int)b.side.size() < n_geom) {
      hipStream_t st;
      HIPCHK(h0, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b.side.push_back(st);
    }
    while ((int)b.ev.size() < n_geom + 1) {
      hipEvent_t e;
      HIPCHK(h0, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b.ev.push_back(e);
    }
    HIPCHK(h0, hipStreamBeginCapture(b.origin, hipStreamCaptureModeThreadLocal));
    int rc = TEFMM_OK;
    hipError_t e = hipEventRecord(b.ev[n_geom], b.origin);
    for (int g = 0; g < n_geom && rc == TEFMM_OK && e == hipSuccess; ++g) {
      e = hipStreamWaitEvent(b.side[g], b.ev[n_geom], 0);
      if (e != hipSuccess) break;
      rc = enqueue_evaluate(hs[g], q[g], nrhs[g], phi[g], b.side[g], false);
      if (rc != TEFMM_OK) break;
      e = hipEventRecord(b.ev[g], b.side[g]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b.origin, b.ev[g], 0);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(b.origin, &graph);
    if (rc != TEFMM_OK || e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != TEFMM_OK) return fail(h0, rc, "capture: " + std::string(h0->err));
      return fail(h0, TEFMM_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b.graph = graph;
    HIPCHK(h0, hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    b.hs.assign(hs, hs + n_geom);
    b.gens.clear();
    for (int g = 0; g < n_geom; ++g) b.gens.push_back(hs[g]->gen);
    b.q.assign(q, q + n_geom);
    b.phi.assign(phi, phi + n_geom);
    b.nrhs.assign(nrhs, nrhs + n_geom);
  }
  HIPCHK(h0, hipGraphLaunch(b.exec, (hipStream_t)stream));
  return TEFMM_OK;
}

// Batched evaluation with the near fields of all geometries in one persistent launch
// (k_nf_queue): the charges of every geometry are put in tree order on the caller's
// stream, then the far fields (a graph with one branch per geometry, captured once) and
// the queue run side by side, then every geometry's final scaling follows both.
extern "C" int tefmm_evaluate_batch_queue(tefmm_t* hs, int n_geom, const double* const* q, const int* nrhs,
                                          double* const* phi, void* stream) {
  if (!hs || n_geom < 1 || !q || !nrhs || !phi || !hs[0]) return TEFMM_ERR_INVALID_ARG;
  tefmm_t h0 = hs[0];
  for (int g = 0; g < n_geom; ++g) {
    if (!hs[g]) return fail(h0, TEFMM_ERR_INVALID_ARG, "null handle in batch");
    for (int g2 = 0; g2 < g; ++g2)
      if (hs[g2] == hs[g]) return fail(h0, TEFMM_ERR_INVALID_ARG, "a handle appears twice in the batch");
    int rc = check_eval_args(hs[g], q[g], nrhs[g], phi[g]);
    if (rc != TEFMM_OK) return fail(h0, rc, "geometry " + std::to_string(g) + ": " + hs[g]->err);
    rc = ensure_rhs(hs[g], nrhs[g]);
    if (rc != TEFMM_OK) return fail(h0, rc, "geometry " + std::to_string(g) + ": " + hs[g]->err);
  }
  std::string why;
  if (!queue_eligible(hs, n_geom, nrhs, why))
    return fail(h0, TEFMM_ERR_UNSUPPORTED, "near-field queue: " + why + " (use tefmm_evaluate_batch)");
  hipStream_t s = (hipStream_t)stream;
  tefmm_ctx::Batch& b = h0->batch;
  // the work list (one entry per geometry and layer group) is uploaded when the handle
  // list or a handle's buffers changed
  bool same = b.queue && (int)b.hs.size() == n_geom;
  for (int g = 0; same && g < n_geom; ++g) same = b.hs[g] == hs[g] && b.gens[g] == hs[g]->gen;
  while ((int)b.side.size() < n_geom) {
    hipStream_t st;
    HIPCHK(h0, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    b.side.push_back(st);
  }
  while ((int)b.ev.size() < n_geom + 1) {
    hipEvent_t e;
    HIPCHK(h0, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b.ev.push_back(e);
  }
  if (!same) {
    batch_clear(h0, b);
    if (!b.nf) HIPCHK(h0, hipStreamCreateWithFlags(&b.nf, hipStreamNonBlocking));
    if (!b.ev_nf) HIPCHK(h0, hipEventCreateWithFlags(&b.ev_nf, hipEventDisableTiming));
    std::vector<NFQueueGeom> geo;
    // items: (estimated cost, geometry << 24 | work index); pair items sorted longest
    // first, so that the queue's tail holds the short ones; empty leaves have no item
    std::vector<std::pair<double, unsigned>> pitems;
    std::vector<unsigned> gitems;
    for (int g = 0; g < n_geom; ++g) {
      tefmm_t h = hs[g];
      for (auto& gr : h->groups) {
        NFQueueGeom e;
        std::memset(&e, 0, sizeof(e));
        PassArgs& a = e.a;
        a.p = h->opt.p, a.nC = h->nC, a.k = h->med.k[gr.layer], a.n = h->n, a.xs = h->d_xs, a.q = h->d_q;
        a.phi = h->d_phi_near, a.leaf_start = h->d_leaf_start, a.leaf_count = h->d_leaf_count;
        a.leaf_base = gr.leaf_base, a.mi = h->d_mi;
        for (int c = 0; c < 3; ++c) a.lo[c] = gr.lo[c];
        a.nbox_dim = 1 << gr.depth, a.h = gr.side / (1 << gr.depth);
        const int nl = 1 << (3 * gr.depth);
        e.np = gr.np, e.part = h->d_part, e.G = gr.p2p_split, e.tpl = gr.p2p_tpl;
        e.poly = h->opt.precision == TEFMM_MIXED_FP32 && gr.np_on ? 1 : 0;
        const int gi = (int)geo.size(), nb = 1 << gr.depth, tp = 64 * e.tpl;
        const int* lcg = h->leaf_count_host.data() + gr.leaf_base;
        int np = 0;
        for (int leaf = 0; leaf < nl; ++leaf) {
          const int cnt = lcg[leaf];
          if (!cnt) continue;
          gitems.push_back((unsigned)gi << 24 | (unsigned)leaf);
          // sources of a pass: the leaf itself and its forward half of neighbours
          const int ix = leaf / (nb * nb), iy = (leaf / nb) % nb, iz = leaf % nb;
          int64_t src = cnt;
          for (int dx = 0; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dz = -1; dz <= 1; ++dz) {
                const bool fwd = dx == 1 || (dx == 0 && dy == 1) || (dx == 0 && dy == 0 && dz == 1);
                const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
                if (!fwd || jx >= nb || jy < 0 || jy >= nb || jz < 0 || jz >= nb) continue;
                src += lcg[((int64_t)jx * nb + jy) * nb + jz];
              }
          for (int half = 0; half < e.G && half * tp < cnt; ++half) {
            int64_t tg = 0;
            for (int c0 = half * tp; c0 < cnt; c0 += e.G * tp) tg += std::min(tp, cnt - c0);
            pitems.push_back({(double)tg * (double)src, (unsigned)gi << 24 | (unsigned)(leaf * e.G + half)});
            ++np;
          }
        }
        e.p2p_items = np, e.gather_items = 0;
        geo.push_back(e);
      }
    }
    const int ng = (int)geo.size();
    if (ng > 255 || pitems.size() > 0x7fffffffu)
      return fail(h0, TEFMM_ERR_UNSUPPORTED, "near-field queue: at most 255 layer groups in a batch");
    std::stable_sort(pitems.begin(), pitems.end(),
                     [](const std::pair<double, unsigned>& x, const std::pair<double, unsigned>& y) {
                       return x.first > y.first;
                     });
    std::vector<unsigned> starts;  // the pair items, then the gather items
    for (auto& it : pitems) starts.push_back(it.second);
    starts.insert(starts.end(), gitems.begin(), gitems.end());
    b.n_p2p = (int)pitems.size(), b.n_gather = (int)gitems.size();
    HIPCHK(h0, dmalloc(h0, &b.d_geo, sizeof(NFQueueGeom) * ng));
    HIPCHK(h0, dmalloc(h0, &b.d_start, sizeof(unsigned) * std::max<size_t>(starts.size(), 1)));
    HIPCHK(h0, dmalloc(h0, &b.d_ctr, sizeof(unsigned) * (1 + ng)));
    HIPCHK(h0, dmalloc(h0, &b.d_err, sizeof(int)));
    HIPCHK(h0, hipMemcpy(b.d_geo, geo.data(), sizeof(NFQueueGeom) * ng, hipMemcpyHostToDevice));
    if (!starts.empty())
      HIPCHK(h0, hipMemcpy(b.d_start, starts.data(), sizeof(unsigned) * starts.size(), hipMemcpyHostToDevice));
    HIPCHK(h0, hipMemset(b.d_err, 0, sizeof(int)));
    b.ngeo = ng;
    b.qgrid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)starts.size(), 1280));
    b.f32q = hs[0]->opt.precision == TEFMM_MIXED_FP32;
    // the far fields of all geometries, captured once as a graph with one branch per
    // geometry (forks from and joins to the origin stream only)
    if (!b.origin) HIPCHK(h0, hipStreamCreateWithFlags(&b.origin, hipStreamNonBlocking));
    if (!b.ev_q) HIPCHK(h0, hipEventCreateWithFlags(&b.ev_q, hipEventDisableTiming));
    if (!b.ev_ff) HIPCHK(h0, hipEventCreateWithFlags(&b.ev_ff, hipEventDisableTiming));
    HIPCHK(h0, hipStreamBeginCapture(b.origin, hipStreamCaptureModeThreadLocal));
    int rc = TEFMM_OK;
    hipError_t e = hipEventRecord(b.ev[n_geom], b.origin);
    for (int g = 0; g < n_geom && rc == TEFMM_OK && e == hipSuccess; ++g) {
      e = hipStreamWaitEvent(b.side[g], b.ev[n_geom], 0);
      if (e != hipSuccess) break;
      rc = enqueue_evaluate(hs[g], q[g], nrhs[g], phi[g], b.side[g], false, true);
      if (rc != TEFMM_OK) break;
      e = hipEventRecord(b.ev[g], b.side[g]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b.origin, b.ev[g], 0);
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b.origin, &graph);
    if (rc != TEFMM_OK || e != hipSuccess || e2 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != TEFMM_OK) return fail(h0, rc, "capture: " + std::string(h0->err));
      return fail(h0, TEFMM_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b.graph = graph;
    HIPCHK(h0, hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    b.hs.assign(hs, hs + n_geom);
    b.gens.clear();
    for (int g = 0; g < n_geom; ++g) b.gens.push_back(hs[g]->gen);
    b.queue = true;
  }
  NFQueueArgs qa;
  std::memset(&qa, 0, sizeof(qa));
  qa.geo = b.d_geo, qa.ngeo = b.ngeo, qa.items = b.d_start, qa.n_p2p = b.n_p2p, qa.n_gather = b.n_gather;
  qa.ticket = b.d_ctr, qa.done = b.d_ctr + 1, qa.err = b.d_err, qa.spin_limit = 1 << 22;
  // charges in tree order on the caller's stream; then the far-field graph and the queue
  // side by side; then every geometry's final scaling on the caller's stream
  for (int g = 0; g < n_geom; ++g) {
    const int rc = enqueue_gather_q(hs[g], q[g], nrhs[g], s);
    if (rc != TEFMM_OK) return fail(h0, rc, "geometry " + std::to_string(g) + ": " + hs[g]->err);
  }
  HIPCHK(h0, hipEventRecord(b.ev_q, s));
  HIPCHK(h0, hipStreamWaitEvent(b.origin, b.ev_q, 0));
  HIPCHK(h0, hipGraphLaunch(b.exec, b.origin));
  HIPCHK(h0, hipEventRecord(b.ev_ff, b.origin));
  HIPCHK(h0, hipStreamWaitEvent(b.nf, b.ev_q, 0));
  hipLaunchKernelGGL(k_nf_queue_reset, dim3(1), dim3(64), 0, b.nf, qa.ticket, qa.done, qa.ngeo, qa.err);
  HIPCHK(h0, hipGetLastError());
  if (b.f32q)
    hipLaunchKernelGGL(k_nf_queue<float>, dim3(b.qgrid), dim3(256), 0, b.nf, qa);
  else
    hipLaunchKernelGGL(k_nf_queue<double>, dim3(b.qgrid), dim3(256), 0, b.nf, qa);
  HIPCHK(h0, hipGetLastError());
  HIPCHK(h0, hipEventRecord(b.ev_nf, b.nf));
  HIPCHK(h0, hipStreamWaitEvent(s, b.ev_ff, 0));
  HIPCHK(h0, hipStreamWaitEvent(s, b.ev_nf, 0));
  for (int g = 0; g < n_geom; ++g) {
    const int rc = enqueue_finalize(hs[g], nrhs[g], phi[g], s);
    if (rc != TEFMM_OK) return fail(h0, rc, "geometry " + std::to_string(g) + ": " + hs[g]->err);
  }
  return TEFMM_OK;
}

extern "C" int tefmm_batch_check(tefmm_t h, void* stream) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  HIPCHK(h, hipStreamSynchronize((hipStream_t)stream));
  if (!h->batch.queue || !h->batch.d_err) return TEFMM_OK;
  int err = 0;
  HIPCHK(h, hipMemcpy(&err, h->batch.d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (err) return fail(h, TEFMM_ERR_STATE, "near-field queue: a gather item stopped waiting (its result is wrong)");
  return TEFMM_OK;
}

__global__ static void k_fill_ones(double2* q, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) q[i] = make_double2(1.0, 0.0);
}

// Autotuner (E2): times the evaluation for tree depths d-1, d, d+1 and both M2L
// tile widths on the handle's own geometry and keeps the fastest.
extern "C" int tefmm_autotune(tefmm_t h, void* stream, int* depth_out, int* ncb_out) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  if (!h->ready || !h->d_xyz_user) return fail(h, TEFMM_ERR_STATE, "set_particles has not succeeded");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = h->n;
  const int d0 = h->groups[0].depth;
  const int depth_opt = h->opt.depth;
  double2 *q1 = nullptr, *phi1 = nullptr;
  HIPCHK(h, dmalloc(h, &q1, sizeof(double2) * n));
  HIPCHK(h, dmalloc(h, &phi1, sizeof(double2) * n));
  hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, q1, n);
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  float best = 1e30f;
  int bd = d0, bn = 0, rc = TEFMM_OK;
  for (int cand = std::max(2, d0 - 1); cand <= std::min(7, d0 + 1) && rc == TEFMM_OK; ++cand) {
    h->opt.depth = cand;
    rc = tefmm_set_particles(h, n, h->d_xyz_user, 1, stream);
    if (rc == TEFMM_OK) rc = ensure_rhs(h, 1);
    for (int ncb = 1; ncb <= 2 && rc == TEFMM_OK; ++ncb) {
      h->m2l_ncb = ncb;
      (void)hipEventRecord(e0, s);
      rc = enqueue_evaluate(h, (const double*)q1, 1, (double*)phi1, s, false);
      if (rc != TEFMM_OK) break;
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float warm = 0;
      (void)hipEventElapsedTime(&warm, e0, e1);
      // a candidate whose first (untimed) evaluation takes three times the best so far
      // cannot win; its other tile width is not tried either
      if (best < 1e30f && warm > 1.5f * best) break;
      (void)hipEventRecord(e0, s);
      for (int it = 0; it < 2 && rc == TEFMM_OK; ++it) rc = enqueue_evaluate(h, (const double*)q1, 1, (double*)phi1, s, false);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rc == TEFMM_OK && ms < best) best = ms, bd = cand, bn = ncb;
    }
  }
  if (rc != TEFMM_OK) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dfree(h, q1);
    dfree(h, phi1);
    h->opt.depth = depth_opt;
    return rc;
  }
  h->opt.depth = bd;
  rc = tefmm_set_particles(h, n, h->d_xyz_user, 1, stream);
  h->m2l_ncb = bn;
  // the fork point of the near field, for the chosen depth and tile width (set_particles
  // rebuilt the levels: their moment and local buffers first)
  if (rc == TEFMM_OK) rc = ensure_rhs(h, 1);
  if (rc == TEFMM_OK) {
    // the three choices in turn, five rounds of four evaluations, the best time of each
    // (the differences can be a percent or two)
    float bt[3] = {1e30f, 1e30f, 1e30f};
    for (int round = 0; round < 5 && rc == TEFMM_OK; ++round)
      for (int fm = 0; fm <= 2 && rc == TEFMM_OK; ++fm) {
        h->fork_late = fm;
        rc = enqueue_evaluate(h, (const double*)q1, 1, (double*)phi1, s, false);
        if (rc != TEFMM_OK) break;
        (void)hipEventRecord(e0, s);
        for (int it = 0; it < 4 && rc == TEFMM_OK; ++it) rc = enqueue_evaluate(h, (const double*)q1, 1, (double*)phi1, s, false);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rc == TEFMM_OK) bt[fm] = std::min(bt[fm], ms);
      }
    int bfm = 0;
    for (int fm = 1; fm <= 2; ++fm)
      if (bt[fm] < bt[bfm]) bfm = fm;
    h->fork_late = rc == TEFMM_OK ? bfm : -1;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dfree(h, q1);
  dfree(h, phi1);
  if (depth_out) *depth_out = bd;
  if (ncb_out) *ncb_out = bn;
  return rc;
}

extern "C" int tefmm_get_stats(tefmm_t h, tefmm_stats* st) {
  if (!h || !st) return TEFMM_ERR_INVALID_ARG;
  if (!h->ev.empty() && h->ev_count > 0) {
    // average over the evaluations recorded since the last timer reset (at most EV_RING)
    double t[8] = {0}, tot = 0;
    for (int c = 0; c < h->ev_count; ++c) {
      const int set = ((h->ev_next - 1 - c) % EV_RING + EV_RING) % EV_RING;
      hipEvent_t* e = &h->ev[9 * set];
      HIPCHK(h, hipEventSynchronize(e[7]));
      // far-field phases on the caller's stream: 0 start, 1..5 after P2M, M2M, M2L,
      // L2L, L2P; near field on the second stream: 8 start, 6 end; 7 after finalize
      for (int i = 1; i < 6; ++i) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e[i - 1], e[i]);
        t[i] += ms;
      }
      float mp = 0;
      (void)hipEventElapsedTime(&mp, e[8], e[6]);
      t[6] += mp;
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e[0], e[7]);
      tot += ms;
    }
    const double inv = 1.0 / h->ev_count;
    h->st.t_p2m_ms = t[1] * inv;  // includes the charge gather
    h->st.t_m2m_ms = t[2] * inv;
    h->st.t_m2l_ms = t[3] * inv;
    h->st.t_l2l_ms = t[4] * inv;
    h->st.t_l2p_ms = t[5] * inv;
    h->st.t_p2p_ms = t[6] * inv;
    h->st.t_total_ms = tot * inv;
    h->st.timed_evaluations = h->ev_count;
  }
  *st = h->st;
  return TEFMM_OK;
}

extern "C" int tefmm_reset_timers(tefmm_t h) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  h->ev_count = 0;
  return TEFMM_OK;
}

extern "C" int tefmm_get_moments(tefmm_t h, int gi, int level, double* out, int64_t cap) {
  if (!h || !h->ready || gi < 0 || gi >= (int)h->groups.size()) return TEFMM_ERR_INVALID_ARG;
  Group& g = h->groups[gi];
  if (level < 2 || level > g.depth || g.alpha.empty() || !g.alpha[level]) return TEFMM_ERR_STATE;
  const int64_t cnt = g.nbox[level] * h->nC;
  if (cap < cnt * 2) return TEFMM_ERR_INVALID_ARG;
  HIPCHK(h, hipDeviceSynchronize());
  HIPCHK(h, hipMemcpy(out, g.alpha[level], sizeof(double2) * cnt, hipMemcpyDeviceToHost));
  return TEFMM_OK;
}

extern "C" int tefmm_get_tree(tefmm_t h, int gi, int* layer, int* depth, double* centre3, double* side) {
  if (!h || !h->ready || gi < 0 || gi >= (int)h->groups.size()) return TEFMM_ERR_INVALID_ARG;
  Group& g = h->groups[gi];
  if (layer) *layer = g.layer;
  if (depth) *depth = g.depth;
  if (centre3)
    for (int c = 0; c < 3; ++c) centre3[c] = g.lo[c] + 0.5 * g.side;
  if (side) *side = g.side;
  return TEFMM_OK;
}

extern "C" int tefmm_taylor_coefficients(int n, const double* x, const double* y, const double* zeta, double k,
                                         double hsc, int order, double* out) {
  if (n < 0 || order < 0 || order > 20 || !(hsc > 0)) return TEFMM_ERR_INVALID_ARG;
  if (n == 0) return TEFMM_OK;
  const int nT = mi_count(order);
  std::vector<short> nbr(6 * nT, -1);
  for (int m = 0; m <= order; ++m)
    for (int a = m; a >= 0; --a)
      for (int b = m - a; b >= 0; --b) {
        const int c = m - a - b, i = mi_index(a, b, c);
        if (a >= 1) nbr[6 * i + 0] = (short)mi_index(a - 1, b, c);
        if (b >= 1) nbr[6 * i + 1] = (short)mi_index(a, b - 1, c);
        if (c >= 1) nbr[6 * i + 2] = (short)mi_index(a, b, c - 1);
        if (a >= 2) nbr[6 * i + 3] = (short)mi_index(a - 2, b, c);
        if (b >= 2) nbr[6 * i + 4] = (short)mi_index(a, b - 2, c);
        if (c >= 2) nbr[6 * i + 5] = (short)mi_index(a, b, c - 2);
      }
  short* d_nbr = nullptr;
  if (hipMalloc(&d_nbr, sizeof(short) * 6 * nT) != hipSuccess) return TEFMM_ERR_HIP;
  if (hipMemcpy(d_nbr, nbr.data(), sizeof(short) * 6 * nT, hipMemcpyHostToDevice) != hipSuccess) {
    dfree_raw(d_nbr);
    return TEFMM_ERR_HIP;
  }
  const size_t lds = 2 * sizeof(double2) * nT;
  (void)hipFuncSetAttribute((const void*)k_taylor_points, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_taylor_points, dim3(n), dim3(64), lds, 0, x, y, zeta, k, hsc, order, nT, d_nbr,
                     (double2*)out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  dfree_raw(d_nbr);
  return e == hipSuccess ? TEFMM_OK : TEFMM_ERR_HIP;
}

extern "C" int tefmm_selftest_mfma(void) {
  double* d64 = nullptr;
  float* d32 = nullptr;
  if (hipMalloc(&d64, 256 * sizeof(double)) != hipSuccess) return TEFMM_ERR_HIP;
  if (hipMalloc(&d32, 256 * sizeof(float)) != hipSuccess) return TEFMM_ERR_HIP;
  hipLaunchKernelGGL(k_selftest_mfma, dim3(1), dim3(64), 0, 0, d64, d32);
  double h64[256];
  float h32[256];
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(h64, d64, sizeof(h64), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(h32, d32, sizeof(h32), hipMemcpyDeviceToHost);
  dfree_raw(d64);
  dfree_raw(d32);
  if (e != hipSuccess) return TEFMM_ERR_HIP;
  int bad = 0;
  for (int m = 0; m < 16; ++m)
    for (int nn = 0; nn < 16; ++nn) {
      double ref = 0;
      for (int kk = 0; kk < 4; ++kk) ref += (1.0 + m + 0.25 * kk) * (2.0 - 0.5 * kk + 0.125 * nn);
      if (std::abs(h64[m * 16 + nn] - ref) > 1e-12 * std::abs(ref)) bad |= 1;
      if (std::abs(h32[m * 16 + nn] - ref) > 1e-5 * std::abs(ref)) bad |= 2;
    }
  return bad;
}

// ---------------------------------------------------------------------------
// Surrogate for the Sigma-family tables of one layer.  The network maps a key
// position (x, y, S = z + z') to the compact table entries scaled by the
// envelope of a source at the nearer mirror distance,
//   W_g = D^g K_Sigma(x, y, S) R_e^{|g|+1} / |g|!,
//   R_e = sqrt(x^2 + y^2 + Z_m^2),  Z_m = min(S - 2 d_l, 2 d_{l-1} - S),
// each output further divided by its RMS over the training set.  It is trained
// on tables generated from the complex images (the method itself), and a
// validation map over cells of the (x, y, S) box keeps a cell only if the
// largest error of W found there is within the budget; keys outside the box
// or in rejected cells use the image tables.
// ---------------------------------------------------------------------------
struct tefmm_surrogate {
  tefmm_t ref = nullptr;  // medium and order-p constant tables
  int layer = 0, p = 0, nG = 0, P2 = 0, nH = 0;
  tefmm_surrogate_options o;
  std::vector<cplx> A[2], Z[2];  // Sigma-up and Sigma-down images of the training box
  bool has[2] = {false, false};
  double2* d_img = nullptr;      // the images on the device: A, Z of Sigma-up, then of Sigma-down
  double2* d_qs = nullptr;       // the quasi-static images alone (depth 0: the mirror points)
  int qs_up = 0, qs_dn = 0;
  tefmm::Mlp net;
  std::vector<float> sigma;      // RMS of each normalised output over the training set
  float* d_sigma = nullptr;
  unsigned char* d_gord = nullptr;  // |g| of each compact table entry
  std::vector<unsigned char> cell_ok;
  std::vector<double> cell_err;
  std::string err;
  ~tefmm_surrogate() {
    if (d_sigma) (void)hipFree(d_sigma);
    if (d_gord) (void)hipFree(d_gord);
    if (d_img) (void)hipFree(d_img);
    if (d_qs) (void)hipFree(d_qs);
    if (ref) tefmm_destroy(ref);
  }
};

// distances of a key (X, Y, S) from the two mirror points (1e300 for a family that is
// absent), appended to out: they set the envelope of the surrogate's outputs
static void sigma_mirror_dist(const MediumDesc& med, int l, bool up, bool dn, double X, double Y, double S,
                              std::vector<double>& out) {
  const double r2 = X * X + Y * Y;
  out.push_back(up ? std::sqrt(r2 + (S - 2 * med.d[l]) * (S - 2 * med.d[l])) : 1e300);
  out.push_back(dn ? std::sqrt(r2 + (2 * med.d[l - 1] - S) * (2 * med.d[l - 1] - S)) : 1e300);
}

// cell (i_rho, i_S) of the validation map, -1 outside the training box
static int sur_cell(const tefmm_surrogate* su, double rho, double S) {
  const tefmm_surrogate_options& o = su->o;
  const double u = rho / o.rho_max, w = (S - o.s_lo) / (o.s_hi - o.s_lo);
  if (!(u >= 0 && u <= 1 && w >= 0 && w <= 1)) return -1;
  const int cu = std::min(o.cells_rho - 1, (int)(u * o.cells_rho)), cw = std::min(o.cells_s - 1, (int)(w * o.cells_s));
  return cu * o.cells_s + cw;
}

static bool surrogate_applies(const tefmm_surrogate* su, int layer, bool up, bool dn) {
  return su->layer == layer && su->has[0] == up && su->has[1] == dn;
}

static bool surrogate_serves_leaves(const tefmm_surrogate* su) { return su->o.leaf_level || su->o.h_from_images; }

static bool surrogate_accepts(const tefmm_surrogate* su, double X, double Y, double S) {
  if (su->o.h_from_images) return sur_cell(su, std::hypot(X, Y), S) >= 0;
  const int c = sur_cell(su, std::hypot(X, Y), S);
  return c >= 0 && su->cell_ok[c];
}

// H_{m,c} (rotation-free derivatives of K_Sigma) of the surrogate's images at (rho, S)
static int sur_image_h(tefmm_surrogate* su, const std::vector<double>& rho, const std::vector<double>& S,
                       double2* d_H, hipStream_t s, bool qs_only = false) {
  tefmm_t h = su->ref;
  const MediumDesc& med = h->med;
  const int l = su->layer, n = (int)rho.size();
  if (!n) return TEFMM_OK;
  std::vector<double> w(n);
  for (int i = 0; i < n; ++i) w[i] = rho[i] * rho[i];
  double *d_w = nullptr, *d_s = nullptr;
  HIPCHK(h, hipMalloc(&d_w, sizeof(double) * n));
  HIPCHK(h, hipMalloc(&d_s, sizeof(double) * n));
  HIPCHK(h, hipMemcpyAsync(d_w, w.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(d_s, S.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
  const int nup = qs_only ? su->qs_up : su->has[0] ? (int)su->A[0].size() : 0;
  const int ndn = qs_only ? su->qs_dn : su->has[1] ? (int)su->A[1].size() : 0;
  hipLaunchKernelGGL(k_sigma_h, dim3(n), dim3(64), 0, s, d_w, d_s, n, qs_only ? su->d_qs : su->d_img, nup, ndn,
                     l < med.L ? 2 * med.d[l] : 0.0, l > 0 ? 2 * med.d[l - 1] : 0.0, med.k[l], su->P2, d_H);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(s));
  dfree_raw(d_w);
  dfree_raw(d_s);
  return TEFMM_OK;
}

// network inputs: rho / rho_max and S scaled to [-1, 1].  H is even in rho (a function of
// rho^2), so training also draws negative rho: the axis rho = 0, where the keys straight
// above one another sit, is then inside the input range instead of on its edge.
static void sur_inputs(const tefmm_surrogate* su, const std::vector<double>& rho, const std::vector<double>& S,
                       std::vector<float>& u) {
  const tefmm_surrogate_options& o = su->o;
  u.resize(2 * rho.size());
  for (size_t i = 0; i < rho.size(); ++i) {
    u[2 * i] = (float)(rho[i] / o.rho_max);
    u[2 * i + 1] = (float)((2 * S[i] - o.s_lo - o.s_hi) / (o.s_hi - o.s_lo));
  }
}

// rows sk.key of d_out (level box size hb) from the network's H (or, with
// h_from_images, from the images' H), rebuilt into the compact Cartesian layout
static int surrogate_tables(tefmm_t h, const SigmaKeys& sk, double hb, double2* d_out, hipStream_t s) {
  tefmm_surrogate* su = h->sur;
  const int nk = (int)sk.key.size(), nG = h->nG, nH = su->nH;
  std::vector<double> rho(nk);
  for (int i = 0; i < nk; ++i) rho[i] = std::hypot(sk.X[i], sk.Y[i]);
  double2* d_H = nullptr;
  double *d_x = nullptr, *d_y = nullptr, *d_re = nullptr;
  int* d_key = nullptr;
  HIPCHK(h, dmalloc(h, &d_H, sizeof(double2) * (size_t)nk * nH));
  HIPCHK(h, dmalloc(h, &d_x, sizeof(double) * nk));
  HIPCHK(h, dmalloc(h, &d_y, sizeof(double) * nk));
  HIPCHK(h, dmalloc(h, &d_key, sizeof(int) * nk));
  HIPCHK(h, hipMemcpyAsync(d_x, sk.X.data(), sizeof(double) * nk, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(d_y, sk.Y.data(), sizeof(double) * nk, hipMemcpyHostToDevice, s));
  HIPCHK(h, hipMemcpyAsync(d_key, sk.key.data(), sizeof(int) * nk, hipMemcpyHostToDevice, s));
  if (su->o.h_from_images) {
    int rc = sur_image_h(su, rho, sk.S, d_H, s);
    if (rc != TEFMM_OK) return fail(h, rc, "surrogate: " + su->ref->err);
  } else {
    std::vector<float> u;
    sur_inputs(su, rho, sk.S, u);
    float *d_u = nullptr, *d_net = nullptr;
    HIPCHK(h, dmalloc(h, &d_u, sizeof(float) * u.size()));
    HIPCHK(h, dmalloc(h, &d_net, sizeof(float) * (size_t)nk * 2 * nH));
    HIPCHK(h, dmalloc(h, &d_re, sizeof(double) * 2 * nk));
    HIPCHK(h, hipMemcpyAsync(d_u, u.data(), sizeof(float) * u.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_re, sk.Re.data(), sizeof(double) * 2 * nk, hipMemcpyHostToDevice, s));
    HIPCHK(h, su->net.reserve(std::min(nk, 65536)));
    for (int r0 = 0; r0 < nk; r0 += (int)su->net.cap) {
      const int cnt = std::min<int>((int)su->net.cap, nk - r0);
      HIPCHK(h, su->net.forward(d_u + 2 * (size_t)r0, cnt, d_net + (size_t)r0 * 2 * nH, s));
    }
    // the quasi-static part, exact, then the network's remainder added to it
    int rc = sur_image_h(su, rho, sk.S, d_H, s, true);
    if (rc != TEFMM_OK) return fail(h, rc, "surrogate: " + su->ref->err);
    hipLaunchKernelGGL(k_sur_h_from_net, dim3(nk), dim3(128), 0, s, d_net, d_re, nk, su->P2, su->d_sigma,
                       su->o.envelope, d_H);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(s));
    dfree(h, d_u);
    dfree(h, d_net);
  }
  hipLaunchKernelGGL(k_sigma_restore, dim3(nk), dim3(64), 0, s, d_H, d_x, d_y, nk, d_key, hb,
                     h->med.k[su->layer], su->P2, nG, h->d_g1, h->d_g3, su->d_gord, d_out, nullptr, 0);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(s));
  dfree(h, d_H);
  dfree(h, d_x);
  dfree(h, d_y);
  dfree(h, d_key);
  dfree(h, d_re);
  return TEFMM_OK;
}

extern "C" void tefmm_surrogate_default_options(const tefmm_medium* medium, int layer, tefmm_surrogate_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->layer = layer;
  o->rho_max = 1.1;
  o->s_lo = -1.0, o->s_hi = 1.0;
  MediumDesc med;
  std::string err;
  if (medium && medium_from_desc(medium, med, err) && layer >= 0 && layer <= med.L) {
    const double margin = 0.15;
    const double top = layer == 0 ? (med.L ? med.d[0] + 2.0 : 2.0) : med.d[layer - 1];
    const double bot = layer == med.L ? (med.L ? med.d[med.L - 1] - 2.0 : -2.0) : med.d[layer];
    o->s_lo = 2 * bot + margin, o->s_hi = 2 * top - margin;
  }
  o->n_train = 262144;
  o->epochs = 300;
  o->batch = 1024;
  o->lr = 2e-3f;
  o->width = 128;
  o->n_hidden = 4;
  o->cells_rho = 8;
  o->cells_s = 16;
  o->n_valid = 16;
  o->budget = 4e-4;
  o->seed = 1234;
  o->h_from_images = 0;
  o->envelope = 1;
  o->leaf_level = 0;
  o->split_bf16 = 1;
  o->err_total = 1.2e-3;
}

#define SURCHK(x)                                                \
  do {                                                           \
    int rc_ = (x);                                               \
    if (rc_ != TEFMM_OK) {                                       \
      if (rep) rep->status = rc_;                                \
      delete su;                                                 \
      return rc_;                                                \
    }                                                            \
  } while (0)
#define SURHIP(x) SURCHK(((x) == hipSuccess) ? TEFMM_OK : TEFMM_ERR_HIP)

extern "C" int tefmm_surrogate_train(tefmm_surrogate_t* out, const tefmm_medium* medium, const tefmm_options* opt,
                                     const tefmm_surrogate_options* so, tefmm_surrogate_report* rep,
                                     double* epoch_loss, void* stream) {
  if (!out || !medium || !so) return TEFMM_ERR_INVALID_ARG;
  *out = nullptr;
  if (rep) std::memset(rep, 0, sizeof(*rep));
  const tefmm_surrogate_options& o = *so;
  if (!(o.rho_max > 0) || !(o.s_hi > o.s_lo) || o.n_train < 64 || o.epochs < 0 || o.batch < 1 || !(o.lr > 0) ||
      o.width < 16 || o.n_hidden < 1 || o.cells_rho < 1 || o.cells_s < 1 || o.n_valid < 1 || !(o.budget > 0) ||
      std::isnan(o.err_total))
    return TEFMM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  tefmm_surrogate* su = new tefmm_surrogate();
  su->o = o;
  su->layer = o.layer;
  SURCHK(tefmm_create(&su->ref, medium, opt));
  tefmm_t h = su->ref;
  const MediumDesc& med = h->med;
  const int l = o.layer;
  if (l < 0 || l > med.L) SURCHK(TEFMM_ERR_INVALID_ARG);
  su->p = h->opt.p, su->nG = h->nG, su->P2 = 2 * h->opt.p;
  su->nH = (su->P2 + 1) * (su->P2 + 2) / 2;
  if (su->P2 > SIGMA_P2_MAX) SURCHK(TEFMM_ERR_UNSUPPORTED);
  const int nG = su->nG, nH = su->nH;
  // the training box must lie in the layer (S = z + z' of two points of the layer)
  const double top = med.top(l), bot = med.bottom(l);
  if (!(o.s_lo > 2 * bot) || !(o.s_hi < 2 * top)) SURCHK(TEFMM_ERR_INVALID_ARG);
  auto t0 = std::chrono::steady_clock::now();
  // complex images of the box (Sec. 3.3), as the method's own tables use them
  for (int f = 0; f < 2; ++f) {
    double fe = 0;
    std::string err;
    if (!same_layer_family(med, l, f, 0.5 * o.s_lo, 0.5 * o.s_hi, h->opt.dcim_T1, h->opt.dcim_samples,
                           h->opt.dcim_svd_tol, su->A[f], su->Z[f], fe, err))
      SURCHK(TEFMM_ERR_DCIM_FIT);
    su->has[f] = !su->A[f].empty();
  }
  if (!su->has[0] && !su->has[1]) SURCHK(TEFMM_ERR_UNSUPPORTED);  // no Sigma family in this layer
  {
    std::vector<double2> img;
    for (int f = 0; f < 2; ++f)
      for (size_t j = 0; j < su->A[f].size(); ++j) {
        img.push_back(make_double2(su->A[f][j].real(), su->A[f][j].imag()));
        img.push_back(make_double2(su->Z[f][j].real(), su->Z[f][j].imag()));
      }
    SURHIP(hipMalloc(&su->d_img, sizeof(double2) * std::max<size_t>(img.size(), 1)));
    SURHIP(hipMemcpy(su->d_img, img.data(), sizeof(double2) * img.size(), hipMemcpyHostToDevice));
    // the quasi-static image of each family (the fit places it at depth 0, the mirror point)
    std::vector<double2> qs;
    for (int f = 0; f < 2; ++f)
      for (size_t j = 0; j < su->A[f].size(); ++j)
        if (su->Z[f][j] == cplx(0, 0)) {
          qs.push_back(make_double2(su->A[f][j].real(), su->A[f][j].imag()));
          qs.push_back(make_double2(0.0, 0.0));
          (f == 0 ? su->qs_up : su->qs_dn) += 1;
        }
    SURHIP(hipMalloc(&su->d_qs, sizeof(double2) * std::max<size_t>(qs.size(), 1)));
    if (!qs.empty()) SURHIP(hipMemcpy(su->d_qs, qs.data(), sizeof(double2) * qs.size(), hipMemcpyHostToDevice));
  }
  std::vector<unsigned char> gord(nG);
  for (int n = 0; n <= 2 * su->p; ++n)
    for (int i = g_offset(n); i < g_offset(n + 1); ++i) gord[i] = (unsigned char)n;
  SURHIP(hipMalloc(&su->d_gord, nG));
  SURHIP(hipMemcpy(su->d_gord, gord.data(), nG, hipMemcpyHostToDevice));
  if (o.h_from_images) {  // no network: rows from the images' H (a check of the representation)
    if (rep) rep->status = TEFMM_OK, rep->n_out = 2 * nH;
    *out = su;
    return TEFMM_OK;
  }
  // samples: uniform in the box
  uint64_t st = o.seed;
  auto unif = [&]() {
    st += 0x9e3779b97f4a7c15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  // normalised targets: W = (H - H_quasi-static) (divided by the envelope if asked), and
  // the sums of |W|^2 per entry
  auto targets = [&](const std::vector<double>& R, const std::vector<double>& S, double2* d_W,
                     double* d_sumsq) -> int {
    const int n = (int)R.size();
    double2 *d_H = nullptr, *d_Hq = nullptr;
    double* d_re = nullptr;
    HIPCHK(h, hipMalloc(&d_H, sizeof(double2) * (size_t)n * nH));
    HIPCHK(h, hipMalloc(&d_Hq, sizeof(double2) * (size_t)n * nH));
    HIPCHK(h, hipMalloc(&d_re, sizeof(double) * 2 * n));
    int rc = sur_image_h(su, R, S, d_H, s);
    if (rc == TEFMM_OK) rc = sur_image_h(su, R, S, d_Hq, s, true);
    if (rc != TEFMM_OK) return rc;
    std::vector<double> re;
    for (int i = 0; i < n; ++i) sigma_mirror_dist(med, l, su->has[0], su->has[1], R[i], 0.0, S[i], re);
    HIPCHK(h, hipMemcpyAsync(d_re, re.data(), sizeof(double) * re.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sur_normalize, dim3(n), dim3(128), 0, s, d_H, d_Hq, d_re, n, su->P2, o.envelope, d_W,
                       d_sumsq);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipStreamSynchronize(s));
    dfree_raw(d_H);
    dfree_raw(d_Hq);
    dfree_raw(d_re);
    return TEFMM_OK;
  };
  const int n = o.n_train;
  std::vector<double> R(n), S(n);
  for (int i = 0; i < n; ++i) {
    R[i] = (2 * unif() - 1) * o.rho_max;  // signed: see sur_inputs
    S[i] = o.s_lo + unif() * (o.s_hi - o.s_lo);
  }
  double2* d_W = nullptr;
  double* d_sumsq = nullptr;
  float *d_T = nullptr, *d_X = nullptr;
  SURHIP(hipMalloc(&d_W, sizeof(double2) * (size_t)n * nH));
  SURHIP(hipMalloc(&d_sumsq, sizeof(double) * nH));
  SURHIP(hipMemset(d_sumsq, 0, sizeof(double) * nH));
  SURCHK(targets(R, S, d_W, d_sumsq));
  std::vector<double> sumsq(nH);
  SURHIP(hipMemcpy(sumsq.data(), d_sumsq, sizeof(double) * nH, hipMemcpyDeviceToHost));
  su->sigma.resize(nH);
  for (int g = 0; g < nH; ++g) su->sigma[g] = (float)std::max(std::sqrt(sumsq[g] / n), 1e-30);
  SURHIP(hipMalloc(&su->d_sigma, sizeof(float) * nH));
  SURHIP(hipMemcpy(su->d_sigma, su->sigma.data(), sizeof(float) * nH, hipMemcpyHostToDevice));
  SURHIP(hipMalloc(&d_T, sizeof(float) * (size_t)n * 2 * nH));
  hipLaunchKernelGGL(k_sur_targets, dim3((unsigned)(((size_t)n * nH + 255) / 256)), dim3(256), 0, s, d_W, n, nH,
                     su->d_sigma, d_T);
  SURHIP(hipGetLastError());
  std::vector<float> u;
  sur_inputs(su, R, S, u);
  SURHIP(hipMalloc(&d_X, sizeof(float) * u.size()));
  SURHIP(hipMemcpyAsync(d_X, u.data(), sizeof(float) * u.size(), hipMemcpyHostToDevice, s));
  SURHIP(hipStreamSynchronize(s));
  dfree_raw(d_W);
  dfree_raw(d_sumsq);
  auto t1 = std::chrono::steady_clock::now();
  // training on the matrix cores
  SURHIP(su->net.init(2, o.width, o.n_hidden, 2 * nH, o.seed ^ 0x5bd1e995ull));
  su->net.split = o.split_bf16 ? 1 : 0;
  std::vector<double> losses;
  SURHIP(su->net.train(d_X, d_T, n, o.epochs, o.batch, o.lr, o.seed + 17, losses, s));
  if (epoch_loss)
    for (size_t i = 0; i < losses.size(); ++i) epoch_loss[i] = losses[i];
  dfree_raw(d_X);
  dfree_raw(d_T);
  auto t2 = std::chrono::steady_clock::now();
  // validation map: n_valid fresh points per (rho, S) cell
  const int ncell = o.cells_rho * o.cells_s, nv = ncell * o.n_valid;
  std::vector<double> vR(nv), vS(nv);
  for (int c = 0; c < ncell; ++c) {
    const int cu = c / o.cells_s, cw = c % o.cells_s;
    for (int j = 0; j < o.n_valid; ++j) {
      const int i = c * o.n_valid + j;
      // the first point of every cell on its lower rho edge (rho = 0 for the first column:
      // the keys straight above one another sit there, on the edge of the input range)
      vR[i] = (cu + (j == 0 ? 0.0 : unif())) / o.cells_rho * o.rho_max;
      vS[i] = o.s_lo + (cw + unif()) / o.cells_s * (o.s_hi - o.s_lo);
    }
  }
  double2* d_vW = nullptr;
  float *d_vu = nullptr, *d_vy = nullptr;
  SURHIP(hipMalloc(&d_vW, sizeof(double2) * (size_t)nv * nH));
  SURCHK(targets(vR, vS, d_vW, nullptr));
  std::vector<float> vu;
  sur_inputs(su, vR, vS, vu);
  SURHIP(hipMalloc(&d_vu, sizeof(float) * vu.size()));
  SURHIP(hipMalloc(&d_vy, sizeof(float) * (size_t)nv * 2 * nH));
  SURHIP(hipMemcpy(d_vu, vu.data(), sizeof(float) * vu.size(), hipMemcpyHostToDevice));
  SURHIP(su->net.reserve(std::min(nv, 65536)));
  for (int r0 = 0; r0 < nv; r0 += (int)su->net.cap) {
    const int cnt = std::min<int>((int)su->net.cap, nv - r0);
    SURHIP(su->net.forward(d_vu + 2 * (size_t)r0, cnt, d_vy + (size_t)r0 * 2 * nH, s));
  }
  std::vector<double2> vW((size_t)nv * nH);
  std::vector<float> vy((size_t)nv * 2 * nH);
  SURHIP(hipMemcpyAsync(vW.data(), d_vW, sizeof(double2) * vW.size(), hipMemcpyDeviceToHost, s));
  SURHIP(hipMemcpyAsync(vy.data(), d_vy, sizeof(float) * vy.size(), hipMemcpyDeviceToHost, s));
  SURHIP(hipStreamSynchronize(s));
  dfree_raw(d_vW);
  dfree_raw(d_vu);
  dfree_raw(d_vy);
  su->cell_ok.assign(ncell, 0);
  su->cell_err.assign(ncell, 0.0);
  double emax = 0;
  for (int c = 0; c < ncell; ++c) {
    double e = 0;
    for (int j = 0; j < o.n_valid; ++j) {
      const size_t i = (size_t)c * o.n_valid + j;
      // in envelope units, entry (m, c) weighted by 2^-(m+c): a translation between boxes of
      // side h at distance R >= 2h (the well-separated ones) uses order n of the kernel's
      // expansion with the weight (h / R)^n relative to order 0
      for (int nn = 0, g = 0; nn <= su->P2; ++nn) {
        const double wt = std::ldexp(1.0, -nn);
        for (int m = 0; m <= nn; ++m, ++g) {
          const double pr = vy[(i * nH + g) * 2] * su->sigma[g] - vW[i * nH + g].x,
                       pi = vy[(i * nH + g) * 2 + 1] * su->sigma[g] - vW[i * nH + g].y;
          e = std::max(e, wt * std::hypot(pr, pi));
        }
      }
    }
    su->cell_err[c] = e;
    emax = std::max(emax, e);
  }
  // cells kept in order of increasing error while each is within the budget and the
  // errors of the kept cells sum to at most err_total: every served row moves the
  // potential, so the number of rows, not only their accuracy, has to stay bounded
  int ok = 0;
  {
    std::vector<int> order(ncell);
    for (int c = 0; c < ncell; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return su->cell_err[a] < su->cell_err[b]; });
    double sum = 0;
    for (int c : order) {
      const double e = su->cell_err[c];
      if (!(e <= o.budget) || (o.err_total > 0 && sum + e > o.err_total)) break;
      sum += e;
      su->cell_ok[c] = 1;
      ++ok;
    }
  }
  auto t3 = std::chrono::steady_clock::now();
  if (rep) {
    rep->t_data_s = std::chrono::duration<double>(t1 - t0).count();
    rep->t_train_s = std::chrono::duration<double>(t2 - t1).count();
    rep->t_valid_s = std::chrono::duration<double>(t3 - t2).count();
    rep->final_loss = losses.empty() ? 0.0 : losses.back();
    rep->max_cell_err = emax;
    rep->cells_ok = ok;
    rep->cells_total = ncell;
    rep->n_out = 2 * nH;
    rep->n_params = su->net.P;
    rep->status = TEFMM_OK;
  }
  *out = su;
  return TEFMM_OK;
}
#undef SURCHK
#undef SURHIP

extern "C" void tefmm_surrogate_destroy(tefmm_surrogate_t su) { delete su; }

extern "C" int tefmm_surrogate_cell_ok(tefmm_surrogate_t su, int n, const double* xys, int* ok) {
  if (!su || n < 0 || (n > 0 && (!xys || !ok))) return TEFMM_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) ok[i] = surrogate_accepts(su, xys[3 * i], xys[3 * i + 1], xys[3 * i + 2]) ? 1 : 0;
  return TEFMM_OK;
}

extern "C" int tefmm_surrogate_cell_errors(tefmm_surrogate_t su, double* err) {
  if (!su || !err) return TEFMM_ERR_INVALID_ARG;
  for (size_t c = 0; c < su->cell_err.size(); ++c) err[c] = su->cell_err[c];
  return TEFMM_OK;
}

extern "C" int tefmm_set_surrogate(tefmm_t h, tefmm_surrogate_t su) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  if (su) {
    if (su->p != h->opt.p) return fail(h, TEFMM_ERR_INVALID_ARG, "surrogate trained for another order p");
    const MediumDesc& a = su->ref->med;
    if (a.k != h->med.k || a.d != h->med.d) return fail(h, TEFMM_ERR_INVALID_ARG, "surrogate trained for another medium");
  }
  h->sur = su;
  return TEFMM_OK;
}

// ---------------------------------------------------------------------------
// H_{m,c} of the Sigma families of one layer at given points, by the complex
// images (Sec. 3.3) or by the Sommerfeld integrals (Sec. 4.2).
// ---------------------------------------------------------------------------
extern "C" int tefmm_sigma_derivatives(tefmm_t h, int layer, int method, int64_t n, const double* rho,
                                       const double* S, double* out, void* stream) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  const MediumDesc& med = h->med;
  if (layer < 0 || layer > med.L) return fail(h, TEFMM_ERR_INVALID_ARG, "layer out of range");
  if (method != TEFMM_SIGMA_IMAGES && method != TEFMM_SIGMA_SOMMERFELD)
    return fail(h, TEFMM_ERR_INVALID_ARG, "unknown method");
  if (n < 1 || n > (1 << 22) || !rho || !S || !out) return fail(h, TEFMM_ERR_INVALID_ARG, "need 1 <= n <= 2^22 points");
  const bool up = layer < med.L, dn = layer > 0;
  if (!up && !dn) return fail(h, TEFMM_ERR_UNSUPPORTED, "a medium of one layer has no reaction term");
  const int P2 = 2 * h->opt.p, nH = (P2 + 1) * (P2 + 2) / 2;
  if (P2 > SIGMA_P2_MAX) return fail(h, TEFMM_ERR_UNSUPPORTED, "needs 2p <= " + std::to_string(SIGMA_P2_MAX));
  double zmin = 1e300, rmax = 0.0, slo = 1e300, shi = -1e300;
  for (int64_t i = 0; i < n; ++i) {
    const double zu = up ? S[i] - 2 * med.d[layer] : 1e300, zd = dn ? 2 * med.d[layer - 1] - S[i] : 1e300;
    if (!(rho[i] >= 0 && rho[i] < 1e300) || !(zu > 0) || !(zd > 0))
      return fail(h, TEFMM_ERR_INVALID_ARG, "point " + std::to_string(i) + " outside the layer's Sigma range");
    zmin = std::min(zmin, std::min(zu, zd));
    rmax = std::max(rmax, rho[i]);
    slo = std::min(slo, S[i]), shi = std::max(shi, S[i]);
  }
  hipStream_t s = (hipStream_t)stream;
  const std::vector<double> vr(rho, rho + n), vS(S, S + n);
  double2* d_H = nullptr;
  double2* d_img = nullptr;
  double *d_w = nullptr, *d_s = nullptr;
  auto run = [&]() -> int {
    HIPCHK(h, dmalloc(h, &d_H, sizeof(double2) * (size_t)n * nH));
    if (method == TEFMM_SIGMA_SOMMERFELD) {
      SomPath P;
      sommerfeld_path(med, layer, up, dn, zmin, rmax, P2, P);
      std::vector<int> idx(n);
      for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
      return sommerfeld_h(h, layer, up, dn, P, P2, vr, vS, idx, idx, d_H, s);
    }
    std::vector<double2> img;
    int cnt[2] = {0, 0};
    for (int f = 0; f < 2; ++f) {
      if ((f == 0 && !up) || (f == 1 && !dn)) continue;
      std::vector<cplx> A, Z;
      double fe = 0;
      std::string err;
      if (!same_layer_family(med, layer, f, 0.5 * slo, 0.5 * shi, h->opt.dcim_T1, h->opt.dcim_samples,
                             h->opt.dcim_svd_tol, A, Z, fe, err))
        return fail(h, TEFMM_ERR_DCIM_FIT, err);
      for (size_t j = 0; j < A.size(); ++j) {
        img.push_back(make_double2(A[j].real(), A[j].imag()));
        img.push_back(make_double2(Z[j].real(), Z[j].imag()));
      }
      cnt[f] = (int)A.size();
    }
    std::vector<double> w(n);
    for (int64_t i = 0; i < n; ++i) w[i] = rho[i] * rho[i];
    HIPCHK(h, dmalloc(h, &d_img, sizeof(double2) * std::max<size_t>(img.size(), 1)));
    HIPCHK(h, dmalloc(h, &d_w, sizeof(double) * n));
    HIPCHK(h, dmalloc(h, &d_s, sizeof(double) * n));
    if (!img.empty())
      HIPCHK(h, hipMemcpyAsync(d_img, img.data(), sizeof(double2) * img.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_w, w.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_s, S, sizeof(double) * n, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_sigma_h, dim3((unsigned)n), dim3(64), 0, s, d_w, d_s, (int)n, d_img, cnt[0], cnt[1],
                       up ? 2 * med.d[layer] : 0.0, dn ? 2 * med.d[layer - 1] : 0.0, med.k[layer], P2, d_H);
    HIPCHK(h, hipGetLastError());
    return TEFMM_OK;
  };
  int rc = run();
  if (rc == TEFMM_OK) {
    if (hipMemcpyAsync(out, d_H, sizeof(double2) * (size_t)n * nH, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = fail(h, TEFMM_ERR_HIP, "copy of the derivatives");
  }
  dfree(h, d_H), dfree(h, d_img), dfree(h, d_w), dfree(h, d_s);
  return rc;
}

// ---------------------------------------------------------------------------
// H_{m,c} of the Delta family of one layer (functions of rho and w = z - z'), by the
// complex images (Sec. 3.3) or by the Sommerfeld integrals (Sec. 4.2).
// ---------------------------------------------------------------------------
extern "C" int tefmm_delta_derivatives(tefmm_t h, int layer, int method, int64_t n, const double* rho,
                                       const double* w, double* out, void* stream) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  const MediumDesc& med = h->med;
  if (layer < 0 || layer > med.L) return fail(h, TEFMM_ERR_INVALID_ARG, "layer out of range");
  if (method != TEFMM_SIGMA_IMAGES && method != TEFMM_SIGMA_SOMMERFELD)
    return fail(h, TEFMM_ERR_INVALID_ARG, "unknown method");
  if (n < 1 || n > (1 << 22) || !rho || !w || !out) return fail(h, TEFMM_ERR_INVALID_ARG, "need 1 <= n <= 2^22 points");
  if (layer == 0 || layer == med.L)
    return fail(h, TEFMM_ERR_UNSUPPORTED, "the Delta family needs a layer with two interfaces");
  const int P2 = 2 * h->opt.p, nH = (P2 + 1) * (P2 + 2) / 2;
  if (P2 > SIGMA_P2_MAX) return fail(h, TEFMM_ERR_UNSUPPORTED, "needs 2p <= " + std::to_string(SIGMA_P2_MAX));
  const double D = med.thickness(layer);
  double zmin = 1e300, rmax = 0.0, wmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(rho[i] >= 0 && rho[i] < 1e300) || !(D - std::fabs(w[i]) > 0))
      return fail(h, TEFMM_ERR_INVALID_ARG, "point " + std::to_string(i) + " outside the layer's Delta range");
    zmin = std::min(zmin, D - std::fabs(w[i]));
    rmax = std::max(rmax, rho[i]);
    wmax = std::max(wmax, std::fabs(w[i]));
  }
  hipStream_t s = (hipStream_t)stream;
  const std::vector<double> vr(rho, rho + n), vw(w, w + n);
  double2* d_H = nullptr;
  double2* d_img = nullptr;
  double *d_w = nullptr, *d_s = nullptr;
  auto run = [&]() -> int {
    HIPCHK(h, dmalloc(h, &d_H, sizeof(double2) * (size_t)n * nH));
    if (method == TEFMM_SIGMA_SOMMERFELD) {
      SomPath P;
      sommerfeld_path(med, layer, true, true, zmin, rmax, P2, P, true);
      std::vector<int> idx(n);
      for (int64_t i = 0; i < n; ++i) idx[i] = (int)i;
      return sommerfeld_h(h, layer, true, true, P, P2, vr, vw, idx, idx, d_H, s, true);
    }
    // the images of the family fitted for heights spanning the largest |w|; each enters
    // at D + w and at D - w with the same amplitude
    std::vector<cplx> A, Z;
    double fe = 0;
    std::string err;
    if (!same_layer_family(med, layer, 2, 0.0, wmax, h->opt.dcim_T1, h->opt.dcim_samples, h->opt.dcim_svd_tol, A, Z,
                           fe, err))
      return fail(h, TEFMM_ERR_DCIM_FIT, err);
    std::vector<double2> img;
    for (int f = 0; f < 2; ++f)
      for (size_t j = 0; j < A.size(); ++j) {
        img.push_back(make_double2(A[j].real(), A[j].imag()));
        img.push_back(make_double2(Z[j].real(), Z[j].imag()));
      }
    std::vector<double> r2(n);
    for (int64_t i = 0; i < n; ++i) r2[i] = rho[i] * rho[i];
    HIPCHK(h, dmalloc(h, &d_img, sizeof(double2) * std::max<size_t>(img.size(), 1)));
    HIPCHK(h, dmalloc(h, &d_w, sizeof(double) * n));
    HIPCHK(h, dmalloc(h, &d_s, sizeof(double) * n));
    if (!img.empty())
      HIPCHK(h, hipMemcpyAsync(d_img, img.data(), sizeof(double2) * img.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_w, r2.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(d_s, w, sizeof(double) * n, hipMemcpyHostToDevice, s));
    double two_dl, two_dt;
    som_offsets(med, layer, true, &two_dl, &two_dt);
    hipLaunchKernelGGL(k_sigma_h, dim3((unsigned)n), dim3(64), 0, s, d_w, d_s, (int)n, d_img, (int)A.size(),
                       (int)A.size(), two_dl, two_dt, med.k[layer], P2, d_H);
    HIPCHK(h, hipGetLastError());
    return TEFMM_OK;
  };
  int rc = run();
  if (rc == TEFMM_OK) {
    if (hipMemcpyAsync(out, d_H, sizeof(double2) * (size_t)n * nH, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = fail(h, TEFMM_ERR_HIP, "copy of the derivatives");
  }
  dfree(h, d_H), dfree(h, d_img), dfree(h, d_w), dfree(h, d_s);
  return rc;
}

// ---------------------------------------------------------------------------
// H_{m,c} of the cross-layer kernel (target in `layer`, source in `src_layer`) with the
// source-side z' derivative of order k3, from the Sommerfeld integrals (Sec. 4.2).
// ---------------------------------------------------------------------------
extern "C" int tefmm_cross_derivatives(tefmm_t h, int layer, int src_layer, int k3, int64_t n, const double* rho,
                                       const double* z, const double* zs, double* out, void* stream) {
  if (!h) return TEFMM_ERR_INVALID_ARG;
  const MediumDesc& med = h->med;
  const int L = med.L;
  if (layer < 0 || layer > L || src_layer < 0 || src_layer > L || layer == src_layer)
    return fail(h, TEFMM_ERR_INVALID_ARG, "need two different layers of the medium");
  if (k3 < 0 || k3 > h->opt.p) return fail(h, TEFMM_ERR_INVALID_ARG, "k3 outside 0 .. p");
  if (n < 1 || n > 4096 || !rho || !z || !zs || !out) return fail(h, TEFMM_ERR_INVALID_ARG, "need 1 <= n <= 4096 points");
  const int P2 = 2 * h->opt.p, nH = (P2 + 1) * (P2 + 2) / 2;
  if (P2 > SIGMA_P2_MAX) return fail(h, TEFMM_ERR_UNSUPPORTED, "needs 2p <= " + std::to_string(SIGMA_P2_MAX));
  const bool up = layer < L, dn = layer > 0;
  for (int64_t i = 0; i < n; ++i)
    if (!(rho[i] >= 0 && rho[i] < 1e300) || !(z[i] > med.bottom(layer) && z[i] < med.top(layer)) ||
        !(zs[i] > med.bottom(src_layer) && zs[i] < med.top(src_layer)))
      return fail(h, TEFMM_ERR_INVALID_ARG, "point " + std::to_string(i) + " outside its layer");
  hipStream_t s = (hipStream_t)stream;
  const double offs[2] = {up ? med.d[layer] : 0.0, dn ? med.d[layer - 1] : 0.0};
  const cplx I(0.0, 1.0);
  std::vector<double2> hostH((size_t)n * nH);
  double2* d_H = nullptr;
  int rc = TEFMM_OK;
  for (int64_t i = 0; i < n && rc == TEFMM_OK; ++i) {
    const double za = std::min(up ? z[i] - med.d[layer] : 1e300, dn ? med.d[layer - 1] - z[i] : 1e300);
    const double zb = std::min(src_layer < L ? zs[i] - med.d[src_layer] : 1e300,
                               src_layer > 0 ? med.d[src_layer - 1] - zs[i] : 1e300);
    SomPath P;
    std::vector<cplx> wts, sig;
    som_nodes(med, za + zb, std::max(rho[i], 1e-3), P2 + k3, P.krho, wts);
    for (size_t t = 0; t < P.krho.size(); ++t) {
      reaction_densities(med, src_layer, P.krho[t], sig);
      const cplx kz = vertical_wavenumber(med.k[layer], P.krho[t]), kzp = vertical_wavenumber(med.k[src_layer], P.krho[t]);
      cplx eu = 0.0, ed = 0.0;
      if (src_layer < L) eu = std::pow(I * kzp, (double)k3) * std::exp(I * kzp * (zs[i] - med.d[src_layer]));
      if (src_layer > 0) ed = std::pow(-I * kzp, (double)k3) * std::exp(I * kzp * (med.d[src_layer - 1] - zs[i]));
      const cplx f = wts[t] * I / kz;
      P.kz.push_back(kz);
      P.cu.push_back(up ? f * (sig[layer * 4 + 0] * eu + sig[layer * 4 + 1] * ed) : cplx(0.0));
      P.cd.push_back(dn ? f * (sig[layer * 4 + 2] * eu + sig[layer * 4 + 3] * ed) : cplx(0.0));
    }
    const std::vector<double> vr(1, rho[i]), vz(1, z[i]);
    const std::vector<int> idx(1, 0);
    auto run = [&]() -> int {
      HIPCHK(h, dmalloc(h, &d_H, sizeof(double2) * nH));
      const int r2 = sommerfeld_h(h, layer, up, dn, P, P2, vr, vz, idx, idx, d_H, s, false, offs);
      if (r2 != TEFMM_OK) return r2;
      HIPCHK(h, hipMemcpyAsync(hostH.data() + (size_t)i * nH, d_H, sizeof(double2) * nH, hipMemcpyDeviceToHost, s));
      HIPCHK(h, hipStreamSynchronize(s));
      return TEFMM_OK;
    };
    rc = run();
    dfree(h, d_H);
  }
  if (rc == TEFMM_OK) std::memcpy(out, hostH.data(), sizeof(double2) * (size_t)n * nH);
  return rc;
}

// ---------------------------------------------------------------------------
// The tree build's sort and scan alone (sort_scan.hip).
// ---------------------------------------------------------------------------
extern "C" int tefmm_radix_sort(int64_t n, unsigned* keys, int* vals, int end_bit, void* stream) {
  if (n < 1 || n > 2147483647LL || !keys || !vals || end_bit < 0 || end_bit > 32) return TEFMM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  unsigned* k2 = nullptr;
  int* v2 = nullptr;
  void* sc = nullptr;
  int rc = TEFMM_OK;
  if (hipMalloc(&k2, sizeof(unsigned) * n) != hipSuccess || hipMalloc(&v2, sizeof(int) * n) != hipSuccess ||
      hipMalloc(&sc, sort_scratch_bytes(n)) != hipSuccess ||
      radix_sort_pairs(keys, k2, vals, v2, n, end_bit, sc, s) != hipSuccess ||
      hipMemcpyAsync(keys, k2, sizeof(unsigned) * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(vals, v2, sizeof(int) * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = TEFMM_ERR_HIP;
  if (k2) (void)hipFree(k2);
  if (v2) (void)hipFree(v2);
  if (sc) (void)hipFree(sc);
  return rc;
}

extern "C" int tefmm_exclusive_scan(int64_t n, const unsigned* in, unsigned* out, void* stream) {
  if (n < 1 || n > 2147483647LL || !in || !out) return TEFMM_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  void* sc = nullptr;
  int rc = TEFMM_OK;
  if (hipMalloc(&sc, scan_scratch_bytes(n)) != hipSuccess || exclusive_scan(in, out, n, sc, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    rc = TEFMM_ERR_HIP;
  if (sc) (void)hipFree(sc);
  return rc;
}
