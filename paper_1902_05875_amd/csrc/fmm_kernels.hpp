// Kernel argument blocks and launch declarations of the TE-FMM kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tefmm {

constexpr int MAX_LAYERS = 8;  // layers of the medium (the C ABI's TEFMM_MAX_LAYERS)

// One term of a derivative-table key: coef * f(x, y, zeta) in box units,
// f = exp(i kh R)/R; flip = 1 when the key's variable enters zeta with a minus sign.
struct TableTerm {
  double x, y, zr, zi, cr, ci;
  int flip, pad;
};

struct TableGenArgs {
  const TableTerm* terms;
  const int* term_start;  // [nkeys+1]
  const double* h;        // [nkeys] box size of each key
  double k;
  int order, nG;          // orders 0..order, nG = g_count(order) compact entries (g1 <= 2)
  const short* nbr;       // [nG][6]: g - e_x, g - e_y, g - e_z, g - 2e_x, g - 2e_y, g - 2e_z (-1 if none)
  const unsigned char* g3;  // [nG] third component of g
  const unsigned char* g1;  // [nG] first component of g
  int swap13;             // generate in the (zeta, y, x) frame (flip follows g1 then)
  const double* fact;     // [nG] g!
  double2* out;           // [nkeys][nG]
};

struct TreeGeom {
  int group_of_layer[MAX_LAYERS];
  int depth[MAX_LAYERS];
  double lo[MAX_LAYERS][3];
  double side[MAX_LAYERS];
  int64_t leaf_offset[MAX_LAYERS];
};

// Arguments shared by the per-box passes (P2M, M2M, L2L, L2P, P2P).
struct PassArgs {
  int p, nC;
  int nbox_dim;        // boxes per dimension at this level
  double h;            // box size at this level
  double lo[3];        // root-cube corner
  double k;            // wave number of the group's layer
  int64_t n;           // total particles (sorted arrays' length)
  const double* xs;    // sorted positions SoA [3][n]
  const double2* q;    // sorted charges [rhs][n]
  double2* phi;        // sorted potentials [rhs][n]
  const int* leaf_start;
  const int* leaf_count;
  int64_t leaf_base;   // offset of this group's leaves in leaf_start/count
  const int* mi;       // packed multi-indices k1 | k2<<8 | k3<<16, graded order
  double2* alpha;      // this level [rhs][box][nC]
  double2* beta;
  int64_t rhs_stride;  // per-rhs stride of alpha/beta at this level (elements)
  const double2* alpha_child;
  int64_t rhs_stride_child;
  const double2* beta_parent;
  int64_t rhs_stride_parent;
};

// Per-box change of representation between the full Taylor coefficients (C(p+3,3),
// graded order) and the Helmholtz-reduced set (k1 <= 1, (p+1)^2 entries).
struct ReduceArgs {
  int p, nC, nR;
  double kh2;            // (k h)^2 at this level
  const int* mi;         // [nC] packed graded multi-indices
  const int* rfull;      // [nR] graded index of each reduced entry
  const double* scale;   // [nC] (-1)^{|k|}/k!  (reduce)
  const double* invfact; // [nC] 1/k!          (expand)
  const double2* in;     // reduce: alpha^ [rhs][box][nC];  expand: b [rhs][box][nR]
  double2* out;          // reduce: a [rhs][box][nR];      expand: beta^ [rhs][box][nC]
  float2* out32;         // reduce: if set, a in FP32 here instead of out (mixed precision)
  int64_t in_stride, out_stride;  // per-rhs strides (elements)
  int nsplit;            // expand: partial sets of b to sum (1 if unsplit)
  int64_t split_stride;  // elements between partial sets
};

// One tree level of the M2L launch.
struct M2LLevel {
  int n;                 // boxes per dimension
  int leaf;              // leaf level: neighbour offsets take part
  int tiles_x, tiles_y, ntiles;
  int near_fd, near_s;
  const double2* a;      // reduced scaled moments [rhs][box][nR]
  const float2* a32;     // the same in FP32 (mixed precision)
  double2* b;            // reduced locals [rhs][box][nR]
  int64_t rhs_stride;
  const double2* Tfd;    // [343][nG] free + Delta (|d|>=2) and Delta-only (|d|<=1) or null
  const double2* TS;     // [49 (2n-1)][nG] Sigma family or null
  const float2* Tfd32;   // FP32 copies (mixed precision)
  const float2* TS32;
  int64_t split_stride;  // elements between the partial outputs of the offset splits
  const unsigned char* occ;  // [n^3] 1 where the box holds particles, or null (all counted occupied):
                             // empty targets get zero locals, empty sources are not staged
};

constexpr int M2L_MAX_LEVELS = 8;

struct M2LArgs {
  int nR, nRs, nKB, nRB; // reduced coefficients, LDS row stride, K blocks of 4, row blocks of 16
  int nG, p, P2;         // compact table size, order, 2p + 1
  int nlev;              // levels in this launch; the last one is the widest
  int ncb;               // targets per workgroup / 16: 1 or 2, 0 = automatic
  int nsplit;            // the offsets of a tile are split over nsplit workgroups (blockIdx.z),
                         // each writing its own partial locals (summed in fixed order by k_expand)
  int kph, kpb, nRsP;    // source moments staged in kph phases of kpb blocks of 4 (LDS row stride nRsP)
  int ksplit;            // 1: one or two row-block tiles left over after 4 per wave are split along K
  int tile_start[M2L_MAX_LEVELS + 1];
  M2LLevel lev[M2L_MAX_LEVELS];
  const int* rmi;        // [nR] packed reduced multi-indices
  const int* gpad;       // [nG] position of each compact table entry in the padded LDS layout
};

// Cross-layer translation (target layer group vs source layer groups), list driven.
struct CrossEntry {
  int src;          // source group index
  int dx, dy, izs;  // source box offset (x, y) and absolute z index in the source grid
  int key;          // table key
};

struct M2LCrossLevel {
  int n, tiles_x, tiles_y, ntiles;
  const int* list_start;   // [4 n + 1]: entries of (parity class px + 2 py, iz_t) at 4 iz_t + pc
  const CrossEntry* list;
  double2* b;              // z-reduced locals of the target group [rhs][box][nR]
  int64_t rhs_stride;
  const double2* T[2];     // tables per k3' in {0, 1}: [nkeys][nG] (swapped frame)
  const float2* T32[2];
  const double2* asrc[MAX_LAYERS];  // z-reduced moments of each source group at this level
  int64_t src_stride[MAX_LAYERS];
  int64_t split_stride;    // elements between the partial outputs of the list splits
};

struct M2LCrossArgs {
  int nR, nRs, nKB, nRB, nG, p, P2;
  int nlev;
  int nsplit;              // list entries of a tile split over nsplit workgroups (blockIdx.z)
  int tile_start[M2L_MAX_LEVELS + 1];
  M2LCrossLevel lev[M2L_MAX_LEVELS];
  const int* rzmi;         // [nR] z-reduced multi-indices (packed)
  const int* gpadz;        // [nG] padded LDS position of each swapped-frame entry, -1 if unused
};

hipError_t launch_m2l_cross(const M2LCrossArgs& a, int nrhs, bool fp32, hipStream_t s);

// Direct evaluation of the Sigma-family reaction kernel (the same-layer reaction
// component that depends on z + z') for the leaf pairs whose expansion about the box
// centres would not converge (boxes next to an interface): for each target in a listed
// leaf, phi += sum over its listed source leaves of q_j K(x - x', y - y', z + z') with
// K = sum_img A e^{ikR}/R, R^2 = rho^2 + zeta^2, zeta = z + z' - 2 d_l - Z (up-going
// family) or 2 d_{l-1} - z - z' - Z (down-going family), terms with Re zeta <= 0 left out
// as in the tables.  FP64.
constexpr int SIGMA_DIRECT_MAX_IMAGES = 128;
struct SigmaDirectArgs {
  const double* xs;        // sorted positions SoA [3][n]
  int64_t n;
  const double2* q;        // sorted charges [rhs][n]
  double2* phi;            // sorted potentials [rhs][n] (accumulated)
  const int* leaf_start;
  const int* leaf_count;
  int64_t leaf_base;
  const int* tgt;          // [ntgt] listed target leaves (grid index in the group)
  const int* src_start;    // [ntgt + 1]
  const int* src;          // source leaves of each target leaf
  const double2* img;      // [2 (nup + ndn)]: A_j, Z_j of the up-going images, then the down-going ones
  int nup, ndn;
  double two_dl, two_dt;   // 2 d_l and 2 d_{l-1}
  double k;
};
__global__ void k_sigma_direct(SigmaDirectArgs a);

void upload_binomials();

template <int NW>
__global__ void k_table_gen(TableGenArgs a);  // NW = 1, 2, 4, 8 waves per key
// FP32 copy of an FP64 complex array (the mixed mode's tables)
__global__ void k_to_f32(const double2* in, size_t n, float2* out);
// Rotation-free derivatives H_{m,c} = (2 d_{rho^2})^m d_S^c of the Sigma-family kernel
// (m + c <= P2 <= SIGMA_P2_MAX), their normalisation for the surrogate network, and the
// compact Cartesian table rows rebuilt from them.
constexpr int SIGMA_P2_MAX = 32;
constexpr int SIGMA_H_MAX = (SIGMA_P2_MAX + 1) * (SIGMA_P2_MAX + 2) / 2;
__global__ void k_sigma_h(const double* w, const double* S, int n, const double2* img, int nup, int ndn,
                          double two_dl, double two_dt, double k, int P2, double2* H);
__global__ void k_sur_normalize(const double2* H, const double2* Hq, const double* Re, int n, int P2, int env,
                                double2* W, double* sumsq);
__global__ void k_sur_targets(const double2* W, int n, int nH, const float* sigma, float* T);
__global__ void k_sur_h_from_net(const float* y, const double* Re, int n, int P2, const float* sigma, int env,
                                 double2* H);
__global__ void k_sigma_restore(const double2* H, const double* X, const double* Y, int nk, const int* row, double h,
                                double k, int P2, int nG, const unsigned char* g1s, const unsigned char* g3s,
                                const unsigned char* gord, double2* out, const int* hrow, int accumulate);
// Sigma-family H_{m,c} from the Sommerfeld integrals on the deformed contour
__global__ void k_som_radial(const double2* krho, int nn, const double* rho, int M, double2* A);
__global__ void k_som_vertical(const double2* kz, const double2* cu, const double2* cd, int nn, const double* S,
                               double two_dl, double two_dt, int has_up, int has_dn, double zeta_eps, int M,
                               double2* B);
__global__ void k_som_contract(const double2* A, const double2* B, int nn, int M, const int* pr, const int* ps,
                               double2* H);
__global__ void k_taylor_points(const double* px, const double* py, const double* pz, double k, double h,
                                int order, int nT, const short* nbr, double2* out);
__global__ void k_selftest_mfma(double* out64, float* out32);
__global__ void k_layer_stats(const double* xyz, int64_t n, int nif, const double* ifz, double eps,
                              double* part, int* bad);
__global__ void k_leaf_keys(const double* xyz, int64_t n, int nif, const double* ifz, TreeGeom geo,
                            unsigned* keys, int* perm);
__global__ void k_count_keys(const unsigned* keys, int64_t n, int* count);
__global__ void k_gather_pos(const double* xyz, const int* perm, int64_t n, double* xs);
__global__ void k_gather_q(const double2* q, const int* perm, int64_t n, double2* qs);
__global__ void k_finalize(const double2* phi_s, const double2* phi_near, const int* perm, int64_t start, int64_t cnt,
                           int64_t n, double sr, double si, double2* out);
__global__ void k_p2m(PassArgs a);
__global__ void k_reduce(ReduceArgs a);
__global__ void k_expand(ReduceArgs a);
__global__ void k_reduce_z(ReduceArgs a);
__global__ void k_expand_z_add(ReduceArgs a);
__global__ void k_m2m(PassArgs a);
__global__ void k_l2l(PassArgs a);
__global__ void k_l2p(PassArgs a);
// Coefficients of the FP32 near-field pair value as quadratics in s = r^2 (scaled
// units, r = k |x - y| / (2 pi)): cos(2 pi r) ~ c0 + c1 s + c2 s^2 and
// sin(2 pi r) / r ~ s0 + s1 s + s2 s^2.
struct NearPoly {
  float c0, c1, c2, s0, s1, s2;
};
// Near-field work items (leaves, or leaf G + half for the symmetric kernel) cut into 8
// contiguous segments of about equal pair work, one per XCD: segment x is
// items[start[x] .. start[x + 1]).
struct XcdSegs {
  int start[9];
};
template <typename T, int BS, int RB, bool POLY>
__global__ void k_p2p(PassArgs a, int nrhs, NearPoly np, const unsigned* items, XcdSegs seg);
template <typename R>
struct SymTypes;
template <>
struct SymTypes<float> {
  typedef float4 R4;
  typedef float2 R2;
};
template <>
struct SymTypes<double> {
  typedef double4 R4;
  typedef double2 R2;
};
template <typename R, int T, int NW, bool POLY>
__global__ void k_p2p_sym(PassArgs a, int nrhs, int G, typename SymTypes<R>::R2* part, NearPoly np,
                          const unsigned* items, XcdSegs seg);
template <typename R2>
__global__ void k_p2p_sym_gather(PassArgs a, int nrhs, int tp, int G, const R2* part);

// Near fields of several geometries in one persistent launch: a work queue of
// (geometry, phase, tile) items taken in ticket order, first the symmetric-pair items
// (one per leaf and workgroup index, longest first), then one gather item per
// non-empty leaf, which waits until its geometry's pair items are done.  Items are
// packed geometry << 24 | index.  One charge vector.
struct NFQueueGeom {
  PassArgs a;    // a.phi: the geometry's near-field sums
  NearPoly np;
  void* part;    // source-side slot sums (float2 or double2)
  int G, tpl, poly;
  int p2p_items, gather_items;  // pair items of this geometry in the list; unused
};
struct NFQueueArgs {
  const NFQueueGeom* geo;
  int ngeo;
  const unsigned* items;    // n_p2p pair items, then n_gather gather items
  int n_p2p, n_gather;
  unsigned* ticket;         // next item
  unsigned* done;           // [ngeo] pair items finished
  int* err;                 // set to 1 when a wait gives up (spin_limit polls)
  int spin_limit;
};
template <typename R>
__global__ void k_nf_queue(NFQueueArgs q);
__global__ void k_nf_queue_reset(unsigned* ticket, unsigned* done, int ngeo, int* err);

// GMRES vector kernels (complex128): multi-column dot products in two stages, basis
// updates, axpby.
constexpr int GM_BLOCKS = 512;
__global__ void k_gm_multidot(const double2* V, int64_t ld, int ncol, const double2* w, int64_t n, double2* partial);
__global__ void k_gm_reduce(const double2* partial, int nblk, double2* out);
__global__ void k_gm_update(const double2* V, int64_t ld, int ncol, const double2* coef, double sgn, double2* w,
                            int64_t n);
__global__ void k_gm_axpby(double2 a, const double2* x, double2 b, double2* y, int64_t n);

// M2L launcher (picks the row-block instantiation for nRB).
hipError_t launch_m2l(const M2LArgs& a, int nrhs, bool fp32, hipStream_t s);

}  // namespace tefmm
