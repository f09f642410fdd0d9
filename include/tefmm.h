/*
 * tefmm.h -- C ABI of the MI355X Taylor-expansion FMM for the 3-D Helmholtz
 * sum in horizontally layered media.
 *
 * Computes, for every particle i (sources = targets),
 *
 *   phi_i = sum_{j != i, same layer} q_j exp(i k_l R_ij) / (4 pi R_ij)
 *         + sum_j q_j G^r_{l_i l_j}(r_i, r_j)                       (1)
 *
 * (Eq. totalinteraction, Sec. 3.2; the reaction part G^r is the Sommerfeld
 * integral of Eq. greenfuncomponent / Eq. totaldensity, Sec. 2.1).  The free
 * part excludes j = i, the reaction part includes it.  Results are returned
 * in physical normalisation (the paper's kernels times i k_l / 4 pi) unless
 * TEFMM_NORM_PAPER is requested.
 *
 * The layered medium follows Sec. 2.1: n_layers = L+1 layers, interfaces
 * d_0 > d_1 > ... > d_{L-1}, wave number k_l in layer l, layer 0 on top;
 * transmission conditions u and k du/dz continuous.
 *
 * Error behaviour: every function returns an int status (TEFMM_OK = 0, a
 * negative TEFMM_ERR_* otherwise) and never throws across the ABI; a
 * human-readable message for the last failure on a handle is available from
 * tefmm_last_error().  A handle is not thread safe: one handle serves one
 * host thread and one stream at a time.
 *
 * Memory: pointers marked "device" must be device memory of the current HIP
 * device (e.g. torch tensors on cuda:0); the caller owns them.  The library
 * owns its tree, expansions and tables (device memory it allocates with
 * hipMalloc, or from the caller's allocator of tefmm_set_allocator, and frees
 * by tefmm_destroy).
 */
#ifndef TEFMM_H
#define TEFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TEFMM_OK = 0,
  TEFMM_ERR_INVALID_ARG = -1,
  TEFMM_ERR_PARTICLE_ON_INTERFACE = -2,
  TEFMM_ERR_UNSUPPORTED = -3,
  TEFMM_ERR_HIP = -4,
  TEFMM_ERR_DCIM_FIT = -5,
  TEFMM_ERR_OOM = -6,
  TEFMM_ERR_STATE = -7
};

/* Precision.  TEFMM_FP64: every step in FP64.  TEFMM_MIXED_FP32: the M2L
 * contractions (FP32 MFMA, FP32 accumulation within one launch) and the P2P
 * sums run in FP32.  Near-field pairs closer than 5% of the leaf side, whose FP32
 * coordinate differences have lost digits, take those differences from the FP64
 * positions: with one charge vector (each pair evaluated once) the pair value and
 * its accumulation then stay FP32 (the digits lost were those of the difference);
 * with several vectors the pair is redone in FP64 and summed in FP64.
 * Complex-image fits, table generation, P2M/M2M/L2L/L2P and the final
 * accumulation of the potential stay FP64. */
enum { TEFMM_FP64 = 0, TEFMM_MIXED_FP32 = 1 };
enum { TEFMM_NORM_PHYSICAL = 0, TEFMM_NORM_PAPER = 1 };

typedef struct tefmm_ctx* tefmm_t;

/* Layered medium of Sec. 2.1.  interfaces: n_layers-1 strictly decreasing
 * heights; k: n_layers real wave numbers > 0, top to bottom; at most
 * TEFMM_MAX_LAYERS layers. */
#define TEFMM_MAX_LAYERS 8
typedef struct {
  int n_layers;
  const double* interfaces;
  const double* k;
} tefmm_medium;

/* Method parameters.  p: Taylor order (|k| <= p, full truncation of the
 * translation operators, Sec. 3.1).  depth: uniform octree depth per layer
 * (0 = choose the smallest depth with mean occupancy <= max_leaf).
 * DCIM parameters (Sec. 3.3): dcim_T1 and dcim_samples per level, relative
 * singular-value cut dcim_svd_tol; dcim_T1_cross is the length of the second
 * sampling path for the cross-layer fits (their spectral functions have
 * branch points of the other layers near the path, and a longer second path
 * moves the misfit away from the spatial range used).  interface_eps: minimum
 * distance of a particle from an interface (the Sommerfeld integrals diverge
 * on them). */
typedef struct {
  int p;
  int depth;
  int max_leaf;
  int precision;      /* TEFMM_FP64 or TEFMM_MIXED_FP32 */
  int normalization;  /* TEFMM_NORM_PHYSICAL or TEFMM_NORM_PAPER */
  double dcim_T1;
  int dcim_samples;
  double dcim_svd_tol;
  double interface_eps;
  int n_rhs_max;
  double dcim_T1_cross;
  int m2l_tile;       /* M2L targets per workgroup / 16: 1 or 2 (0 = automatic; tefmm_autotune measures) */
  int p2p_targets;    /* near field with one charge vector: 1, 2 or 4 = each pair of particles in
                         different leaves is evaluated once and its kernel value applied in both
                         directions, with that many targets per GPU lane (FP64: 1 or 2, 4 is
                         rejected); 0 = that kernel with 2 targets per lane above a mean
                         occupancy of 96 over the occupied leaves, else 1; -1 = every ordered
                         pair evaluated on its own
                         (also the kernel for several charge vectors) */
  int p2p_poly;       /* FP32 near field (both kernels): 0 = the pair value e^{ikr}/r from
                         two quadratics in r^2 fitted on the host over the distances of a leaf's
                         3 x 3 x 3 block (k r is small there), used where the fit is within 3e-7 of
                         cos(k r) and sin(k r) (see p2p_poly_err; else, and with -1, the hardware
                         sine and cosine) */
  int sigma_tables;   /* translation tables of the same-layer reaction terms: the Sigma families
                         (which depend on z + z') and the Delta family (on z - z').
                         TEFMM_SIGMA_IMAGES from the complex images (Sec. 3.3);
                         TEFMM_SIGMA_SOMMERFELD from the Sommerfeld integrals of the
                         rotation-free derivatives on the deformed contour of Sec. 4.2 (the
                         integrals of Eq. symmetricdetable, no fit), rebuilt exactly into the
                         Cartesian rows.  Rows answered by an attached surrogate stay the
                         surrogate's; the near-interface pairs evaluated directly keep the
                         images. */
} tefmm_options;
enum { TEFMM_SIGMA_IMAGES = 0, TEFMM_SIGMA_SOMMERFELD = 1 };

/* Timings (ms, measured with HIP events; averages over the evaluations since
 * the last tefmm_reset_timers, at most the last 64) and counters.  The far
 * field (P2M .. L2P) runs on the caller's stream; the near field (P2P) runs
 * concurrently on a second stream of the handle (by default; see
 * tefmm_autotune), joined before the final scaling, so t_p2p_ms overlaps the
 * far-field phases and t_total_ms is the whole evaluation.  Set-up timings of the
 * last tefmm_set_particles: t_setup_tree_ms (bounding cubes, sort, leaf ranges),
 * t_setup_tables_ms (lists, complex images, derivative tables, cross-layer fits and
 * tables), and within it t_setup_dcim_ms (host wall time of the same-layer
 * complex-image fits, Sec. 3.3, run on host threads). */
typedef struct {
  double t_setup_tree_ms, t_setup_tables_ms, t_setup_dcim_ms;
  double t_p2m_ms, t_m2m_ms, t_m2l_ms, t_l2l_ms, t_l2p_ms, t_p2p_ms, t_total_ms;
  int64_t m2l_pairs, p2p_pairs;
  int n_images[3 * TEFMM_MAX_LAYERS];       /* DCIM image counts of the fitted families */
  double dcim_fit_err[3 * TEFMM_MAX_LAYERS]; /* max relative misfit on the sampling paths */
  int depth[TEFMM_MAX_LAYERS]; /* tree depth per layer group (0 if none), groups in layer order */
  int n_families;
  double m2l_flops;      /* algorithmic M2L flops of the last evaluate: 8 (p+1)^4 per
                            (target box, source box, family) contraction, times n_rhs */
  int m2l_launches;      /* M2L kernel launches of the last evaluate */
  int n_rhs;             /* charge vectors of the last evaluate */
  int64_t cross_pairs;   /* cross-layer (target box, source box) translations per charge vector */
  int64_t cross_pairs_forced; /* of those, leaf pairs that fail the acceptance test sqrt(3) h <= 0.6 D
                                 (translated anyway: less accurate; zero with the automatic depth
                                 unless the depth limit 7 is reached) */
  int n_cross_fits;      /* cross-layer complex-image fits of the geometry */
  double cross_fit_err;  /* their largest relative misfit on the sampling paths */
  int64_t sigma_keys;    /* rows of the Sigma-family tables of the geometry */
  int64_t surrogate_keys; /* of those, rows produced by the attached surrogate network */
  int timed_evaluations; /* evaluations the phase times t_p2m_ms .. t_total_ms average over */
  int64_t p2p_pairs_same_leaf; /* of p2p_pairs, the ordered pairs inside one leaf */
  double p2p_poly_err;   /* largest error of the near-field quadratics in use (of cos(k r) and of
                            r sin(k r) / r, relative to the pair value's size 1/r); 0 if none */
  int64_t sigma_direct_pairs; /* particle pairs (per charge vector) whose Sigma-family reaction
                                 term is evaluated directly from the complex images: leaf pairs
                                 next to an interface, where the expansion about the box centres
                                 would converge slowly or not at all (ratio sqrt(3) h / distance
                                 of the key's centre from the mirror point above 0.75) */
  int64_t occupied_leaves; /* leaves holding particles, over all layer groups */
  int64_t max_leaf_count;  /* particles in the fullest leaf */
  int64_t reaction_keys_forced; /* (level, z-slab pair) translations of a reaction family with
                                   that ratio above 0.87 (converging slowly or not at all:
                                   boxes reaching close to an interface, or a layer thin
                                   against the boxes); zero in the usual configurations */
  int64_t sigma_quad_nodes; /* TEFMM_SIGMA_SOMMERFELD: contour nodes of the largest Sigma
                               quadrature of the geometry (0 otherwise) */
  int64_t sigma_quad_keys;  /* TEFMM_SIGMA_SOMMERFELD: Sigma rows produced from the integrals */
} tefmm_stats;

/* Fill an options struct with the defaults (p = 8, depth auto, max_leaf 64,
 * FP64, physical normalisation, T1 = 10, 101 samples, tol 1e-12,
 * interface_eps 1e-9, n_rhs_max 64, T1 = 30 for the cross-layer fits). */
void tefmm_default_options(tefmm_options* opt);

/* Create a handle for a medium: validates the medium and options and uploads
 * the small index tables of order p to the current HIP device.
 * Returns TEFMM_ERR_INVALID_ARG for non-decreasing interfaces, k <= 0,
 * p outside [1, 16] or more than TEFMM_MAX_LAYERS layers, TEFMM_ERR_HIP if the device
 * tables cannot be allocated. */
int tefmm_create(tefmm_t* out, const tefmm_medium* medium, const tefmm_options* opt);

/* Device allocator of a handle (e.g. a framework's caching allocator).  Every
 * device buffer the handle owns (index tables, sorted particles, tree arrays,
 * expansions, derivative tables, set-up temporaries) is then taken from
 * alloc(bytes, user) and given back with free(ptr, user); alloc returns NULL
 * when it cannot serve the request (the call in progress then fails with
 * TEFMM_ERR_OOM).  Both NULL restores hipMalloc / hipFree.  Memory is used on
 * the streams passed to tefmm_set_particles / tefmm_evaluate (and, joined back
 * to them, on the handle's own second stream), and freed at set-up of the next
 * geometry or at tefmm_destroy.  The call releases what the handle holds (with
 * the allocator that gave it) and uploads the index tables again, so the
 * geometry must be set again afterwards.  Synchronous. */
typedef void* (*tefmm_alloc_fn)(size_t bytes, void* user);
typedef void (*tefmm_free_fn)(void* ptr, void* user);
int tefmm_set_allocator(tefmm_t h, tefmm_alloc_fn alloc, tefmm_free_fn free, void* user);

/* Set the particle geometry.  xyz_soa: 3*n doubles, x[0..n) then y then z,
 * device memory (on_device = 1) or host memory (on_device = 0).  Builds the
 * per-layer octrees on the GPU, fits the discrete complex images
 * (Sec. 3.3, two-level GPOF) on the host and generates the derivative
 * tables on the GPU.  stream: hipStream_t (NULL = default stream).  Fails
 * with TEFMM_ERR_PARTICLE_ON_INTERFACE if a particle lies within
 * interface_eps of an interface.  With particles in several layers all layer
 * trees share one x-y box grid, one box side and one depth (the common grid of
 * the cross-layer translations, Algorithm 2); each cube is placed inside its
 * layer when the layer is thick enough, and TEFMM_ERR_UNSUPPORTED is returned
 * when a box holding particles would have its centre outside its layer. */
int tefmm_set_particles(tefmm_t h, int64_t n, const double* xyz_soa, int on_device, void* stream);

/* Evaluate (1) for n_rhs charge vectors.  q: device, complex128 interleaved
 * (re, im), column-major n x n_rhs (vector r starts at q + 2*n*r).
 * phi: device, same layout, written (not accumulated), in the caller's
 * particle order.  Stream ordered on `stream`: the near field forks to the
 * handle's second stream (after the charges are read, or after the upward
 * pass: by default in FP64; the autotuner may also keep it on `stream`) and
 * joins back before the result is written, by events (when `stream` is being
 * captured into a graph the near field stays on `stream`).  Returns after enqueueing (call
 * hipStreamSynchronize to wait). */
int tefmm_evaluate(tefmm_t h, const double* q, int n_rhs, double* phi, void* stream);

/* Integral-equation driver (the application the method serves, Sec. 1: iterative
 * solvers apply the potential operator many times): GMRES(restart) for
 *   (I - tau G) x = b,
 * G the operator of (1) as tefmm_evaluate computes it with one charge vector
 * (physical or paper normalisation per the options), tau a complex scalar (for
 * point scatterers of strength tau this is the Foldy-Lax system of multiple
 * scattering in the layered medium).  b, x: device, complex128 interleaved, n
 * entries in the caller's particle order; x is the initial guess if x0_given,
 * else x = 0 to start; x receives the solution.  Stops when the relative
 * residual ||b - A x|| / ||b|| is <= tol (the true residual, recomputed at each
 * restart) or after max_iter steps; restart in [1, 200].  Work space of
 * (restart + 3) n complex128 from the handle's allocator.  Synchronous on
 * `stream`.  info (may be NULL) gets the steps, operator applications, final
 * relative residual and whether tol was reached. */
typedef struct {
  int iterations;
  int matvecs;
  double rel_residual;
  int converged;
} tefmm_gmres_info;
int tefmm_gmres(tefmm_t h, double tau_re, double tau_im, const double* b, double* x, int x0_given, int restart,
                int max_iter, double tol, void* stream, tefmm_gmres_info* info);

/* Batched evaluation of n_geom handles, each with its own geometry, charges
 * q[g] (n_rhs[g] vectors, layout as in tefmm_evaluate) and output phi[g].
 * The handles' evaluation sequences are captured once into a HIP graph, one
 * stream branch per geometry so that independent geometries run concurrently,
 * and the graph is replayed by later calls with the same handles, pointers and
 * n_rhs (a changed list, or a handle whose geometry or buffers changed since,
 * triggers a new capture).  The graph reads q[g] at replay time.  The graph is
 * owned by hs[0].  Returns after enqueueing on `stream`.  All handles must be
 * distinct and ready; per-phase timings are not recorded for batched calls. */
int tefmm_evaluate_batch(tefmm_t* hs, int n_geom, const double* const* q, const int* n_rhs,
                         double* const* phi, void* stream);

/* The same batched evaluation with the near fields of all geometries in one
 * persistent launch (the C5 batching of the paper's workloads, E2): a work queue
 * of (geometry, phase, tile) items, taken in ticket order by a fixed grid of
 * workgroups: first the symmetric near-field items of every geometry and layer
 * group (workgroup h of leaf A, Sec. 3.2's local direct interactions), then one
 * gather item per leaf, which waits until its geometry's near-field items are done
 * (a bounded wait; see tefmm_batch_check).  The far fields stay graph branches, one
 * per geometry, running beside the queue; each geometry's final scaling follows the
 * queue.  Needs one charge vector per geometry, one precision for all handles and
 * the symmetric near field with 1 or 2 targets per lane (tefmm_options.p2p_targets),
 * else TEFMM_ERR_UNSUPPORTED.  Results equal tefmm_evaluate_batch's bit for bit (the
 * same per-item arithmetic in the same order).  The graph and the queue's work list
 * (allocated with hs[0]'s allocator) are owned by hs[0]. */
int tefmm_evaluate_batch_queue(tefmm_t* hs, int n_geom, const double* const* q, const int* n_rhs,
                               double* const* phi, void* stream);

/* Synchronise `stream` and report whether the last queue launch of the batch owned by
 * h had a gather item stop waiting (after about 4M polls: TEFMM_ERR_STATE, its
 * results are wrong); TEFMM_OK otherwise (also for a batch without a queue). */
int tefmm_batch_check(tefmm_t h, void* stream);

/* Autotuner: times the evaluation of the handle's own geometry (unit charges)
 * for tree depths d-1, d, d+1 (d the current depth, clamped to [2, 7]) and for
 * 16 or 32 target boxes per M2L workgroup, then rebuilds the handle with the
 * fastest choice; for it, also whether the near field runs beside the far field
 * from the start, beside it from the end of the upward pass (P2M, M2M), or before
 * it on the same stream, keeping the fastest.  *depth_out / *ncb_out
 * (may be NULL) receive the depth and tile width.  Synchronous. */
int tefmm_autotune(tefmm_t h, void* stream, int* depth_out, int* ncb_out);

/* Statistics of the last set_particles / evaluate (timings need the stream
 * to have completed; this call synchronises it). */
int tefmm_get_stats(tefmm_t h, tefmm_stats* st);
/* Start a new averaging window for the phase times of tefmm_get_stats. */
int tefmm_reset_timers(tefmm_t h);

const char* tefmm_last_error(tefmm_t h);
void tefmm_destroy(tefmm_t h);

/* ----------------------------------------------------------------------
 * Introspection entry points (host FP64 or single kernels), used to check
 * individual steps against the oracle.
 * ---------------------------------------------------------------------- */

/* Reaction densities sigma^{ab}_{m,lp}(k_rho) of Eq. updownspectraldoamin
 * for a source in layer lp at n complex points krho (interleaved).  out:
 * host, complex interleaved, 4*(L+1)*n entries ordered
 * [m][ab][point] with ab = uu, ud, du, dd (absent entries are zero).
 * Up-going waves are referenced at a layer's lower interface, down-going
 * waves at its upper interface.  Pure host call. */
int tefmm_densities(const tefmm_medium* medium, int lp, int n, const double* krho, double* out);

/* Discrete complex images of the same-layer reaction families of layer l
 * (Sec. 3.3, Eq. compleximageapp, two-level GPOF): family 0 = Sigma-up
 * (sigma^{uu}, exponent z + z' - 2 d_l), 1 = Sigma-down (sigma^{dd},
 * exponent 2 d_{l-1} - z - z'), 2 = Delta (sigma^{ud} = sigma^{du},
 * exponents D +- (z - z')).  z_lo, z_hi: range of particle heights in the
 * layer (sets the decay shift z_min of the paper).  On return *m holds the
 * image count; amp/depth (host, complex interleaved, capacity cap) the
 * amplitudes A_j and complex depths of the kernel representation
 *   K(rho, Z) = sum_j A_j exp(i k R_j) / (4 pi R_j),  R_j = sqrt(rho^2 + (Z - depth_j)^2)
 * where Z is the family's exponent.  *fit_err gets the largest relative
 * misfit on the sampling paths.  Pure host call. */
int tefmm_dcim_family(const tefmm_medium* medium, const tefmm_options* opt, int l, int family,
                      double z_lo, double z_hi, int cap, int* m, double* amp, double* depth,
                      double* fit_err);

/* Cross-layer complex images (Sec. 3.3: one fit per source height and z'
 * derivative order): target layer l, source layer lp != l, target-side wave
 * a (0 = up-going, 1 = down-going), source height zs, derivative order k3p;
 * z_lo, z_hi: the target particles' height range.  The kernel
 *   d^{k3p}/dz'^{k3p} G^{(a)}_{l,lp}(r, r') / k3p!  at z' = zs
 * equals sum_j A_j exp(i k_l R_j) / (4 pi R_j), R_j = sqrt(rho^2 + (Z - depth_j)^2),
 * Z = z - d_l (a = 0) or d_{l-1} - z (a = 1).  Output as for tefmm_dcim_family.
 * Pure host call. */
int tefmm_dcim_cross(const tefmm_medium* medium, const tefmm_options* opt, int l, int lp, int a, double zs,
                     int k3p, double z_lo, double z_hi, int cap, int* m, double* amp, double* depth,
                     double* fit_err);

/* Rotation-free derivatives of the Sigma-family kernel of layer `layer`
 * (Sec. 4.2; the same-layer reaction terms with sigma^{uu} and sigma^{dd},
 * which depend on rho and S = z + z'):
 *   H_{m,c}(rho, S) = (2 d_w)^m d_S^c K,  w = rho^2,  m + c <= 2p (p of the handle),
 * K = 4 pi G in the physical normalisation (the form sum_j A_j e^{ikR_j}/R_j of the
 * images), stored at index (m + c)(m + c + 1)/2 + m.  With u = x + i y the Cartesian
 * derivatives follow as (d_x + i d_y)^m d_S^c K = u^m H_{m,c}.
 * method TEFMM_SIGMA_IMAGES: from the complex images of the layer's families, fitted
 * for the height range min(S)/2 .. max(S)/2 (Sec. 3.3);
 * TEFMM_SIGMA_SOMMERFELD: from the Sommerfeld integrals on the deformed contour of
 * Sec. 4.2 (the integrals of Eq. symmetricdetable in rotation-free form; the
 * k_rho -> infinity limit of each density is the image at the mirror point, added
 * exactly).  rho, S: host arrays of n >= 1 values, S with both mirror distances
 * S - 2 d_l and 2 d_{l-1} - S positive where the interface exists; out: host array
 * of n (2p+1)(2p+2)/2 complex values (re, im interleaved), written on success.
 * Needs no particles; synchronous on `stream`.  Errors: TEFMM_ERR_INVALID_ARG (bad
 * layer, method, size or a point outside the layer), TEFMM_ERR_UNSUPPORTED (layer
 * without interfaces, or 2p above 32), TEFMM_ERR_DCIM_FIT, TEFMM_ERR_HIP. */
int tefmm_sigma_derivatives(tefmm_t h, int layer, int method, int64_t n, const double* rho, const double* S,
                            double* out, void* stream);

/* The same for the Delta family of layer `layer` (the same-layer reaction terms with
 * sigma^{ud} e^{i k_z (D + w)} and sigma^{du} e^{i k_z (D - w)}, D the layer's thickness,
 * which depend on rho and w = z - z'; Sec. 3.3 and Sec. 4.2):
 *   H_{m,c}(rho, w) = (2 d_v)^m d_w^c K,  v = rho^2,  m + c <= 2p,
 * stored as for tefmm_sigma_derivatives; d_w is the target's z derivative.
 * TEFMM_SIGMA_IMAGES: from the family's complex images, fitted for heights spanning the
 * largest |w|, each at D + w and D - w; TEFMM_SIGMA_SOMMERFELD: from the Sommerfeld
 * integrals on the contour of Sec. 4.2 (these densities vanish as k_rho grows, so there
 * is no mirror-point image).  rho, w: host arrays of n >= 1 values with |w| < D; out:
 * host array of n (2p+1)(2p+2)/2 complex values, written on success.  Needs no
 * particles; synchronous on `stream`.  Errors: TEFMM_ERR_INVALID_ARG (bad layer, method,
 * size or |w| >= D), TEFMM_ERR_UNSUPPORTED (a layer without two interfaces, or 2p above
 * 32), TEFMM_ERR_DCIM_FIT, TEFMM_ERR_HIP. */
int tefmm_delta_derivatives(tefmm_t h, int layer, int method, int64_t n, const double* rho, const double* w,
                            double* out, void* stream);

/* Rotation-free derivatives of the cross-layer reaction kernel, target in layer `layer`
 * and source in layer `src_layer` (Algorithm 2's components between different layers;
 * Sec. 4.2): H_{m,c}(rho, z, z') = (2 d_v)^m d_z^c d_{z'}^{k3} K, v = rho^2, m + c <= 2p,
 * K = i int k_rho J0(k_rho rho) / k_z sum_{a,b} P_a(z) sigma^{ab} E_b(z') dk_rho in the
 * physical normalisation (k_z of the target layer, P_a the target layer's waves, E_b
 * the source layer's), stored as for tefmm_sigma_derivatives, from the Sommerfeld
 * integrals on the contour of Sec. 4.2 (the route of the cross tables under
 * TEFMM_SIGMA_SOMMERFELD).  rho, z, zs: host arrays of n (1 .. 4096) values with z inside
 * `layer` and zs inside `src_layer`; 0 <= k3 <= p; out: host array of n (2p+1)(2p+2)/2
 * complex values, written on success.  Synchronous on `stream`.  Errors:
 * TEFMM_ERR_INVALID_ARG (equal or bad layers, k3, size, or a point outside its layer),
 * TEFMM_ERR_UNSUPPORTED (2p above 32), TEFMM_ERR_HIP. */
int tefmm_cross_derivatives(tefmm_t h, int layer, int src_layer, int k3, int64_t n, const double* rho,
                            const double* z, const double* zs, double* out, void* stream);

/* TEFMM-II (Sec. 4.1) in free space, symmetric basis (n, m, s), 0 <= s <= m <= n,
 * ordered by n, then m, then s (C(N+3,3) entries up to order N).
 * tefmm_sym_derivatives: D^s_{nm} h0(k|R|) (Eq. sysdifferential applied to h0, derivatives
 * in the first argument) for n <= order <= 32 at n_pts displacements R (host, 3 doubles
 * each, none zero), from the Theorem 4.2 ladder on Omega^m_n = h_n Y^m_n; out: host,
 * n_pts * C(order+3,3) complex (re, im interleaved).
 * tefmm_sym_m2l: the translation of Eq. M2Ltransop, beta_i = L(R_i) alpha_i with
 *   L[(n,m,s),(n',m',s')] = (-1)^n' D^{s+s'}_{n+n',m+m'} h0(k|R_i|) / (F(n,m,s) F(n',m',s')),
 *   F(n,m,s) = 2^m (n-m)! s! (m-s)!,
 * R_i = target centre - source centre (host, 3 doubles each, none zero); alpha, beta:
 * device arrays of n_pairs * C(p+3,3) complex (Eq. mecoefficients moments in, the local
 * coefficients of Corollary 4.1 out), p <= 16.  Both synchronous on `stream`, scratch from
 * hipMalloc; TEFMM_ERR_INVALID_ARG or TEFMM_ERR_HIP on failure. */
int tefmm_sym_derivatives(double k, int order, int64_t n_pts, const double* R, double* out, void* stream);
int tefmm_sym_m2l(double k, int p, int64_t n_pairs, const double* R, const double* alpha, double* beta,
                  void* stream);

/* Scaled Taylor coefficients h^{|g|} D^g f / g! of f = exp(i k R)/R at n
 * points (x, y, zeta) with complex zeta (device arrays x, y: n doubles;
 * zeta: 2n doubles interleaved), orders |g| <= order, on the GPU with the
 * derivative recurrence.  out: device, n * C(order+3,3) complex
 * interleaved, graded order (|g| ascending, then g1 descending, then g2
 * descending).  Single kernel, synchronous. */
int tefmm_taylor_coefficients(int n, const double* x, const double* y, const double* zeta,
                              double k, double h, int order, double* out);

/* The tree build's primitives, for checking them alone.  tefmm_radix_sort: stable
 * sort of n (key, value) pairs by the key bits [0, end_bit) (least significant digit
 * first, 4-bit digits, per-tile counts scanned in digit-major order; deterministic);
 * keys and vals are device arrays of n entries, sorted in place; 1 <= n <= 2^31 - 1,
 * 0 <= end_bit <= 32.  tefmm_exclusive_scan: out[i] = sum_{j < i} in[j] in unsigned
 * 32-bit arithmetic (wrapping), device arrays, in and out may be the same array.
 * Both take their scratch from hipMalloc, free it before returning and are
 * synchronous on `stream`.  Errors: TEFMM_ERR_INVALID_ARG, TEFMM_ERR_HIP. */
int tefmm_radix_sort(int64_t n, unsigned* keys, int* vals, int end_bit, void* stream);
int tefmm_exclusive_scan(int64_t n, const unsigned* in, unsigned* out, void* stream);

/* Multipole moments of the last evaluate (rhs 0) for layer group g at tree
 * level l: host copy, n_box * C(p+3,3) complex interleaved, boxes in
 * grid order (ix * n + iy) * n + iz, moments normalised by the box size. */
int tefmm_get_moments(tefmm_t h, int g, int level, double* out, int64_t cap);

/* Geometry of layer group g: *layer, *depth, centre/side of the root cube. */
int tefmm_get_tree(tefmm_t h, int g, int* layer, int* depth, double* centre3, double* side);

/* MFMA lane-layout self test: multiplies fixed 16x4 by 4x16 matrices in FP64
 * and FP32 on the GPU and returns 0 when the results match the host. */
int tefmm_selftest_mfma(void);

/* ------------------------------------------------------------------------
 * Surrogate network (an extension beyond the paper: a learned replacement for
 * the reaction derivative tables, trained from the method's own complex-image
 * tables).  A fully connected tanh network
 *   a_0 = x,  a_{l+1} = tanh(W_l a_l + b_l)  (l < n_hidden, width units),
 *   y = W_out a_{n_hidden} + b_out,
 * trained on the mean-squared loss L = mean over samples and outputs of
 * (y - t)^2 with Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * The hidden layers' matrix products use BF16 operands with FP32 accumulation
 * on the matrix cores; the first layer and the output layer (and their
 * gradients) are FP32 on the vector units; weights, gradients and moments are
 * FP32.  Parameter vector (float): W_0, b_0, W_1, b_1, ...,
 * W_out, b_out, matrices row-major with W[j][i] the weight from input i to
 * unit j.  Data arrays are device memory, row-major, one row per sample.
 * Calls are stream ordered on `stream` unless stated; one handle serves one
 * stream at a time.
 * ------------------------------------------------------------------------ */
typedef struct tefmm_mlp* tefmm_mlp_t;

/* Create a network (n_in <= 4, width <= 4096, 1 <= n_hidden <= 16) with
 * Glorot-uniform weights from `seed` and zero biases. */
int tefmm_mlp_create(tefmm_mlp_t* out, int n_in, int width, int n_hidden, int n_out, uint64_t seed);
void tefmm_mlp_destroy(tefmm_mlp_t m);
int64_t tefmm_mlp_num_params(tefmm_mlp_t m);
const char* tefmm_mlp_last_error(tefmm_mlp_t m);
/* Host parameter vectors (num_params floats); set also clears the Adam state. */
int tefmm_mlp_set_params(tefmm_mlp_t m, const float* theta_host);
int tefmm_mlp_get_params(tefmm_mlp_t m, float* theta_host);
/* split = 1: the hidden products carry each FP32 operand as two BF16 values
 * (hi = bf16(x), lo = bf16(x - hi)) and take three BF16 MFMAs with FP32
 * accumulation (lo hi + hi lo + hi hi), ~16 mantissa bits per operand instead of
 * 8; split = 0 (the default): one MFMA on the rounded operands.  Applies to the
 * forward pass, the loss gradient and training.  Anything else: INVALID_ARG. */
int tefmm_mlp_set_split(tefmm_mlp_t m, int split);
/* y[n x n_out] = network(x[n x n_in]) (device arrays). */
int tefmm_mlp_forward(tefmm_mlp_t m, const float* x, int64_t n, float* y, void* stream);
/* Forward pass that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops).  Same kernels and
 * result as tefmm_mlp_forward (bitwise), y[n x n_out] = network(x[n x n_in]),
 * x and y device arrays owned by the caller; the hidden activations live in a
 * fixed device array of the library (TEFMM_MLP_SCRATCH_BYTES per GPU, held
 * until the process ends) instead of the handle's workspace, so at most
 * TEFMM_MLP_SCRATCH_BYTES / (8 width) rows per call (more: TEFMM_ERR_INVALID_ARG,
 * nothing enqueued).  The first call on a device looks up that device's copy.
 * Every call on one GPU shares the array, so calls that overlap on one GPU
 * (other streams or host threads) race and must be serialised by the caller.
 * Stream ordered on `stream`. */
#define TEFMM_MLP_SCRATCH_BYTES (32LL << 20)
int tefmm_mlp_forward_noalloc(tefmm_mlp_t m, const float* x, int64_t n, float* y, void* stream);
/* Loss of (x, t) (device, n rows) and its gradient: *loss and grad_host
 * (num_params floats) on the host, either may be NULL.  Synchronous. */
int tefmm_mlp_loss_grad(tefmm_mlp_t m, const float* x, const float* t, int64_t n, double* loss, float* grad_host,
                        void* stream);
/* One Adam step with the gradient of the last tefmm_mlp_loss_grad.  Synchronous. */
int tefmm_mlp_adam_step(tefmm_mlp_t m, float lr, void* stream);
/* Minibatch Adam over (x, t) (device, n rows): `epochs` passes in a shuffled
 * order (seeded), batches of `batch` rows.  epoch_loss (host, epochs
 * doubles, may be NULL) gets each epoch's mean batch loss.  Synchronous. */
int tefmm_mlp_train(tefmm_mlp_t m, const float* x, const float* t, int64_t n, int epochs, int batch, float lr,
                    uint64_t seed, double* epoch_loss, void* stream);

/* ------------------------------------------------------------------------
 * Surrogate for the Sigma-family derivative tables of one layer (the
 * reaction component whose kernel depends on x - x', y - y' and S = z + z',
 * Sec. 3.2; an extension beyond the paper).  That kernel K is axisymmetric in
 * (x, y), so with u = x + i y and w = rho^2 every derivative reduces to the
 * rotation-free functions (the phase e^{i m phi} of the cylindrical derivatives
 * of Sec. 4.2, carried by u^m)
 *   H_{m,c}(rho, S) = (2 d_w)^m d_S^c K,  (d_x + i d_y)^m d_S^c K = u^m H_{m,c},
 * m + c <= 2p, (2p+1)(2p+2)/2 complex functions of two variables.  The network
 * maps (rho, S) in the training box [0, rho_max] x [s_lo, s_hi] to them, each
 * scaled by the envelope of a source at the nearer mirror distance R_e
 * (W = H R_e^(2m+c+1) / ((2m-1)!! c!)) and by its RMS over the training set.
 * The compact Cartesian table rows h^|g| d^g K of a key (x, y, S) are rebuilt
 * from H exactly: d_x = (D+ + D-)/2, d_y = (D+ - D-)/(2i), D+- = d_x +- i d_y, and
 * D+ D- = -(d_S^2 + k^2) (the kernel solves the Helmholtz equation).  Training
 * data are H of the method's own complex images (Sec. 3.3) at n_train uniform
 * points of the box (GPU FP64); training is minibatch Adam on the GPU
 * (tefmm_mlp kernels).  A validation map over cells_rho x cells_s cells keeps a
 * cell when the largest |W_network - W_images| over n_valid fresh points in it
 * is <= budget, taking cells in order of increasing error until their errors
 * sum to err_total (each served row moves the potential).  Attached to a
 * handle, the surrogate produces the Sigma table rows whose keys fall in kept
 * cells; every other row (outside the box,
 * rejected cells, other layers) comes from the complex images as before.
 * ------------------------------------------------------------------------ */
typedef struct tefmm_surrogate* tefmm_surrogate_t;

typedef struct {
  int layer;           /* layer whose Sigma tables are learned */
  double rho_max;      /* horizontal key distance rho <= rho_max in the box */
  double s_lo, s_hi;   /* z + z' range of the box (inside the layer) */
  int n_train;         /* training points */
  int epochs, batch;
  float lr;
  int width, n_hidden; /* network shape (2 -> width x n_hidden -> 2 (2p+1)(2p+2)/2) */
  int cells_rho, cells_s, n_valid;
  double budget;       /* largest accepted error of W in a cell */
  uint64_t seed;
  int h_from_images;   /* 1: no network; the rows of every key in the box come from the images'
                          H through the same rebuilding (a check of the representation) */
  int envelope;        /* 1: outputs also divided by the envelope of the two mirror distances */
  int leaf_level;      /* 1: keys of the leaf level are answered too (0: only the levels above it,
                          whose translations carry less of the potential per row) */
  int split_bf16;      /* 1: the network's hidden products as BF16 hi + lo pairs (see
                          tefmm_mlp_set_split); 0: plain BF16 operands */
  double err_total;    /* cells are kept in order of increasing error while the kept cells'
                          errors sum to at most err_total (<= 0: no such limit) */
} tefmm_surrogate_options;

typedef struct {
  int status;
  double t_data_s, t_train_s, t_valid_s;  /* host wall time of the three phases */
  double final_loss;                      /* mean loss of the last epoch (normalised outputs) */
  double max_cell_err;                    /* largest cell error of W */
  int cells_ok, cells_total;
  int n_out;
  int64_t n_params;
} tefmm_surrogate_report;

/* Defaults for `layer` of `medium`: rho_max 1.1, S range the layer's z + z'
 * range less 0.15 at each interface (2 units beyond the interface in a
 * half-space), n_train 262144, 300 epochs of 1024, lr 2e-3, width 128,
 * 4 hidden layers, 8 x 16 cells with 16 points, budget 4e-4 (the error of W
 * in envelope units, entry (m, c) weighted by 2^-(m+c)), envelope on, leaf
 * level off, split BF16 products on, err_total 1.2e-3. */
void tefmm_surrogate_default_options(const tefmm_medium* medium, int layer, tefmm_surrogate_options* o);
/* Fit the images of the box, generate the training and validation targets,
 * train, build the validation map.  opt gives p and the image parameters
 * (NULL: defaults).  epoch_loss (host, `epochs` doubles) may be NULL.
 * Synchronous on `stream`; fails with TEFMM_ERR_UNSUPPORTED if the layer has
 * no Sigma family, TEFMM_ERR_INVALID_ARG if the box leaves the layer. */
int tefmm_surrogate_train(tefmm_surrogate_t* out, const tefmm_medium* medium, const tefmm_options* opt,
                          const tefmm_surrogate_options* so, tefmm_surrogate_report* rep, double* epoch_loss,
                          void* stream);
void tefmm_surrogate_destroy(tefmm_surrogate_t s);
/* ok[i] = 1 if the key (x, y, S) = xys[3i..3i+2] lies in a kept cell. */
int tefmm_surrogate_cell_ok(tefmm_surrogate_t s, int n, const double* xys, int* ok);
/* Largest validation error of W in each cell (cells_rho cells_s doubles,
 * cell (i, j) of rho, S at i cells_s + j). */
int tefmm_surrogate_cell_errors(tefmm_surrogate_t s, double* err);
/* Attach (or with NULL detach) a surrogate; it is used by the following
 * tefmm_set_particles calls and must outlive them.  Rejects a surrogate of
 * another order p or medium. */
int tefmm_set_surrogate(tefmm_t h, tefmm_surrogate_t s);

#ifdef __cplusplus
}
#endif
#endif /* TEFMM_H */
