/*
 * mfs.h -- C ABI of the MI355X (gfx950) implementation of the peanut-compressed
 * two-body method of fundamental solutions for 2D Stokes flow around nearly
 * touching rigid disks (Broms, Tornberg & Barnett, arXiv 2606.11273).
 *
 * The calls follow the paper's problem statement and the phases of Alg. 2:
 *   mfs_setup             geometry, coarse discretisation, one-body bases, contact list
 *                         (Sec. 3.1, Sec. 4.1, Sec. 6);
 *   mfs_precompute_pairs  per-close-pair compressed corrections A, E (Sec. 3.2-3.4, 4.3-4.4, 5;
 *                         Alg. 2 precompute loop);
 *   mfs_apply             the preconditioned matrix-vector product T mu (Alg. 3);
 *   mfs_gmres_solve       RHS -> GMRES -> post-processing (Alg. 2; Sec. 4.4 for mobility);
 *   mfs_flow_eval         the flow at any points from a solve's density (Alg. 2 flowEval,
 *                         Sec. 3.3), mfs_boundary_residual its relative boundary error
 *                         (Sec. 6.1);
 *   mfs_server_*          many independent solves sharing one device.
 *
 * Conventions shared by every call:
 *  - Every call returns mfs_status.  On error nothing is written to the outputs,
 *    except MFS_ERR_NOCONV from mfs_gmres_solve, which writes the best iterate's
 *    outputs and info.  mfs_last_error() returns a message for the last failing
 *    call on that context.
 *  - "host" pointers are read or written during the call only.  "device" pointers
 *    must be device memory of the current HIP device, at least the stated size;
 *    they are accessed on the context's stream and the call returns after that
 *    work is enqueued (mfs_apply, mfs_kernel_sum) or completed (everything else).
 *  - Coarse collocation data (mu, u, b) have n = 2 * sum(n_col) entries: per node
 *    (x, y) interleaved, nodes of body 0 first.  Source strengths have
 *    2 * sum(n_src) entries, same layout.  Per-body triples are (x, y, rotational).
 *  - Node q of body i sits at c_i + a_i (cos 2 pi q / n_col_i, sin 2 pi q / n_col_i);
 *    source j at c_i + r_src_i a_i (cos 2 pi j / n_src_i, sin 2 pi j / n_src_i)
 *    (equispaced rings, first point at angle 0 in the global frame).
 *  - Forces are sums of Stokeslet strengths: the force exerted on the fluid.  Torque
 *    is the (x - c)^perp moment with (x1, x2)^perp = (-x2, x1) (Sec. 1).
 *  - A context is used by one host thread at a time.
 */
#ifndef MFS_H
#define MFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfs_ctx mfs_ctx;

typedef enum {
  MFS_OK = 0,
  MFS_ERR_ARG = 1,       /* invalid argument, size or unsupported configuration */
  MFS_ERR_GEOMETRY = 2,  /* overlapping or touching disks (gap <= 0) */
  MFS_ERR_OOM = 3,       /* device allocation failed */
  MFS_ERR_DEVICE = 4,    /* HIP / rocBLAS / rocSOLVER error */
  MFS_ERR_STATE = 5,     /* call out of order (e.g. apply before precompute) */
  MFS_ERR_NOCONV = 6,    /* GMRES stopped at max_iter above tolerance (outputs = best iterate) */
  MFS_ERR_NUMERIC = 7    /* NaN or Inf in the input or the iteration */
} mfs_status;

typedef enum { MFS_RESISTANCE = 0, MFS_MOBILITY = 1 } mfs_problem;

/* Arithmetic of the all-pairs Stokeslet sum (step 2a of Alg. 3).  Every other step
 * is FP64 in both modes.  MFS_MIXED evaluates the near disks' ring expansions (FP64
 * moments, offsets rounded once) in FP32 with FP64 accumulation, and translates far cells
 * into the local expansions in FP64 at a lower order; mfs_gmres_solve then runs GMRES with
 * the operator relaxed from FP64 to mixed as the residual falls, inside an FP64 refinement
 * on the true residual. */
typedef enum { MFS_FP64 = 0, MFS_MIXED = 1 } mfs_precision;

/* Method parameters; mfs_default_params fills the paper's values (Sec. 5, Sec. 6). */
typedef struct {
  double mu;              /* viscosity (1) */
  double delta_c;         /* contact threshold on the gap: |c_i - c_k| <= a_i + a_k + delta_c (0.2) */
  double eps_trunc;       /* one-body and peanut pseudoinverse truncation, relative to sigma_1 (1e-14) */
  double eps_trunc_fine;  /* fine pair pseudoinverse truncation (1e-11) */
  double eps_ring;        /* ring rule R = 1 - ln(1/eps)/N (1e-12) */
  int32_t n_fp;           /* fine proxy sources per disk (150) */
  int32_t n_ell;          /* shielding-ellipse sampling parameter (80) */
  int32_t m_p;            /* peanut collocation nodes (200) */
  int32_t a_ell;          /* Moebius fine nodes = a_ell * n_ell (5) */
  double gamma;           /* ellipse tip parameter (0.3) */
  double a_f;             /* equispaced fine nodes = ceil(a_f * n_fp) (1.2) */
  double mobius_r;        /* Moebius clustering parameter (0.6) */
} mfs_params;

typedef struct {
  int32_t iters_total;    /* inner GMRES iterations summed over refinement steps */
  int32_t outer_steps;    /* FP64 refinement steps (1 for MFS_FP64) */
  double rel_resid;       /* final FP64 true residual |b - T x| / |b| */
  double* resid_hist;     /* host, optional: relative residual estimate per inner iteration */
  int32_t hist_cap;       /* capacity of resid_hist */
  int32_t hist_len;       /* entries written */
  double ms_rhs, ms_iterate, ms_post;   /* wall-clock phases of the solve */
  int64_t n_pairs;
  int32_t matvecs_fp64;   /* operator applications with the FP64 kernel sum (refinement residuals) */
  int32_t matvecs_mixed;  /* operator applications with the mixed kernel sum */
  /* Work of all kernel sums of the solve (eq. getall).  dense_pairs counts the (node, source)
   * pairs of the plain direct sums they stand for; the kernels evaluate direct_pairs of them one
   * by one and replace the rest by ring_expansions evaluations of a disk's ring expansion (each
   * per node, of orders summing to expansion_terms) and by local_translations of a cell's
   * moments into a wave's local expansion, evaluated local_evaluations times (per node slot),
   * as counted by the kernels themselves (mfs_kernel_sum_work). */
  int64_t dense_pairs;
  int64_t direct_pairs;
  int64_t ring_expansions;
  int64_t expansion_terms;
  int64_t local_translations;
  int64_t local_evaluations;
} mfs_solve_info;

/* Fill *prm with the paper's defaults.  prm: host, written. */
void mfs_default_params(mfs_params* prm);

/* Create a context for P disks.
 * centers: host, P x 2 row-major; radii: host, P (> 0); n_src, n_col: host, P each
 * (1 <= n_src < n_col, n_col <= 512, even counts; disks with equal (radius, n_src,
 * n_col, r_src) share one-body factors); r_src: host, P, source-ring radius as a
 * fraction of the disk radius in (0, 1), or <= 0 for 1 - ln(1/eps_ring)/n_src (Sec. 6).
 * prm: host or NULL for defaults.  stream: the hipStream_t every call of this context
 * runs on (NULL: the null stream).  Builds the coarse rings, the one-body factors of
 * every disk class by SVD (eq. howG+, eq. SL) and the contact list.
 * Errors: MFS_ERR_ARG (sizes, parameters), MFS_ERR_GEOMETRY (some gap <= 0),
 * MFS_ERR_OOM, MFS_ERR_DEVICE.  *ctx is NULL on error. */
mfs_status mfs_setup(mfs_ctx** ctx, int32_t P, const double* centers, const double* radii,
                     const int32_t* n_src, const int32_t* n_col, const double* r_src,
                     const mfs_params* prm, void* stream);

/* Device-memory callbacks of a context.  alloc returns bytes (> 0) of device memory
 * usable by work on the context's stream, or NULL when it cannot (the call that needed
 * it then fails with MFS_ERR_OOM or MFS_ERR_DEVICE); free releases a pointer that alloc
 * returned.  The library frees a buffer only after the work on the context's stream
 * that uses it has completed.  user is passed through.  Both callbacks stay valid until
 * mfs_destroy of the context returns, and are called from the thread that makes the
 * library call. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} mfs_allocator;

/* mfs_setup with every device buffer of the context (geometry, one-body factors, pair
 * matrices, fine factors, Krylov basis, work space and per-call temporaries) taken
 * from allocator, e.g. a framework's caching allocator; NULL behaves as mfs_setup
 * (hipMalloc / hipFree).  rocBLAS and rocSOLVER keep their own internal work space.
 * MFS_ERR_ARG if allocator is given with a NULL callback. */
mfs_status mfs_setup_ex(mfs_ctx** ctx, int32_t P, const double* centers, const double* radii,
                        const int32_t* n_src, const int32_t* n_col, const double* r_src,
                        const mfs_params* prm, void* stream, const mfs_allocator* allocator);

/* Precompute, on the device, the compressed correction A^c (eq. Amat) and the
 * extraction matrix E^c (velocities for mobility, eq. rbm2; forces/torques for
 * resistance, eq. force_ext read with a transpose and sign) of every close pair,
 * for problem prob.  n_pairs_out: host or NULL.  The fine pair discretisation of
 * Sec. 5 is the paper's for unit disks; a disk of radius a gets fine counts scaled by
 * a, the limit point of the pair's two circles for its shielding ellipse and a
 * rolling unit circle for the peanut, so pairs of unequal radii and classes are
 * accepted.  With mfs_keep_fine_factors set it also keeps the fine maps for
 * mfs_flow_eval.  Calling it again for the other problem keeps both sets. */
mfs_status mfs_precompute_pairs(mfs_ctx* ctx, mfs_problem prob, int64_t* n_pairs_out);

/* Number of close pairs and the list itself.  pairs: host, n_pairs x 2 (i < k),
 * lexicographic order, or NULL to query only the count. */
mfs_status mfs_get_pairs(const mfs_ctx* ctx, int64_t* n_pairs, int32_t* pairs);

/* The disk order of the kernel sums and the clusters of the two-level FP64 sum (for tests
 * and inspection).  Disks are sorted along a Morton curve over their centres and cut
 * into clusters of consecutive disks (at most 16 disks and 1024 sources each, within one
 * quadtree cell).  In the FP64 sum at arbitrary points (mfs_flow_eval), a cluster farther
 * than 4 radii from a target is summed through one order-26 expansion about its centre
 * (moments A_k, B_k and D_k = sum sigma conj(w) w^k of its sources; the paper's fast
 * multipole method plays this part, Sec. 6).  The same disk order is the leaf order of the
 * hierarchical sum's quadtree (mfs_get_fmm).
 * n_clusters: host, written.  Each of the others is host memory or NULL: slot_body (P):
 * the disk at each position of the order; cl_start (n_clusters + 1): first position of
 * each cluster; centre (2 n_clusters): mean of its disks' centres; radius (n_clusters):
 * the radius of the far test, at least the largest |c_b - centre| + rho_b over its disks
 * (rho_b: source ring radius) and at least (3 max a + delta_c + that) / 4, so that a far
 * cluster never holds a target's disk or one of its contact partners. */
mfs_status mfs_get_clusters(const mfs_ctx* ctx, int32_t* n_clusters, int32_t* slot_body, int32_t* cl_start,
                            double* centre, double* radius);

/* The hierarchical far field of the kernel sum over the context's own nodes (inspection,
 * for tests and measurement; the paper evaluates this sum with a fast multipole method,
 * Sec. 6).  Cells: a quadtree over the disks in the order of mfs_get_clusters (slot_body),
 * leaf s < P the disk in slot s, an internal cell the slots [cell_lo, cell_hi) of one curve
 * prefix; centre the mean of its disks' centres, radius max |c_b - centre| + a_b (a_b the disk
 * radius).  Waves: runs of at most 128 consecutive nodes of the visiting order (the nodes of
 * the disks in slot order), cut where the next disk lies more than 3 radii from the run's
 * first disk; wave w holds positions [wave_start[w], wave_start[w + 1]), centre wave_c (the
 * midpoint of its nodes' bounding box).  A wave's m2l list holds the cells translated into its
 * local expansion (|centre - wave_c| >= sep (radius + r), r the wave's largest node distance
 * from wave_c, sep 4 for MFS_FP64 and 3 for MFS_MIXED, and no node's own disk or contact
 * partner inside); its near list the other disks (slots, increasing), each summed from the
 * disk's ring expansion at the lowest of the orders 27, 40, 56 (MFS_FP64) or 14, 24, 44
 * (MFS_MIXED) whose squared distance tier_d2 every node of the wave exceeds (skipped nodes
 * aside), else directly.  prob: the one-body map whose strengths set tier_d2.  sizes (host,
 * 4, written): ncell, nwave, m2l and near list lengths.  Every other pointer is host memory of
 * the size it implies or NULL (not written): cell_lo, cell_hi, cell_r (ncell), cell_c
 * (2 ncell), wave_start, m2l_off, near_off (nwave + 1), wave_c (2 nwave), m2l, near, tier_d2
 * (3 P, slot order). */
mfs_status mfs_get_fmm(const mfs_ctx* ctx, mfs_problem prob, mfs_precision prec, int64_t* sizes,
                       int32_t* cell_lo, int32_t* cell_hi, double* cell_c, double* cell_r, int32_t* wave_start,
                       double* wave_c, int32_t* m2l_off, int32_t* m2l, int32_t* near_off, int32_t* near,
                       double* tier_d2);

/* Import (set) or export (get) the pair matrices of problem prob in the pair
 * order of mfs_get_pairs.  A: host, sum over pairs of (2 n_src_i + 2 n_src_k)^2,
 * each pair's matrix row-major; E: host, sum of 6 x (2 n_src_i + 2 n_src_k),
 * row-major.  Setting marks prob as precomputed (used to run the matvec on
 * matrices computed elsewhere, e.g. at an earlier time step). */
mfs_status mfs_set_pair_matrices(mfs_ctx* ctx, mfs_problem prob, const double* A, const double* E);
mfs_status mfs_get_pair_matrices(const mfs_ctx* ctx, mfs_problem prob, double* A, double* E);

/* u_out = T mu_in, the matvec of Alg. 3 for problem prob (steps 1a, 1b, 2a, 2b and
 * the identity fix), for n_rhs stacked vectors.  mu_in, u_out: device, n_rhs x n
 * doubles, must not overlap.  The all-pairs sum skips each disk's own sources
 * and those of its contact partners; the pair step adds, in FP64, each partner's
 * corrections from its other contacts; the result equals Alg. 3 in exact
 * arithmetic (the self and near blocks that Alg. 3 adds and then subtracts are
 * never formed).  Errors: MFS_ERR_STATE before precompute of prob, MFS_ERR_ARG. */
mfs_status mfs_apply(mfs_ctx* ctx, mfs_problem prob, mfs_precision prec, int32_t n_rhs,
                     const double* mu_in, double* u_out);

/* mfs_apply for one vector (n_rhs = 1) that allocates no device memory, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The kernel sum's expansion records of the vector (the disks' ring expansions and
 * the cells' moments and records, mfs_get_fmm), which mfs_apply keeps in buffers of the
 * context, go to a static scratch array of 128 MiB that every context on the device shares
 * (each device holds its own copy until the process ends).  Calls that overlap in time on one
 * device race on that array: run them on one stream, or order them.  The result equals
 * mfs_apply's (same kernels).  It launches kernels only (no allocation, copy, fill or
 * synchronisation), so on a context whose stream is capturing it records into a HIP graph,
 * and each replay reads mu_in and writes u_out at the captured addresses.  mu_in, u_out:
 * device, n doubles, not overlapping.  Errors: as
 * mfs_apply; MFS_ERR_ARG when this context's records (16 (ncell (81 + 108) + 174 P) + 8 x 140 P
 * bytes, 78 MB at P = 10^4) exceed the array. */
mfs_status mfs_apply_noalloc(mfs_ctx* ctx, mfs_problem prob, mfs_precision prec, const double* mu_in,
                             double* u_out);

/* All-pairs Stokeslet sum over the context's coarse sources and nodes (eq. getall):
 * u[t] = sum_s S(x_t, y_s) sigma[s].  skip = 0: every source; skip = 1: sources of the
 * target's own disk are left out; skip = 2: also those of the disk's contact partners (the
 * form step 2a of mfs_apply uses, with the skipped blocks applied in FP64 by the pair step).
 * sigma: device, 2 * sum(n_src); u: device, 2 * sum(n_col).  This is the kernel of step 2a,
 * exposed for tests and measurement.  The far field is hierarchical (mfs_get_fmm; the paper
 * uses a fast multipole method, Sec. 6): per wave of up to 128 nodes, cells far from the wave
 * are translated into the wave's local expansion (FP64, order 26 with MFS_FP64, 20 with
 * MFS_MIXED; truncation below 4^-27 and 3^-21 of the sources' strength sums), the other disks
 * are summed from their ring expansions (FP64 moments; evaluated in FP64, or in FP32 with
 * MFS_MIXED) at an order that keeps the truncation below 1e-15 (FP64) or 1e-9 (FP32) of the
 * field of unit boundary data through the one-body map and below 1e-16 / 1e-9 of sum |sigma|
 * for any strengths, or directly in FP64 when a node is too close for every order. */
mfs_status mfs_kernel_sum(mfs_ctx* ctx, mfs_precision prec, const double* sigma, double* u,
                          int32_t skip);

/* Measurement form of mfs_kernel_sum: packs sigma and forms its expansion records once, then
 * launches the sum kernel reps times (each writes the same u), timed with HIP events on the
 * context's stream.  ms_records (host, written): packing and records; ms_sum (host, written):
 * the average duration of one sum launch.  Synchronises the stream.  Arguments as
 * mfs_kernel_sum; reps >= 1. */
mfs_status mfs_time_kernel_sum(mfs_ctx* ctx, mfs_precision prec, const double* sigma, double* u, int32_t skip,
                               int32_t reps, double* ms_records, double* ms_sum);

/* Work counted by the context's kernel sums (eq. getall) since setup or the last reset:
 * work[0] direct (node, source) pair evaluations, work[1] evaluations of a disk's ring
 * expansion and work[2] their orders summed (each per node; a wave of 64 threads, 2 nodes
 * each, takes one path per near disk for all its nodes, and every thread counts what it
 * executes), work[3] translations of a cell's moments into a wave's local expansion (one wave
 * each), work[4] evaluations of local expansions (per node slot of a wave with translations).
 * Flow-evaluation points are not counted.  work: host, 5, written.  Synchronises the
 * context's stream; reset != 0 then zeroes the counters.  mfs_gmres_solve resets them at its
 * start. */
mfs_status mfs_kernel_sum_work(mfs_ctx* ctx, int64_t* work, int32_t reset);

/* Right-hand side of the preconditioned system.  given: host, P x 3 (forces and
 * torques for mobility, velocities for resistance); b: device, n.  Mobility:
 * b = -u_0 with u_0 the completion flow of lambda_0 = K (K^T K)^{-1} [f; t] summed over
 * all disks (eq. u0_def); resistance: b = B [v; omega] at every node (eq. rigidbc). */
mfs_status mfs_rhs(mfs_ctx* ctx, mfs_problem prob, const double* given, double* b);

/* Post-processing of a solution mu (device, n): out (host, P x 3) = velocities
 * [v; omega] = -K^T lambda_bar + sum_c E^c x_c (mobility) or forces/torques
 * K^T lambda_bar + sum_c E^c x_c (resistance), lambda_bar = one-body pseudoinverse of mu. */
mfs_status mfs_post(mfs_ctx* ctx, mfs_problem prob, const double* mu, double* out);

/* Full solve (Alg. 2; Sec. 4.4).  rhs: host, n_rhs x P x 3; out: host, n_rhs x P x 3.
 * x0: device, n_rhs x n initial mu, or NULL for zero.  tol: relative residual of
 * the square system; max_iter: cap on GMRES iterations per solve (unrestarted).
 * MFS_FP64 runs GMRES on the FP64 operator.  MFS_MIXED refines in FP64 on the true
 * residual around a GMRES whose operator applications switch to the mixed kernel sum
 * once its residual estimate is below tol_inner / delta (relaxed inexact Krylov;
 * delta = 1e-6 for mobility, 1e-3 for resistance; environment MFS_MIXED_DELTA).
 * Right-hand sides run in lockstep groups of up to 8 (stacked products, one Krylov
 * basis each).  Each stops on its own
 * tolerance.  info: host or NULL; with several right-hand sides iters_total sums their
 * inner iterations, rel_resid is the largest, and matvecs count vectors. */
mfs_status mfs_gmres_solve(mfs_ctx* ctx, mfs_problem prob, mfs_precision prec, int32_t n_rhs,
                           const double* rhs, double* out, const double* x0, double tol,
                           int32_t max_iter, mfs_solve_info* info);

/* ---------------------------------------------------------------------------------
 * Flow evaluation after a solve (Sec. 3.3, eq. chi: the source triplet lambda,
 * lambda_bar, beta that Alg. 2 returns when flowEval is set) and the relative boundary
 * residual (Sec. 6.1, eqs. residual_x and residual).
 *
 * The flow at a point is the sum of every disk's coarse strengths, Pi (lambda_bar +
 * the compressed pair corrections lambda_tilde), plus for mobility the force/torque
 * sources lambda_0 = K (K^T K)^{-1} [f; t]; at a point near a close pair (on one of its
 * two disks, or in the fluid inside its peanut) that pair's compressed strengths are
 * replaced by its fine sources, -S(x, Yf) Pi_f G [lambda_bar_i; lambda_bar_k] (eq. bfm
 * in the symmetric form, Pi_f the fine rigid projection for mobility).  All FP64. */

/* Keep (keep != 0) or drop each pair's fine map G (2 (nf_i + nf_k) x 2 (N_i + N_k)
 * doubles, about 0.9 MB per unit-disk pair), fine source points and peanut geometry in
 * the next mfs_precompute_pairs calls, for mfs_flow_eval.  Default: not kept.  Matrices
 * imported with mfs_set_pair_matrices carry no fine factors. */
mfs_status mfs_keep_fine_factors(mfs_ctx* ctx, int32_t keep);

/* Density mu (device, n = 2 N_t doubles, layout of mfs_apply) of right-hand side rhs
 * (0-based) of the latest mfs_gmres_solve on ctx (also after MFS_ERR_NOCONV: the
 * iterate).  MFS_ERR_STATE before any solve, MFS_ERR_ARG for rhs out of range. */
mfs_status mfs_get_density(const mfs_ctx* ctx, int32_t rhs, double* mu);

/* Velocity u (device, 2 n_pts: (u_x, u_y) per point) at points pts (device, 2 n_pts,
 * absolute (x, y)) from the density mu (device, n) of problem prob.  body (device,
 * n_pts): the disk whose boundary holds the point, or -1 for a point in the fluid;
 * fluid points must lie outside every disk.  given (host, 3P): the forces and torques
 * of a mobility solve (the lambda_0 sources); ignored for resistance (may be NULL).
 * Needs the pair precompute of prob with fine factors kept when there are pairs
 * (MFS_ERR_STATE otherwise).  Synchronous on the context's stream. */
mfs_status mfs_flow_eval(mfs_ctx* ctx, mfs_problem prob, const double* mu, const double* given,
                         int64_t n_pts, const double* pts, const int32_t* body, double* u);

/* Relative boundary residual of a solution: n_per_body points per disk at angles
 * 2 pi (j + 1/2) / n_per_body, eps(x) = |u(x) - (v_i + omega_i (x - c_i)^perp)| with u
 * from mfs_flow_eval, and *eps_max (host) = max eps / max |v_i + omega_i (x - c_i)^perp|.
 * rigid (host, 3P): the rigid motions (mobility: the solve's velocities; resistance:
 * the prescribed velocities); given as for mfs_flow_eval.  eps (device, P n_per_body,
 * disk-major) receives the pointwise residuals, or NULL.  1 <= n_per_body <= 2^20. */
mfs_status mfs_boundary_residual(mfs_ctx* ctx, mfs_problem prob, const double* mu, const double* given,
                                 const double* rigid, int32_t n_per_body, double* eps, double* eps_max);

/* Sizes: P, total sources N_s, total nodes N_t (n = 2 N_t), pairs.  Any pointer may be NULL. */
mfs_status mfs_get_sizes(const mfs_ctx* ctx, int32_t* P, int64_t* n_sources, int64_t* n_nodes,
                         int64_t* n_pairs);

/* Release every device and host resource of ctx (NULL is accepted). */
mfs_status mfs_destroy(mfs_ctx* ctx);

/* Message of the last failing call on ctx (or of the last failing mfs_setup when
 * ctx is NULL).  Valid until the next call on that context. */
const char* mfs_last_error(const mfs_ctx* ctx);

/* ---------------------------------------------------------------------------------
 * Serving: continuous batching of independent suspension solves on one device.
 *
 * A server owns max_slots HIP streams, each driven by a host worker thread.  A
 * submitted request (geometry + given forces/torques or velocities) is queued; a
 * free slot admits the oldest queued request whose device-memory footprint fits in
 * what the budget has left (requests that arrive while others run are admitted as
 * slots and memory free up).  An admitted request runs setup, the pair precompute
 * and the solve (mfs_setup, mfs_precompute_pairs, mfs_gmres_solve) on its slot's
 * stream, so the work of different requests overlaps on the device; its context,
 * pair matrices and Krylov basis stay resident until it completes.  Each request's
 * arithmetic does not depend on what else runs: the same request gives the same
 * result alone and in a mix.  The solve follows Alg. 2 (Sec. 4.4 for mobility).
 * --------------------------------------------------------------------------------- */
typedef struct mfs_server mfs_server;

typedef struct {
  int32_t P;                /* number of disks */
  const double* centers;    /* host, P x 2 */
  const double* radii;      /* host, P */
  const int32_t* n_src;     /* host, P */
  const int32_t* n_col;     /* host, P */
  const double* r_src;      /* host, P (see mfs_setup) */
  mfs_problem problem;
  mfs_precision precision;
  const double* given;      /* host, P x 3: (fx, fy, t) for mobility, (vx, vy, omega) for resistance */
  double tol;               /* relative residual tolerance of the solve */
  int32_t max_iter;         /* inner iteration limit, 1..1000 */
} mfs_request;

typedef struct {
  double ms_queue;          /* submit -> admission */
  double ms_service;        /* admission -> completion (setup, precompute, solve) */
  double ms_total;          /* submit -> completion: the time to solution */
  double ms_precompute;     /* pair precompute inside the service time */
  int64_t footprint_bytes;  /* device memory reserved for the request while it ran */
  mfs_solve_info solve;     /* as from mfs_gmres_solve (resid_hist not filled) */
} mfs_ticket_info;

/* Create a server.  hbm_budget_bytes: device memory the admitted requests may hold
 * together (0: 80% of the memory free on the current device now).  max_slots:
 * concurrent requests, 1..64.  prm: host or NULL for the defaults; applies to every
 * request.  Errors: MFS_ERR_ARG, MFS_ERR_DEVICE (stream creation).  *srv is NULL on
 * error. */
mfs_status mfs_server_create(mfs_server** srv, size_t hbm_budget_bytes, int32_t max_slots, const mfs_params* prm);

/* Device-memory footprint the server reserves for a request (an upper bound of what
 * its context, pair matrices, precompute work space and Krylov basis allocate).
 * The host inputs are read during the call.  Errors: MFS_ERR_ARG, MFS_ERR_GEOMETRY. */
mfs_status mfs_server_footprint(const mfs_server* srv, const mfs_request* req, int64_t* bytes);

/* Queue a request; returns at once with its ticket (> 0).  The inputs are copied.
 * Errors: MFS_ERR_ARG (sizes, or a footprint above the whole budget),
 * MFS_ERR_GEOMETRY (some gap <= 0), MFS_ERR_STATE (server shutting down). */
mfs_status mfs_server_submit(mfs_server* srv, const mfs_request* req, int64_t* ticket);

/* Wait for a ticket to complete.  out: host, P x 3 ((vx, vy, omega) for mobility,
 * (fx, fy, t) for resistance); info: host or NULL.  timeout_ms < 0 waits without
 * limit.  Returns the request's own status (outputs are written for MFS_OK and
 * MFS_ERR_NOCONV); the ticket is released.  On a timeout returns MFS_ERR_STATE and
 * keeps the ticket.  An unknown ticket gives MFS_ERR_ARG. */
mfs_status mfs_server_wait(mfs_server* srv, int64_t ticket, double* out, mfs_ticket_info* info,
                           int32_t timeout_ms);

/* Message for the last failing server call or request (valid until the next call). */
const char* mfs_server_last_error(const mfs_server* srv);

/* Stop admitting, finish the running requests, drop the queued ones and release
 * every resource.  srv may be NULL.  No other call on srv may be in progress or made
 * afterwards (a ticket still queued is dropped, not completed). */
mfs_status mfs_server_destroy(mfs_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* MFS_H */
