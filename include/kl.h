/* kl.h -- C ABI of the matrix-free isogeometric Galerkin Karhunen-Loeve library for
 * one AMD MI355X (gfx950).
 *
 * Problem (Mika et al., "A matrix-free isogeometric Galerkin method for Karhunen-Loeve
 * approximation of random fields ...", arXiv 2011.13861):
 *   Sec. 3.4 eq. (weakform):   Galerkin discretisation of the Fredholm eigenproblem
 *                              T phi = lambda phi in the trial space of eq. (basis).
 *   Sec. 4.1 eq. (cholesky):   standard form  A' v' = lambda v',  v' = L^T v.
 *   Sec. 4.2-4.4.1:            interpolation based quadrature gives
 *                              A~' = L^{-1} M^T Bt^{-1} J Gamma J Bt^{-T} M L^{-T}.
 *   Sec. 4.4.2, Algorithm 1:   the matrix-free product v' -> A~' v'.
 *
 * Conventions
 *   - Every function returns kl_status (0 = KL_OK, negative = error).  Nothing aborts,
 *     throws or exits across the ABI; kl_last_error() returns a thread-local message
 *     describing the most recent failure on the calling thread.
 *   - Vectors are in vec order (Sec. 2.2): the multi-index (i_1..i_d) maps to
 *     i_1 + n_1 (i_2 + n_2 i_3), first index fastest.  Blocks of vectors are
 *     column-major with a leading dimension >= N.
 *   - "device" pointers are HIP device allocations owned by the caller; "host" pointers
 *     are ordinary host memory owned by the caller.  The library owns the kl_problem
 *     handle and all of its internal device buffers (points, weights, factors and
 *     workspaces), allocated once by kl_setup and released by kl_destroy.
 *   - Validation happens before any device work; on error, outputs and the handle are
 *     left untouched, except where a function documents partial results.
 *   - A handle is not thread-safe: use one handle per host thread / stream.
 */
#ifndef KL_H
#define KL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kl_problem kl_problem;   /* opaque, library-owned */

typedef enum {
    KL_OK = 0,
    KL_EINVAL = -1,      /* invalid argument or description */
    KL_ENOMEM = -2,      /* device or host allocation failed */
    KL_EHIP = -3,        /* a HIP runtime call failed */
    KL_EDOMAIN = -4,     /* det DF <= 0 at a Greville point (Sec. 3.4 assumes det DF > 0) */
    KL_ESINGULAR = -5,   /* univariate Gramian not SPD, or collocation matrix singular */
    KL_ENUMERIC = -6,    /* NaN or Inf met in an input block or in the eigensolver */
    KL_ENOCONV = -7      /* eigensolver hit max_applies; best pairs are still returned */
} kl_status;

/* Arithmetic of stage 5 (the covariance-times-block kernel).  The Kronecker stages
 * always run in FP64. */
typedef enum {
    KL_F64 = 0,      /* FP64 kernel evaluation, FP64 MFMA contraction */
    KL_F32 = 1,      /* FP32 kernel evaluation, FP32 MFMA contraction, FP32 accumulation */
    KL_BF16 = 2,     /* FP32 kernel evaluation rounded to BF16, BF16 MFMA, FP32 accumulation */
    KL_BF16X3 = 3    /* BF16 hi/lo split of both operands, three BF16 MFMAs, FP32 accumulation */
} kl_precision;

/* Covariance kernels (Sec. 3.1, eq. (kernel)); rho = ||diag(ell)^{-1}(x - x')||_2.
 * EXP: sigma2 exp(-rho); SQEXP: sigma2 exp(-rho^2).  EXP_L1, CONST and LIN are test
 * kernels: sigma2 exp(-sum |dx_k|/ell_k), sigma2, sigma2 (1 + x . x'). */
typedef enum { KL_COV_EXP = 0, KL_COV_SQEXP = 1, KL_COV_EXP_L1 = 2, KL_COV_CONST = 3,
               KL_COV_LIN = 4 } kl_cov_kind;

/* Geometry maps F : [0,1]^d -> D (Sec. 2.4).  map_params:
 *   BOX:            lo[0..d-1] in params[0..2], hi[0..d-1] in params[3..5]
 *   ANNULUS_NURBS:  (2D) r0 = params[0], r1 = params[1]; exact rational quadratic arc
 *   ANNULUS_POLAR:  (2D) r0, r1 as above; polar parametrisation of the same domain
 *   SINE_CUBE:      F(u) = u + eps amp prod_k sin(pi u_k); eps = params[0],
 *                   amp = params[1..3]
 *   TENSOR_NURBS:   a general tensor-product NURBS map (Sec. 2.3-2.4) given by the map_*
 *                   fields of kl_desc: F(u) = sum_a w_a P_a prod_k N_{a_k}(u_k) / W(u),
 *                   W(u) = sum_a w_a prod_k N_{a_k}(u_k), with its own degrees and open
 *                   knot vectors on [0, 1] per direction; map_params is not read.   */
typedef enum { KL_MAP_IDENTITY = 0, KL_MAP_BOX = 1, KL_MAP_ANNULUS_NURBS = 2,
               KL_MAP_ANNULUS_POLAR = 3, KL_MAP_SINE_CUBE = 4, KL_MAP_TENSOR_NURBS = 5 } kl_map_kind;

/* Knot vectors (Sec. 2.3), when given explicitly: nondecreasing, open (the first and the
 * last value repeated p + 1 times), from 0 to 1, at least 2 p + 2 entries; the space has
 * nknots - p - 1 functions.  Trial and interpolation knot vectors may repeat an interior
 * value up to p + 1 times: a discontinuous (C^-1) space, as Sec. 6 uses for the
 * interpolation space across a C^0 line of the geometry, and, in the trial space, the
 * non-conforming coupling of two patches (Sec. 3.6).  The last function left of such a
 * knot and the first one right of it have the same Greville abscissa (the knot); each of
 * these points is evaluated as the limit from the side of its own function, the basis
 * functions and det DF alike.  Map knot vectors repeat interior values at most p times
 * (the map is continuous).  Host arrays, read during kl_setup only. */
typedef struct {
    int32_t dim;                 /* spatial dimension d, 1..3 */
    int32_t degree[3];           /* trial-space degree p_k >= 1 */
    int32_t nelem[3];            /* trial-space elements per direction >= 1; open uniform
                                    knots with C^{p-1} continuity, n_k = nelem_k + p_k.
                                    Not read for a direction with explicit knots. */
    const double *knots[3];      /* optional explicit trial knot vector of direction k
                                    (NULL = open uniform from nelem) */
    int32_t nknots[3];           /* its length */
    int32_t interp_degree[3];    /* interpolation space (Sec. 4.2); 0 = same as trial */
    int32_t interp_nelem[3];     /* 0 = same as trial */
    int32_t interp_mult[3];      /* multiplicity m of every interior breakpoint of the
                                    interpolation knot vector, 1 <= m <= interp degree pt
                                    + 1: continuity C^{pt-m}, nt_k = pt + 1 + (net_k - 1) m;
                                    m = pt gives the C^0 interpolation spaces that Sec. 4.2
                                    and Sec. 6 prefer for the exponential kernel, m = pt + 1
                                    a discontinuous one.  0 = 1 (C^{pt-1}). */
    const double *interp_knots[3];   /* optional explicit interpolation knot vector
                                    (NULL = from interp_nelem / interp_mult; with explicit
                                    trial knots and interp_degree, interp_nelem and
                                    interp_mult all 0 or equal to the trial ones, the trial
                                    knot vector); its degree is interp_degree (0 = trial) */
    int32_t interp_nknots[3];
    int32_t map_kind;            /* kl_map_kind */
    double  map_params[8];
    int32_t map_degree[3];       /* TENSOR_NURBS: degree per direction >= 1 */
    const double *map_knots[3];  /* TENSOR_NURBS: open knot vector per direction (host) */
    int32_t map_nknots[3];
    const double *map_ctrl;      /* TENSOR_NURBS: control points, prod_k m_k points of d
                                    coordinates each (m_k = map_nknots[k] - map_degree[k] - 1),
                                    in vec order (first index fastest), point-major (host) */
    const double *map_weights;   /* TENSOR_NURBS: prod_k m_k weights > 0, or NULL (all 1) */
    int32_t cov_kind;            /* kl_cov_kind */
    double  sigma2;              /* variance > 0 */
    double  corr_len[3];         /* correlation length per physical direction > 0 */
} kl_desc;

/* Builds the problem: knots, Greville points, Z_k and its Cholesky factor L_k, the
 * collocation matrices Bt_k and their LU factors, the mixed mass matrices M_k, the
 * composed factors C_k = Bt_k^{-T} M_k L_k^{-T}, mapped Greville points X = F(xhat)
 * and J = sqrt(det DF(xhat)) (Sec. 3.5, 4.1-4.3), in FP64 on the host; then uploads
 * them on `stream` (a hipStream_t, NULL = default stream) and allocates all workspaces.
 * Synchronous: returns after the uploads on `stream` have completed.  The setup time is
 * kept with the handle (kl_eigs_report.t_setup).  Errors: KL_EINVAL, KL_EDOMAIN,
 * KL_ESINGULAR, KL_ENOMEM, KL_EHIP.  *out is written only on success. */
kl_status kl_setup(const kl_desc *desc, void *stream, kl_problem **out);

/* Host part of kl_setup only (no device work, usable without a GPU): the handle
 * supports kl_info, kl_get_points, kl_get_factor and kl_destroy; kl_apply, kl_stage5
 * and kl_eigs reject it with KL_EINVAL.  Same errors as kl_setup otherwise. */
kl_status kl_setup_host(const kl_desc *desc, kl_problem **out);

/* A domain made of several patches (Sec. 3.6, non-conforming multipatch): every patch
 * has its own description (trial and interpolation spaces, map); they must share dim and
 * the covariance (kind, sigma2, corr_len), else KL_EINVAL.  The trial space is the direct
 * sum of the patch spaces (C^-1 between patches); the patches are coupled by the
 * covariance alone: stage 5 runs over the Greville points of all patches, the Kronecker
 * stages patch by patch.  Vectors hold patch 0's N_0 standard-form coefficients (in vec
 * order), then patch 1's, and so on; points and J likewise (kl_patch_info gives the
 * offsets).  The handle works with every single-problem entry point (kl_apply,
 * kl_apply_noalloc, kl_stage5, kl_eigs with coeffs, kl_kle_field, kl_set_cov, the
 * configuration and profiling calls) except kl_get_factor (KL_EINVAL: one factor per
 * patch).  patches: host array of npatch descriptions, read during the call.  Same
 * stream semantics and errors as kl_setup; a patch's own error is reported with its
 * index. */
kl_status kl_setup_patches(int32_t npatch, const kl_desc *patches, void *stream, kl_problem **out);

/* Number of patches of a problem (1 for kl_setup), 0 for NULL. */
int32_t kl_patch_count(const kl_problem *P);

/* Patch i: its trial dofs N_i and interpolation points Ntilde_i, and the offsets of its
 * dofs and points in the problem's vectors.  Any output pointer may be NULL.  KL_EINVAL
 * for a NULL handle or i outside 0 .. kl_patch_count - 1. */
kl_status kl_patch_info(const kl_problem *P, int32_t i, int64_t *N, int64_t *Ntilde, int64_t *dof_offset,
                        int64_t *point_offset);

/* Sizes: N = prod n_k trial dofs, Ntilde = prod nt_k interpolation dofs (the sums over
 * the patches for kl_setup_patches); n and nt (host arrays of 3) receive the
 * per-direction sizes (patch 0's for several patches; 1 beyond dim).  Any pointer may
 * be NULL. */
kl_status kl_info(const kl_problem *P, int64_t *N, int64_t *Ntilde, int32_t *n, int32_t *nt);

/* Replaces the covariance of an existing problem (Sec. 4.3: the kernel enters only
 * through stage 5): kind, variance sigma2 > 0 and correlation lengths corr_len[0..dim-1]
 * > 0 (host array).  Mesh, map and the Kronecker factors are kept, so a sweep over
 * covariance parameters costs one small upload per value.  Waits for outstanding device
 * work before it replaces the scaled points.  Errors: KL_EINVAL, KL_EHIP. */
kl_status kl_set_cov(kl_problem *P, int32_t cov_kind, double sigma2, const double *corr_len);

/* y = A~' x for nvec columns (Algorithm 1): forward Kronecker stages 1-4 (composed
 * into one factor per direction), stage 5 in the given kl_precision, backward stages
 * 6-9.  x, y: device, FP64, column-major, ld >= N; x and y must not overlap.
 * Asynchronous on `stream` (a hipStream_t, NULL = default stream); allocates nothing.
 * Errors: KL_EINVAL (bad sizes/precision/pointers), KL_EHIP (launch failure). */
kl_status kl_apply(kl_problem *P, int32_t precision, int32_t nvec,
                   const double *x, int64_t ldx, double *y, int64_t ldy, void *stream);

/* kl_apply for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same y = A~' x, with every
 * intermediate (Kronecker buffers, stage-5 input, split partials and output) taken from a
 * static device array of the library (64 MiB on each device, held until the process ends)
 * instead of the problem's workspace; it calls no allocating routine.  All calls on one
 * device share that array, so calls that overlap on one device (other streams, other
 * threads) race and must be ordered by the caller; the array keeps the last call's
 * contents, and the call clears what must start at zero itself.  Arguments and errors as
 * kl_apply; a problem whose intermediates exceed the array is KL_EINVAL (the message gives
 * the size needed); with fewer stage-5 split partials fitting than kl_apply would use, the
 * split count is lowered (results agree with kl_apply to rounding). */
kl_status kl_apply_noalloc(kl_problem *P, int32_t precision, int32_t nvec,
                           const double *x, int64_t ldx, double *y, int64_t ldy, void *stream);

/* Stage 5 alone (Algorithm 1, stage 5): z = Gamma y on the Greville grid, for
 * nvec columns of y (device, FP64, column-major, ld >= Ntilde).  z receives FP64.
 * sigma2 is applied; J is not.  Used to test the kernel in isolation. */
kl_status kl_stage5(kl_problem *P, int32_t precision, int32_t nvec,
                    const double *y, int64_t ldy, double *z, int64_t ldz, void *stream);

/* Launch structure of kl_apply (Sec. 2.2, the d mode products of each side): with
 * fuse_directions = 1 (the default) and d >= 2, the first two directions of the forward
 * side run as one launch over 2-D slabs, and so do those of the backward side, which
 * also adds the stage-5 split partials and applies sigma^2 J (2d - 1 launches per
 * 32-column block); with 0, one launch per direction plus the split sums.  Sizes whose
 * slab does not fit the fused kernel's LDS take the per-direction form either way.  The
 * setting also covers the evaluation of the eigenfunctions in kl_kle_field (its forward side).
 * fused_out (may be NULL) receives whether a 32-column apply would be fused.
 * Errors: KL_EINVAL. */
kl_status kl_apply_config(kl_problem *P, int32_t fuse_directions, int32_t *fused_out);

/* Stage-5 launch configuration for one kl_precision (used by the autotuner):
 * rb = 32-row blocks per wave of the FP32/BF16 kernels (1, 2 or 4; 8 selects the FP32
 * form with two blocks per wave and 8 waves per workgroup; 0 keeps the current value;
 * the FP64 kernel always uses four 16-row blocks); nsplit = number of l-splits
 * (1..64 forces it, 0 = automatic load-balancing choice, -1 keeps the current setting).
 * rb_out / nsplit_out (may be NULL) receive the effective values.  Errors: KL_EINVAL. */
kl_status kl_stage5_config(kl_problem *P, int32_t precision, int32_t rb, int32_t nsplit,
                           int32_t *rb_out, int32_t *nsplit_out);

/* Symmetric stage 5 (Sec. 7 names exploiting the symmetry of the covariance as further
 * work).  Gamma(x, x') = Gamma(x', x), so each kernel value of a pair of point blocks below
 * the diagonal serves both products z_r += Gamma y_c and z_c += Gamma y_r: about half the
 * kernel evaluations of the plain kernel for the same matrix products.  The partial sums of
 * the two sides (FP64 for KL_F64, FP32 for KL_BF16 / KL_BF16X3) are added in a fixed order
 * (deterministic results; rounding differs from the plain kernel's).  precision = KL_F64,
 * KL_BF16 or KL_BF16X3 (KL_EINVAL otherwise); on = 1 selects the form for that precision's
 * applies of this handle (kl_apply, kl_stage5, kl_eigs) and allocates the buffers, shared
 * by the precisions (about Ntpad^2 / 16 doubles of partial sums, Ntpad = Ntilde rounded up to
 * 256; this call synchronises the device when it (re)allocates); on = 0 returns that
 * precision to the plain kernel and keeps the buffers until kl_destroy.  chunk = 64-point
 * row tiles per work item (0 = automatic, about three items per compute unit; a new chunk
 * re-plans for every precision); items_out (may be NULL) receives the number of work items.
 * kl_apply_noalloc always uses the plain kernels.  Errors: KL_EINVAL, KL_ENOMEM. */
kl_status kl_stage5_symmetric(kl_problem *P, int32_t precision, int32_t on, int32_t chunk, int32_t *items_out);

/* Copies of the setup data (host arrays, caller-owned):  X: Ntilde x dim row-major
 * physical Greville points; J: Ntilde weights sqrt(det DF); C: the nt_k x n_k
 * row-major composed factor of direction k (0-based).  Any output may be NULL. */
kl_status kl_get_points(const kl_problem *P, double *X, double *J);

/* Truncated KL expansion (Sec. 3.2) at the Ntilde mapped Greville points of kl_get_points:
 *   F[:, s] = sum_{i<M} sqrt(lam_i) phi_i(x) xi[i, s]   zero-mean field samples, s < m
 *   var     = sum_{i<M} lam_i phi_i(x)^2                the truncated variance
 * with phi_i = (sum_j v_j B_j) / sqrt(det DF) in the trial basis of Sec. 3.4 and v = L^{-T} v'
 * for the standard-form eigenvector v' (Sec. 4.1; column i of evecs, as kl_eigs returns it).
 * lam: host, M eigenvalues (finite, >= 0).  evecs: device, N x M column-major, ld ldv >= N.
 * xi: device, M x m column-major, ld ldxi >= M (read only when F is requested).  F: device,
 * Ntilde x m column-major, ld ldf >= Ntilde, or NULL; ceil(Ntilde / 64) ceil(m / 64) < 2^31.  var: device, Ntilde, or NULL (not
 * both NULL).  Inputs and outputs must not overlap.  Asynchronous on `stream`; uses the
 * problem's workspaces, so calls on one problem must not run concurrently with each other or
 * with kl_apply.  Errors: KL_EINVAL (sizes, pointers, eigenvalues, host-only handle),
 * KL_EHIP. */
kl_status kl_kle_field(kl_problem *P, int32_t M, const double *lam, const double *evecs, int64_t ldv,
                       int32_t m, const double *xi, int64_t ldxi, double *F, int64_t ldf, double *var,
                       void *stream);
kl_status kl_get_factor(const kl_problem *P, int32_t k, double *C);

typedef struct {
    int32_t k;              /* wanted eigenpairs (largest first), >= 1 */
    int32_t block;          /* block size b of the block eigensolver; 0 = 32 */
    int32_t max_applies;    /* cap on single-vector operator applications; 0 = default */
    double  tol;            /* relative residual tolerance; 0 = 1e-6 */
    double  abs_floor;      /* absolute floor relative to lambda_1; 0 = 1e-12 */
    int32_t precision;      /* kl_precision of the inner applies */
    int32_t refine_fp64;    /* 1: finish with FP64 applies so that the criterion below
                               holds under the FP64 operator (forced for KL_F64) */
    uint64_t seed;          /* seed of the random start block */
    int32_t guard;          /* extra Ritz vectors kept beyond k; 0 = default */
    int32_t max_basis;      /* largest search-space dimension; 0 = default */
    double  lo_floor;       /* low-precision phase: relative residual (times theta_1) it
                               runs down to before the FP64 phase; 0 = default (FP32 2e-6,
                               BF16x3 5e-5, BF16 5e-3) */
    int32_t coeffs;         /* 0: evecs receive the standard-form eigenvectors v' (unit
                               2-norm); 1: the B-spline coefficients v = L^{-T} v' of the
                               eigenfunctions phi_h = sum_j v_j B_j / sqrt(det DF) (Sec. 4.1,
                               Sec. 3.4), which have unit L2 norm */
} kl_eigs_opts;

typedef struct {
    int32_t n_applies[4];   /* single-vector applications per kl_precision */
    int32_t n_block_applies[4];
    int32_t n_restarts;
    int32_t converged;      /* number of leading pairs meeting the criterion */
    double  t_setup;        /* seconds spent in kl_setup for this handle (host setup and
                               uploads), reported separately as the paper does (Sec. 6) */
    double  t_solve;        /* seconds, wall clock */
    double  t_host_eig;     /* seconds spent in host dense eigensolves (Rayleigh-Ritz) */
    double  max_rel_residual;   /* max_i ||A~' x_i - theta_i x_i|| / theta_i over i <= k */
} kl_eigs_report;

/* k leading eigenpairs of A~' (descending), block Krylov eigensolver with FP64
 * Rayleigh-Ritz and FP64 reorthogonalisation.  Converged when for every i <= k
 *   ||A~' x_i - theta_i x_i||_2 <= max(tol * theta_i, abs_floor * theta_1),  ||x_i|| = 1.
 * x0: optional device FP64 start block (N x nvec0, ld N), or NULL for a seeded random
 * start.  evals: host, k values.  evecs: device FP64, N x k, leading dimension ldv;
 * unit 2-norm columns v' (so phi_h has unit L2 norm, Sec. 4.1), or their B-spline
 * coefficients with opts->coeffs = 1.  rep may be NULL.
 * Ordering: the solver runs on its own stream, which first waits for the work queued on
 * `stream` (a hipStream_t, NULL = default stream) at the time of the call, so x0 may be
 * produced there; the call returns after evecs has been written (synchronous).
 * On KL_ENOCONV evals/evecs hold the best Ritz pairs found.
 * The solver's device buffers and stream are created on the first call
 * and kept with the handle (grown when a later call needs more) until kl_destroy, so
 * calls on one handle must not overlap with each other or with kl_apply / kl_stage5 /
 * kl_kle_field on the same handle (they share its workspaces). */
kl_status kl_eigs(kl_problem *P, const kl_eigs_opts *opts, const double *x0, int32_t nvec0,
                  double *evals, double *evecs, int64_t ldv, kl_eigs_report *rep, void *stream);

/* Stage-5 kernel timing for measurement tools: while enabled, every stage-5 launch of
 * this handle (from kl_apply, kl_stage5 and kl_eigs) is bracketed by two HIP events
 * recorded on its stream right before and after the covariance kernel (the split sums
 * that follow it are outside), created without the system-scope fence so that the
 * interval holds no cache writeback; up to 8192 launches until the next read.
 * kl_profile_enable(P, 1) creates the event pool (once) and resets the counters;
 * kl_profile_enable(P, 0) stops recording.  kl_profile_read waits for the recorded
 * events and returns, per kl_precision (host arrays of 4), the number of timed launches
 * and their total duration in milliseconds accumulated since the last enable. */
kl_status kl_profile_enable(kl_problem *P, int32_t enable);
kl_status kl_profile_read(kl_problem *P, int64_t *count, double *ms);

/* Dense symmetric eigensolver used by the Rayleigh-Ritz step of kl_eigs (host, FP64):
 * A is n x n row-major symmetric (host, read only); w receives the n eigenvalues in
 * descending order, Z (host, n x n column-major) the orthonormal eigenvectors.
 * Householder tridiagonalisation + implicit QR with Wilkinson shifts.
 * Errors: KL_EINVAL, KL_ENUMERIC (non-finite input), KL_ENOCONV. */
kl_status kl_symeig(int32_t n, const double *A, double *w, double *Z);

/* As kl_symeig, but only the eigenvectors of the nv largest eigenvalues (Z: host, n x nv
 * column-major; all n eigenvalues in w): eigenvalues by QR on the tridiagonal form
 * without vectors, eigenvectors by inverse iteration on the tridiagonal form (vectors
 * of eigenvalues closer than 1e-3 ||T|| orthogonalised against each other), then the
 * Householder back-transformation.  Errors: KL_EINVAL, KL_ENUMERIC, KL_ENOCONV. */
kl_status kl_symeig_partial(int32_t n, const double *A, double *w, double *Z, int32_t nv);

/* The nv largest eigenvalues only (w: host, nv entries, descending) and their orthonormal
 * eigenvectors (Z: host, n x nv column-major) of the n x n row-major symmetric A (host, read
 * only): Householder tridiagonalisation, the eigenvalues by bisection on Sturm counts (to an
 * interval of 2 eps |lambda|), eigenvectors by inverse iteration as in kl_symeig_partial, and
 * the back-transformation; the bisection, the inverse iteration (in groups of whole clusters)
 * and the back-transformation run on a persistent team of up to 8 host threads when it is
 * free, with results independent of the team.  The solver used by the Rayleigh-Ritz step of
 * kl_eigs.  Errors: KL_EINVAL, KL_ENUMERIC (non-finite input), KL_ENOCONV. */
kl_status kl_symeig_top(int32_t n, const double *A, int32_t nv, double *w, double *Z);

/* The eigensolver's tall-skinny FP64 product (Ritz vectors X = V S, projections):
 * Out (N x c) = alpha A (N x m) S (m x c) + beta Out, device arrays, column-major with leading
 * dimensions lda >= N, lds >= m, ldo >= N; beta = 0 does not read Out; m = 0 gives beta Out
 * (A and S may then be NULL).  Out must not overlap A or S.  On the FP64 matrix cores: a
 * workgroup owns 32 rows and up to 128 columns (S staged in LDS in chunks of the
 * contraction, A read from memory with the next chunk in flight), or for more than 32
 * columns and at least 16384 rows 64 rows with each wave owning 16 rows and every column
 * tile; every output entry adds its m products in the order of k either way.  Asynchronous
 * on `stream` (a hipStream_t, NULL = default stream); allocates nothing.  N <= 2^36.
 * Errors: KL_EINVAL (sizes, leading dimensions, NULL pointers), KL_EHIP (launch failure). */
kl_status kl_gemm_tall(int64_t N, int32_t m, int32_t c, const double *A, int64_t lda, const double *S,
                       int64_t lds, double alpha, double beta, double *Out, int64_t ldo, void *stream);

/* The eigensolver's Gram product on the device: C (m x c, column-major, leading dimension
 * exactly m) = A^T B for tall A (N x m, ld lda >= N) and B (N x c, ld ldb >= N), FP64 device
 * arrays.  The N rows are split into up to 256 ranges of at least 128 rows; each range's
 * partial products (FP64 matrix cores, 64 rows of C by up to 128 columns per workgroup) go to
 * `work` (device, kl_gram_tall_workspace(N, m, c) doubles, caller-owned) and are added in range
 * order, so the result does not depend on scheduling.  m = 0 or c = 0: nothing is done; N = 0:
 * C = 0.  C must not overlap A, B or work; calls sharing `work` must not overlap.
 * Asynchronous on `stream`; allocates nothing.  N <= 2^36.  Errors: KL_EINVAL (sizes, leading
 * dimensions, NULL pointers, workspace too small), KL_EHIP. */
int64_t kl_gram_tall_workspace(int64_t N, int32_t m, int32_t c);
kl_status kl_gram_tall(int64_t N, int32_t m, int32_t c, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *C, double *work, int64_t work_elems, void *stream);

/* ---- Batches of problems -------------------------------------------------------------
 * Many problems of uneven size (same dimension) solved together: one apply of the whole
 * batch is one replay of a captured HIP graph of 2 dim + 3 launches (batched Kronecker
 * directions, a persistent stage-5 kernel that takes (problem, row tile, l-split) items
 * longest first, split sums).  Block arenas: problem i's block of nvec columns starts
 * at element nvec * row_offset_i of the arena and has leading dimension N_i
 * (row_offset_i = N_0 + ... + N_{i-1}, see kl_batch_info).  Calls on one batch must be
 * ordered (one stream); the batched path supports KL_F64 and KL_F32. */
typedef struct kl_batch kl_batch;

/* Sets up n problems (host setup as kl_setup for each; all with the same dim).  Errors
 * as kl_setup (the message names the failing problem). */
kl_status kl_setup_batch(int32_t n, const kl_desc *descs, kl_batch **out);
kl_status kl_batch_info(const kl_batch *B, int32_t i, int64_t *N, int64_t *Ntilde, int64_t *row_offset);

/* y_i = A~'_i x_i for every problem i with active[i] != 0 (active: host array of n flags,
 * NULL = all); y_i of inactive problems is left untouched.  x, y: device FP64 arenas as
 * above, 1 <= nvec <= 32, x and y must not overlap.  Asynchronous on stream.  The first
 * call per precision builds and captures the graph (synchronous).  Errors: KL_EINVAL,
 * KL_ENOMEM, KL_EHIP. */
kl_status kl_apply_batch(kl_batch *B, int32_t precision, int32_t nvec, const double *x, double *y,
                         const int32_t *active, void *stream);

/* Tile configuration of the batched stage-5 kernel (for the autotuner): rb = 32-row
 * blocks per wave of the FP32 kernel (2 or 4, 0 keeps), lchunk = l-points per split
 * (0 = automatic: the largest power of two >= 512 that leaves >= 4 queue items per
 * resident workgroup).  Rebuilds the graph if the setting changed (waits for the device).
 * grid_out / items_out (may be NULL): resident workgroups and queue length. */
kl_status kl_batch_config(kl_batch *B, int32_t precision, int32_t rb, int64_t lchunk, int32_t *grid_out,
                          int32_t *items_out);

/* kl_eigs for every problem of the batch with the same options, in lockstep: each
 * iteration applies the operators of all unfinished problems in one graph replay
 * (finished ones masked off).  evals: host, n x k (row i = problem i).  evecs: device
 * arena, problem i's N_i x k block at element k * row_offset_i, leading dimension N_i.
 * reps: host array of n reports, or NULL.  Ordering as kl_eigs: the solver streams first
 * wait for the work queued on `stream`; the call returns after evecs has been written.
 * Returns KL_ENOCONV if any problem did not converge (its report says how far it got), or
 * the first error. */
kl_status kl_eigs_batch(kl_batch *B, const kl_eigs_opts *opts, double *evals, double *evecs, kl_eigs_report *reps,
                        void *stream);
kl_status kl_batch_destroy(kl_batch *B);

/* ---- Warm-start network -----------------------------------------------------------
 * A multilayer perceptron that maps covariance parameters to a block of leading
 * eigenvector coefficients, used as the start block of kl_eigs.  It is an addition to
 * the method (the paper starts its Lanczos iteration from a generic vector, Sec. 4.4.2).
 * Layers l = 0..n_layers-1 map sizes[l] -> sizes[l+1]; hidden layers apply tanh, the
 * output layer is linear.  Parameters (device, FP32, flat): per layer W_l (sizes[l] x
 * sizes[l+1], row-major) then b_l (sizes[l+1]).  Inputs and outputs are row-major FP32
 * device arrays, one row per sample.  Calls on one handle must not overlap. */
typedef struct kl_mlp kl_mlp;

/* Creates the network: W_l ~ U(-1/sqrt(sizes[l]), 1/sqrt(sizes[l])) drawn from
 * splitmix64(seed), b_l = 0, Adam moments zero.  sizes: host array of n_layers + 1
 * widths (1..2^24), 1 <= n_layers <= 16.  Errors: KL_EINVAL, KL_ENOMEM, KL_EHIP. */
kl_status kl_mlp_create(int32_t n_layers, const int32_t *sizes, uint64_t seed, kl_mlp **out);
kl_status kl_mlp_num_params(const kl_mlp *M, int64_t *n);
/* Host copies of the flat parameter vector; set also clears the Adam state. */
kl_status kl_mlp_set_params(kl_mlp *M, const float *params);
kl_status kl_mlp_get_params(const kl_mlp *M, float *params);

/* y (batch x sizes[n_layers]) = network(x (batch x sizes[0])).  Asynchronous on
 * stream; grows internal activation buffers on first use of a larger batch. */
kl_status kl_mlp_forward(kl_mlp *M, int32_t batch, const float *x, float *y, void *stream);

/* Loss and gradients for one batch (no update).  group = 0: loss = 0.5/B sum (y - t)^2;
 * group = g > 0 (g divides the output width): every output row is split into groups of
 * g values (one eigenvector each) and loss = 0.5/B sum_groups min_{s=+-1} ||y_g - s t_g||^2,
 * s = +1 when <y_g, t_g> >= 0 (eigenvectors are defined up to sign).  The gradients are
 * kept for kl_mlp_adam and, if grads != NULL, copied there (device, flat layout).
 * loss (host, may be NULL) receives the batch loss; then the call waits for the stream. */
kl_status kl_mlp_gradients(kl_mlp *M, int32_t batch, const float *x, const float *t, int32_t group,
                           double *loss, float *grads, void *stream);

/* One Adam step (Kingma and Ba, with bias correction) with the gradients of the last
 * kl_mlp_gradients call.  The bias corrections are applied through their reciprocals and
 * the square root and final reciprocal are the hardware's (about 1 ulp each). */
kl_status kl_mlp_adam(kl_mlp *M, float lr, float beta1, float beta2, float eps, void *stream);

/* Minibatch training on n samples x (n x sizes[0]) and targets t (n x sizes[L]), both
 * device: per epoch a splitmix64(seed) shuffle, batches of `batch` rows (the last may be
 * smaller), loss as in kl_mlp_gradients, Adam (0.9, 0.999, 1e-8) with a learning rate
 * going geometrically from lr0 (first epoch) to lr1 (last).  epoch_loss (host, epochs
 * values, may be NULL) receives the mean per-sample loss of each epoch.  Synchronous.
 * Each step gives the bits of kl_mlp_gradients + kl_mlp_adam on the same rows, but the
 * Adam step of a layer's weights and biases runs inside its weight-gradient product where
 * the product allows it, so afterwards the kept gradients are not those of the last batch:
 * call kl_mlp_gradients before a separate kl_mlp_adam.
 * Errors: KL_EINVAL, KL_ENOMEM, KL_EHIP, KL_ENUMERIC (non-finite loss). */
kl_status kl_mlp_train(kl_mlp *M, int64_t n, const float *x, const float *t, int32_t group, int32_t epochs,
                       int32_t batch, float lr0, float lr1, uint64_t seed, double *epoch_loss, void *stream);
/* Weight mu >= 0 of the subspace term of the grouped loss (0, the default, leaves it
 * out).  With group > 0, kl_mlp_gradients and kl_mlp_train then add, per row and output
 * group y_g, mu * 0.5 / batch * ||(I - P) y_g||^2 with P = sum_j t_j t_j^T / <t_j, t_j>
 * over the row's target groups: the part of the prediction outside the span of the
 * targets, which does not change when eigenvectors of a cluster are rotated among
 * themselves (the targets must be mutually orthogonal, as eigenvectors are, for P to be
 * the projector).  At most 32 groups per row (KL_EINVAL at the call otherwise).  Errors:
 * KL_EINVAL (NULL handle, negative or non-finite weight). */
kl_status kl_mlp_set_subspace(kl_mlp *M, float weight);
kl_status kl_mlp_destroy(kl_mlp *M);

/* Releases the handle and every device buffer it owns.  NULL is accepted. */
kl_status kl_destroy(kl_problem *P);

/* Thread-local description of the last error ("" if none). */
const char *kl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KL_H */
