/*
 * cdcs.h -- C-ABI of the MI355X (gfx950) library for chordally decomposed ADMM
 * on sparse semidefinite programs.
 *
 * Method: Zheng, Fantuzzi, Papachristodoulou, Goulart, Wynn, "Fast ADMM for
 * Semidefinite Programs with Chordal Sparsity" (arXiv:1609.06068).
 *   - problem forms: Sec. I, (E:PrimalSDP) and (E:DualSDP);
 *   - decomposition: Sec. II-B/II-C (E_k, Grone's and Agler's theorems),
 *     Sec. III-A (H_k = E_k (x) E_k, (E:PrimalVectorForm)), Sec. IV-A
 *     ((E:DualDecomposedSDPVector));
 *   - iteration: Algorithm 1 (primal form) and Algorithm 2 (dual form).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pattern entries.  The aggregate sparsity pattern is passed as a list of
 * nnz distinct lower-triangular entries e = (i[e], j[e]), i >= j, diagonal
 * included.  Every "global" vector of length nnz (x, C, columns of A) is indexed
 * by that list position and holds matrix values (an off-diagonal entry stands
 * for both (i, j) and (j, i)).  Inner products and norms of global vectors
 * weight off-diagonal entries by 2, so they equal the paper's vec() products.
 * (Inside a handle the entries are renumbered by first appearance in the
 * packed clique blocks, so that the gather and scatter between global vectors
 * and blocks stream through memory; every entry point converts its global
 * vectors from and to the pattern order given here.)
 *
 * Cliques.  p cliques as a CSR (ptr[p+1], vert[]), vertices strictly
 * increasing inside a clique (the natural order of Sec. II-B).  The pattern
 * must equal the union of C_k x C_k (lower triangles).  Clique sizes are
 * limited to 1..CDCS_MAX_CLIQUE.  cdcs_setup without cliques computes a
 * chordal extension of the pattern and its maximal cliques itself
 * (cdcs_chordal_extension).
 *
 * Packed clique blocks.  Per-clique matrices (x_k, z_k, v_k, lambda_k, W_k,
 * P(W_k)) are stored as packed lower triangles, row-major: element (a, b),
 * a >= b, of clique k sits at off[k] + a(a+1)/2 + b, where off[] is the
 * prefix sum of s_k(s_k+1)/2 (cdcs_clique_offsets).  a, b index the clique's
 * sorted vertex list.  These blocks are FP32; global vectors are FP64.
 *
 * Memory.  Pointers documented "host" are read during the call only and may
 * be freed on return.  Pointers documented "device" are caller-owned device
 * memory (e.g. torch tensors); the library never frees them.  The handle owns
 * its internal device data.  A handle is not thread-safe; calls on one handle
 * must be serialised by the caller, and the device work they enqueue must not
 * overlap (one stream, or streams ordered by events): the handle's work
 * buffers, the iterate among them, are shared by its calls.
 *
 * Streams.  Work is enqueued on the caller's stream (0 = legacy default
 * stream).  Entry points return after enqueueing, except cdcs_setup and
 * cdcs_admm_solve, which synchronise on that stream.
 *
 * Errors.  Every entry point returns a cdcs_status and never aborts; the
 * message of the last failure on the calling thread is cdcs_last_error().
 */
#ifndef CDCS_H
#define CDCS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest clique of a handle.  Cliques of up to CDCS_MAX_BATCHED_CLIQUE
 * vertices are projected by Jacobi eigensolves in one workgroup's LDS (the
 * handle-free cdcs_psd_project_batched and the adjoint take only these);
 * larger ones by the matrix sign function on the matrix cores. */
#define CDCS_MAX_CLIQUE 1024
#define CDCS_MAX_BATCHED_CLIQUE 126

typedef enum {
    CDCS_OK = 0,
    CDCS_E_ARG = 1,            /* bad argument, size or pointer */
    CDCS_E_PATTERN = 2,        /* cliques/pattern/data inconsistent */
    CDCS_E_RANK = 3,           /* A D^-1 A^T not positive definite: A rank deficient */
    CDCS_E_DEVICE = 4,         /* HIP runtime failure */
    CDCS_E_NOMEM = 5,          /* device allocation failed */
    CDCS_E_NOT_CONVERGED = 6,  /* iteration cap reached; results are written */
    CDCS_E_NUMERIC = 7,        /* an eigensolve hit its sweep cap, or NaN/Inf in the iterate */
    CDCS_PRIMAL_INFEASIBLE = 8, /* HSDE solve: certificate of primal infeasibility found */
    CDCS_DUAL_INFEASIBLE = 9   /* HSDE solve: certificate of dual infeasibility (unbounded primal) found */
} cdcs_status;

typedef enum { CDCS_PRIMAL = 0, /* Algorithm 1 */ CDCS_DUAL = 1 /* Algorithm 2 */ } cdcs_form;

typedef struct cdcs_handle cdcs_handle;

/* Aggregate sparsity pattern G(V, E) (Sec. III-A), lower triangle. */
typedef struct {
    int32_t n;            /* matrix order */
    int64_t nnz;          /* number of entries */
    const int32_t *i;     /* host [nnz], row index, 0 <= j[e] <= i[e] < n */
    const int32_t *j;     /* host [nnz] */
} cdcs_pattern;

/* Maximal cliques C_1..C_p of the (chordal) pattern (Sec. II-A). */
typedef struct {
    int32_t p;
    const int64_t *ptr;   /* host [p+1], ptr[0] = 0 */
    const int32_t *vert;  /* host [ptr[p]] */
} cdcs_cliques;

/* Constraint matrices A_1..A_m of the operator A(X) = [<A_i, X>] (Sec. I),
 * each given by its values on pattern entries.  dense = 1: val is m x nnz
 * row-major (ptr, idx ignored).  dense = 0: CSR rows (ptr[m+1], idx[] pattern
 * entry of each value, val[]); duplicates are summed.  A dense matrix, or a
 * CSR one with more than a fifth of its m x nnz entries present, is stored on
 * the device in FP32 (off-diagonal values doubled, exactly) as a dense array
 * and its transpose; a sparser CSR matrix is kept sparse in FP64 (rows for
 * A u, the nonzero columns for A^T y).  The KKT factor is built from the
 * stored values.  Batch handles (cdcs_setup_batch) always store A densely. */
typedef struct {
    int32_t m;
    int32_t dense;
    const int64_t *ptr;   /* host [m+1] (dense = 0) */
    const int32_t *idx;   /* host [ptr[m]] (dense = 0) */
    const double *val;    /* host */
} cdcs_constraints;

typedef struct {
    double rho;           /* ADMM penalty, > 0 (the paper leaves it free) */
    double tol;           /* stop when max(eps_p, eps_d) <= tol; 0 runs max_iter */
    int32_t max_iter;     /* iteration cap (>= 1) */
    int32_t form;         /* cdcs_form */
    int32_t check_every;  /* iterations per captured HIP graph (0: no graph, eager launches) */
} cdcs_options;

typedef struct {
    int32_t iters;        /* completed iterations */
    int32_t status;       /* cdcs_status of the solve */
    int32_t converged;    /* 1 if max(eps_p, eps_d) <= tol */
    int32_t jacobi_cap_hits; /* eigensolves that stopped at the sweep cap */
    double eps_p, eps_d;  /* relative residuals of the last iteration */
    double obj_primal;    /* <C, X> of the primal iterate */
    double obj_dual;      /* <b, y> of the dual iterate */
    double loop_s;        /* wall time of the iteration loop */
    int64_t jacobi_sweeps; /* Jacobi sweeps summed over all eigensolves of the solve (and the
                              Newton-Schulz steps of cliques above the LDS limit) */
} cdcs_info;

/* Caller-owned ADMM state (device memory).  Zero-filled state is the
 * paper-neutral initial guess; a previous solve's state is a warm start.
 *   x   [nnz]    FP64  global x (Alg. 1: the primal X on the pattern;
 *                      Alg. 2: the multiplier, X_sdp = -rho x)
 *   y   [m]      FP64  KKT multiplier y (Alg. 1: y_sdp = -rho y; Alg. 2: y_sdp = y)
 *   blk [nslots] FP32  x_k (Alg. 1) or z_k (Alg. 2), packed
 *   lam [nslots] FP32  lambda_k, packed
 *   v   [nslots] FP32  v_k (Alg. 2 only; NULL allowed for Alg. 1)
 *   vw  [nwarm]  FP32  eigenvectors of each clique's last projection (k x k
 *                      blocks, row-major, clique order, offsets the prefix
 *                      sums of s_k^2): the starting basis of the clique's
 *                      next Jacobi eigensolve (Sec. III-B.2: one small
 *                      eigendecomposition per cone and iteration).  Must hold
 *                      orthogonal blocks; cdcs_warm_reset writes identities.
 *                      With vw the warm start carries over from one solve
 *                      call to the next, so splitting a solve into several
 *                      calls does not change its iterates.  NULL: the handle
 *                      keeps its own copy and restarts it at identity in
 *                      every solve. */
typedef struct {
    double *x;
    double *y;
    float *blk;
    float *lam;
    float *v;
    float *vw;
} cdcs_state;

/* Sizes of a handle.  sparse_a = 1 if A is kept sparse (nnz_a coefficients),
 * 0 if it is stored densely (nnz_a = m * nnz).  sparse_factor = 1 if the
 * inverse Cholesky factor is kept as CSR (nnz_factor nonzeros in L^-1), 0 if
 * it is dense (nnz_factor = m (m + 1) / 2, and the handle keeps the dense
 * inverse M^-1 = L^-T L^-1 of A D^-1 A^T, m x m, in its place).  nnz_l > 0: the factor of
 * A D^-1 A^T was computed sparse (symbolic elimination order, then the
 * numeric factor on the device; no dense m x m matrix), with nnz_l nonzeros
 * in L; 0: it was factored dense. */
typedef struct {
    int32_t n, m, p, smax;
    int64_t nnz, nslots;
    int32_t sparse_a, sparse_factor;
    int64_t nnz_a;
    int64_t nnz_factor;
    int64_t nwarm;        /* sum of s_k^2: length of cdcs_state.vw */
    int64_t nnz_l;        /* nonzeros of the sparse Cholesky factor (0: dense factor) */
    int32_t nvcones;      /* vector cones (cdcs_setup_cones) */
    int32_t pad_;
    int64_t nslots_psd;   /* packed slots of the cliques; the cones' slots follow them */
} cdcs_sizes;

/*
 * Chordal extension of an arbitrary aggregate pattern and its maximal cliques
 * (Sec. II-A, Definition 1; finding a minimum-fill extension is NP-complete,
 * so a heuristic is used): the graph of the pattern (vertices that occur in
 * an entry, edges the off-diagonal entries) is tested for chordality by
 * maximum cardinality search; a chordal graph is kept as it is, any other is
 * filled by minimum-degree elimination (smallest label on ties).  The maximal
 * cliques come from the resulting perfect elimination ordering, in that
 * order, each with its vertices sorted.  Deterministic.
 *   pattern: as for cdcs_setup.  Outputs (host): nfill added entries
 *   (fill_i[e] >= fill_j[e], not in the pattern), p cliques with nvert
 *   vertices in all (clique_ptr [p+1], clique_vert [nvert]).  Call once with
 *   NULL arrays for the sizes, then with arrays of those sizes (any NULL
 *   array is skipped).
 * cdcs_setup with cliques = NULL runs this and appends the fill entries to
 * the caller's entries, with zero values of C and of every A_i on them: the
 * handle's global vectors then have nnz + nfill entries, the caller's first
 * (so x[0 .. nnz) is X on the caller's pattern and x beyond it is the
 * positive semidefinite completion's value on the fill).
 * Errors: CDCS_E_ARG, CDCS_E_PATTERN (entry out of range, duplicate).
 */
cdcs_status cdcs_chordal_extension(const cdcs_pattern *pattern, int64_t *nfill, int32_t *p, int64_t *nvert,
                                   int32_t *fill_i, int32_t *fill_j, int64_t *clique_ptr, int32_t *clique_vert);

/*
 * Setup step of Algorithms 1 and 2: the chordal decomposition data and the
 * cached factor of the KKT system (Sec. III-B.1).  Validates the pattern and
 * cliques, builds the entry selectors H_k and the overlap counts
 * D = sum_k H_k^T H_k (Sec. III-B.1), uploads the data, factors
 * M = A diag(w/D) A^T (Cholesky, FP64, on the device) and caches the inverse
 * factor for the affine projection (as CSR when sparse, else the dense inverse
 * M^-1 = L^-T L^-1 formed from it), and times the launch forms of
 * the batched projection (cdcs_get_tuning).  The factor is sparse when A is
 * kept sparse and the inverse factor stays sparse: a symbolic step on the
 * host orders M's rows (constraints sharing a pattern entry are adjacent;
 * perfect elimination order when that graph is chordal, else minimum degree)
 * and the device computes L column by column, level by level of the
 * elimination tree, then L^-1 along the tree paths (CSR, no m x m matrix).
 * Otherwise M is formed and factored dense (m <= 8192) and L^-1 kept as CSR
 * when it has under an eighth of a triangle's entries.
 *   b [m] host FP64, c [nnz] host FP64 (values of C on the entries).
 *   opts may be NULL (rho = 1).  The cached factor does not depend on rho.
 *   cliques may be NULL: the pattern is then extended to a chordal one and
 *   its maximal cliques found (cdcs_chordal_extension); the fill entries
 *   follow the caller's (dense A is read as m x nnz for the caller's nnz).
 *   A clique above CDCS_MAX_CLIQUE is rejected with CDCS_E_ARG.
 * Errors: CDCS_E_ARG, CDCS_E_PATTERN (unsorted/duplicate clique vertex, clique
 * pair missing from the pattern, entry in no clique, index out of range),
 * CDCS_E_RANK (A not of full row rank), CDCS_E_NOMEM, CDCS_E_DEVICE.
 * On error *out is NULL.
 */
cdcs_status cdcs_setup(const cdcs_pattern *pattern, const cdcs_constraints *A,
                       const double *b, const double *c, const cdcs_cliques *cliques,
                       const cdcs_options *opts, hipStream_t stream, cdcs_handle **out);

/*
 * Vector cones beside the PSD cliques (the cone types other than PSD that
 * CDCS accepts, Sec. IV: the free cone R^q, the nonnegative orthant R^q_+ and
 * the second-order cone {(t, z) : ||z|| <= t}).  Cone q covers the diagonal
 * entries of vertices vert[ptr[q] .. ptr[q+1]) (host arrays), in that order;
 * a second-order cone has at least 2 vertices, the first holding t.  A cone
 * vertex lies in no clique and in no other cone, and the pattern holds its
 * diagonal entry and no off-diagonal entry of it (so its variables are
 * ordinary vector variables, w_e = 1).  Each cone is one more block of the
 * decomposition: its selector H_k reads the cone's entries as a vector and
 * D_e = 1 on them.  Its slots follow the clique blocks' slots in cone order
 * (one slot per vertex), so state buffers hold nslots = nslots_psd + the cone
 * sizes (cdcs_get_sizes).  Algorithm 1 (and the HSDE solver) projects a cone
 * block onto its cone, Algorithm 2 onto the dual cone (the free cone's dual
 * cone is {0}; the orthant and the second-order cone are self-dual).
 */
typedef enum { CDCS_CONE_FREE = 0, CDCS_CONE_ORTHANT = 1, CDCS_CONE_SOC = 2 } cdcs_cone_kind;

typedef struct {
    int32_t ncones;
    const int32_t *kind;  /* host [ncones] cdcs_cone_kind */
    const int64_t *ptr;   /* host [ncones+1], ptr[0] = 0 */
    const int32_t *vert;  /* host [ptr[ncones]] */
} cdcs_vcones;

/*
 * cdcs_setup with vector cones (cones NULL or empty: the same as cdcs_setup).
 * With cones the clique list may be empty (p = 0: a linear or second-order
 * cone program).  cliques = NULL: the chordal extension covers the pattern
 * without the cone vertices.  Handles with cones run Algorithms 1 and 2 and
 * the HSDE solver; the differentiation entry points reject them (CDCS_E_ARG).
 * Errors: as for cdcs_setup; CDCS_E_PATTERN for a cone that breaks the rules
 * above, CDCS_E_ARG for an unknown kind.
 */
cdcs_status cdcs_setup_cones(const cdcs_pattern *pattern, const cdcs_constraints *A, const double *b,
                             const double *c, const cdcs_cliques *cliques, const cdcs_vcones *cones,
                             const cdcs_options *opts, hipStream_t stream, cdcs_handle **out);

/* One SDP of a batch (all pointers host, as for cdcs_setup). */
typedef struct {
    const cdcs_pattern *pattern;
    const cdcs_constraints *A;
    const double *b;
    const double *c;
    const cdcs_cliques *cliques;
} cdcs_problem;

/*
 * Many independent SDPs in one handle (the batching form of the hot path;
 * the paper only notes that the per-clique projections are independent and
 * parallel, Sec. III-B.2).  Instance q's entries, cliques, packed slots and
 * constraint rows follow instance q-1's, so state buffers are the
 * concatenations of the per-instance buffers (sizes from cdcs_get_sizes,
 * packed offsets from cdcs_clique_offsets; instance boundaries are the
 * prefix sums of the per-instance nnz, slots and m).  One projection launch
 * covers every instance's cliques; the affine step uses one cached factor per
 * instance (block-diagonal A).  cdcs_admm_solve (Algorithm 1 or 2) stops each
 * instance on its own residuals: once max(eps_p, eps_d) <= tol, that
 * instance's state is frozen and its time to tolerance is recorded
 * (cdcs_batch_info).  Each instance needs m <= 256.  Errors as cdcs_setup
 * (the message names the failing problem).
 */
cdcs_status cdcs_setup_batch(int32_t nprob, const cdcs_problem *probs, const cdcs_options *opts,
                             hipStream_t stream, cdcs_handle **out);

typedef struct {
    int32_t iters;        /* iterations when the instance stopped */
    int32_t status;       /* CDCS_OK (converged) or CDCS_E_NOT_CONVERGED */
    double eps_p, eps_d;  /* residuals at the last check of the instance */
    double obj_primal, obj_dual;
    double time_to_tol_s; /* device wall time from solve start to the instance's stop */
} cdcs_instance_info;

/* Per-instance results of the last solve on a batch handle (host [nprob]). */
cdcs_status cdcs_batch_info(const cdcs_handle *h, int32_t nprob, cdcs_instance_info *out_host);

cdcs_status cdcs_get_sizes(const cdcs_handle *h, cdcs_sizes *out);

/* Packed-slot offsets off[0..p] (host array of p+1 int64 written). */
cdcs_status cdcs_clique_offsets(const cdcs_handle *h, int64_t *off_host);

/*
 * Batched projection onto the product of PSD cones, P_k[W_k] of (E:XkUpdate)
 * and (E:zkUpdate): P(W) = Q max(Lambda, 0) Q^T for each of nb independent
 * symmetric blocks, FP32 (round-robin parallel Jacobi, one workgroup per
 * block).  Handle-free.
 *   sizes [nb] device int32, each in 1..CDCS_MAX_BATCHED_CLIQUE
 *   off   [nb+1] device int64, packed offsets (prefix sums of s(s+1)/2)
 *   W, P  [off[nb]] device FP32 packed lower triangles (may not alias)
 *   evals [sum s] device FP32 or NULL: eigenvalues, block t at eoff[t]
 *   evecs [sum s^2] device FP32 or NULL: eigenvectors as columns of a
 *         row-major s x s matrix, block t at voff[t]
 *   eoff, voff device int64 [nb+1] (required when evals/evecs are given)
 *   smax  host: the largest size in sizes[] (selects the kernel variant)
 * Accuracy: the sweeps stop once the off-diagonal part left in the rotated
 * block is at most 2^-20 ||W||_F; since the projection onto the PSD cone is
 * 1-Lipschitz in the Frobenius norm, P is then within 2^-20 ||W||_F (plus FP32
 * rounding) of P(W).  When evals or evecs are requested the sweeps run to
 * 2^-23 ||W||_F, so the eigenpairs themselves are converged.
 * A block whose size lies outside 1..smax is skipped (its P is not written);
 * nb <= 0 is a no-op.  Errors: CDCS_E_ARG (smax outside 1..CDCS_MAX_BATCHED_CLIQUE,
 * NULL W/P/sizes/off), CDCS_E_DEVICE.
 */
cdcs_status cdcs_psd_project_batched(int32_t nb, int32_t smax, const int32_t *sizes,
                                     const int64_t *off, const float *W, float *P,
                                     float *evals, const int64_t *eoff,
                                     float *evecs, const int64_t *voff, hipStream_t stream);

/*
 * The same projection for the cliques of a handle, launched with the handle's
 * tuned plan (cdcs_get_tuning: one persistent work-queue launch or one launch
 * per size bucket), as inside cdcs_admm_solve but on given blocks and from a
 * cold start (Jacobi from the identity, no eigenvector warm start).
 *   W, P [nslots] device FP32 packed clique blocks (cdcs_clique_offsets), no
 *        aliasing.  Accuracy as cdcs_psd_project_batched without eigenpairs.
 * Errors: CDCS_E_ARG (NULL argument), CDCS_E_DEVICE.
 */
cdcs_status cdcs_psd_project_cliques(cdcs_handle *h, const float *W, float *P, hipStream_t stream);

/*
 * Adjoint of the batched projection, for differentiating through
 * (E:XkUpdate) / (E:zkUpdate): given the eigenpairs written by
 * cdcs_psd_project_batched (evals, evecs with the same eoff/voff) and the
 * cotangent gP of P (packed), writes the cotangent gW of W (packed):
 *   Wbar = V (Gamma o (V^T G V)) V^T   (Daleckii-Krein form),
 * Gamma_ij = (max(l_i,0) - max(l_j,0)) / (l_i - l_j), 1 if both l > 0, 0 if
 * both l <= 0 (the derivative of max(., 0) at 0 is taken as 0).  An
 * off-diagonal packed value stands for both triangles: G holds half of it on
 * each side and gW adds both triangles of Wbar.  gW may not alias gP.
 * Errors: CDCS_E_ARG, CDCS_E_DEVICE.
 */
cdcs_status cdcs_psd_project_vjp(int32_t nb, int32_t smax, const int32_t *sizes, const int64_t *off,
                                 const float *evals, const int64_t *eoff, const float *evecs,
                                 const int64_t *voff, const float *gP, float *gW, hipStream_t stream);

/*
 * Entry selectors of Sec. III-A in FP64, for building differentiable
 * iterations: cdcs_gather writes H_k x for every clique into packed slots
 * (x [nnz] -> packed [nslots]); cdcs_scatter writes sum_k H_k^T applied to
 * packed clique blocks (packed [nslots] -> out [nnz]; each packed slot adds to
 * its entry once, so the two are transposes of each other).  Device buffers;
 * no aliasing.  Errors: CDCS_E_ARG.
 */
cdcs_status cdcs_gather(const cdcs_handle *h, const double *x, double *packed, hipStream_t stream);
cdcs_status cdcs_scatter(const cdcs_handle *h, const double *packed, double *out, hipStream_t stream);

/*
 * Affine projection: solve the KKT system of (E:OptCondMinYPrimal)
 * [D A^T; A 0][x; y] = [r1; r2] by block elimination with the cached factor
 * (the same matrix serves (E:OptCondMinYDual), Sec. IV-B.1):
 *   y = M^-1 (A (w r1 / D) - r2),   x = (r1 - A^T y) / D.
 *   r1, x [nnz] device FP64; r2, y [m] device FP64.  x may alias r1.
 */
cdcs_status cdcs_affine_project(const cdcs_handle *h, const double *r1, const double *r2,
                                double *x, double *y, hipStream_t stream);

/*
 * ADMM iterations of Algorithm 1 (opts->form = CDCS_PRIMAL) or Algorithm 2
 * (CDCS_DUAL) on the caller's state, until max(eps_p, eps_d) <= tol or
 * max_iter iterations.  Residuals (Boyd et al. 2011, Sec. 3.3, relative form):
 *   Alg. 1: eps_p = ||x_k - H_k x|| / max(||H_k x||, ||x_k||),
 *           eps_d = rho ||sum_k H_k^T (x_k - x_k_prev)|| / ||sum_k H_k^T lambda_k||;
 *   Alg. 2: eps_p = ||z_k - v_k|| / max(||z_k||, ||v_k||),
 *           eps_d = rho ||v_k - v_k_prev|| / ||lambda_k||.
 * With check_every > 0, check_every iterations are captured in one HIP graph
 * and replayed (a last graph holds the max_iter % check_every remaining
 * iterations, so exactly max_iter iterations are launched); every kernel of
 * an iteration after convergence returns at once.  Synchronises on stream.
 * Returns CDCS_OK when converged (or when tol = 0 and max_iter iterations
 * ran), CDCS_E_NOT_CONVERGED at the cap, CDCS_E_NUMERIC if an eigensolve hit
 * its sweep cap or a residual is not finite (a NaN or Inf in the state or
 * the data reaches the residual sums within one iteration; the solve stops
 * there, on a batch handle the instance stops).  info may be NULL.
 */
cdcs_status cdcs_admm_solve(cdcs_handle *h, const cdcs_state *st, const cdcs_options *opts,
                            cdcs_info *info, hipStream_t stream);

/*
 * Capture and instantiate, without running any iteration, the HIP graphs that
 * cdcs_admm_solve with the same handle, state buffers and options launches
 * (max_iter / check_every graphs of check_every iterations, then one graph of
 * the remaining max_iter % check_every iterations), so that the solve itself
 * spends no time on capture.  Nothing is enqueued on `stream`; the state is
 * not read.  check_every = 0 (eager launches) is a no-op.
 * Errors: as cdcs_admm_solve's argument checks; CDCS_E_DEVICE.
 */
cdcs_status cdcs_admm_prepare(cdcs_handle *h, const cdcs_state *st, const cdcs_options *opts,
                              hipStream_t stream);

/* Write identity blocks into a caller's warm-start buffer (cdcs_state.vw,
 * nwarm floats, device memory) on `stream`: the basis a new state starts
 * from.  Errors: CDCS_E_ARG (NULL handle or buffer). */
cdcs_status cdcs_warm_reset(const cdcs_handle *h, float *vw, hipStream_t stream);

/* One iteration (eager launches) continuing from the state; equivalent to
 * cdcs_admm_solve with max_iter = 1, tol = 0, check_every = 0. */
cdcs_status cdcs_admm_step(cdcs_handle *h, const cdcs_state *st, int32_t form, double rho,
                           hipStream_t stream);

/*
 * Differentiation through unrolled iterations (not in the paper: the
 * adjoint of the map (c, b) -> x after K iterations of Algorithm 1).
 *
 * cdcs_unrolled_step: one iteration of Algorithm 1 on the caller's state,
 * exactly as cdcs_admm_step (primal form) runs it, but with the cost c
 * [nnz, pattern order] and right-hand side b [m] taken from the caller's
 * device buffers (FP64) instead of the handle's data, and writing the
 * eigenpairs of every clique's projection (E:XkUpdate): evals [sum_k s_k]
 * (clique k at the prefix sum of s_j, j < k) and evecs [nwarm] (k x k
 * row-major, eigenvectors in columns, offsets the prefix sums of s_k^2), FP32
 * device buffers, each may be NULL.  With c and b equal to the handle's data
 * the new state equals cdcs_admm_step's bit for bit.  The eigenvectors are
 * those the state's warm start (vw) keeps; give the state a vw buffer, or
 * every step restarts Jacobi from the identity.
 *
 * cdcs_unrolled_step_vjp: its adjoint.  Inputs: the step's saved evals and
 * evecs; the cotangents of the step's outputs: xbar [nnz, pattern order] of
 * its x (NULL: zero), blkbar and lambar [nslots] FP64 of its x_k and
 * lambda_k (packed coordinates: the derivative with respect to each packed
 * value; an off-diagonal value stands for both mirrored entries).  Outputs:
 * blkbar and lambar are overwritten with the cotangents of the step's input
 * x_k and lambda_k; cbar [nnz, pattern order] and bbar [m] accumulate the
 * cotangents of c and b.  The projection's adjoint is the Daleckii-Krein
 * form of cdcs_psd_project_vjp (FP32); the affine adjoint is the cached
 * KKT solve applied to the cotangent (FP64): for x = F(r1, b),
 * rbar1 = w F(xbar / w, 0) and bbar is that solve's y.
 *
 * cdcs_affine_project_adjoint: the affine part alone, for
 * x = cdcs_affine_project(r1, r2): r1bar [nnz] = w F(xbar / w, 0) and
 * r2bar [m] = that solve's y (both overwritten; pattern order).
 *
 * All buffers are device memory; no aliasing between outputs and inputs
 * except as stated.  The handle allocates its work buffers at the first call.
 * Errors: CDCS_E_ARG (NULL argument, rho <= 0, a batch handle for the
 * unrolled step), CDCS_E_NOMEM, CDCS_E_DEVICE; cdcs_unrolled_step returns
 * cdcs_admm_step's status.
 */
cdcs_status cdcs_unrolled_step(cdcs_handle *h, const cdcs_state *st, const double *c, const double *b, double rho,
                               float *evals, float *evecs, hipStream_t stream);
cdcs_status cdcs_unrolled_step_vjp(cdcs_handle *h, double rho, const float *evals, const float *evecs,
                                   const double *xbar, double *blkbar, double *lambar, double *cbar, double *bbar,
                                   hipStream_t stream);
cdcs_status cdcs_affine_project_adjoint(cdcs_handle *h, const double *xbar, double *r1bar, double *r2bar,
                                        hipStream_t stream);

/*
 * cdcs_affine_project_adjoint without any device allocation, for callers
 * that cannot allocate (code under HIP graph capture, serving loops, hosts
 * that forbid hipMalloc after initialisation).  Same inputs, outputs and
 * results as cdcs_affine_project_adjoint (the same kernels); its staging
 * buffers (the KKT solve's x and y) are a fixed array in device memory,
 * 8,454,144 bytes per device, held until the process ends, instead of the
 * buffers cdcs_affine_project_adjoint allocates at its first call.  Limits:
 * the handle's pattern entries at most 2^20 and its constraints at most 8192,
 * each counted as the handle pads them (single-SDP handles: entries to a
 * multiple of 64, constraints to a multiple of 32).
 * Calls that overlap on one device race on that array (serialise them, e.g.
 * one stream).  Errors: CDCS_E_ARG (NULL argument, handle above the limits),
 * CDCS_E_DEVICE.
 */
cdcs_status cdcs_affine_project_adjoint_noalloc(cdcs_handle *h, const double *xbar, double *r1bar, double *r2bar,
                                                hipStream_t stream);

/*
 * Homogeneous self-dual embedding (HSDE) of the decomposed problem: the
 * variant the paper names as future work so that infeasibility can be
 * detected (Sec. VI), solved by the operator-splitting iteration of
 * O'Donoghue, Chu, Parikh and Boyd (2016) without over-relaxation.
 *
 * The decomposed primal problem min <c, x>_w s.t. A(x) = b, H_k x in K_k
 * (cliques: PSD cones; vector cones) is the conic program
 * min <c, x> s.t. Ahat x + s = bhat, s in {0}^m x K_1 x ... x K_p, with
 * Ahat = [A; -H_1; ...; -H_p] and bhat = (b, 0).  Its embedding seeks
 * u = (x, y, z, tau) in R^nnz x R^m x K* x R_+ and v = (0, 0, s, kappa) in
 * {0} x {0} x K x R_+ with v = Q u,
 *   Q = [[0, Ahat^T, c], [-Ahat, 0, bhat], [-c^T, -bhat^T, 0]].
 * An iteration is ut = (I + Q)^-1 (u + v), u = Pi(ut - v), v = v - ut + u:
 * the linear step eliminates down to the m x m matrix
 * M' = I + A diag(w / (1 + D)) A^T, whose factor is cached like Algorithm 1's
 * (dense, CSR inverse or sparse, built at the first HSDE call on a handle),
 * and the cone step is the Algorithm-1 projection kernel with rho = 1
 * (s_k = P(H_k x - z_k), z_k = s_k - (H_k x - z_k)).  After each iteration
 * the residuals, from differences of successive iterates (no extra pass over
 * A), decide the outcome, in this order (tau > 0 for the first):
 *   solved:   ||(A(x) - tau b, s - Hx)|| <= tol tau (1 + ||b||),
 *             ||A^T y - sum_k H_k^T z_k + tau c||_w <= tol tau (1 + ||c||_w),
 *             |<c, x>_w + b^T y| <= tol (tau + |<c, x>_w| + |b^T y|);
 *   primal infeasible: b^T y < 0, ||A^T y - sum_k H_k^T z_k||_w ||b|| <= tol (-b^T y);
 *   dual infeasible:   <c, x>_w < 0, ||(A(x), s - Hx)|| ||c||_w <= tol (-<c, x>_w).
 * Solved: X = x / tau solves the primal SDP, y_sdp = -y / tau the dual one,
 * Z = sum_k H_k^T z_k / tau.  Primal infeasible: y / (b^T y) is a Farkas
 * certificate (b^T y_c = 1, A^T y_c in -K*).  Dual infeasible:
 * x / (-<c, x>_w) is a ray (A(x_c) = 0, x_c in K, <c, x_c> = -1).
 *
 * State (device, caller-owned; sizes from cdcs_get_sizes):
 *   x  [nnz]    FP64  u_x, pattern order
 *   y  [m]      FP64  u_y on the equality rows
 *   s  [nslots] FP32  the cone slacks s_k, packed as cdcs_state.blk
 *   z  [nslots] FP32  the cone duals z_k, packed
 *   tk [2]      FP64  tau, kappa
 *   vw [nwarm]  FP32  eigenvector warm start as in cdcs_state (NULL: the
 *                     handle's copy, restarted at identity by every solve)
 */
typedef struct {
    double *x;
    double *y;
    float *s;
    float *z;
    double *tk;
    float *vw;
} cdcs_hsde_state;

typedef struct {
    int32_t iters;        /* completed iterations */
    int32_t status;       /* CDCS_OK (solved), CDCS_PRIMAL_INFEASIBLE, CDCS_DUAL_INFEASIBLE,
                             CDCS_E_NOT_CONVERGED or CDCS_E_NUMERIC */
    int32_t jacobi_cap_hits;
    int32_t pad_;
    double res_pri, res_dual, gap;  /* the solved test's three ratios at the last iterate */
    double obj_primal;    /* <C, X> with X = x / tau (NaN if tau = 0) */
    double obj_dual;      /* b^T y_sdp with y_sdp = -y / tau (NaN if tau = 0) */
    double tau, kappa;
    double loop_s;
    int64_t jacobi_sweeps;
} cdcs_hsde_info;

/* Starting point u = (0, 0, 0, 1), v = (0, 0, 0, 1) (every buffer of st
 * written; vw set to identities when given).  Errors: CDCS_E_ARG. */
cdcs_status cdcs_hsde_init(cdcs_handle *h, const cdcs_hsde_state *st, hipStream_t stream);

/*
 * Up to opts->max_iter HSDE iterations from st (opts->tol, max_iter,
 * check_every as for cdcs_admm_solve; rho and form are not used).  Builds the
 * HSDE factor on the first call (CDCS_E_RANK if M' is not positive definite,
 * which needs A rank deficient beyond rounding).  The outcome is in
 * info->status and the return value.  Synchronises on stream.
 * Errors: CDCS_E_ARG (NULL buffers, batch handle), CDCS_E_NOMEM, CDCS_E_DEVICE.
 */
cdcs_status cdcs_hsde_solve(cdcs_handle *h, const cdcs_hsde_state *st, const cdcs_options *opts,
                            cdcs_hsde_info *info, hipStream_t stream);

/*
 * The primal and dual points of the state cdcs_hsde_solve returned, by its
 * outcome `which`: 0 (solved) X = x / tau [nnz] and y_sdp = -y / tau [m];
 * 1 (primal infeasible) y / (b^T y) into y_out (X_out untouched);
 * 2 (dual infeasible) x / (-<c, x>_w) into X_out (y_out untouched).
 * X_out and y_out device FP64, pattern order; the scale factors are the ones
 * the solve's last check computed.  Errors: CDCS_E_ARG.
 */
cdcs_status cdcs_hsde_solution(cdcs_handle *h, const cdcs_hsde_state *st, int32_t which, double *X_out,
                               double *y_out, hipStream_t stream);

/* cdcs_hsde_solve with eager launches and HIP events around each kernel kind
 * of every iteration, as cdcs_admm_solve_timed does for Algorithms 1 and 2
 * (kinds: the projection, the A u partials, the solve with M^-1, A^T y,
 * the scatter; the tau row and the update of x run unbracketed, the check
 * inside the A u launch as for Algorithm 1).
 * The iterates are those of cdcs_hsde_solve with the same state and options.
 * Errors: those of cdcs_hsde_solve; CDCS_E_ARG for NULL kernel_ms or launches. */
cdcs_status cdcs_hsde_solve_timed(cdcs_handle *h, const cdcs_hsde_state *st, const cdcs_options *opts,
                                  cdcs_hsde_info *info, double *kernel_ms, int64_t *launches, hipStream_t stream);

/* Residual history of the last HSDE solve: n_host triples (res_pri,
 * res_dual, gap) of the solved test, one per iteration, host. */
cdcs_status cdcs_hsde_history(const cdcs_handle *h, double *hist_host, int32_t n_host);

/* Kernels of one iteration, for cdcs_profile_kernel. */
typedef enum {
    CDCS_K_PROJECT = 0,   /* fused gather + Jacobi projection + epilogue, all size buckets */
    CDCS_K_GEMV_AU = 1,   /* partials of A (w r1 / D)    (affine step, first half; without the
                             small reduction to t = A (w r1 / D) - r2 that follows it) */
    CDCS_K_TRMV = 2,      /* y = M^-1 t                  (one product with the dense M^-1 = L^-T L^-1,
                             or two with the sparse inverse factor L^-1 and its transpose) */
    CDCS_K_GEMV_ATY = 3,  /* x = (r1 - A^T y) / D        (affine step, second half) */
    CDCS_K_SCATTER = 4    /* r1 = sum_k H_k^T (...)      (right-hand side scatter) */
} cdcs_kernel;

/*
 * Instrumentation: cdcs_admm_solve with eager launches (opts->check_every is
 * not used) that brackets each kernel kind of every iteration with HIP events
 * on `stream`.  The launches, their order and so the iterates are those of
 * cdcs_admm_solve with the same state and options, so replaying a timed
 * cdcs_admm_solve from a copy of its starting state gives its per-kernel
 * durations.  On return kernel_ms[k] holds the summed milliseconds and
 * launches[k] the number of bracketed launches of kind k (arrays of 5,
 * indexed by cdcs_kernel, owned by the caller; CDCS_K_GEMV_AU without the
 * small reduction that follows it).  Batch handles: CDCS_K_GEMV_AU covers the
 * whole affine step, CDCS_K_TRMV and CDCS_K_GEMV_ATY stay 0.  The residual
 * checks run unbracketed, except Algorithm 1's on a single-SDP handle, which
 * runs as the first workgroup of the A u launch (overlapping the product; a
 * separate launch only when the partial sums number more than 8192) and so
 * falls inside CDCS_K_GEMV_AU.  Synchronises on stream.
 * Errors: those of cdcs_admm_solve; CDCS_E_ARG for NULL kernel_ms or launches.
 */
cdcs_status cdcs_admm_solve_timed(cdcs_handle *h, const cdcs_state *st, const cdcs_options *opts,
                                  cdcs_info *info, double *kernel_ms, int64_t *launches,
                                  hipStream_t stream);

/*
 * Instrumentation: enqueue `reps` back-to-back launches of one kernel of an
 * iteration of the given form, with the arguments it has inside
 * cdcs_admm_solve on this state (y, blk, lam, v, vw are updated as by those
 * launches).  The x these launches read and write is the handle's own copy of
 * the iterate, which equals st->x after a cdcs_admm_solve or cdcs_admm_step
 * on this state; st->x itself is neither read nor written, so nothing but the
 * named kernel runs.  Lets a caller bracket one kernel with events on
 * `stream` to time it.
 * Errors: CDCS_E_ARG (unknown kernel, reps < 1, NULL state buffers).
 */
cdcs_status cdcs_profile_kernel(cdcs_handle *h, const cdcs_state *st, int32_t form, double rho,
                                int32_t kernel, int32_t reps, hipStream_t stream);

/*
 * Launch plan of the batched projection inside the ADMM loop ("thousands of
 * cliques of uneven sizes" in one step, Sec. III-B.2): cliques are padded to
 * size buckets S in {16, 32, 48, 64, 80, 96, 112, 128}.  Either one persistent launch
 * draws every clique, largest first, from a device work queue
 * (persistent = 1, `threads` per workgroup, `grid` workgroups), or each
 * bucket gets its own launch with its own workgroup size, one after the other
 * in the caller's stream (persistent = 0) or on parallel streams forked from
 * it and joined back into it (persistent = 2: the launches' tails overlap;
 * the same kernels, so the same bits as 0).  Setup picks the fastest form by
 * timing all three on the handle's cliques (queue_us, buckets_us = sum of
 * bucket_us, parallel_us: microseconds per projection of all cliques on
 * generated nearly diagonal blocks; -1 where a form does not apply).
 */
typedef struct {
    int32_t persistent;
    int32_t threads;
    int32_t grid;
    int32_t nbuckets;
    int32_t bucket_size[8];
    int32_t bucket_threads[8];
    int32_t bucket_count[8];
    float bucket_us[8];      /* best per-bucket launch time */
    float queue_us;
    float buckets_us;
    float parallel_us;
} cdcs_tuning;

cdcs_status cdcs_get_tuning(const cdcs_handle *h, cdcs_tuning *out);

/*
 * Override the tuned plan: persistent = 1 with threads 256 or 512 (512 only
 * when a clique has more than 96 vertices) and `grid`
 * workgroups (0: as many as stay resident, at most one per clique; a smaller
 * grid makes every workgroup project several cliques), or persistent = 0 with
 * threads 64, 256 or 512 for every bucket that has that size built (64:
 * buckets 16 and 32 only, the others keep 256; 256 and 512: every bucket),
 * or 0 to keep the tuned per-bucket sizes (grid is ignored); persistent = 2
 * is persistent = 0 with the buckets on parallel streams.
 * Synchronizes the device and drops captured graphs.  Errors: CDCS_E_ARG
 * (also for a grid above the resident workgroups), CDCS_E_DEVICE.
 */
cdcs_status cdcs_set_projection_plan(cdcs_handle *h, int32_t persistent, int32_t threads, int32_t grid);

/* Residual history of the last solve: n_host pairs (eps_p, eps_d), host. */
cdcs_status cdcs_residual_history(const cdcs_handle *h, double *hist_host, int32_t n_host);

cdcs_status cdcs_destroy(cdcs_handle *h);

/* Message of the last error on the calling thread ("" if none). */
const char *cdcs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CDCS_H */
