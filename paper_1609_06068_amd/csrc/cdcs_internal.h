// Internal declarations of the gfx950 library: the handle, the device-side
// control block and the kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cdcs.h"

namespace cdcs {

// Device control block of an ADMM solve.  Kernels of an iteration read
// `stop` first and return at once when it is set, so a captured graph of
// several iterations becomes a no-op after convergence.
struct Ctl {
    int32_t iter;       // completed iterations
    int32_t stop;       // 0 running, 1 converged, 2 iteration cap, 3 NaN/Inf in the residuals,
                        // 4 / 5 primal / dual infeasibility certificate (HSDE)
    int32_t max_iter;
    int32_t jacobi_cap; // eigensolves that hit the sweep cap
    int32_t sweeps;     // Jacobi sweeps summed over all eigensolves
    int32_t pad_;
    double tol;
    double eps_p, eps_d;
};

// Arguments of the batched projection kernel.
enum ProjMode : int32_t {
    PROJ_STANDALONE = 0,  // W given packed, P written packed
    PROJ_PRIMAL = 1,      // Alg. 1: W = H_k x - lam/rho; x_k = P(W); lam += rho (x_k - H_k x)
    PROJ_DUAL = 2,        // Alg. 2: W = v - lam/rho; z_k = P(W)
};

struct ProjArgs {
    int32_t mode;
    int32_t nblk;              // blocks in this launch
    const int32_t *ids;        // [nblk] block ids (NULL: identity)
    const int32_t *size;       // [*] block sizes
    const int64_t *off;        // [*] packed offsets
    // standalone
    const float *Win;
    float *Pout;
    float *evals;
    const int64_t *eoff;
    float *evecs;
    const int64_t *voff;
    // ADMM
    const int32_t *gather;     // [nslots] pattern entry of each packed slot
    const double *x;           // [nnz]
    float *blk;                // [nslots]
    float *lam;                // [nslots]
    const float *v;            // [nslots]
    double rho;
    double inv_rho;            // 1 / rho (computed on the host: one FP64 multiply per slot, not a divide)
    const int32_t *kinst;      // [*] instance of each block (many-SDP handles), or NULL
    const int32_t *istop;      // [nprob] per-instance stop flags, or NULL
    float *vwarm;              // eigenvector warm start, NULL: cold
    const int64_t *vwoff;      // [*] offsets of the k x k blocks in vwarm
    int32_t warm_store;        // write the new eigenvectors back to vwarm
    double *cpart;             // [p][4] per-block partial sums
    float *dslot;              // [nslots] Alg. 1: x_k(new) - x_k(old) per slot (the dual residual's terms), or NULL
    Ctl *ctl;                  // may be NULL (standalone)
};

// Size bucket (padded clique size) of the projection kernel for cliques <= smax:
// 16, 32, 48, 64, 80, 96, 112 or 128 (cliques of at most 126 vertices).
int proj_bucket(int smax);
// Workgroup sizes built for a bucket: 64 (S <= 32), 256, 512 (S >= 48).
bool proj_threads_ok(int S, int nthreads);
// One launch over a.nblk cliques of one bucket (workgroup b: clique a.ids[b]).
void launch_project(const ProjArgs &a, int smax, int nthreads, hipStream_t s);
// Persistent launch over a.nblk cliques of every bucket up to smax, drawn in
// a.ids order from the ticket counter (nthreads 256 or 512).
void launch_project_queue(const ProjArgs &a, int smax, int nthreads, int grid, unsigned long long *ticket,
                          hipStream_t s);
// Resident workgroups per CU of the persistent launch.
int project_queue_occupancy(int smax, int nthreads);

// Vector cones: blocks of at most kVecChunk slots, one workgroup each
// (kernels_cones.hip).  vblk rows are (kind, first slot, end slot, cone; for
// a second-order cone its index among those cones); the blocks' residual
// partial sums go to cpart rows p + b.  A second-order cone's norm comes
// from per-block partial sums (soc_part) that each of its blocks adds up.
constexpr int kVecChunk = 1024;
struct Dev;
void launch_project_vec(const ProjArgs &a, const Dev &d, hipStream_t s);

// Cliques above the LDS-resident limit (kMaxLdsClique vertices): projection
// through the Newton-Schulz sign iteration on N x N blocks (kernels_big.hip).
constexpr int kMaxLdsClique = 126;
constexpr int kNsSteps = 48;
struct BigCliques {
    int32_t nbig = 0;              // large cliques
    int32_t tmax2 = 0;             // largest (N / 64)^2: 64 x 64 tiles of one block
    const int32_t *ids = nullptr;  // [nbig] clique ids
    const int32_t *n = nullptr;    // [nbig] sizes
    const int32_t *N = nullptr;    // [nbig] sizes rounded up to 64
    const int64_t *boff = nullptr; // [nbig + 1] offsets of the N x N blocks
    float *W = nullptr;            // [boff[nbig]] W, zero padded
    float *X0 = nullptr, *X1 = nullptr;  // Newton-Schulz iterates
    float *Y = nullptr;            // products; P at the end
    double *part = nullptr;        // [4 * nbig * tmax2] per-tile partial sums
    double *inv_norm = nullptr;    // [nbig] 1 / ||W||_F
    int32_t *stop = nullptr;       // [nbig] Newton-Schulz step at which the clique stopped, -1 running
};
void launch_big_projection(const ProjArgs &a, const BigCliques &b, hipStream_t s);

// Arguments of the projection adjoint (Daleckii-Krein) kernel.
struct VjpArgs {
    int32_t nblk;
    const int32_t *size;
    const int64_t *off;        // packed offsets
    const float *evals;
    const int64_t *eoff;
    const float *evecs;        // k x k row-major, eigenvectors in columns
    const int64_t *voff;
    const float *gP;           // packed cotangent of P
    float *gW;                 // packed cotangent of W
};
void launch_project_vjp(const VjpArgs &a, int smax, hipStream_t s);
// Autotuning input: nearly diagonal symmetric packed blocks (see the kernel).
void launch_tune_blocks(const int32_t *size, const int64_t *off, int p, float *W, hipStream_t s);
// Set every k x k block of V (at voff[k]) to the identity.
void launch_identity_blocks(const int32_t *size, const int64_t *voff, int p, float *V, hipStream_t s);

// Many independent SDPs in one handle: index ranges and per-instance state.
// Column chunk (entries) of one job of the batched A u product: long rows
// are split so that jobs are of similar size.
constexpr int kBatchAuChunk = 4096;
constexpr int kXcds = 8;  // XCDs of the MI355X (workgroups are dispatched to them round robin)

struct Batch {
    int32_t nprob = 0;
    int64_t *U_off = nullptr;      // [nprob+1] entry ranges
    int32_t *m_off = nullptr;      // [nprob+1] constraint-row ranges
    int32_t *k_off = nullptr;      // [nprob+1] clique ranges
    int64_t *A_off = nullptr;      // [nprob] offset of A_q (w-scaled FP32, m_q x A_ld[q])
    int32_t *A_ld = nullptr;       // [nprob]
    int64_t *F_off = nullptr;      // [nprob] offset of the m_q x m_q FP64 factors
    int32_t *einst = nullptr;      // [nU] instance of each entry
    int32_t *rinst = nullptr;      // [m] instance of each row
    int32_t *kinst = nullptr;      // [p] instance of each clique
    int32_t *sblk = nullptr;       // [nsblk * 4] scatter blocks (q, e0, e1, 0)
    int32_t *sblk_off = nullptr;   // [nprob+1] scatter-block ranges
    int32_t nsblk = 0;
    int32_t *syrk_jobs = nullptr;  // [nsyrk * 4] (q, I, J, 0) tiles of M_q
    int32_t nsyrk = 0;
    int32_t *trtri_jobs = nullptr; // [m * 2] (q, j)
    int32_t *rjobs = nullptr;      // [nrjobs * 4] (q, first row, rows <= 4, column chunk) of the A u product, by XCD; rows 0 = unused slot
    int32_t *nch = nullptr;        // [nprob] column chunks of kBatchAuChunk entries per row of A_q
    int64_t *p_off = nullptr;      // [nprob] offset of instance q's per-chunk partial sums in tpart
    double *tpart = nullptr;       // [sum over split instances of m_q * nch_q] partial sums of A u
    int32_t split = 0;             // some instance has rows of more than one chunk
    int32_t nrjobs = 0;
    int32_t *ejobs = nullptr;      // [nejobs * 2] (q, first entry in q) of 1024-entry A^T y blocks
    int32_t nejobs = 0;
    int32_t *vblk = nullptr;       // [nvblk * 4] slot blocks (q, s0, s1, 0) of the Alg. 2 epilogue
    int32_t *vblk_off = nullptr;   // [nprob+1] slot-block ranges
    int32_t nvblk = 0;
    int32_t *istop = nullptr;      // [nprob] 0 running, 1 converged, 2 iteration cap, 3 NaN/Inf
    int32_t *iiters = nullptr;     // [nprob] iterations at stop
    uint64_t *itime = nullptr;     // [nprob] device wall clock at stop
    uint64_t *t0 = nullptr;        // [1] device wall clock at solve start
    double *ieps = nullptr;        // [nprob * 2] last eps_p, eps_d
    double *iobj = nullptr;        // [nprob * 2] <c, x>_w and <b, y>
    int32_t *nrunning = nullptr;   // [1] instances still running
    int32_t *finfo = nullptr;      // [nprob] factorisation status
};

// Affine-step, scatter, residual and setup kernels (kernels_affine.hip).
struct Dev {
    // problem
    int32_t n = 0, m = 0, p = 0, smax = 0;
    int64_t nU = 0, nslots = 0;
    int64_t nslots_psd = 0;        // slots of the cliques; the vector cones' slots follow
    int32_t nvc = 0, nvb = 0;      // vector cones and their work blocks
    int32_t *vblk = nullptr;       // [nvb * 4] (kind, s0, s1, cone)
    int32_t nsoc = 0;              // second-order cones
    int32_t *soc = nullptr;        // [nsoc * 3] (first slot, first block, end block)
    int32_t nsocb = 0;             // work blocks of the second-order cones
    int32_t *socb = nullptr;       // [nsocb] their indices among the nvb blocks
    double *soc_part = nullptr;    // [nvb] per-block sums of z^2 (second-order cone blocks)
    int64_t ldU = 0;               // row stride of Aw (nU rounded up to 64)
    int64_t ldM = 0;               // row stride of AwT (m rounded up to 32; 4 on batch handles)
    int32_t *clq_size = nullptr;   // [p]
    int64_t *clq_off = nullptr;    // [p+1]
    int32_t *gather = nullptr;     // [nslots] internal entry of each packed slot
    int32_t *perm = nullptr;       // [nU] pattern position of each internal entry
    int32_t *inv_ptr = nullptr;    // [nU+1]
    int32_t *inv_slot = nullptr;   // [nslots]
    int32_t *heavy = nullptr;      // [nheavy] entries with long inverse lists
    int32_t nheavy = 0;
    double *invD = nullptr;        // [nU]  1 / D_e
    double *s2 = nullptr;          // [nU]  1 / (w_e D_e)
    double *wt = nullptr;          // [nU]  w_e (1 diagonal, 2 off-diagonal)
    double *c = nullptr;           // [nU]
    double *b = nullptr;           // [m]
    float *Aw = nullptr;           // [m * ldU] row-major, w_e * A_ie, zero padded
    float *AwT = nullptr;          // [nU * ldM] row-major transpose of Aw, zero padded
    // sparse A (CSR input of low density): rows for A u, touched columns for A^T y
    int32_t sparse = 0;
    int64_t nnzA = 0;
    int32_t ntc = 0;               // pattern entries with at least one constraint coefficient
    int32_t *sp_ptr = nullptr;     // [m+1]   row pointers
    int32_t *sp_col = nullptr;     // [nnzA]  entry of each coefficient (sorted within a row)
    double *sp_val = nullptr;      // [nnzA]  w_e * A_ie
    int32_t *tc_e = nullptr;       // [ntc]   touched entries, increasing
    int32_t *tc_ptr = nullptr;     // [ntc+1]
    int32_t *tc_row = nullptr;     // [nnzA]  row of each coefficient, by touched entry
    double *tc_val = nullptr;      // [nnzA]  w_e * A_ie, by touched entry
    // sparse inverse factors (used when L^-1 has few nonzeros): CSR rows of
    // L^-1 (lower) and of L^-T (upper), FP64
    int32_t sparse_linv = 0;
    int64_t nnz_linv = 0;
    int32_t spchol = 0;            // L computed sparse (symbolic + numeric), no dense M ever formed
    int64_t nnz_l = 0;             // its nonzeros
    int32_t *li_ptr = nullptr, *li_col = nullptr;
    double *li_val = nullptr;
    int32_t *lt_ptr = nullptr, *lt_col = nullptr;
    double *lt_val = nullptr;
    double *Linv = nullptr;        // [m * m] row-major, L^-1 (lower); setup only (batch handles: per instance)
    double *LinvT = nullptr;       // [m * m] row-major, L^-T (upper); setup only (batch handles: per instance)
    double *Minv = nullptr;        // [m * m] row-major, M^-1 = L^-T L^-1 (dense factor of a single-SDP handle)
    int32_t *order = nullptr;      // [p_lds] cliques of at most kMaxLdsClique vertices, by decreasing size
    int32_t p_lds = 0;             // cliques projected in LDS (the others: big)
    int32_t smax_lds = 0;          // largest of them
    BigCliques big;
    int64_t *vwoff = nullptr;      // [p+1] offsets of k x k blocks (prefix sums of s_k^2)
    float *vwarm = nullptr;        // [sum s_k^2] eigenvectors of the last projection
    int64_t nwarm = 0;             // sum s_k^2
    // work
    double *u = nullptr;           // [ldU] r1 / D, zero padded
    double *xi = nullptr;          // [ldU] x in internal entry order (the solver's iterate)
    double *xtmp = nullptr;        // [ldU] entry-space scratch of the interface calls
    double *t = nullptr;           // [m]
    double *tpart = nullptr;       // [8 * m] split-K partials of A u
    double *y1 = nullptr;          // [m]
    float *dslot = nullptr;        // [nslots] x_k(new) - x_k(old) of the last Alg. 1 projection, per slot
    uint32_t *wbits = nullptr;     // [(nU + 31) / 32] bit e: entry e is off the diagonal (w_e = 2)
    double *cpart = nullptr;       // [(p + nvb) * 4]
    double *spart = nullptr;       // [nsblk * 2]
    double *vpart = nullptr;       // [nvblk * 5]
    double *hist = nullptr;        // [hist_cap * 2]
    double *obj = nullptr;         // [2]
    double *opart = nullptr;       // [objective_partials()] partial sums of the objectives
    int32_t hist_cap = 0;
    int32_t *info = nullptr;       // [4] setup status words
    Ctl *ctl = nullptr;
    Ctl *ctl_host = nullptr;       // pinned mirror
    Batch *batch = nullptr;        // many-SDP handles only
};

// many-SDP kernels (kernels_batch.hip)
void launch_breset(const Dev &d, hipStream_t s);
void launch_bscatter_primal(const Dev &d, const float *blk, const float *lam, double rho, hipStream_t s);
void launch_bcheck_primal(const Dev &d, double rho, hipStream_t s);
void launch_bscatter_dual(const Dev &d, const float *blk, const float *lam, double rho, hipStream_t s);
void launch_bvupdate(const Dev &d, const double *x, const float *blk, float *lam, float *v, double rho,
                     hipStream_t s);
void launch_bcheck_dual(const Dev &d, double rho, hipStream_t s);
void launch_baffine(const Dev &d, const double *r2, double r2scale, double *x, double *y, const Ctl *ctl,
                    const int32_t *istop, hipStream_t s);
void launch_bsetup(const Dev &d, double *M, hipStream_t s);
void launch_bobjectives(const Dev &d, const double *x, const double *y, double *out, hipStream_t s);

// Homogeneous self-dual embedding (kernels_hsde.hip): per-handle data, built
// at the first HSDE call.  sc: [0] h^T g, [1] <c, g_x>_w, [2] ||b||,
// [3] ||c||_w, [4] ut (tau row of the last linear step), [5] tau - ut,
// [6] ||A(x) - tau b||^2, [7] ||A(x)||^2, [8] b^T y, [9] <c, x>_w,
// [10..12] the solved test's ratios of the last check.
struct HsdeDev {
    double *invE = nullptr, *s2E = nullptr;  // [ldU] 1 / E, 1 / (w E), E = 1 + D
    double *gx = nullptr;                     // [ldU] g_x (internal entry order)
    double *gy = nullptr;                     // [ldM] g_y
    double *a = nullptr;                      // [ldU] x rows of the linear step
    double *yh = nullptr;                     // [ldM] y rows of the linear step
    double *dx = nullptr;                     // [ldU] x(previous) - x
    double *sc = nullptr;                     // [16]
    double *hpart = nullptr;                  // [scatter_blocks * 2]
    double *dpart = nullptr;                  // [hsde_dot_blocks]
    double *hist = nullptr;                   // [3 * hist_cap] res_pri, res_dual, gap per iteration
    int32_t hist_cap = 0;
};
int hsde_dot_blocks(const Dev &d);
void launch_hsde_scales(const Dev &d, const HsdeDev &hs, hipStream_t s);
void launch_hsde_cu(const Dev &d, const HsdeDev &hs, hipStream_t s);
void launch_hsde_consts(const Dev &d, const HsdeDev &hs, hipStream_t s);
void launch_hsde_init(const Dev &d, double *x, double *y, float *sl, float *z, double *tk, hipStream_t s);
void launch_hsde_scatter(const Dev &d, const HsdeDev &hs, const float *sl, const float *z, const double *tk,
                         hipStream_t s);
void launch_hsde_check(const Dev &d, const HsdeDev &hs, const double *tk, hipStream_t s);
// the HSDE check in the first workgroup of the A u launch of its linear step
// (dh: the HSDE's Dev, d: the handle's; r2, r2scale as for its part 0), when
// check_in_au(d)
void launch_au_with_hsde_check(const Dev &dh, const Dev &d, const HsdeDev &hs, const double *tk, const double *r2,
                               double r2scale, const Ctl *ctl, hipStream_t s);
void launch_hsde_tau(const Dev &d, const HsdeDev &hs, double *y, double *tk, hipStream_t s);
void launch_hsde_axpy(const Dev &d, const HsdeDev &hs, hipStream_t s);
void launch_hsde_solution(const Dev &d, const HsdeDev &hs, int which, const double *x, const double *y,
                          const double *tk, double *X, double *Y, hipStream_t s);

// scatter / residual / affine kernels
int scatter_blocks(const Dev &d);
int scatter_light_blocks(const Dev &d);
// The Algorithm 1 and HSDE scatters give each thread of a light block
// kScatterEPT entries: their block counts (light, and light + heavy).
constexpr int kScatterEPT = 4;
int pscatter_blocks(const Dev &d);
int pscatter_light_blocks(const Dev &d);
int heavy_threshold();
int vupdate_blocks(const Dev &d);
void launch_reset_ctl(const Dev &d, int max_iter, double tol, hipStream_t s);
void launch_scatter_primal(const Dev &d, const float *blk, const float *lam, double rho, hipStream_t s);
void launch_check_primal(const Dev &d, double rho, hipStream_t s);
// true when Algorithm 1's residual check can run as the first workgroup of
// the A u launch (launch_au_with_check: part 0 of the affine step with the
// same r2, r2scale) instead of a launch of its own
bool check_in_au(const Dev &d);
void launch_au_with_check(const Dev &d, const double *r2, double r2scale, double rho, const Ctl *ctl,
                          hipStream_t s);
void launch_scatter_dual(const Dev &d, const float *blk, const float *lam, double rho, hipStream_t s);
void launch_vupdate(const Dev &d, const double *x, const float *blk, float *lam, float *v, double rho,
                    hipStream_t s);
void launch_check_dual(const Dev &d, double rho, hipStream_t s);
void launch_scale_u(const Dev &d, const double *r1, hipStream_t s);
void launch_affine(const Dev &d, const double *r2, double r2scale, double *x, double *y, const Ctl *ctl,
                   hipStream_t s);
// One part of the affine step: 0 split-K A u partials, 3 their reduction to t,
// 1 both triangular products, 2 gemv_ATy.
void launch_affine_part(const Dev &d, int part, const double *r2, double r2scale, double *x, double *y,
                        const Ctl *ctl, hipStream_t s);
// FP64 gather (entries -> packed slots) and scatter-add (packed -> entries).
void launch_gather_f64(const Dev &d, const double *x, double *packed, hipStream_t s);
void launch_perm_in(const Dev &d, const double *x_pattern, double *x_internal, hipStream_t s);
void launch_perm_out(const Dev &d, const double *x_internal, double *x_pattern, hipStream_t s);
void launch_scatter_f64(const Dev &d, const double *packed, double *out, hipStream_t s);
void launch_objectives(const Dev &d, const double *x, const double *y, hipStream_t s);
int objective_partials();
// Adjoint of one unrolled Algorithm-1 iteration (packed coordinates):
// gP = blkbar + rho lambar; hbar = gW - rho lambar, lambar -= gW / rho;
// d.u = s2 (sum_k H_k^T hbar + xbar) (hbar, xbar_pat nullable; xbar in pattern
// order); r1bar = w x kept in x, out_pat[perm] (+)= scale r1bar;
// blkbar = H_k r1bar, lambar += H_k r1bar / rho; out (+)= v.
void launch_adjoint_in(const Dev &d, const double *blkbar, const double *lambar, double rho, float *gP,
                       hipStream_t s);
void launch_adjoint_mid(const Dev &d, const float *gW, double *lambar, double rho, double *hbar, hipStream_t s);
void launch_adjoint_scatter(const Dev &d, const double *hbar, const double *xbar_pat, hipStream_t s);
void launch_adjoint_post(const Dev &d, double *x, double *out_pat, double scale, int accumulate, hipStream_t s);
void launch_adjoint_slots(const Dev &d, const double *r1bar, double *blkbar, double *lambar, double rho,
                          hipStream_t s);
void launch_add_to(const double *v, double *out, int n, int accumulate, hipStream_t s);

// api.cpp helpers for the entry points of other translation units.
cdcs_status set_error(cdcs_status st, const std::string &msg);   // message of cdcs_last_error
void handle_dims(const cdcs_handle *h, int64_t *ldU, int64_t *ldM);
cdcs_status affine_adjoint_into(cdcs_handle *h, const double *xbar, double *r1bar, double *r2bar, double *xs,
                                double *ys, hipStream_t stream);

// Chordal extension of a pattern and its maximal cliques (chordal.cpp, host).
struct ChordalExt {
    bool chordal_input = false;           // the pattern was chordal already (no fill)
    std::vector<int32_t> fill_i, fill_j;  // added lower-triangular entries, in clique order
    std::vector<int64_t> ptr;             // maximal cliques, CSR, vertices sorted
    std::vector<int32_t> vert;
};
cdcs_status chordal_extension(int32_t n, int64_t nnz, const int32_t *ei, const int32_t *ej, ChordalExt &out,
                              std::string &err);
// Elimination order of the graph adj (vertices with used[v]): the maximum
// cardinality search order when it is perfect (returns true: no fill), else
// minimum degree; later[v] = the neighbours of v eliminated after it in the
// filled graph (the structure of column v of the Cholesky factor).
bool elimination_order(int32_t n, const std::vector<std::vector<int32_t>> &adj, const std::vector<char> &used,
                       std::vector<int32_t> &order, std::vector<std::vector<int32_t>> &later);

// Sparse Cholesky factor of M (sparse A): structure from the host's symbolic
// step, values on the device (kernels_setup.hip).  All device arrays.
struct SpFactor {
    const int32_t *cp = nullptr;        // [m+1] column pointers of L (factor order)
    const int32_t *ri = nullptr;        // [nnzL] rows, increasing per column, diagonal first
    const int32_t *order = nullptr;     // [m] original row of factor index j
    const int32_t *pinv = nullptr;      // [m] factor index of original row r
    const int32_t *rk_ptr = nullptr;    // [m+1] per row j: the columns k < j with L_jk != 0
    const int32_t *rk_col = nullptr;    // [nnzL - m] k, increasing
    const int32_t *rk_pos = nullptr;    // [nnzL - m] position of row j within column k
    const int32_t *level_cols = nullptr;  // columns by elimination-tree level (leaves first)
    const int64_t *xp = nullptr;        // [m+1] column pointers of X = L^-1 (paths to the root)
    const int32_t *xr = nullptr;        // [nnzX] rows of X
    double *Lv = nullptr;               // [nnzL] values of L
    double *diag0 = nullptr;            // [m] diagonal of M (factor order)
    double *xv = nullptr;               // [nnzX] values of X
};
// shift: added to the diagonal of M (0 for A D^-1 A^T, 1 for the HSDE matrix I + A E^-1 A^T)
void launch_spchol_fill(const Dev &d, const SpFactor &f, const int32_t *tid, double shift, hipStream_t s);
void launch_spchol(const Dev &d, const SpFactor &f, const std::vector<int32_t> &level_off, int32_t *info,
                   hipStream_t s);
int spinv_max_path();
void launch_gather_vals(const double *in, const int64_t *idx, double *out, int64_t n, hipStream_t s);

// setup kernels (kernels_setup.hip)
void launch_syrk(const float *Aw, int64_t ld, const double *s2, int m, double *M, hipStream_t s);
// M (zeroed, m x m) = sum over coefficients of a sparse A; tid[q] = touched-entry index of sp_col[q]
void launch_sp_syrk(const Dev &d, const int32_t *tid, double *M, hipStream_t s);
void launch_potrf(double *M, int m, double *diag0, int32_t *info, hipStream_t s);
void launch_add_diag(double *M, int m, double shift, hipStream_t s);
void launch_trtri(const double *L, int m, double *LinvT, double *Linv, hipStream_t s);
void launch_inv_product(const double *LinvT, int m, double *Minv, hipStream_t s);
// Nonzeros of each row of a dense m x m triangle (lower: columns <= row,
// upper: columns >= row) -> cnt[m]; then the CSR copy given ptr[m+1].
void launch_tri_count(const double *T, int m, int upper, int32_t *cnt, hipStream_t s);
void launch_tri_compress(const double *T, int m, int upper, const int32_t *ptr, int32_t *col, double *val,
                         hipStream_t s);

}  // namespace cdcs
