/*
 * CPU FP64 oracle for chordally decomposed ADMM -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU library.
 *
 * Contents (plain, slow, obviously correct; no BLAS/LAPACK):
 *   - cyclic-by-row Jacobi eigensolver for a symmetric matrix
 *     (Golub & Van Loan, "Matrix Computations", Sec. 8.5: the 2x2 symmetric
 *     Schur decomposition followed by J^T A J over all (p, q), p < q, in row
 *     order), used for the projection onto the PSD cone P_k of
 *     equations (E:XkUpdate) / (E:zkUpdate) of the paper:
 *         P(W) = Q max(Lambda, 0) Q^T,   W = Q Lambda Q^T;
 *   - dense Cholesky factorisation M = L L^T (Golub & Van Loan, Sec. 4.2),
 *     the "KKT factorization" cached in the Setup step of Algorithms 1 and 2;
 *   - forward and backward substitution with L and L^T (block elimination of
 *     the KKT systems (E:OptCondMinYPrimal) and (E:OptCondMinYDual)).
 *
 * All matrices are dense, row-major, double precision.
 * Threads (OpenMP): the batch entry points project independent cliques
 * concurrently and the Cholesky factorisation computes the rows below each
 * pivot concurrently; every output element is still computed by one thread
 * in the sequential order, so the results do not depend on the thread count.
 * Status codes: 0 ok, 1 bad argument, 3 non-positive pivot (rank),
 *               7 sweep cap reached without convergence.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG 1
#define OR_E_RANK 3
#define OR_E_NUMERIC 7

/* Frobenius norm of the strictly off-diagonal part and of the whole matrix. */
static void off_and_fro(int k, const double *A, double *off, double *fro)
{
    double so = 0.0, sf = 0.0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double v = A[(size_t)i * k + j];
            sf += v * v;
            if (i != j) so += v * v;
        }
    *off = sqrt(so);
    *fro = sqrt(sf);
}

/*
 * Symmetric eigendecomposition A = V diag(evals) V^T by cyclic-by-row Jacobi.
 * Rotation for the pair (p, q): tau = (a_qq - a_pp) / (2 a_pq),
 * t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1/sqrt(1 + t^2), s = t c,
 * J = identity except J_pp = J_qq = c, J_pq = s, J_qp = -s; A <- J^T A J,
 * V <- V J.  Stops when off(A) <= tol * ||A||_F (tol = 4 k 2^-52), at most
 * max_sweeps sweeps.  A_in is not modified.  V is k x k row-major with the
 * eigenvectors in its columns.  Returns a status; *sweeps_out gets the count.
 */
int oracle_jacobi_eigh(int k, const double *A_in, double *evals, double *V,
                       int max_sweeps, int *sweeps_out)
{
    if (k < 0 || (k > 0 && (!A_in || !evals || !V))) return OR_E_ARG;
    double *A = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k * k : 1));
    if (!A) return OR_E_ARG;
    memcpy(A, A_in, sizeof(double) * (size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) V[(size_t)i * k + j] = (i == j) ? 1.0 : 0.0;

    const double tol = 4.0 * (double)k * ldexp(1.0, -52);
    int sweeps = 0, status = OR_E_NUMERIC;
    for (;;) {
        double off, fro;
        off_and_fro(k, A, &off, &fro);
        if (off <= tol * fro) { status = OR_OK; break; }
        if (sweeps >= max_sweeps) break;
        ++sweeps;
        for (int p = 0; p < k - 1; ++p) {
            for (int q = p + 1; q < k; ++q) {
                double apq = A[(size_t)p * k + q];
                if (apq == 0.0) continue;
                double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* columns p, q of A: A <- A J */
                for (int i = 0; i < k; ++i) {
                    double aip = A[(size_t)i * k + p], aiq = A[(size_t)i * k + q];
                    A[(size_t)i * k + p] = c * aip - s * aiq;
                    A[(size_t)i * k + q] = s * aip + c * aiq;
                }
                /* rows p, q of A: A <- J^T A */
                for (int j = 0; j < k; ++j) {
                    double apj = A[(size_t)p * k + j], aqj = A[(size_t)q * k + j];
                    A[(size_t)p * k + j] = c * apj - s * aqj;
                    A[(size_t)q * k + j] = s * apj + c * aqj;
                }
                /* V <- V J */
                for (int i = 0; i < k; ++i) {
                    double vip = V[(size_t)i * k + p], viq = V[(size_t)i * k + q];
                    V[(size_t)i * k + p] = c * vip - s * viq;
                    V[(size_t)i * k + q] = s * vip + c * viq;
                }
            }
        }
    }
    for (int i = 0; i < k; ++i) evals[i] = A[(size_t)i * k + i];
    free(A);
    if (sweeps_out) *sweeps_out = sweeps;
    return status;
}

/*
 * Projection onto the PSD cone: P = V max(Lambda, 0) V^T, then symmetrised
 * as (P + P^T)/2.  Optionally returns the eigenpairs (evals, V may be NULL).
 */
int oracle_psd_project(int k, const double *W, double *P, double *evals_out, double *V_out)
{
    if (k < 0) return OR_E_ARG;
    if (k == 0) return OR_OK;
    double *ev = (double *)malloc(sizeof(double) * (size_t)k);
    double *V = (double *)malloc(sizeof(double) * (size_t)k * k);
    if (!ev || !V) { free(ev); free(V); return OR_E_ARG; }
    int sw = 0;
    int st = oracle_jacobi_eigh(k, W, ev, V, 100, &sw);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double acc = 0.0;
            for (int t = 0; t < k; ++t)
                if (ev[t] > 0.0) acc += V[(size_t)i * k + t] * ev[t] * V[(size_t)j * k + t];
            P[(size_t)i * k + j] = acc;
        }
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) {
            double a = 0.5 * (P[(size_t)i * k + j] + P[(size_t)j * k + i]);
            P[(size_t)i * k + j] = a;
            P[(size_t)j * k + i] = a;
        }
    if (evals_out) memcpy(evals_out, ev, sizeof(double) * (size_t)k);
    if (V_out) memcpy(V_out, V, sizeof(double) * (size_t)k * k);
    free(ev);
    free(V);
    return st;
}

/*
 * Batch of independent projections (one per clique).  W and P hold the full
 * k_t x k_t row-major matrices back to back; offsets[t] is the start of
 * matrix t.  status[t] receives each projection's status; the return value is
 * the first non-zero status (or 0).
 */
int oracle_psd_project_batch(int nb, const int64_t *sizes, const int64_t *offsets,
                             const double *W, double *P, int *status)
{
    int first = OR_OK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < nb; ++t) {
        int st = oracle_psd_project((int)sizes[t], W + offsets[t], P + offsets[t], NULL, NULL);
        if (status) status[t] = st;
        if (st != OR_OK) {
            #pragma omp critical
            if (first == OR_OK) first = st;
        }
    }
    return first;
}

/* Same batch, also returning eigenvalues (concatenated, sum k_t) and
 * eigenvectors (full k_t x k_t each, at offsets[t]). */
int oracle_psd_project_batch_eig(int nb, const int64_t *sizes, const int64_t *offsets,
                                 const int64_t *eoffsets, const double *W, double *P,
                                 double *evals, double *V)
{
    int first = OR_OK;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < nb; ++t) {
        int st = oracle_psd_project((int)sizes[t], W + offsets[t], P + offsets[t],
                                    evals + eoffsets[t], V + offsets[t]);
        if (st != OR_OK) {
            #pragma omp critical
            if (first == OR_OK) first = st;
        }
    }
    return first;
}

/*
 * Cholesky factorisation M = L L^T of a symmetric positive definite m x m
 * matrix (lower triangle of M read).  L is written row-major with zeros above
 * the diagonal.  A pivot s_j <= 2^-40 M_jj (the Schur complement has lost all
 * but rounding noise of the diagonal) means M is numerically singular, i.e. A
 * does not have full row rank: returns OR_E_RANK.
 */
int oracle_cholesky(int m, const double *M, double *L)
{
    if (m < 0 || (m > 0 && (!M || !L))) return OR_E_ARG;
    memset(L, 0, sizeof(double) * (size_t)m * m);
    for (int j = 0; j < m; ++j) {
        double s = M[(size_t)j * m + j];
        const double *Lj = L + (size_t)j * m;
        for (int k = 0; k < j; ++k) s -= Lj[k] * Lj[k];
        if (!(s > ldexp(M[(size_t)j * m + j], -40))) return OR_E_RANK;
        double ljj = sqrt(s);
        L[(size_t)j * m + j] = ljj;
        #pragma omp parallel for schedule(static)
        for (int i = j + 1; i < m; ++i) {
            const double *Li = L + (size_t)i * m;
            double t = M[(size_t)i * m + j];
            for (int k = 0; k < j; ++k) t -= Li[k] * Lj[k];
            L[(size_t)i * m + j] = t / ljj;
        }
    }
    return OR_OK;
}

/* Solve (L L^T) y = t by forward substitution L z = t then back substitution
 * L^T y = z.  t and y may alias. */
int oracle_chol_solve(int m, const double *L, const double *t, double *y)
{
    if (m < 0) return OR_E_ARG;
    double *z = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    if (!z) return OR_E_ARG;
    for (int i = 0; i < m; ++i) {
        double s = t[i];
        const double *Li = L + (size_t)i * m;
        for (int k = 0; k < i; ++k) s -= Li[k] * z[k];
        z[i] = s / Li[i];
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < m; ++k) s -= L[(size_t)k * m + i] * y[k];
        y[i] = s / L[(size_t)i * m + i];
    }
    free(z);
    return OR_OK;
}
