// Setup of the affine projection ("Setup: ... KKT factorization" of
// Algorithms 1 and 2; Sec. III-B.1: the KKT matrix is constant, so its
// factorisation is computed once and cached).
//
//   M = A diag(w / D) A^T = Aw diag(s2) Aw^T     (Aw = w A, s2 = 1 / (w D)), FP64
//   M = L L^T                                    (blocked right-looking Cholesky)
//   L^-1 and L^-T                                (blocked, 64-row block rows)
//   M^-1 = L^-T L^-1                             (when L^-1 does not stay sparse)
//
// The solve y = M^-1 t of each iteration is then one matrix-vector product
// with the cached inverse (or two sparse triangular ones with the inverse
// factor), which spreads over the whole GPU instead of a length-m chain of
// dependent substitution steps.
#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int TS = 64;   // output tile of the SYRK kernels
constexpr int KC = 32;   // reduction chunk
constexpr int NB = 64;   // Cholesky panel width

__device__ __forceinline__ int tri_row_i(int64_t s) {
    int64_t a = (int64_t)((sqrt(8.0 * (double)s + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= s) ++a;
    while (a * (a + 1) / 2 > s) --a;
    return (int)a;
}

// M[i][j] (i >= j tiles) = sum_e Aw[i][e] * Aw[j][e] * s2[e].
__global__ __launch_bounds__(256) void k_syrk(const float *__restrict__ Aw, int64_t ld,
                                              const double *__restrict__ s2, int m, double *__restrict__ M) {
    __shared__ double As[TS][KC + 1];
    __shared__ double Bs[TS][KC + 1];
    const int tb = blockIdx.x;
    const int I = tri_row_i(tb), J = tb - I * (I + 1) / 2;
    const int i0 = I * TS, j0 = J * TS;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int64_t e0 = 0; e0 < ld; e0 += KC) {
        for (int idx = threadIdx.x; idx < TS * KC; idx += 256) {
            const int r = idx / KC, q = idx - r * KC;
            const int64_t e = e0 + q;
            const double sc = s2[e];
            const int ri = i0 + r, rj = j0 + r;
            As[r][q] = (ri < m) ? (double)Aw[(int64_t)ri * ld + e] * sc : 0.0;
            Bs[r][q] = (rj < m) ? (double)Aw[(int64_t)rj * ld + e] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < KC; ++q) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[ty * 4 + a][q];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[tx * 4 + b][q];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
            if (i < m && j < m) M[(int64_t)i * m + j] = acc[a][b];
        }
}

// Minv[i][j] = Minv[j][i] = sum_k LinvT[i][k] LinvT[j][k] over i >= j tiles,
// i.e. (L^-T L^-1)[i][j] = (L L^T)^-1[i][j].  L^-T is upper triangular, so the
// sum starts at the row tile's first column; both triangles are written, from
// the same sums, so Minv is exactly symmetric.
__global__ __launch_bounds__(256) void k_inv_product(const double *__restrict__ LinvT, int m,
                                                     double *__restrict__ Minv) {
    __shared__ double As[TS][KC + 1];
    __shared__ double Bs[TS][KC + 1];
    const int tb = blockIdx.x;
    const int I = tri_row_i(tb), J = tb - I * (I + 1) / 2;
    const int i0 = I * TS, j0 = J * TS;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int e0 = i0; e0 < m; e0 += KC) {
        for (int idx = threadIdx.x; idx < TS * KC; idx += 256) {
            const int r = idx / KC, q = idx - r * KC;
            const int e = e0 + q;
            const int ri = i0 + r, rj = j0 + r;
            As[r][q] = (ri < m && e < m) ? LinvT[(int64_t)ri * m + e] : 0.0;
            Bs[r][q] = (rj < m && e < m) ? LinvT[(int64_t)rj * m + e] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < KC; ++q) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[ty * 4 + a][q];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[tx * 4 + b][q];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
            if (i < m && j < m) {
                Minv[(int64_t)i * m + j] = acc[a][b];
                Minv[(int64_t)j * m + i] = acc[a][b];
            }
        }
}

__global__ void k_copy_diag(const double *__restrict__ M, int m, double *__restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) d[i] = M[(int64_t)i * m + i];
}

__global__ void k_add_diag(double *__restrict__ M, int m, double shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) M[(int64_t)i * m + i] += shift;
}

// Unblocked Cholesky of the diagonal block [kb, kb+nb)^2 (lower) in LDS.
// A pivot <= 2^-40 times the original diagonal flags rank deficiency
// (info[0] = 1, info[1] = row) and is replaced by 1 to keep the rest finite.
__global__ __launch_bounds__(256) void k_potrf_diag(double *__restrict__ M, int m, int kb, int nb,
                                                    const double *__restrict__ diag0, int32_t *info) {
    __shared__ double L[NB][NB + 1];
    for (int idx = threadIdx.x; idx < nb * nb; idx += 256) {
        const int i = idx / nb, j = idx - i * nb;
        L[i][j] = (j <= i) ? M[(int64_t)(kb + i) * m + kb + j] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (threadIdx.x == 0) {
            double piv = L[j][j];
            if (!(piv > ldexp(diag0[kb + j], -40))) {
                if (info[0] == 0) {
                    info[0] = 1;
                    info[1] = kb + j;
                }
                piv = 1.0;
            }
            L[j][j] = sqrt(piv);
        }
        __syncthreads();
        const double ljj = L[j][j];
        for (int i = j + 1 + threadIdx.x; i < nb; i += 256) L[i][j] /= ljj;
        __syncthreads();
        // trailing update of the block: L[i][l] -= L[i][j] L[l][j], j < l <= i
        const int rem = nb - j - 1;
        for (int idx = threadIdx.x; idx < rem * rem; idx += 256) {
            const int i = j + 1 + idx / rem, l = j + 1 + idx % rem;
            if (l <= i) L[i][l] -= L[i][j] * L[l][j];
        }
        __syncthreads();
    }
    for (int idx = threadIdx.x; idx < nb * nb; idx += 256) {
        const int i = idx / nb, j = idx - i * nb;
        if (j <= i) M[(int64_t)(kb + i) * m + kb + j] = L[i][j];
    }
}

// Panel below the diagonal block: rows r >= kb+nb solve X L11^T = A21.
// One thread per row; the row lives in LDS.
__global__ __launch_bounds__(64) void k_trsm_panel(double *__restrict__ M, int m, int kb, int nb) {
    __shared__ double L[NB][NB + 1];
    __shared__ double X[64][NB + 1];
    for (int idx = threadIdx.x; idx < nb * nb; idx += 64) {
        const int i = idx / nb, j = idx - i * nb;
        L[i][j] = M[(int64_t)(kb + i) * m + kb + j];
    }
    const int r0 = kb + nb + blockIdx.x * 64;
    for (int idx = threadIdx.x; idx < 64 * nb; idx += 64) {
        const int rr = idx / nb, j = idx - rr * nb;
        X[rr][j] = (r0 + rr < m) ? M[(int64_t)(r0 + rr) * m + kb + j] : 0.0;
    }
    __syncthreads();
    const int rr = threadIdx.x;
    if (r0 + rr < m) {
        for (int j = 0; j < nb; ++j) {
            double s = X[rr][j];
            for (int l = 0; l < j; ++l) s -= X[rr][l] * L[j][l];
            X[rr][j] = s / L[j][j];
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * nb; idx += 64) {
        const int q = idx / nb, j = idx - q * nb;
        if (r0 + q < m) M[(int64_t)(r0 + q) * m + kb + j] = X[q][j];
    }
}

// Trailing update M22 -= L21 L21^T on lower tiles of the trailing matrix.
__global__ __launch_bounds__(256) void k_syrk_update(double *__restrict__ M, int m, int kb, int nb) {
    __shared__ double As[TS][NB + 1];
    __shared__ double Bs[TS][NB + 1];
    const int t0 = kb + nb;
    const int tb = blockIdx.x;
    const int I = tri_row_i(tb), J = tb - I * (I + 1) / 2;
    const int i0 = t0 + I * TS, j0 = t0 + J * TS;
    for (int idx = threadIdx.x; idx < TS * nb; idx += 256) {
        const int r = idx / nb, q = idx - r * nb;
        As[r][q] = (i0 + r < m) ? M[(int64_t)(i0 + r) * m + kb + q] : 0.0;
        Bs[r][q] = (j0 + r < m) ? M[(int64_t)(j0 + r) * m + kb + q] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int q = 0; q < nb; ++q) {
        double av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = As[ty * 4 + a][q];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Bs[tx * 4 + b][q];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
            if (i < m && j <= i) M[(int64_t)i * m + j] -= acc[a][b];
        }
}

// Blocked triangular inverse X = L^-1, block row I at a time (64-row blocks):
//   X_IC = L_II^-1 (delta_IC I - sum_{C <= K < I} L_IK X_KC),  C <= I.
// One workgroup per column block C of the current block row; the sum is a
// 64 x 64 tile product over the already finished block rows, the L_II^-1
// application a forward substitution of 64 columns in parallel.
__global__ __launch_bounds__(256) void k_trtri_blockrow(const double *__restrict__ L, int m, int I,
                                                        double *__restrict__ X) {
    constexpr int B = 64, KC = 16;
    __shared__ double Ls[B][B + 1];  // L_II, later the right-hand sides
    __shared__ double As[B][KC + 1];
    __shared__ double Bs[KC][B + 1];
    const int C = blockIdx.x;
    const int r0 = I * B, c0 = C * B;
    const int nr = min(B, m - r0), nc = min(B, m - c0);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    // S = sum over K in [C, I) of L_IK X_KC (columns k0 = C*B .. r0-1)
    for (int k0 = c0; k0 < r0; k0 += KC) {
        for (int idx = threadIdx.x; idx < B * KC; idx += 256) {
            const int r = idx / KC, q = idx % KC;
            As[r][q] = (r < nr) ? L[(int64_t)(r0 + r) * m + k0 + q] : 0.0;
        }
        for (int idx = threadIdx.x; idx < KC * B; idx += 256) {
            const int q = idx / B, c = idx % B;
            Bs[q][c] = (c < nc) ? X[(int64_t)(k0 + q) * m + c0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < KC; ++q) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[ty * 4 + a][q];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[q][tx * 4 + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
        }
        __syncthreads();
    }
    // right-hand sides T = delta - S in Bs-sized scratch: reuse Ls after loading L_II below
    __shared__ double T[B][B + 1];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = ty * 4 + a, c = tx * 4 + b;
            T[r][c] = ((I == C && r == c) ? 1.0 : 0.0) - acc[a][b];
        }
    for (int idx = threadIdx.x; idx < B * B; idx += 256) {
        const int r = idx / B, c = idx % B;
        Ls[r][c] = (r < nr && c <= r) ? L[(int64_t)(r0 + r) * m + r0 + c] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    // forward substitution L_II Xcol = Tcol, one column per thread (64 columns)
    if (threadIdx.x < B) {
        const int c = threadIdx.x;
        for (int r = 0; r < nr; ++r) {
            double v = T[r][c];
            for (int q = 0; q < r; ++q) v -= Ls[r][q] * T[q][c];
            T[r][c] = v / Ls[r][r];
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < B * B; idx += 256) {
        const int r = idx / B, c = idx % B;
        if (r < nr && c < nc) X[(int64_t)(r0 + r) * m + c0 + c] = (I == C && c > r) ? 0.0 : T[r][c];
    }
}

// Sparse A: row i of M = sum over the coefficients (i, e) of row i and the
// coefficients (i', e) of the same entry e of Aw_ie Aw_i'e s2_e.  One thread
// owns row i (fixed summation order, no atomics).
__global__ __launch_bounds__(256) void k_sp_syrk(const int32_t *__restrict__ sp_ptr,
                                                 const int32_t *__restrict__ sp_col,
                                                 const double *__restrict__ sp_val,
                                                 const int32_t *__restrict__ tid,
                                                 const int32_t *__restrict__ tc_ptr,
                                                 const int32_t *__restrict__ tc_row,
                                                 const double *__restrict__ tc_val,
                                                 const double *__restrict__ s2, int m, double *__restrict__ M) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    double *row = M + (int64_t)i * m;
    for (int32_t q = sp_ptr[i]; q < sp_ptr[i + 1]; ++q) {
        const double a = sp_val[q] * s2[sp_col[q]];
        const int32_t t = tid[q];
        for (int32_t r = tc_ptr[t]; r < tc_ptr[t + 1]; ++r) row[tc_row[r]] += a * tc_val[r];
    }
}

// Nonzeros of row i of a triangle, one wave per row.
__global__ __launch_bounds__(256) void k_tri_count(const double *__restrict__ T, int m, int upper,
                                                   int32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const int lo = upper ? row : 0, hi = upper ? m : row + 1;
    int c = 0;
    for (int j = lo + lane; j < hi; j += 64) c += (T[(int64_t)row * m + j] != 0.0);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane == 0) cnt[row] = c;
}

// CSR copy of the triangle's nonzeros, columns increasing; one wave per row,
// 64 columns at a time compacted with a ballot.
__global__ __launch_bounds__(256) void k_tri_compress(const double *__restrict__ T, int m, int upper,
                                                      const int32_t *__restrict__ ptr, int32_t *__restrict__ col,
                                                      double *__restrict__ val) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const int lo = upper ? row : 0, hi = upper ? m : row + 1;
    int pos = ptr[row];
    for (int j0 = lo; j0 < hi; j0 += 64) {
        const int j = j0 + lane;
        const double v = (j < hi) ? T[(int64_t)row * m + j] : 0.0;
        const bool nz = v != 0.0;
        const unsigned long long mask = __ballot(nz);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (nz) {
            col[pos + before] = j;
            val[pos + before] = v;
        }
        pos += __popcll(mask);
    }
}

__global__ void k_transpose(const double *__restrict__ in, int m, double *__restrict__ out) {
    __shared__ double tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int i = by + r, j = bx + threadIdx.x;
        tile[r][threadIdx.x] = (i < m && j < m) ? in[(int64_t)i * m + j] : 0.0;
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += blockDim.y) {
        const int i = bx + r, j = by + threadIdx.x;
        if (i < m && j < m) out[(int64_t)i * m + j] = tile[threadIdx.x][r];
    }
}

}  // namespace

void launch_syrk(const float *Aw, int64_t ld, const double *s2, int m, double *M, hipStream_t s) {
    const int T = (m + TS - 1) / TS;
    hipLaunchKernelGGL(k_syrk, dim3(T * (T + 1) / 2), dim3(256), 0, s, Aw, ld, s2, m, M);
}

void launch_inv_product(const double *LinvT, int m, double *Minv, hipStream_t s) {
    const int T = (m + TS - 1) / TS;
    hipLaunchKernelGGL(k_inv_product, dim3(T * (T + 1) / 2), dim3(256), 0, s, LinvT, m, Minv);
}

void launch_add_diag(double *M, int m, double shift, hipStream_t s) {
    hipLaunchKernelGGL(k_add_diag, dim3((m + 255) / 256), dim3(256), 0, s, M, m, shift);
}

void launch_potrf(double *M, int m, double *diag0, int32_t *info, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_diag, dim3((m + 255) / 256), dim3(256), 0, s, (const double *)M, m, diag0);
    for (int kb = 0; kb < m; kb += NB) {
        const int nb = std::min(NB, m - kb);
        hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, M, m, kb, nb, (const double *)diag0, info);
        const int rem = m - kb - nb;
        if (rem > 0) {
            hipLaunchKernelGGL(k_trsm_panel, dim3((rem + 63) / 64), dim3(64), 0, s, M, m, kb, nb);
            const int T = (rem + TS - 1) / TS;
            hipLaunchKernelGGL(k_syrk_update, dim3(T * (T + 1) / 2), dim3(256), 0, s, M, m, kb, nb);
        }
    }
}

void launch_tri_count(const double *T, int m, int upper, int32_t *cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_count, dim3((m + 3) / 4), dim3(256), 0, s, T, m, upper, cnt);
}

void launch_tri_compress(const double *T, int m, int upper, const int32_t *ptr, int32_t *col, double *val,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_tri_compress, dim3((m + 3) / 4), dim3(256), 0, s, T, m, upper, ptr, col, val);
}

void launch_sp_syrk(const Dev &d, const int32_t *tid, double *M, hipStream_t s) {
    (void)hipMemsetAsync(M, 0, (size_t)d.m * d.m * sizeof(double), s);
    hipLaunchKernelGGL(k_sp_syrk, dim3((d.m + 255) / 256), dim3(256), 0, s, (const int32_t *)d.sp_ptr,
                       (const int32_t *)d.sp_col, (const double *)d.sp_val, tid, (const int32_t *)d.tc_ptr,
                       (const int32_t *)d.tc_row, (const double *)d.tc_val, (const double *)d.s2, d.m, M);
}

void launch_trtri(const double *L, int m, double *LinvT, double *Linv, hipStream_t s) {
    // Linv must be zero above the diagonal blocks: written block row by block row
    (void)hipMemsetAsync(Linv, 0, (size_t)m * m * sizeof(double), s);
    const int nb = (m + 63) / 64;
    for (int I = 0; I < nb; ++I)
        hipLaunchKernelGGL(k_trtri_blockrow, dim3(I + 1), dim3(256), 0, s, L, m, I, Linv);
    hipLaunchKernelGGL(k_transpose, dim3((m + 31) / 32, (m + 31) / 32), dim3(32, 8), 0, s, (const double *)Linv, m,
                       LinvT);
}

namespace {

// ---- Sparse factor of M = A D^-1 A^T (sparse A) ----------------------------
// The rows and columns of M are taken in an elimination order (a perfect one
// when M's graph is chordal, else minimum degree; host symbolic step): column
// j of the factor L holds the rows cp[j] .. cp[j+1] of ri[] (increasing, the
// diagonal first).  Numeric work on the device, deterministic order.

// Column j of L <- the entries of M in column j's structure (rows >= j of
// M's row order[j], in the factor's order): one thread per column, adding the
// products of the coefficients that share each pattern entry, as k_sp_syrk.
__global__ __launch_bounds__(256) void k_spchol_fill(const int32_t *__restrict__ cp, const int32_t *__restrict__ ri,
                                                     const int32_t *__restrict__ order,
                                                     const int32_t *__restrict__ pinv,
                                                     const int32_t *__restrict__ sp_ptr,
                                                     const int32_t *__restrict__ sp_col,
                                                     const double *__restrict__ sp_val,
                                                     const int32_t *__restrict__ tid,
                                                     const int32_t *__restrict__ tc_ptr,
                                                     const int32_t *__restrict__ tc_row,
                                                     const double *__restrict__ tc_val,
                                                     const double *__restrict__ s2, double shift, int m,
                                                     double *__restrict__ Lv, double *__restrict__ diag0) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const int32_t c0 = cp[j], c1 = cp[j + 1];
    for (int32_t p = c0; p < c1; ++p) Lv[p] = 0.0;
    const int32_t r = order[j];
    for (int32_t q = sp_ptr[r]; q < sp_ptr[r + 1]; ++q) {
        const double a = sp_val[q] * s2[sp_col[q]];
        const int32_t t = tid[q];
        for (int32_t u = tc_ptr[t]; u < tc_ptr[t + 1]; ++u) {
            const int32_t i = pinv[tc_row[u]];
            if (i < j) continue;
            int32_t lo = c0, hi = c1 - 1;  // i is in the column's structure
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (ri[mid] < i) lo = mid + 1;
                else hi = mid;
            }
            Lv[lo] += a * tc_val[u];
        }
    }
    Lv[c0] += shift;  // the diagonal leads the column
    diag0[j] = Lv[c0];
}

// Left-looking Cholesky of the columns of one elimination-tree level (their
// descendants are done): column j -= L_jk L(rows >= j, k) over the columns k
// with L_jk != 0 (rk lists: k increasing, with the position of row j in
// column k), then scaled by 1 / sqrt of its diagonal.  One workgroup per
// column; threads over the rows of column k.  A pivot <= 2^-40 times M_jj
// flags rank deficiency (info[0] = 1, info[1] = the original row) and is
// replaced by 1.
__global__ __launch_bounds__(256) void k_spchol_level(const int32_t *__restrict__ cols, const int32_t *__restrict__ cp,
                                                      const int32_t *__restrict__ ri,
                                                      const int32_t *__restrict__ rk_ptr,
                                                      const int32_t *__restrict__ rk_col,
                                                      const int32_t *__restrict__ rk_pos,
                                                      const int32_t *__restrict__ order,
                                                      const double *__restrict__ diag0, double *__restrict__ Lv,
                                                      int32_t *info) {
    __shared__ double s_ljj;
    const int j = cols[blockIdx.x];
    const int32_t c0 = cp[j], c1 = cp[j + 1];
    for (int32_t q = rk_ptr[j]; q < rk_ptr[j + 1]; ++q) {
        const int32_t k = rk_col[q];
        const int32_t k0 = cp[k] + rk_pos[q], k1 = cp[k + 1];
        const double ljk = Lv[k0];
        for (int32_t p = k0 + threadIdx.x; p < k1; p += 256) {
            const int32_t i = ri[p];
            int32_t lo = c0, hi = c1 - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (ri[mid] < i) lo = mid + 1;
                else hi = mid;
            }
            Lv[lo] -= Lv[p] * ljk;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double piv = Lv[c0];
        if (!(piv > ldexp(diag0[j], -40))) {
            if (atomicCAS(&info[0], 0, 1) == 0) info[1] = order[j];
            piv = 1.0;
        }
        s_ljj = sqrt(piv);
        Lv[c0] = s_ljj;
    }
    __syncthreads();
    const double inv = 1.0 / s_ljj;
    for (int32_t p = c0 + 1 + threadIdx.x; p < c1; p += 256) Lv[p] *= inv;
}

// Column j of X = L^-1: nonzero on the elimination-tree path from j to its
// root (xr[xp[j] .. xp[j+1]), increasing); X_jj = 1 / L_jj and, along the
// path, X_ij = -(sum over path rows k < i with L_ik != 0 of L_ik X_kj) / L_ii.
// One wave per column; the path and its values in LDS (at most 256).
constexpr int kMaxPath = 256;
__global__ __launch_bounds__(64) void k_spinv_col(const int32_t *__restrict__ cp, const int32_t *__restrict__ ri,
                                                  const int32_t *__restrict__ rk_ptr,
                                                  const int32_t *__restrict__ rk_col,
                                                  const int32_t *__restrict__ rk_pos,
                                                  const double *__restrict__ Lv, const int64_t *__restrict__ xp,
                                                  const int32_t *__restrict__ xr, double *__restrict__ xv, int m) {
    __shared__ int32_t path[kMaxPath];
    __shared__ double val[kMaxPath];
    const int j = blockIdx.x;
    if (j >= m) return;
    const int lane = threadIdx.x;
    const int64_t p0 = xp[j];
    const int P = (int)(xp[j + 1] - p0);
    for (int t = lane; t < P; t += 64) path[t] = xr[p0 + t];
    if (lane == 0) val[0] = 1.0 / Lv[cp[j]];
    __syncthreads();
    for (int t = 1; t < P; ++t) {
        const int i = path[t];
        double acc = 0.0;
        for (int32_t q = rk_ptr[i] + lane; q < rk_ptr[i + 1]; q += 64) {
            const int32_t k = rk_col[q];
            if (k < j) continue;
            int lo = 0, hi = t - 1;  // is k on the path below i?
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (path[mid] < k) lo = mid + 1;
                else hi = mid;
            }
            if (path[lo] == k) acc += Lv[cp[k] + rk_pos[q]] * val[lo];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) val[t] = -acc / Lv[cp[i]];
        __syncthreads();
    }
    for (int t = lane; t < P; t += 64) xv[p0 + t] = val[t];
}

// out[q] = in[idx[q]] (value layouts of the CSR copies)
__global__ __launch_bounds__(256) void k_gather_vals(const double *__restrict__ in, const int64_t *__restrict__ idx,
                                                     double *__restrict__ out, int64_t n) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < n) out[q] = in[idx[q]];
}

}  // namespace

void launch_spchol_fill(const Dev &d, const SpFactor &f, const int32_t *tid, double shift, hipStream_t s) {
    hipLaunchKernelGGL(k_spchol_fill, dim3((d.m + 255) / 256), dim3(256), 0, s, f.cp, f.ri, f.order, f.pinv,
                       (const int32_t *)d.sp_ptr, (const int32_t *)d.sp_col, (const double *)d.sp_val, tid,
                       (const int32_t *)d.tc_ptr, (const int32_t *)d.tc_row, (const double *)d.tc_val,
                       (const double *)d.s2, shift, d.m, f.Lv, f.diag0);
}

void launch_spchol(const Dev &d, const SpFactor &f, const std::vector<int32_t> &level_off, int32_t *info,
                   hipStream_t s) {
    for (size_t l = 0; l + 1 < level_off.size(); ++l) {
        const int ncol = level_off[l + 1] - level_off[l];
        if (ncol > 0)
            hipLaunchKernelGGL(k_spchol_level, dim3(ncol), dim3(256), 0, s, f.level_cols + level_off[l], f.cp, f.ri,
                               f.rk_ptr, f.rk_col, f.rk_pos, f.order, (const double *)f.diag0, f.Lv, info);
    }
    hipLaunchKernelGGL(k_spinv_col, dim3(d.m), dim3(64), 0, s, f.cp, f.ri, f.rk_ptr, f.rk_col, f.rk_pos,
                       (const double *)f.Lv, f.xp, f.xr, f.xv, d.m);
}

int spinv_max_path() { return kMaxPath; }

void launch_gather_vals(const double *in, const int64_t *idx, double *out, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, idx, out, n);
}

}  // namespace cdcs
