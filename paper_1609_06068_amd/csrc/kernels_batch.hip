// Many independent SDPs in one handle.  The instances' pattern entries,
// cliques, packed slots and constraint rows are concatenated; the projection
// runs over every instance's cliques in one launch (kernels_project.hip).  The
// affine step is block diagonal: each constraint row and each factor belongs to
// one instance.  Every instance has its own residuals and stop flag: once
// max(eps_p, eps_d) <= tol for instance q, all kernels skip q's work, so q's
// state stays at the iterate that met the tolerance, and a device wall-clock
// stamp records when that happened.
#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kNT = 256;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum_d(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum_d(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < kNT / 64; ++i) r += red[i];
    return r;
}

__global__ void k_breset(int32_t *istop, int32_t *iiters, uint64_t *itime, int32_t *nrunning, int nprob,
                         uint64_t *t0) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nprob) {
        istop[q] = 0;
        iiters[q] = 0;
        itime[q] = 0;
    }
    if (q == 0) {
        *nrunning = nprob;
        *t0 = wall_clock64();
    }
}

// Alg. 1 right-hand side per scatter block (q, e0, e1): entries of one
// instance; per-block partial sums of the dual-residual terms.
__global__ __launch_bounds__(kNT) void k_bscatter_primal(const int4 *__restrict__ sblk,
                                                         const int32_t *__restrict__ istop,
                                                         const int32_t *__restrict__ inv_ptr,
                                                         const int32_t *__restrict__ inv_slot,
                                                         const float *__restrict__ blk, const float *__restrict__ lam,
                                                         const float *__restrict__ dslot,
                                                         const double *__restrict__ c,
                                                         const uint32_t *__restrict__ wbits, double *__restrict__ u,
                                                         double *__restrict__ spart, double rho, const Ctl *ctl) {
    __shared__ double red[kNT / 64];
    if (ctl->stop) return;
    const int4 bk = sblk[blockIdx.x];
    if (istop[bk.x]) return;
    const int64_t e = (int64_t)bk.y + threadIdx.x;
    double ds2 = 0.0, sl2 = 0.0;
    if (e < bk.z) {
        double s_x = 0.0, s_l = 0.0, s_d = 0.0;
        const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
        for (int32_t q = q0; q < q1; ++q) {
            const int32_t sl = inv_slot[q];
            s_x += (double)blk[sl];
            s_l += (double)lam[sl];
            s_d += (double)dslot[sl];
        }
        u[e] = (s_x + s_l / rho - c[e] / rho) / (double)(q1 - q0);
        const double w = ((wbits[e >> 5] >> (e & 31)) & 1u) ? 2.0 : 1.0;
        ds2 = w * s_d * s_d;
        sl2 = w * s_l * s_l;
    }
    ds2 = block_sum_d(ds2, red);
    sl2 = block_sum_d(sl2, red);
    if (threadIdx.x == 0) {
        spart[2 * (int64_t)blockIdx.x + 0] = ds2;
        spart[2 * (int64_t)blockIdx.x + 1] = sl2;
    }
}

// Alg. 2 right-hand side per scatter block: u = (c - sum_k H_k^T (z_k + lam_k / rho)) / D.
__global__ __launch_bounds__(kNT) void k_bscatter_dual(const int4 *__restrict__ sblk,
                                                       const int32_t *__restrict__ istop,
                                                       const int32_t *__restrict__ inv_ptr,
                                                       const int32_t *__restrict__ inv_slot,
                                                       const float *__restrict__ blk, const float *__restrict__ lam,
                                                       const double *__restrict__ c,
                                                       double *__restrict__ u, double rho, const Ctl *ctl) {
    if (ctl->stop) return;
    const int4 bk = sblk[blockIdx.x];
    if (istop[bk.x]) return;
    const int64_t e = (int64_t)bk.y + threadIdx.x;
    if (e >= bk.z) return;
    double acc = 0.0;
    const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
    for (int32_t q = q0; q < q1; ++q) {
        const int32_t sl = inv_slot[q];
        acc += (double)blk[sl] + (double)lam[sl] / rho;
    }
    u[e] = (c[e] - acc) / (double)(q1 - q0);
}

// Alg. 2 epilogue per slot block (q, s0, s1) of one instance: v_k = z_k +
// lam_k / rho + H_k x (E:vkEqn), lam_k += rho (z_k - v_k) (E:MultUpdateDualSDP),
// and the block's residual partial sums.
__global__ __launch_bounds__(kNT) void k_bvupdate(const int4 *__restrict__ vblk, const int32_t *__restrict__ istop,
                                                  const int32_t *__restrict__ gather, const double *__restrict__ x,
                                                  const double *__restrict__ wt, const float *__restrict__ blk,
                                                  float *__restrict__ lam, float *__restrict__ v,
                                                  double *__restrict__ vpart, double rho, const Ctl *ctl) {
    __shared__ double red[kNT / 64];
    if (ctl->stop) return;
    const int4 bk = vblk[blockIdx.x];
    if (istop[bk.x]) return;
    const int64_t s = (int64_t)bk.y + threadIdx.x;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0, q4 = 0.0;
    if (s < bk.z) {
        const int32_t e = gather[s];
        const double hx = x[e];
        const double z = blk[s], l = lam[s], vo = v[s];
        const double vn = z + l / rho + hx;
        const double ln = l + rho * (z - vn);
        v[s] = (float)vn;
        lam[s] = (float)ln;
        const double w = wt[e];
        q0 = w * (z - vn) * (z - vn);
        q1 = w * z * z;
        q2 = w * vn * vn;
        q3 = w * (vn - vo) * (vn - vo);
        q4 = w * ln * ln;
    }
    q0 = block_sum_d(q0, red);
    q1 = block_sum_d(q1, red);
    q2 = block_sum_d(q2, red);
    q3 = block_sum_d(q3, red);
    q4 = block_sum_d(q4, red);
    if (threadIdx.x == 0) {
        double *o = vpart + 5 * (int64_t)blockIdx.x;
        o[0] = q0;
        o[1] = q1;
        o[2] = q2;
        o[3] = q3;
        o[4] = q4;
    }
}

// Alg. 2 per-instance residual check of the iteration just completed
// (n = ctl->iter + 1): one wave per instance over its slot blocks.
__global__ __launch_bounds__(kNT) void k_bcheck_dual(const double *__restrict__ vpart,
                                                     const int32_t *__restrict__ vblk_off, int nprob, double rho,
                                                     int32_t *__restrict__ istop, int32_t *__restrict__ iiters,
                                                     uint64_t *__restrict__ itime, double *__restrict__ ieps,
                                                     int32_t *nrunning, const Ctl *ctl) {
    if (ctl->stop) return;
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
    if (q >= nprob || istop[q]) return;
    const int n = ctl->iter + 1;
    double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = vblk_off[q] + lane; b < vblk_off[q + 1]; b += 64)
#pragma unroll
        for (int i = 0; i < 5; ++i) r[i] += vpart[5 * (int64_t)b + i];
#pragma unroll
    for (int i = 0; i < 5; ++i) r[i] = wave_sum_d(r[i]);
    if (lane != 0) return;
    const double den_p = fmax(sqrt(r[1]), sqrt(r[2]));
    const double eps_p = den_p > 0.0 ? sqrt(r[0]) / den_p : sqrt(r[0]);
    const double den_d = sqrt(r[4]);
    const double eps_d = den_d > 0.0 ? rho * sqrt(r[3]) / den_d : rho * sqrt(r[3]);
    ieps[2 * q + 0] = eps_p;
    ieps[2 * q + 1] = eps_d;
    const bool finite = isfinite(eps_p) && isfinite(eps_d);  // NaN or Inf in the instance's iterate: 3
    int st = 0;
    if (!finite) st = 3;
    else if (fmax(eps_p, eps_d) <= ctl->tol) st = 1;
    else if (n >= ctl->max_iter) st = 2;
    if (st) {
        istop[q] = st;
        iiters[q] = n;
        itime[q] = wall_clock64();
        atomicSub(nrunning, 1);
    }
}

// Global bookkeeping after the per-instance Alg. 2 checks.
__global__ void k_bcheck_dual_finish(const int32_t *nrunning, Ctl *ctl) {
    if (threadIdx.x != 0 || ctl->stop) return;
    ctl->iter = ctl->iter + 1;
    if (*nrunning <= 0) ctl->stop = 1;
}

// Per-instance residual check of iteration n = ctl->iter: one wave per instance.
__global__ __launch_bounds__(kNT) void k_bcheck_primal(const double *__restrict__ cpart,
                                                       const int32_t *__restrict__ k_off,
                                                       const double *__restrict__ spart,
                                                       const int32_t *__restrict__ sblk_off, int nprob, double rho,
                                                       int32_t *__restrict__ istop, int32_t *__restrict__ iiters,
                                                       uint64_t *__restrict__ itime, double *__restrict__ ieps,
                                                       int32_t *nrunning, const Ctl *ctl) {
    if (ctl->stop) return;
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
    if (q >= nprob || istop[q]) return;
    const int n = ctl->iter;
    if (n >= 1) {
        double r2 = 0.0, h2 = 0.0, x2 = 0.0, d2 = 0.0, l2 = 0.0;
#pragma unroll 4
        for (int k = k_off[q] + lane; k < k_off[q + 1]; k += 64) {
            r2 += cpart[4 * (int64_t)k + 0];
            h2 += cpart[4 * (int64_t)k + 1];
            x2 += cpart[4 * (int64_t)k + 2];
        }
#pragma unroll 4
        for (int b = sblk_off[q] + lane; b < sblk_off[q + 1]; b += 64) {
            d2 += spart[2 * (int64_t)b + 0];
            l2 += spart[2 * (int64_t)b + 1];
        }
        r2 = wave_sum_d(r2);
        h2 = wave_sum_d(h2);
        x2 = wave_sum_d(x2);
        d2 = wave_sum_d(d2);
        l2 = wave_sum_d(l2);
        if (lane == 0) {
            const double den_p = fmax(sqrt(h2), sqrt(x2));
            const double eps_p = den_p > 0.0 ? sqrt(r2) / den_p : sqrt(r2);
            const double den_d = sqrt(l2);
            const double eps_d = den_d > 0.0 ? rho * sqrt(d2) / den_d : rho * sqrt(d2);
            ieps[2 * q + 0] = eps_p;
            ieps[2 * q + 1] = eps_d;
            const bool finite = isfinite(eps_p) && isfinite(eps_d);  // NaN or Inf in the instance's iterate: 3
            if (!finite || fmax(eps_p, eps_d) <= ctl->tol) {
                istop[q] = finite ? 1 : 3;
                iiters[q] = n;
                itime[q] = wall_clock64();
                atomicSub(nrunning, 1);
                return;
            }
        }
    }
    if (lane == 0 && n >= ctl->max_iter) {
        istop[q] = 2;
        iiters[q] = n;
        itime[q] = wall_clock64();
        atomicSub(nrunning, 1);
    }
}

// Global bookkeeping after the per-instance checks.
__global__ void k_bcheck_finish(const int32_t *nrunning, Ctl *ctl) {
    if (threadIdx.x != 0 || ctl->stop) return;
    if (*nrunning <= 0) ctl->stop = 1;
    else ctl->iter = ctl->iter + 1;
}

// t = A_q (w u_q) - r2scale r2 for up to 8 consecutive rows of one instance
// and one column chunk of kBatchAuChunk entries per wave (job (q, first row,
// rows, chunk)): each u element loaded once serves all the wave's rows.  Lanes
// stride the chunk in float4 groups; FP64 accumulation.  An instance whose
// rows span several chunks writes per-chunk partial sums, which
// k_bAu_reduce adds in chunk order (deterministic).  A job with rows = 0 is an
// unused slot of the per-XCD job layout.
constexpr int kRowsPerWave = 8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMaxBatchRows = 256;  // constraints per instance (checked at setup)
static_assert(kBatchAuChunk % 256 == 0, "chunks hold whole float4 groups of a wave");

__global__ __launch_bounds__(kNT) void k_bgemv_Au(const float *__restrict__ A, const int64_t *__restrict__ A_off,
                                                  const int32_t *__restrict__ A_ld, const int4 *__restrict__ rjobs,
                                                  int njobs, const int32_t *__restrict__ m_off,
                                                  const int64_t *__restrict__ U_off, const int32_t *__restrict__ nch,
                                                  const int64_t *__restrict__ p_off, double *__restrict__ tpart,
                                                  const int32_t *__restrict__ istop, const double *__restrict__ u,
                                                  const double *__restrict__ r2, double r2scale,
                                                  double *__restrict__ t, const Ctl *ctl) {
    if (ctl != nullptr && ctl->stop) return;
    const int lane = threadIdx.x & 63;
    const int jb = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
    if (jb >= njobs) return;
    const int4 job = rjobs[jb];  // (q, first row (global), rows, chunk)
    const int q = job.x, r0 = job.y, nr = job.z, ch = job.w;
    if (nr == 0 || (istop != nullptr && istop[q])) return;
    const int64_t u0 = U_off[q];
    const int nU = (int)(U_off[q + 1] - u0);
    const int ld = A_ld[q];
    const float *base = A + A_off[q] + (int64_t)(r0 - m_off[q]) * ld;
    const double *uq = u + u0;
    const int jhi = min(nU, (ch + 1) * kBatchAuChunk);
    double acc[kRowsPerWave];
#pragma unroll
    for (int v = 0; v < kRowsPerWave; ++v) acc[v] = 0.0;
    for (int j = ch * kBatchAuChunk + lane * 4; j < jhi; j += 256) {
        double uj[4];  // (u_q may start at an odd entry: scalar loads)
#pragma unroll
        for (int v = 0; v < 4; ++v) uj[v] = (j + v < nU) ? uq[j + v] : 0.0;
#pragma unroll
        for (int v = 0; v < kRowsPerWave; ++v) {
            if (v < nr) {
                // A is streamed once per product: non-temporal loads keep u in the caches
                const f32x4 a = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(base + (int64_t)v * ld + j));
                acc[v] += (double)a.x * uj[0] + (double)a.y * uj[1] + (double)a.z * uj[2] + (double)a.w * uj[3];
            }
        }
    }
    const int nc = nch[q];
#pragma unroll
    for (int v = 0; v < kRowsPerWave; ++v) {
        const double sv = wave_sum_d(acc[v]);
        if (lane == 0 && v < nr) {
            if (nc == 1) t[r0 + v] = sv - r2scale * r2[r0 + v];
            else tpart[p_off[q] + (int64_t)(r0 + v - m_off[q]) * nc + ch] = sv;
        }
    }
}

// t_r = sum of row r's chunk partial sums (in chunk order) - r2scale r2_r, for
// the rows of instances split into several chunks.
__global__ __launch_bounds__(kNT) void k_bAu_reduce(const int32_t *__restrict__ rinst,
                                                    const int32_t *__restrict__ m_off,
                                                    const int32_t *__restrict__ nch,
                                                    const int64_t *__restrict__ p_off,
                                                    const double *__restrict__ tpart,
                                                    const int32_t *__restrict__ istop, const double *__restrict__ r2,
                                                    double r2scale, double *__restrict__ t, int mtot, const Ctl *ctl) {
    if (ctl != nullptr && ctl->stop) return;
    const int r = blockIdx.x * kNT + threadIdx.x;
    if (r >= mtot) return;
    const int q = rinst[r];
    const int nc = nch[q];
    if (nc == 1 || (istop != nullptr && istop[q])) return;
    const double *pr = tpart + p_off[q] + (int64_t)(r - m_off[q]) * nc;
    double sacc = 0.0;
#pragma unroll 8
    for (int c = 0; c < nc; ++c) sacc += pr[c];
    t[r] = sacc - r2scale * r2[r];
}

// One triangular product per instance: out_q = T_q in_q, T_q lower (upper = 0)
// or upper (upper = 1), m_q x m_q row-major at F_off[q].  One wave per row.
__global__ __launch_bounds__(kNT) void k_btrmv(const double *__restrict__ T, const int64_t *__restrict__ F_off,
                                               const int32_t *__restrict__ rinst, const int32_t *__restrict__ m_off,
                                               const int32_t *__restrict__ istop, int upper,
                                               const double *__restrict__ vin, double *__restrict__ vout, int mtot,
                                               const Ctl *ctl) {
    if (ctl != nullptr && ctl->stop) return;
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
    if (r >= mtot) return;
    const int q = rinst[r];
    if (istop != nullptr && istop[q]) return;
    const int m0 = m_off[q], mq = m_off[q + 1] - m0, i = r - m0;
    const double *tr = T + F_off[q] + (int64_t)i * mq;
    const double *v = vin + m0;
    const int lo = upper ? i : 0, hi = upper ? mq : i + 1;
    double acc = 0.0;
    for (int j = lo + lane; j < hi; j += 64) acc += tr[j] * v[j];
    acc = wave_sum_d(acc);
    if (lane == 0) vout[r] = acc;
}

// x_e = u_e - s2_e (A_q^T y_q)_e: a workgroup takes 1024 consecutive entries
// of one instance (job (q, first entry within the instance)), each thread 4
// of them with float4 loads down the instance's m_q rows (coalesced across
// the workgroup's threads).
__global__ __launch_bounds__(kNT) void k_bgemv_ATy(const float *__restrict__ A, const int64_t *__restrict__ A_off,
                                                   const int32_t *__restrict__ A_ld, const int2 *__restrict__ ejobs,
                                                   const int32_t *__restrict__ m_off,
                                                   const int64_t *__restrict__ U_off,
                                                   const int32_t *__restrict__ istop, const double *__restrict__ y,
                                                   const double *__restrict__ u, const double *__restrict__ s2,
                                                   double *__restrict__ x, const Ctl *ctl) {
    __shared__ double ys[kMaxBatchRows];
    if (ctl != nullptr && ctl->stop) return;
    const int2 job = ejobs[blockIdx.x];
    const int q = job.x;
    if (istop != nullptr && istop[q]) return;
    const int64_t u0 = U_off[q];
    const int nU = (int)(U_off[q + 1] - u0);
    {
        const int m0 = m_off[q], mq = m_off[q + 1] - m0;
        for (int i = threadIdx.x; i < mq; i += kNT) ys[i] = y[m0 + i];
        __syncthreads();
    }
    const int j = job.y + 4 * (int)threadIdx.x;
    if (j >= nU) return;
    const int ld = A_ld[q];
    const int m0 = m_off[q], mq = m_off[q + 1] - m0;
    const float *col = A + A_off[q] + j;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 8
    for (int i = 0; i < mq; ++i) {
        const f32x4 a = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(col + (int64_t)i * ld));
        const double yi = ys[i];
        a0 += (double)a.x * yi;
        a1 += (double)a.y * yi;
        a2 += (double)a.z * yi;
        a3 += (double)a.w * yi;
    }
    const double av[4] = {a0, a1, a2, a3};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t e = u0 + j + v;
        if (j + v < nU) x[e] = u[e] - s2[e] * av[v];
    }
}

// ---- setup: per-instance M_q = A_q diag(s2_q) A_q^T, Cholesky, inverse ----

// Job (q, I, J): 32 x 32 tile of M_q (I >= J), 256 threads, 2 x 2 outputs each.
__global__ __launch_bounds__(256) void k_bsyrk(const int4 *__restrict__ jobs, const float *__restrict__ A,
                                               const int64_t *__restrict__ A_off, const int32_t *__restrict__ A_ld,
                                               const int32_t *__restrict__ m_off, const int64_t *__restrict__ U_off,
                                               const double *__restrict__ s2, const int64_t *__restrict__ F_off,
                                               double *__restrict__ M) {
    constexpr int TS = 32, KC = 32;
    __shared__ double As[TS][KC + 1];
    __shared__ double Bs[TS][KC + 1];
    const int4 jb = jobs[blockIdx.x];
    const int q = jb.x, I = jb.y, J = jb.z;
    const int mq = m_off[q + 1] - m_off[q];
    const int64_t u0 = U_off[q];
    const int nU = (int)(U_off[q + 1] - u0);
    const int ld = A_ld[q];
    const float *Aq = A + A_off[q];
    const int i0 = I * TS, j0 = J * TS;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int e0 = 0; e0 < nU; e0 += KC) {
        for (int idx = threadIdx.x; idx < TS * KC; idx += 256) {
            const int r = idx / KC, qq = idx % KC;
            const int e = e0 + qq;
            const bool ok = e < nU;
            const double sc = ok ? s2[u0 + e] : 0.0;
            As[r][qq] = (ok && i0 + r < mq) ? (double)Aq[(int64_t)(i0 + r) * ld + e] * sc : 0.0;
            Bs[r][qq] = (ok && j0 + r < mq) ? (double)Aq[(int64_t)(j0 + r) * ld + e] : 0.0;
        }
        __syncthreads();
        for (int qq = 0; qq < KC; ++qq) {
            const double a0 = As[ty * 2][qq], a1 = As[ty * 2 + 1][qq];
            const double b0 = Bs[tx * 2][qq], b1 = Bs[tx * 2 + 1][qq];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
    double *Mq = M + F_off[q];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int i = i0 + ty * 2 + a, j = j0 + tx * 2 + b;
            if (i < mq && j < mq) Mq[(int64_t)i * mq + j] = acc[a][b];
        }
}

// Right-looking Cholesky of M_q in place (lower), one workgroup per instance.
// Pivot <= 2^-40 of the original diagonal: rank deficient (info[q] = 1 + row).
__global__ __launch_bounds__(256) void k_bpotrf(double *__restrict__ M, const int64_t *__restrict__ F_off,
                                                const int32_t *__restrict__ m_off, int32_t *__restrict__ info) {
    __shared__ double diag0[256];
    __shared__ double ljj;
    const int q = blockIdx.x;
    const int mq = m_off[q + 1] - m_off[q];
    double *Mq = M + F_off[q];
    for (int i = threadIdx.x; i < mq; i += 256) diag0[i] = Mq[(int64_t)i * mq + i];
    __syncthreads();
    for (int j = 0; j < mq; ++j) {
        if (threadIdx.x == 0) {
            double piv = Mq[(int64_t)j * mq + j];
            if (!(piv > ldexp(diag0[j], -40))) {
                if (info[q] == 0) info[q] = 1 + j;
                piv = 1.0;
            }
            ljj = sqrt(piv);
            Mq[(int64_t)j * mq + j] = ljj;
        }
        __syncthreads();
        const double l = ljj;
        for (int i = j + 1 + threadIdx.x; i < mq; i += 256) Mq[(int64_t)i * mq + j] /= l;
        __syncthreads();
        const int rem = mq - j - 1;
        for (int idx = threadIdx.x; idx < rem * rem; idx += 256) {
            const int i = j + 1 + idx / rem, c = j + 1 + idx % rem;
            if (c <= i) Mq[(int64_t)i * mq + c] -= Mq[(int64_t)i * mq + j] * Mq[(int64_t)c * mq + j];
        }
        __syncthreads();
    }
}

// Row j of L_q^-T (column j of L_q^-1): one wave per job (q, j); z in LDS.
__global__ __launch_bounds__(64) void k_btrtri(const int2 *__restrict__ jobs, const double *__restrict__ L,
                                               const int64_t *__restrict__ F_off, const int32_t *__restrict__ m_off,
                                               double *__restrict__ LinvT, double *__restrict__ Linv) {
    __shared__ double z[256];
    const int2 jb = jobs[blockIdx.x];
    const int q = jb.x, j = jb.y;
    const int mq = m_off[q + 1] - m_off[q];
    const double *Lq = L + F_off[q];
    double *outT = LinvT + F_off[q] + (int64_t)j * mq;
    double *outL = Linv + F_off[q];
    const int lane = threadIdx.x;
    for (int i = lane; i < j; i += 64) {
        outT[i] = 0.0;
        outL[(int64_t)i * mq + j] = 0.0;
    }
    for (int i = j; i < mq; ++i) {
        const double *li = Lq + (int64_t)i * mq;
        double acc = 0.0;
        for (int l = j + lane; l < i; l += 64) acc += li[l] * z[l];
        acc = wave_sum_d(acc);
        const double zi = ((i == j ? 1.0 : 0.0) - acc) / li[i];
        if (lane == 0) {
            z[i] = zi;
            outT[i] = zi;
            outL[(int64_t)i * mq + j] = zi;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kNT) void k_bobjectives(const double *__restrict__ c, const double *__restrict__ wt,
                                                     const double *__restrict__ x,
                                                     const int64_t *__restrict__ U_off, const double *__restrict__ b,
                                                     const double *__restrict__ y, const int32_t *__restrict__ m_off,
                                                     int nprob, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int q = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
    if (q >= nprob) return;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t e = U_off[q] + lane; e < U_off[q + 1]; e += 64) s1 += wt[e] * c[e] * x[e];
    for (int i = m_off[q] + lane; i < m_off[q + 1]; i += 64) s2 += b[i] * y[i];
    s1 = wave_sum_d(s1);
    s2 = wave_sum_d(s2);
    if (lane == 0) {
        out[2 * q + 0] = s1;
        out[2 * q + 1] = s2;
    }
}

inline unsigned waves_blocks(int64_t n) { return (unsigned)((n + kNT / 64 - 1) / (kNT / 64)); }

}  // namespace

void launch_breset(const Dev &d, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_breset, dim3((B.nprob + 255) / 256), dim3(256), 0, s, B.istop, B.iiters, B.itime,
                       B.nrunning, B.nprob, B.t0);
}

void launch_bscatter_primal(const Dev &d, const float *blk, const float *lam, double rho, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bscatter_primal, dim3(B.nsblk), dim3(kNT), 0, s, (const int4 *)B.sblk,
                       (const int32_t *)B.istop, (const int32_t *)d.inv_ptr, (const int32_t *)d.inv_slot, blk, lam,
                       (const float *)d.dslot, (const double *)d.c, (const uint32_t *)d.wbits, d.u, d.spart, rho,
                       (const Ctl *)d.ctl);
}

void launch_bcheck_primal(const Dev &d, double rho, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bcheck_primal, dim3(waves_blocks(B.nprob)), dim3(kNT), 0, s, (const double *)d.cpart,
                       (const int32_t *)B.k_off, (const double *)d.spart, (const int32_t *)B.sblk_off, B.nprob, rho,
                       B.istop, B.iiters, B.itime, B.ieps, B.nrunning, (const Ctl *)d.ctl);
    hipLaunchKernelGGL(k_bcheck_finish, dim3(1), dim3(64), 0, s, (const int32_t *)B.nrunning, d.ctl);
}

void launch_bscatter_dual(const Dev &d, const float *blk, const float *lam, double rho, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bscatter_dual, dim3(B.nsblk), dim3(kNT), 0, s, (const int4 *)B.sblk, (const int32_t *)B.istop,
                       (const int32_t *)d.inv_ptr, (const int32_t *)d.inv_slot, blk, lam, (const double *)d.c,
                       d.u, rho, (const Ctl *)d.ctl);
}

void launch_bvupdate(const Dev &d, const double *x, const float *blk, float *lam, float *v, double rho,
                     hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bvupdate, dim3(B.nvblk), dim3(kNT), 0, s, (const int4 *)B.vblk, (const int32_t *)B.istop,
                       (const int32_t *)d.gather, x, (const double *)d.wt, blk, lam, v, d.vpart, rho,
                       (const Ctl *)d.ctl);
}

void launch_bcheck_dual(const Dev &d, double rho, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bcheck_dual, dim3(waves_blocks(B.nprob)), dim3(kNT), 0, s, (const double *)d.vpart,
                       (const int32_t *)B.vblk_off, B.nprob, rho, B.istop, B.iiters, B.itime, B.ieps, B.nrunning,
                       (const Ctl *)d.ctl);
    hipLaunchKernelGGL(k_bcheck_dual_finish, dim3(1), dim3(64), 0, s, (const int32_t *)B.nrunning, d.ctl);
}

void launch_baffine(const Dev &d, const double *r2, double r2scale, double *x, double *y, const Ctl *ctl,
                    const int32_t *istop, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bgemv_Au, dim3(waves_blocks(B.nrjobs)), dim3(kNT), 0, s, (const float *)d.Aw,
                       (const int64_t *)B.A_off, (const int32_t *)B.A_ld, (const int4 *)B.rjobs, B.nrjobs,
                       (const int32_t *)B.m_off, (const int64_t *)B.U_off, (const int32_t *)B.nch,
                       (const int64_t *)B.p_off, B.tpart, istop, (const double *)d.u, r2, r2scale, d.t, ctl);
    if (B.split)
        hipLaunchKernelGGL(k_bAu_reduce, dim3((d.m + kNT - 1) / kNT), dim3(kNT), 0, s, (const int32_t *)B.rinst,
                           (const int32_t *)B.m_off, (const int32_t *)B.nch, (const int64_t *)B.p_off,
                           (const double *)B.tpart, istop, r2, r2scale, d.t, d.m, ctl);
    hipLaunchKernelGGL(k_btrmv, dim3(waves_blocks(d.m)), dim3(kNT), 0, s, (const double *)d.Linv,
                       (const int64_t *)B.F_off, (const int32_t *)B.rinst, (const int32_t *)B.m_off, istop, 0,
                       (const double *)d.t, d.y1, d.m, ctl);
    hipLaunchKernelGGL(k_btrmv, dim3(waves_blocks(d.m)), dim3(kNT), 0, s, (const double *)d.LinvT,
                       (const int64_t *)B.F_off, (const int32_t *)B.rinst, (const int32_t *)B.m_off, istop, 1,
                       (const double *)d.y1, y, d.m, ctl);
    hipLaunchKernelGGL(k_bgemv_ATy, dim3((unsigned)B.nejobs), dim3(kNT), 0, s, (const float *)d.Aw,
                       (const int64_t *)B.A_off, (const int32_t *)B.A_ld, (const int2 *)B.ejobs,
                       (const int32_t *)B.m_off, (const int64_t *)B.U_off, istop, (const double *)y,
                       (const double *)d.u, (const double *)d.s2, x, ctl);
}

void launch_bsetup(const Dev &d, double *M, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bsyrk, dim3(B.nsyrk), dim3(256), 0, s, (const int4 *)B.syrk_jobs, (const float *)d.Aw,
                       (const int64_t *)B.A_off, (const int32_t *)B.A_ld, (const int32_t *)B.m_off,
                       (const int64_t *)B.U_off, (const double *)d.s2, (const int64_t *)B.F_off, M);
    hipLaunchKernelGGL(k_bpotrf, dim3(B.nprob), dim3(256), 0, s, M, (const int64_t *)B.F_off,
                       (const int32_t *)B.m_off, B.finfo);
    hipLaunchKernelGGL(k_btrtri, dim3(d.m), dim3(64), 0, s, (const int2 *)B.trtri_jobs, (const double *)M,
                       (const int64_t *)B.F_off, (const int32_t *)B.m_off, d.LinvT, d.Linv);
}

void launch_bobjectives(const Dev &d, const double *x, const double *y, double *out, hipStream_t s) {
    const Batch &B = *d.batch;
    hipLaunchKernelGGL(k_bobjectives, dim3(waves_blocks(B.nprob)), dim3(kNT), 0, s, (const double *)d.c,
                       (const double *)d.wt, x, (const int64_t *)B.U_off, (const double *)d.b, y,
                       (const int32_t *)B.m_off, B.nprob, out);
}

}  // namespace cdcs
