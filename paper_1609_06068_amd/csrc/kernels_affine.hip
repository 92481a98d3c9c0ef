// Scatter-add with overlap counts, affine projection, multiplier epilogue of
// Algorithm 2 and the residual / stopping reductions.
//
// Paper anchors: the right-hand sides of (E:OptCondMinYPrimal) and
// (E:OptCondMinYDual) (sums of H_k^T over cliques), block elimination with the
// cached factor (Sec. III-B.1), (E:vkEqn) and (E:MultUpdateDualSDP), and the
// stopping rule of Algorithms 1 and 2.
//
// Determinism: the scatter is owner-computes over the inverse map (each pattern
// entry sums its own clique slots in a fixed order) and every reduction is a
// fixed-shape tree, so repeated runs give identical bits.
#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kNT = 256;
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kGemvSlices = 8;  // column slices of the split-K A u product

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sum (kNT threads), result valid in every thread.
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

// The residual checks reduce the partial sums of the scatter and projection
// launches in one workgroup of CNT threads (1024 when there are tens of
// thousands of partials, 256 otherwise), fixed order (bitwise reproducible):
// five sums at once, each a wave sum and then the waves in order, with one
// barrier (every sum has its own row of `red`).
template <int CNT>
__device__ __forceinline__ void check_sum5_d(double (&v)[5], double (*red)[CNT / 64]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 5; ++i) v[i] = wave_sum_d(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < 5; ++i) red[i][w] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double r = 0.0;
#pragma unroll
        for (int j = 0; j < CNT / 64; ++j) r += red[i][j];
        v[i] = r;
    }
}

__global__ __launch_bounds__(kNT) void k_reset_ctl(Ctl *ctl, int max_iter, double tol) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->iter = 0;
        ctl->stop = 0;
        ctl->max_iter = max_iter;
        ctl->jacobi_cap = 0;
        ctl->sweeps = 0;
        ctl->tol = tol;
        ctl->eps_p = 0.0;
        ctl->eps_d = 0.0;
    }
}

// Entries whose inverse list (clique slots covering the entry) is longer than
// this are summed by a whole wave in extra workgroups of the same launch; the
// others by one thread each.  Both orders are fixed, so results are bitwise
// reproducible.
constexpr int kHeavy = 32;

// w_e from the packed flags: 2 off the diagonal, 1 on it.
__device__ __forceinline__ double entry_weight(const uint32_t *__restrict__ wbits, int64_t e) {
    return ((wbits[e >> 5] >> (e & 31)) & 1u) ? 2.0 : 1.0;
}

// Alg. 1 right-hand side r1 = sum_k H_k^T (x_k + lam_k / rho) - c / rho,
// u = r1 / D (D_e = the number of slots of e, read from the inverse map), plus
// the dual-residual terms ||sum_k H_k^T (x_k - x_k_prev)||_w^2 (from the
// projection's per-slot differences) and ||sum_k H_k^T lam_k||_w^2 as
// per-block partial sums.  Light blocks: kScatterEPT entries per thread
// (entry e0 + u kNT for u < kScatterEPT), whose inverse-map pointers and
// first slots are all loaded before their values, so that the loads of the
// entries are in flight together (almost every entry has one slot); the
// further slots of an entry follow in order.  Entries with more than kHeavy
// slots are left to the heavy blocks, one wave each.
__global__ __launch_bounds__(kNT) void k_scatter_primal(const int32_t *__restrict__ inv_ptr,
                                                        const int32_t *__restrict__ inv_slot,
                                                        const int32_t *__restrict__ heavy, int nheavy,
                                                        int nlight_blocks, const float *__restrict__ blk,
                                                        const float *__restrict__ lam,
                                                        const float *__restrict__ dslot,
                                                        const double *__restrict__ c,
                                                        const uint32_t *__restrict__ wbits, double *__restrict__ u,
                                                        double *__restrict__ spart, int64_t nU, double rho,
                                                        const Ctl *ctl) {
    __shared__ double red[kNT / 64];
    if (ctl->stop) return;
    const int lane = threadIdx.x & 63;
    double ds2 = 0.0, sl2 = 0.0;
    if ((int)blockIdx.x < nlight_blocks) {
        constexpr int U = kScatterEPT;
        const int64_t e0 = (int64_t)blockIdx.x * (kNT * U) + threadIdx.x;
        int32_t q0[U], q1[U], sl[U];
#pragma unroll
        for (int v = 0; v < U; ++v) {
            const int64_t e = e0 + (int64_t)v * kNT;
            q0[v] = e < nU ? inv_ptr[e] : 0;
            q1[v] = e < nU ? inv_ptr[e + 1] : 0;
        }
#pragma unroll
        for (int v = 0; v < U; ++v) sl[v] = q1[v] > q0[v] ? inv_slot[q0[v]] : 0;
        float fx[U], fl[U], fd[U];
#pragma unroll
        for (int v = 0; v < U; ++v) {
            fx[v] = blk[sl[v]];
            fl[v] = lam[sl[v]];
            fd[v] = dslot[sl[v]];
        }
#pragma unroll
        for (int v = 0; v < U; ++v) {
            const int64_t e = e0 + (int64_t)v * kNT;
            const int32_t D = q1[v] - q0[v];
            if (e >= nU || D > kHeavy) continue;
            double s_x = 0.0, s_l = 0.0, s_d = 0.0;
            if (D > 0) {
                s_x = (double)fx[v];
                s_l = (double)fl[v];
                s_d = (double)fd[v];
            }
            for (int32_t q = q0[v] + 1; q < q1[v]; ++q) {
                const int32_t t = inv_slot[q];
                s_x += (double)blk[t];
                s_l += (double)lam[t];
                s_d += (double)dslot[t];
            }
            const double r1 = s_x + s_l / rho - c[e] / rho;
            u[e] = r1 / (double)D;
            const double w = entry_weight(wbits, e);
            ds2 += w * s_d * s_d;
            sl2 += w * s_l * s_l;
        }
    } else {
        const int hw = ((int)blockIdx.x - nlight_blocks) * (kNT / 64) + (threadIdx.x >> 6);
        if (hw < nheavy) {
            const int64_t e = heavy[hw];
            const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
            double s_x = 0.0, s_l = 0.0, s_d = 0.0;
            for (int32_t q = q0 + lane; q < q1; q += 64) {
                const int32_t sl = inv_slot[q];
                s_x += (double)blk[sl];
                s_l += (double)lam[sl];
                s_d += (double)dslot[sl];
            }
            s_x = wave_sum_d(s_x);
            s_l = wave_sum_d(s_l);
            s_d = wave_sum_d(s_d);
            if (lane == 0) {
                const double r1 = s_x + s_l / rho - c[e] / rho;
                u[e] = r1 / (double)(q1 - q0);
                const double w = entry_weight(wbits, e);
                ds2 = w * s_d * s_d;
                sl2 = w * s_l * s_l;
            }
        }
    }
    ds2 = block_sum_d(ds2, red);
    sl2 = block_sum_d(sl2, red);
    if (threadIdx.x == 0) {
        spart[2 * (int64_t)blockIdx.x + 0] = ds2;
        spart[2 * (int64_t)blockIdx.x + 1] = sl2;
    }
}

// Alg. 1 residual check of iteration n = ctl->iter (if any), then start the next one.
// The partial sums' loads are issued before the control block is waited for
// (the buffers always hold p and nsblk entries; before the first iteration
// their values are not used).  Every thread reads the control block before a
// barrier that precedes any write to it, so all waves take the same branches.
// Run by one workgroup of CNT threads.
template <int CNT>
__device__ __forceinline__ void check_primal_block(const double *__restrict__ cpart, int p,
                                                   const double *__restrict__ spart, int nsblk, double rho,
                                                   double *__restrict__ hist, int hist_cap, Ctl *ctl,
                                                   double (*red)[CNT / 64]) {
    const int tid = threadIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // |x_k - H_k x|^2, |H_k x|^2, |x_k|^2, |dS|^2, |S_lam|^2
#pragma unroll 4
    for (int k = tid; k < p; k += CNT) {
        const double4 c4 = *reinterpret_cast<const double4 *>(cpart + 4 * (int64_t)k);
        v[0] += c4.x;
        v[1] += c4.y;
        v[2] += c4.z;
    }
#pragma unroll 8
    for (int b = tid; b < nsblk; b += CNT) {
        const double2 s2v = *reinterpret_cast<const double2 *>(spart + 2 * (int64_t)b);
        v[3] += s2v.x;
        v[4] += s2v.y;
    }
    const int stop = ctl->stop, n = ctl->iter, max_iter = ctl->max_iter;
    const double tol = ctl->tol;
    __syncthreads();
    if (stop) return;
    if (n >= 1) {
        check_sum5_d<CNT>(v, red);
        if (tid == 0) {
            const double den_p = fmax(sqrt(v[1]), sqrt(v[2]));
            const double num_p = sqrt(v[0]);
            const double eps_p = den_p > 0.0 ? num_p / den_p : num_p;
            const double num_d = rho * sqrt(v[3]);
            const double den_d = sqrt(v[4]);
            const double eps_d = den_d > 0.0 ? num_d / den_d : num_d;
            ctl->eps_p = eps_p;
            ctl->eps_d = eps_d;
            if (n - 1 < hist_cap) {
                hist[2 * (int64_t)(n - 1) + 0] = eps_p;
                hist[2 * (int64_t)(n - 1) + 1] = eps_d;
            }
            // a NaN or Inf anywhere in the iterate reaches these sums
            if (!(isfinite(eps_p) && isfinite(eps_d))) {
                ctl->stop = 3;
                return;
            }
            if (fmax(eps_p, eps_d) <= tol) {
                ctl->stop = 1;
                return;
            }
        }
    }
    if (tid == 0) {
        if (n >= max_iter) ctl->stop = 2;
        else ctl->iter = n + 1;
    }
}

template <int CNT>
__global__ __launch_bounds__(CNT) void k_check_primal(const double *__restrict__ cpart, int p,
                                                      const double *__restrict__ spart, int nsblk, double rho,
                                                      double *__restrict__ hist, int hist_cap, Ctl *ctl) {
    __shared__ double red[5][CNT / 64];
    check_primal_block<CNT>(cpart, p, spart, nsblk, rho, hist, hist_cap, ctl, red);
}

// HSDE check of the iterate of iteration n = ctl->iter (n >= 1), then start
// the next one.  sc[6] = ||(y' - y) + (ut - tau') b||^2, sc[7] = ||(y' - y) +
// ut b||^2 (= ||A(x')||^2), sc[8] = b^T y', sc[9] = <c, x'>_w come from the tau
// kernel; the projection's partial sums give ||s' - H x'||^2 and the HSDE
// scatter's (hpart) the dual residual and ||A^T y'||^2.  Writes the three
// ratios of the solved test to sc[10..12] and the history; stop 1 solved,
// 2 iteration limit, 3 non-finite, 4 primal infeasible (certificate y'),
// 5 dual infeasible (certificate x').  Run by one workgroup of CNT threads.
template <int CNT>
__device__ __forceinline__ void hsde_check_block(const double *__restrict__ cpart, int ncp,
                                                 const double *__restrict__ hpart, int nhb, double *__restrict__ sc,
                                                 const double *__restrict__ tk, double *__restrict__ hist,
                                                 int hist_cap, Ctl *ctl, double (*red)[CNT / 64]) {
    const int tid = threadIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // consensus, dual residual, |A^T y'|^2
    for (int k = tid; k < ncp; k += CNT) v[0] += cpart[4 * (int64_t)k];
    for (int b = tid; b < nhb; b += CNT) {
        v[1] += hpart[2 * (int64_t)b + 0];
        v[2] += hpart[2 * (int64_t)b + 1];
    }
    const int stop = ctl->stop, n = ctl->iter, max_iter = ctl->max_iter;
    const double tol = ctl->tol;
    __syncthreads();
    if (stop) return;
    if (n >= 1) {
        check_sum5_d<CNT>(v, red);
        const double cons = v[0], rd2 = v[1], at2 = v[2];
        if (tid == 0) {
            const double tau = tk[0];
            const double nb = sc[2], nc = sc[3], by = sc[8], cx = sc[9];
            const double pri = sqrt(sc[6] + cons), ray = sqrt(sc[7] + cons);
            const double inf = __builtin_huge_val();
            const double rp = tau > 0.0 ? pri / (tau * (1.0 + nb)) : inf;
            const double rdv = tau > 0.0 ? sqrt(rd2) / (tau * (1.0 + nc)) : inf;
            const double gden = tau + fabs(cx) + fabs(by);
            const double gp = gden > 0.0 ? fabs(cx + by) / gden : 0.0;
            sc[10] = rp;
            sc[11] = rdv;
            sc[12] = gp;
            ctl->eps_p = rp;
            ctl->eps_d = fmax(rdv, gp);
            if (n - 1 < hist_cap) {
                hist[3 * (int64_t)(n - 1) + 0] = rp;
                hist[3 * (int64_t)(n - 1) + 1] = rdv;
                hist[3 * (int64_t)(n - 1) + 2] = gp;
            }
            if (!(isfinite(pri) && isfinite(rd2) && isfinite(at2) && isfinite(by) && isfinite(cx) &&
                  isfinite(tau) && isfinite(tk[1]))) {
                ctl->stop = 3;
                return;
            }
            if (tau > 0.0 && fmax(rp, fmax(rdv, gp)) <= tol) {
                ctl->stop = 1;
                return;
            }
            if (by < 0.0 && sqrt(at2) * nb <= tol * (-by)) {
                ctl->stop = 4;
                return;
            }
            if (cx < 0.0 && ray * nc <= tol * (-cx)) {
                ctl->stop = 5;
                return;
            }
        }
    }
    if (tid == 0) {
        if (n >= max_iter) ctl->stop = 2;
        else ctl->iter = n + 1;
    }
}

template <int CNT>
__global__ __launch_bounds__(CNT) void k_hsde_check(const double *__restrict__ cpart, int ncp,
                                                    const double *__restrict__ hpart, int nhb, double *__restrict__ sc,
                                                    const double *__restrict__ tk, double *__restrict__ hist,
                                                    int hist_cap, Ctl *ctl) {
    __shared__ double red[5][CNT / 64];
    hsde_check_block<CNT>(cpart, ncp, hpart, nhb, sc, tk, hist, hist_cap, ctl, red);
}

// Alg. 2 right-hand side r1 = c - sum_k H_k^T (z_k + lam_k / rho), u = r1 / D.
__global__ __launch_bounds__(kNT) void k_scatter_dual(const int32_t *__restrict__ inv_ptr,
                                                      const int32_t *__restrict__ inv_slot,
                                                      const int32_t *__restrict__ heavy, int nheavy,
                                                      int nlight_blocks, const float *__restrict__ blk,
                                                      const float *__restrict__ lam,
                                                      const double *__restrict__ c, double *__restrict__ u,
                                                      int64_t nU, double rho,
                                                      const Ctl *ctl) {
    if (ctl->stop) return;
    const int lane = threadIdx.x & 63;
    if ((int)blockIdx.x < nlight_blocks) {
        const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
        if (e >= nU) return;
        const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
        if (q1 - q0 > kHeavy) return;
        double s = 0.0;
#pragma unroll 4
        for (int32_t q = q0; q < q1; ++q) {
            const int32_t sl = inv_slot[q];
            s += (double)blk[sl] + (double)lam[sl] / rho;
        }
        u[e] = (c[e] - s) / (double)(q1 - q0);
    } else {
        const int hw = ((int)blockIdx.x - nlight_blocks) * (kNT / 64) + (threadIdx.x >> 6);
        if (hw >= nheavy) return;
        const int32_t e = heavy[hw];
        const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
        double s = 0.0;
        for (int32_t q = q0 + lane; q < q1; q += 64) {
            const int32_t sl = inv_slot[q];
            s += (double)blk[sl] + (double)lam[sl] / rho;
        }
        s = wave_sum_d(s);
        if (lane == 0) u[e] = (c[e] - s) / (double)(q1 - q0);
    }
}

// Alg. 2 epilogue: v_k = z_k + lam_k / rho + H_k x (E:vkEqn),
// lam_k += rho (z_k - v_k) (E:MultUpdateDualSDP), and residual partial sums.
__global__ __launch_bounds__(kNT) void k_vupdate(const int32_t *__restrict__ gather,
                                                 const double *__restrict__ x, const double *__restrict__ wt,
                                                 const float *__restrict__ blk, float *__restrict__ lam,
                                                 float *__restrict__ v, double *__restrict__ vpart,
                                                 int64_t nslots, double rho, const Ctl *ctl) {
    __shared__ double red[kNT / 64];
    if (ctl->stop) return;
    const int64_t s = (int64_t)blockIdx.x * kNT + threadIdx.x;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0, q4 = 0.0;
    if (s < nslots) {
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

// Alg. 2 residual check of the iteration just completed (loads issued before
// the control block is waited for; its only writer is thread 0, after the
// reduction's barrier).
template <int CNT>
__global__ __launch_bounds__(CNT) void k_check_dual(const double *__restrict__ vpart, int nvblk, double rho,
                                                    double *__restrict__ hist, int hist_cap, Ctl *ctl) {
    __shared__ double red[5][CNT / 64];
    const int tid = threadIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int b = tid; b < nvblk; b += CNT) {
        const double *o = vpart + 5 * (int64_t)b;
#pragma unroll
        for (int i = 0; i < 5; ++i) v[i] += o[i];
    }
    const int stop = ctl->stop, n = ctl->iter + 1, max_iter = ctl->max_iter;
    const double tol = ctl->tol;
    if (stop) return;
    check_sum5_d<CNT>(v, red);
    if (tid == 0) {
        const double den_p = fmax(sqrt(v[1]), sqrt(v[2]));
        const double eps_p = den_p > 0.0 ? sqrt(v[0]) / den_p : sqrt(v[0]);
        const double den_d = sqrt(v[4]);
        const double eps_d = den_d > 0.0 ? rho * sqrt(v[3]) / den_d : rho * sqrt(v[3]);
        ctl->eps_p = eps_p;
        ctl->eps_d = eps_d;
        ctl->iter = n;
        if (n - 1 < hist_cap) {
            hist[2 * (int64_t)(n - 1) + 0] = eps_p;
            hist[2 * (int64_t)(n - 1) + 1] = eps_d;
        }
        if (!(isfinite(eps_p) && isfinite(eps_d))) ctl->stop = 3;  // NaN or Inf in the iterate
        else if (fmax(eps_p, eps_d) <= tol) ctl->stop = 1;
        else if (n >= max_iter) ctl->stop = 2;
    }
}

// Gather H_k x for every clique into packed slots (FP64).
__global__ __launch_bounds__(kNT) void k_gather_f64(const int32_t *__restrict__ gather,
                                                    const double *__restrict__ x, double *__restrict__ out,
                                                    int64_t nslots) {
    const int64_t s = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (s < nslots) out[s] = x[gather[s]];
}

// sum_k H_k^T over packed slots (FP64), owner-computes like the ADMM scatter.
__global__ __launch_bounds__(kNT) void k_scatter_f64(const int32_t *__restrict__ inv_ptr,
                                                     const int32_t *__restrict__ inv_slot,
                                                     const int32_t *__restrict__ heavy, int nheavy,
                                                     int nlight_blocks, const double *__restrict__ packed,
                                                     double *__restrict__ out, int64_t nU) {
    const int lane = threadIdx.x & 63;
    if ((int)blockIdx.x < nlight_blocks) {
        const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
        if (e >= nU) return;
        const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
        if (q1 - q0 > kHeavy) return;
        double acc = 0.0;
#pragma unroll 4
        for (int32_t q = q0; q < q1; ++q) acc += packed[inv_slot[q]];
        out[e] = acc;
    } else {
        const int hw = ((int)blockIdx.x - nlight_blocks) * (kNT / 64) + (threadIdx.x >> 6);
        if (hw >= nheavy) return;
        const int32_t e = heavy[hw];
        const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
        double acc = 0.0;
        for (int32_t q = q0 + lane; q < q1; q += 64) acc += packed[inv_slot[q]];
        acc = wave_sum_d(acc);
        if (lane == 0) out[e] = acc;
    }
}

__global__ __launch_bounds__(kNT) void k_scale_u(const double *__restrict__ r1, const double *__restrict__ invD,
                                                 double *__restrict__ u, int64_t nU) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e >= nU) return;
    u[e] = r1[e] * invD[e];
}

// The residual check (Algorithm 1's, or the HSDE's when sc is set) run by the
// first workgroup of the A u launch that follows it (ctl == nullptr: none).
struct CheckArgs {
    const double *cpart;
    const double *spart;  // the scatter's partial sums (HSDE: hpart)
    double *hist;
    Ctl *ctl;
    double rho;
    int p, nsblk, hist_cap;
    double *sc;           // HSDE solved-test scalars, or nullptr
    const double *tk;     // HSDE (tau, kappa)
};

// The leading workgroup of an A u launch that carries a check runs it.
__device__ __forceinline__ void run_check(const CheckArgs &ck, double (*red)[kNT / 64]) {
    if (ck.sc != nullptr)
        hsde_check_block<kNT>(ck.cpart, ck.p, ck.spart, ck.nsblk, ck.sc, ck.tk, ck.hist, ck.hist_cap, ck.ctl, red);
    else
        check_primal_block<kNT>(ck.cpart, ck.p, ck.spart, ck.nsblk, ck.rho, ck.hist, ck.hist_cap, ck.ctl, red);
}

// Sparse A: t_i = sum over the coefficients of row i of Aw_ie u_e - r2scale r2_i.
// One wave per row, lanes over the coefficients.
// With a check (ck.ctl set) the first workgroup runs it and the rows start at
// the second: t is scratch, and the triangular products that read it test the
// stop flag, so a stop decided while this launch runs changes nothing.
__global__ __launch_bounds__(kNT) void k_spmv_Au(const int32_t *__restrict__ sp_ptr,
                                                 const int32_t *__restrict__ sp_col,
                                                 const double *__restrict__ sp_val, const double *__restrict__ u,
                                                 const double *__restrict__ r2, double r2scale,
                                                 double *__restrict__ t, int m, const Ctl *ctl, CheckArgs ck) {
    __shared__ double ckred[5][kNT / 64];
    const int lead = ck.ctl != nullptr ? 1 : 0;
    if (lead && blockIdx.x == 0) {
        run_check(ck, ckred);
        return;
    }
    if (ctl != nullptr && ctl->stop) return;
    const int lane = threadIdx.x & 63;
    const int row = ((int)blockIdx.x - lead) * (kNT / 64) + (threadIdx.x >> 6);
    if (row >= m) return;
    double acc = 0.0;
    for (int32_t q = sp_ptr[row] + lane; q < sp_ptr[row + 1]; q += 64) acc += sp_val[q] * u[sp_col[q]];
    acc = wave_sum_d(acc);
    if (lane == 0) t[row] = acc - r2scale * r2[row];
}

// Sparse A, second half of the x-update: x = u (k_copy_u), then x_e = u_e -
// s2_e (Aw^T y)_e on the entries that carry coefficients (k_sp_xcorr, one
// thread per touched entry).  Both are gated by the stop flag like the rest
// of the affine step, so a solve that stops inside an iteration (after its
// scatter and check) keeps the last completed iterate in x.
__global__ __launch_bounds__(kNT) void k_copy_u(const double *__restrict__ u, double *__restrict__ x, int64_t n,
                                                const Ctl *ctl) {
    if (ctl != nullptr && ctl->stop) return;
    const int64_t e = 2 * ((int64_t)blockIdx.x * kNT + threadIdx.x);
    if (e + 1 < n) {
        *reinterpret_cast<double2 *>(x + e) = *reinterpret_cast<const double2 *>(u + e);
    } else if (e < n) {
        x[e] = u[e];
    }
}

__global__ __launch_bounds__(kNT) void k_sp_xcorr(const int32_t *__restrict__ tc_e,
                                                  const int32_t *__restrict__ tc_ptr,
                                                  const int32_t *__restrict__ tc_row,
                                                  const double *__restrict__ tc_val, const double *__restrict__ y,
                                                  const double *__restrict__ u, const double *__restrict__ s2,
                                                  double *__restrict__ x, int ntc, const Ctl *ctl) {
    if (ctl != nullptr && ctl->stop) return;
    const int t = blockIdx.x * kNT + threadIdx.x;
    if (t >= ntc) return;
    double acc = 0.0;
    for (int32_t r = tc_ptr[t]; r < tc_ptr[t + 1]; ++r) acc += tc_val[r] * y[tc_row[r]];
    const int32_t e = tc_e[t];
    x[e] = u[e] - s2[e] * acc;
}

// Split-K partial products of t = A (w u): tpart[slice][row] is the dot
// product of row `row` of the FP32 matrix Aw (= w A, row-major, leading
// dimension ld, zero padded) with u over the columns of one slice.  RG rows per
// workgroup, so each u slice is read once per RG rows; FP64 accumulation.
// With a check (ck.ctl set) the grid has one more column of workgroups in
// front: workgroup (0, 0) runs the residual check of the iteration before
// (dispatched first, so it overlaps the product), the rest of that column
// returns.  The product only writes tpart, which the reduction that follows
// reads only when the check did not stop the solve, so it does not matter
// whether a product workgroup starts before or after the check's decision.
template <int RG>
__global__ __launch_bounds__(kNT, 5) void k_gemv_Au(const float *__restrict__ Aw, int64_t ld,
                                                    const double *__restrict__ u, double *__restrict__ tpart, int m,
                                                    int64_t slice_cols, const Ctl *ctl, CheckArgs ck) {
    __shared__ double red[kNT / 64];
    __shared__ double ckred[5][kNT / 64];
    const int lead = ck.ctl != nullptr ? 1 : 0;
    if (lead && blockIdx.x == 0) {
        if (blockIdx.y == 0) run_check(ck, ckred);
        return;
    }
    if (ctl != nullptr && ctl->stop) return;
    const int row0 = ((int)blockIdx.x - lead) * RG;
    const int64_t c0 = (int64_t)blockIdx.y * slice_cols;
    const int64_t c1 = min(ld, c0 + slice_cols);
    double acc[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) acc[r] = 0.0;
    const float *base[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) base[r] = Aw + (int64_t)min(row0 + r, m - 1) * ld;
#pragma unroll 2
    for (int64_t c = c0 + (int64_t)threadIdx.x * 4; c < c1; c += (int64_t)kNT * 4) {
        const double2 u01 = *reinterpret_cast<const double2 *>(u + c);
        const double2 u23 = *reinterpret_cast<const double2 *>(u + c + 2);
        f32x4 av[RG];
#pragma unroll
        for (int r = 0; r < RG; ++r) av[r] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(base[r] + c));
#pragma unroll
        for (int r = 0; r < RG; ++r)
            acc[r] += (double)av[r].x * u01.x + (double)av[r].y * u01.y + (double)av[r].z * u23.x +
                      (double)av[r].w * u23.y;
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        const double sum = block_sum_d(acc[r], red);
        if (threadIdx.x == 0 && row0 + r < m) tpart[(int64_t)blockIdx.y * m + row0 + r] = sum;
    }
}

// t = sum of the slice partials - r2scale * r2 (fixed slice order).
__global__ __launch_bounds__(kNT) void k_reduce_t(const double *__restrict__ tpart, int nslice,
                                                  const double *__restrict__ r2, double r2scale,
                                                  double *__restrict__ t, int m, const Ctl *ctl) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i >= m) return;
    double sum = 0.0;  // nslice <= kGemvSlices; the loads issue together, before the stop flag is waited for
#pragma unroll
    for (int q = 0; q < kGemvSlices; ++q)
        if (q < nslice) sum += tpart[(int64_t)q * m + i];
    const double r2i = r2[i];
    if (ctl != nullptr && ctl->stop) return;
    t[i] = sum - r2scale * r2i;
}

// Product out = T vin of a row-major m x m matrix over the column range
// [lo, hi) of each row: lower triangle (mode 0): [0, i]; upper (mode 1):
// [i, m); full (mode 2, T = M^-1): [0, m).  One workgroup per row, its elements
// spread over all kNT threads (coalesced), so every wave waits on only a few
// loads and enough of them are in flight to keep HBM busy; triangle rows are
// dispatched longest first.  Fixed-order block sum.
__global__ __launch_bounds__(kNT) void k_trmv(const double *__restrict__ T, int m, int mode,
                                              const double *__restrict__ vin, double *__restrict__ vout,
                                              const Ctl *ctl) {
    __shared__ double red[kNT / 64];
    if (ctl != nullptr && ctl->stop) return;
    const int row = mode != 0 ? (int)blockIdx.x : m - 1 - (int)blockIdx.x;
    const int lo = mode == 1 ? row : 0, hi = mode == 0 ? row + 1 : m;
    const double *tr = T + (int64_t)row * m;
    double a0 = 0.0, a1 = 0.0;
    int j = lo + (int)threadIdx.x;
    for (; j + kNT < hi; j += 2 * kNT) {
        a0 += tr[j] * vin[j];
        a1 += tr[j + kNT] * vin[j + kNT];
    }
    if (j < hi) a0 += tr[j] * vin[j];
    const double acc = block_sum_d(a0 + a1, red);
    if (threadIdx.x == 0) vout[row] = acc;
}

// Sparse triangular product out = T vin with T in CSR (sparse inverse
// factors): one wave per row, fixed summation order.
__global__ __launch_bounds__(kNT) void k_csr_mv(const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                const double *__restrict__ val, const double *__restrict__ vin,
                                                double *__restrict__ vout, int m, const Ctl *ctl) {
    if (ctl != nullptr && ctl->stop) return;
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
    if (row >= m) return;
    double acc = 0.0;
    for (int32_t q = ptr[row] + lane; q < ptr[row + 1]; q += 64) acc += val[q] * vin[col[q]];
    acc = wave_sum_d(acc);
    if (lane == 0) vout[row] = acc;
}

// x = u - s2 * (Aw^T y): four rows of AwT (= (w A)^T, row-major, leading
// dimension ldm, zero padded) per wave, 16 per workgroup; y staged in LDS.
constexpr int kAtyRows = 16;

__global__ __launch_bounds__(kNT) void k_gemv_ATy(const float *__restrict__ AwT, int64_t ldm,
                                                  const double *__restrict__ y, const double *__restrict__ u,
                                                  const double *__restrict__ s2, double *__restrict__ x,
                                                  int64_t nU, int m, const Ctl *ctl) {
    constexpr int CH = 2048;
    __shared__ double ys[CH];
    if (ctl != nullptr && ctl->stop) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t rb = (int64_t)blockIdx.x * kAtyRows + 4 * w;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const float *ar[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ar[q] = AwT + min(rb + q, nU - 1) * ldm;
    for (int c0 = 0; c0 < m; c0 += CH) {
        const int cn = min(CH, m - c0);
        __syncthreads();
        for (int i = threadIdx.x; i < CH; i += kNT) ys[i] = (i < cn) ? y[c0 + i] : 0.0;
        __syncthreads();
        for (int i = lane * 4; i < cn; i += 256) {
            const double y0 = ys[i], y1 = ys[i + 1], y2 = ys[i + 2], y3 = ys[i + 3];
            f32x4 av[4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                av[q] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(ar[q] + c0 + i));
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[q] += (double)av[q].x * y0 + (double)av[q].y * y1 + (double)av[q].z * y2 + (double)av[q].w * y3;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double sum = wave_sum_d(acc[q]);
        const int64_t row = rb + q;
        if (lane == 0 && row < nU) x[row] = u[row] - s2[row] * sum;
    }
}

// Objective terms <c, x>_w and <b, y>: fixed-shape two-pass reduction
// (kObjBlocks grid-stride partials, then one workgroup in block order).
constexpr int kObjBlocks = 512;

__global__ __launch_bounds__(kNT) void k_objectives(const double *__restrict__ c, const double *__restrict__ wt,
                                                    const double *__restrict__ x, int64_t nU,
                                                    const double *__restrict__ b, const double *__restrict__ y,
                                                    int m, double *__restrict__ part) {
    __shared__ double red[kNT / 64];
    double s1 = 0.0, s2 = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < nU; e += (int64_t)kObjBlocks * kNT)
        s1 += wt[e] * c[e] * x[e];
    for (int i = blockIdx.x * kNT + threadIdx.x; i < m; i += kObjBlocks * kNT) s2 += b[i] * y[i];
    s1 = block_sum_d(s1, red);
    s2 = block_sum_d(s2, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = s1;
        part[2 * blockIdx.x + 1] = s2;
    }
}

__global__ __launch_bounds__(kNT) void k_objectives_finish(const double *__restrict__ part,
                                                           double *__restrict__ out) {
    __shared__ double red[kNT / 64];
    double s1 = 0.0, s2 = 0.0;
    for (int q = threadIdx.x; q < kObjBlocks; q += kNT) {
        s1 += part[2 * q];
        s2 += part[2 * q + 1];
    }
    s1 = block_sum_d(s1, red);
    s2 = block_sum_d(s2, red);
    if (threadIdx.x == 0) {
        out[0] = s1;
        out[1] = s2;
    }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kNT - 1) / kNT); }

// Entry-space vectors cross the interface in pattern order; inside they are
// kept in the internal order (perm[e]: pattern position of internal entry e).
__global__ __launch_bounds__(kNT) void k_perm_in(const double *__restrict__ xp, const int32_t *__restrict__ perm,
                                                 double *__restrict__ xi, int64_t nU) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e < nU) xi[e] = xp[perm[e]];
}

__global__ __launch_bounds__(kNT) void k_perm_out(const double *__restrict__ xi, const int32_t *__restrict__ perm,
                                                  double *__restrict__ xp, int64_t nU) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e < nU) xp[perm[e]] = xi[e];
}

// ---- Adjoint of one unrolled iteration of Algorithm 1 ----------------------
// Packed coordinates: a cotangent of a packed slot is the derivative with
// respect to the slot's value (an off-diagonal slot stands for both mirrored
// entries of the clique matrix).  Forward: r1 = sum_k H_k^T (x_k + lam_k / rho)
// - c / rho, x = F(r1, b), h = H_k x, P = P_+(h - lam / rho),
// lam' = lam + rho (P - h), x_k' = P.

// gP = xbar_k' + rho lambar'  (cotangent of P, FP32 for the projection adjoint)
__global__ __launch_bounds__(kNT) void k_adj_in(const double *__restrict__ blkbar, const double *__restrict__ lambar,
                                                double rho, float *__restrict__ gP, int64_t nslots) {
    const int64_t s = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (s < nslots) gP[s] = (float)(blkbar[s] + rho * lambar[s]);
}

// hbar = gW - rho lambar' (cotangent of h), lambar <- lambar' - gW / rho
__global__ __launch_bounds__(kNT) void k_adj_mid(const float *__restrict__ gW, double *__restrict__ lambar,
                                                 double rho, double inv_rho, double *__restrict__ hbar,
                                                 int64_t nslots) {
    const int64_t s = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (s >= nslots) return;
    const double g = (double)gW[s], l = lambar[s];
    hbar[s] = g - rho * l;
    lambar[s] = l - g * inv_rho;
}

// xbar_e = sum over the slots of e of hbar (the gather's transpose) plus the
// caller's cotangent of x (pattern order), then u = xbar / (w D): the input
// of the affine solve F(xbar / w, 0), whose x times w is the cotangent of r1
// (F's Jacobian in r1 is diag(w)^-1 J^T diag(w)) and whose y is the cotangent
// of b.  hbar and xbar_pat may be NULL.  Owner-computes, fixed order.
__global__ __launch_bounds__(kNT) void k_adj_scatter(const int32_t *__restrict__ inv_ptr,
                                                     const int32_t *__restrict__ inv_slot,
                                                     const int32_t *__restrict__ heavy, int nheavy, int nlight_blocks,
                                                     const double *__restrict__ hbar,
                                                     const double *__restrict__ xbar_pat,
                                                     const int32_t *__restrict__ perm,
                                                     const double *__restrict__ s2, double *__restrict__ u,
                                                     int64_t nU) {
    const int lane = threadIdx.x & 63;
    int64_t e = -1;
    double acc = 0.0;
    bool owner = false;
    if ((int)blockIdx.x < nlight_blocks) {
        e = (int64_t)blockIdx.x * kNT + threadIdx.x;
        if (e >= nU) return;
        const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
        if (hbar != nullptr && q1 - q0 > kHeavy) return;
        if (hbar != nullptr)
            for (int32_t q = q0; q < q1; ++q) acc += hbar[inv_slot[q]];
        owner = true;
    } else {
        if (hbar == nullptr) return;
        const int hw = ((int)blockIdx.x - nlight_blocks) * (kNT / 64) + (threadIdx.x >> 6);
        if (hw >= nheavy) return;
        e = heavy[hw];
        const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
        for (int32_t q = q0 + lane; q < q1; q += 64) acc += hbar[inv_slot[q]];
        acc = wave_sum_d(acc);
        owner = lane == 0;
    }
    if (!owner) return;
    if (xbar_pat != nullptr) acc += xbar_pat[perm[e]];
    u[e] = s2[e] * acc;
}

// r1bar = w x (x of the solve F(xbar / w, 0)); out[perm[e]] = scale r1bar_e
// (accumulate: +=).  r1bar is kept in x.
__global__ __launch_bounds__(kNT) void k_adj_post(const double *__restrict__ wt, double *__restrict__ x,
                                                  const int32_t *__restrict__ perm, double *__restrict__ out,
                                                  double scale, int accumulate, int64_t nU) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e >= nU) return;
    const double r = wt[e] * x[e];
    x[e] = r;
    const int32_t pe = perm[e];
    out[pe] = accumulate ? out[pe] + scale * r : scale * r;
}

// Cotangents of the iteration's inputs: xbar_k = H_k r1bar, lambar += H_k r1bar / rho.
__global__ __launch_bounds__(kNT) void k_adj_slots(const int32_t *__restrict__ gather,
                                                   const double *__restrict__ r1bar, double *__restrict__ blkbar,
                                                   double *__restrict__ lambar, double inv_rho, int64_t nslots) {
    const int64_t s = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (s >= nslots) return;
    const double r = r1bar[gather[s]];
    blkbar[s] = r;
    lambar[s] += r * inv_rho;
}

__global__ __launch_bounds__(kNT) void k_add_to(const double *__restrict__ v, double *__restrict__ out, int n,
                                                int accumulate) {
    const int i = blockIdx.x * kNT + threadIdx.x;
    if (i < n) out[i] = accumulate ? out[i] + v[i] : v[i];
}

}  // namespace

int scatter_light_blocks(const Dev &d) { return (int)blocks_for(d.nU); }
int scatter_blocks(const Dev &d) { return scatter_light_blocks(d) + (d.nheavy + kNT / 64 - 1) / (kNT / 64); }
int pscatter_light_blocks(const Dev &d) { return (int)((d.nU + kNT * kScatterEPT - 1) / (kNT * kScatterEPT)); }
int pscatter_blocks(const Dev &d) { return pscatter_light_blocks(d) + (d.nheavy + kNT / 64 - 1) / (kNT / 64); }
int heavy_threshold() { return kHeavy; }
int vupdate_blocks(const Dev &d) { return (int)blocks_for(d.nslots); }

void launch_reset_ctl(const Dev &d, int max_iter, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(kNT), 0, s, d.ctl, max_iter, tol);
}

void launch_scatter_primal(const Dev &d, const float *blk, const float *lam, double rho,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_primal, dim3(pscatter_blocks(d)), dim3(kNT), 0, s, d.inv_ptr, d.inv_slot,
                       (const int32_t *)d.heavy, d.nheavy, pscatter_light_blocks(d), blk, lam,
                       (const float *)d.dslot, (const double *)d.c, (const uint32_t *)d.wbits, d.u, d.spart, d.nU,
                       rho, (const Ctl *)d.ctl);
}

bool check_in_au(const Dev &d) { return d.p + d.nvb + pscatter_blocks(d) <= 8192; }

void launch_check_primal(const Dev &d, double rho, hipStream_t s) {
    // partial sums of the cliques, then of the vector cones' blocks
    const int ncp = d.p + d.nvb;
    if (ncp + pscatter_blocks(d) > 8192)
        hipLaunchKernelGGL(k_check_primal<1024>, dim3(1), dim3(1024), 0, s, (const double *)d.cpart, ncp,
                           (const double *)d.spart, pscatter_blocks(d), rho, d.hist, d.hist_cap, d.ctl);
    else
        hipLaunchKernelGGL(k_check_primal<kNT>, dim3(1), dim3(kNT), 0, s, (const double *)d.cpart, ncp,
                           (const double *)d.spart, pscatter_blocks(d), rho, d.hist, d.hist_cap, d.ctl);
}

void launch_scatter_dual(const Dev &d, const float *blk, const float *lam, double rho,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_dual, dim3(scatter_blocks(d)), dim3(kNT), 0, s, d.inv_ptr, d.inv_slot,
                       (const int32_t *)d.heavy, d.nheavy, scatter_light_blocks(d), blk, lam, d.c, d.u,
                       d.nU, rho, (const Ctl *)d.ctl);
}

void launch_vupdate(const Dev &d, const double *x, const float *blk, float *lam, float *v, double rho,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_vupdate, dim3(blocks_for(d.nslots)), dim3(kNT), 0, s, d.gather, x, d.wt, blk, lam, v,
                       d.vpart, d.nslots, rho, (const Ctl *)d.ctl);
}

void launch_check_dual(const Dev &d, double rho, hipStream_t s) {
    if (vupdate_blocks(d) > 8192)
        hipLaunchKernelGGL(k_check_dual<1024>, dim3(1), dim3(1024), 0, s, (const double *)d.vpart, vupdate_blocks(d),
                           rho, d.hist, d.hist_cap, d.ctl);
    else
        hipLaunchKernelGGL(k_check_dual<kNT>, dim3(1), dim3(kNT), 0, s, (const double *)d.vpart, vupdate_blocks(d),
                           rho, d.hist, d.hist_cap, d.ctl);
}

void launch_scale_u(const Dev &d, const double *r1, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_u, dim3(blocks_for(d.nU)), dim3(kNT), 0, s, r1, (const double *)d.invD, d.u, d.nU);
}

// Affine projection from u = r1 / D: t = A (w u) - r2scale r2, y = L^-T L^-1 t,
// x = u - (A^T y) / D.
int gemv_slices(const Dev &d) {
    const int64_t ncb = (d.ldU + 1023) / 1024;
    return (int)std::min<int64_t>(kGemvSlices, ncb);
}

void launch_gemv_au(const Dev &d, const Ctl *ctl, const CheckArgs &ck, hipStream_t s) {
    constexpr int RG = 8;
    const int ns = gemv_slices(d);
    const int64_t ncb = (d.ldU + 1023) / 1024;
    const int64_t slice_cols = (ncb + ns - 1) / ns * 1024;
    const int lead = ck.ctl != nullptr ? 1 : 0;
    hipLaunchKernelGGL((k_gemv_Au<RG>), dim3((d.m + RG - 1) / RG + lead, ns), dim3(kNT), 0, s, (const float *)d.Aw,
                       d.ldU, (const double *)d.u, d.tpart, d.m, slice_cols, ctl, ck);
}

void launch_spmv_au(const Dev &d, const double *r2, double r2scale, const Ctl *ctl, const CheckArgs &ck,
                    hipStream_t s) {
    const int lead = ck.ctl != nullptr ? 1 : 0;
    hipLaunchKernelGGL(k_spmv_Au, dim3((d.m + kNT / 64 - 1) / (kNT / 64) + lead), dim3(kNT), 0, s,
                       (const int32_t *)d.sp_ptr, (const int32_t *)d.sp_col, (const double *)d.sp_val,
                       (const double *)d.u, r2, r2scale, d.t, d.m, ctl, ck);
}

// The A u part of the affine step (part 0) with the check in its first workgroup.
void launch_au_with_check(const Dev &d, const double *r2, double r2scale, double rho, const Ctl *ctl,
                          hipStream_t s) {
    CheckArgs ck{(const double *)d.cpart, (const double *)d.spart, d.hist, d.ctl, rho, d.p + d.nvb,
                 pscatter_blocks(d), d.hist_cap, nullptr, nullptr};
    if (d.sparse) launch_spmv_au(d, r2, r2scale, ctl, ck, s);
    else launch_gemv_au(d, ctl, ck, s);
}

void launch_au_with_hsde_check(const Dev &dh, const Dev &d, const HsdeDev &hs, const double *tk, const double *r2,
                               double r2scale, const Ctl *ctl, hipStream_t s) {
    CheckArgs ck{(const double *)d.cpart, (const double *)hs.hpart, hs.hist, d.ctl, 0.0, d.p + d.nvb,
                 pscatter_blocks(d), hs.hist_cap, hs.sc, tk};
    if (dh.sparse) launch_spmv_au(dh, r2, r2scale, ctl, ck, s);
    else launch_gemv_au(dh, ctl, ck, s);
}

void launch_hsde_check(const Dev &d, const HsdeDev &hs, const double *tk, hipStream_t s) {
    const int ncp = d.p + d.nvb, nhb = pscatter_blocks(d);
    if (ncp + nhb > 8192)
        hipLaunchKernelGGL(k_hsde_check<1024>, dim3(1), dim3(1024), 0, s, (const double *)d.cpart, ncp,
                           (const double *)hs.hpart, nhb, hs.sc, tk, hs.hist, hs.hist_cap, d.ctl);
    else
        hipLaunchKernelGGL(k_hsde_check<kNT>, dim3(1), dim3(kNT), 0, s, (const double *)d.cpart, ncp,
                           (const double *)hs.hpart, nhb, hs.sc, tk, hs.hist, hs.hist_cap, d.ctl);
}

void launch_affine_part(const Dev &d, int part, const double *r2, double r2scale, double *x, double *y,
                        const Ctl *ctl, hipStream_t s) {
    if (d.sparse && part == 0) {
        launch_spmv_au(d, r2, r2scale, ctl, CheckArgs{}, s);
    } else if (d.sparse && part == 3) {
        // A u already carries - r2scale r2
    } else if (d.sparse && part == 2) {
        hipLaunchKernelGGL(k_copy_u, dim3(blocks_for((d.nU + 1) / 2)), dim3(kNT), 0, s, (const double *)d.u, x, d.nU,
                           ctl);
        if (d.ntc > 0)
            hipLaunchKernelGGL(k_sp_xcorr, dim3(blocks_for(d.ntc)), dim3(kNT), 0, s, (const int32_t *)d.tc_e,
                               (const int32_t *)d.tc_ptr, (const int32_t *)d.tc_row, (const double *)d.tc_val,
                               (const double *)y, (const double *)d.u, (const double *)d.s2, x, d.ntc, ctl);
    } else if (part == 0) {
        launch_gemv_au(d, ctl, CheckArgs{}, s);
    } else if (part == 3) {
        hipLaunchKernelGGL(k_reduce_t, dim3((d.m + kNT - 1) / kNT), dim3(kNT), 0, s, (const double *)d.tpart,
                           gemv_slices(d), r2, r2scale, d.t, d.m, ctl);
    } else if (part == 1 && d.sparse_linv) {
        const unsigned tb = (unsigned)((d.m + kNT / 64 - 1) / (kNT / 64));
        hipLaunchKernelGGL(k_csr_mv, dim3(tb), dim3(kNT), 0, s, (const int32_t *)d.li_ptr, (const int32_t *)d.li_col,
                           (const double *)d.li_val, (const double *)d.t, d.y1, d.m, ctl);
        hipLaunchKernelGGL(k_csr_mv, dim3(tb), dim3(kNT), 0, s, (const int32_t *)d.lt_ptr, (const int32_t *)d.lt_col,
                           (const double *)d.lt_val, (const double *)d.y1, y, d.m, ctl);
    } else if (part == 1) {
        hipLaunchKernelGGL(k_trmv, dim3(d.m), dim3(kNT), 0, s, (const double *)d.Minv, d.m, 2, (const double *)d.t, y,
                           ctl);
    } else {
        const unsigned gb = (unsigned)((d.nU + kAtyRows - 1) / kAtyRows);
        hipLaunchKernelGGL(k_gemv_ATy, dim3(gb), dim3(kNT), 0, s, (const float *)d.AwT, d.ldM, (const double *)y,
                           (const double *)d.u, (const double *)d.s2, x, d.nU, d.m, ctl);
    }
}

void launch_affine(const Dev &d, const double *r2, double r2scale, double *x, double *y, const Ctl *ctl,
                   hipStream_t s) {
    launch_affine_part(d, 0, r2, r2scale, x, y, ctl, s);
    launch_affine_part(d, 3, r2, r2scale, x, y, ctl, s);
    launch_affine_part(d, 1, r2, r2scale, x, y, ctl, s);
    launch_affine_part(d, 2, r2, r2scale, x, y, ctl, s);
}

void launch_perm_in(const Dev &d, const double *x_pattern, double *x_internal, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_in, dim3(blocks_for(d.nU)), dim3(kNT), 0, s, x_pattern, (const int32_t *)d.perm,
                       x_internal, d.nU);
}

void launch_perm_out(const Dev &d, const double *x_internal, double *x_pattern, hipStream_t s) {
    hipLaunchKernelGGL(k_perm_out, dim3(blocks_for(d.nU)), dim3(kNT), 0, s, x_internal, (const int32_t *)d.perm,
                       x_pattern, d.nU);
}

void launch_gather_f64(const Dev &d, const double *x, double *packed, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_f64, dim3(blocks_for(d.nslots)), dim3(kNT), 0, s, (const int32_t *)d.gather, x, packed,
                       d.nslots);
}

void launch_scatter_f64(const Dev &d, const double *packed, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_f64, dim3(scatter_blocks(d)), dim3(kNT), 0, s, (const int32_t *)d.inv_ptr,
                       (const int32_t *)d.inv_slot, (const int32_t *)d.heavy, d.nheavy, scatter_light_blocks(d),
                       packed, out, d.nU);
}

int objective_partials() { return 2 * kObjBlocks; }

void launch_adjoint_in(const Dev &d, const double *blkbar, const double *lambar, double rho, float *gP,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_adj_in, dim3(blocks_for(d.nslots)), dim3(kNT), 0, s, blkbar, lambar, rho, gP, d.nslots);
}

void launch_adjoint_mid(const Dev &d, const float *gW, double *lambar, double rho, double *hbar, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_mid, dim3(blocks_for(d.nslots)), dim3(kNT), 0, s, gW, lambar, rho, 1.0 / rho, hbar,
                       d.nslots);
}

void launch_adjoint_scatter(const Dev &d, const double *hbar, const double *xbar_pat, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_scatter, dim3(scatter_blocks(d)), dim3(kNT), 0, s, (const int32_t *)d.inv_ptr,
                       (const int32_t *)d.inv_slot, (const int32_t *)d.heavy, d.nheavy, scatter_light_blocks(d), hbar,
                       xbar_pat, (const int32_t *)d.perm, (const double *)d.s2, d.u, d.nU);
}

void launch_adjoint_post(const Dev &d, double *x, double *out_pat, double scale, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_post, dim3(blocks_for(d.nU)), dim3(kNT), 0, s, (const double *)d.wt, x,
                       (const int32_t *)d.perm, out_pat, scale, accumulate, d.nU);
}

void launch_adjoint_slots(const Dev &d, const double *r1bar, double *blkbar, double *lambar, double rho,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_adj_slots, dim3(blocks_for(d.nslots)), dim3(kNT), 0, s, (const int32_t *)d.gather, r1bar,
                       blkbar, lambar, 1.0 / rho, d.nslots);
}

void launch_add_to(const double *v, double *out, int n, int accumulate, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_add_to, dim3(blocks_for(n)), dim3(kNT), 0, s, v, out, n, accumulate);
}

void launch_objectives(const Dev &d, const double *x, const double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_objectives, dim3(kObjBlocks), dim3(kNT), 0, s, (const double *)d.c, (const double *)d.wt, x,
                       d.nU, (const double *)d.b, y, d.m, d.opart);
    hipLaunchKernelGGL(k_objectives_finish, dim3(1), dim3(kNT), 0, s, (const double *)d.opart, d.obj);
}

}  // namespace cdcs
