// Homogeneous self-dual embedding (HSDE) of the decomposed problem: the
// variant the paper names as future work (Sec. VI), iterated as in
// O'Donoghue, Chu, Parikh and Boyd (2016), without over-relaxation.
//
// Notation (entries w-weighted as everywhere in the library): the conic
// program min <c, x> s.t. Ahat x + s = bhat, s in {0}^m x K with
// Ahat = [A; -H_1; ...; -H_p], bhat = (b, 0); u = (x, y, z, tau),
// v = (0, 0, s, kappa).  One iteration, with E = 1 + D and the cached factor
// of M' = I + A diag(w / E) A^T:
//   scatter   p = x + sum_k H_k^T (s_k + z_k),  u_e = p_e / E_e
//   affine    t = A(w u) + y,  yh = M'^-1 t,  a = u - (A^T yh) / E
//   dot/tau   ut = (tau + kappa + <c, a>_w + b^T yh) / (1 + h^T g),
//             y <- yh - ut g_y,  tau <- max(ut - kappa, 0),  kappa <- kappa - ut + tau
//   axpy      x <- a - ut g_x
//   cones     s_k <- P(H_k x - z_k),  z_k <- s_k - (H_k x - z_k)  (projection kernel, rho = 1)
// where g = M^-1 (c, bhat) is cached ((g_x, g_y); its cone part is never
// needed).  The linear step is ut = (I + Q)^-1 (u + v) by block elimination:
// its x, y rows form M zeta = (x, y, z + s) (v's x and y parts are zero), and
// with zeta_x = a, zeta_y = yh, the clique rows zeta_k = z_k + s_k - H_k a
// enter the cone step as z_k + s_k - H_k x after the tau correction.
//
// Residuals without extra passes over A (identities of the linear step, with
// primes for the new iterate and ut its tau row):
//   A(x') - tau' b            = (y' - y) + (ut - tau') b
//   s'_k - H_k x'             = |x_k - H_k x|-term of the projection kernel
//   A^T y' - sum H^T z' + tau' c = (x - x') - sum_k H_k^T (s'_k - s_k) + (tau' - ut) c
// The first comes out of the tau kernel, the third out of the next
// iteration's scatter (it has x - x' and the per-slot differences s' - s), so
// the check of an iterate runs at the start of the next iteration, as the
// Algorithm-1 check does.
//
// Deterministic: owner-computes scatter, fixed-order reductions.
#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kNT = 256;
constexpr int kHeavy = 32;  // the scatter's split between thread- and wave-owned entries
constexpr int kDotPer = 8;  // entries per thread of the dot kernel

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum_d(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += red[i];
    return r;
}

__device__ __forceinline__ double entry_weight(const uint32_t *__restrict__ wbits, int64_t e) {
    return ((wbits[e >> 5] >> (e & 31)) & 1u) ? 2.0 : 1.0;
}

// 1 / E and 1 / (w E) with E = 1 + D (from 1 / D); zero on the padding.
__global__ __launch_bounds__(kNT) void k_hsde_scales(const double *__restrict__ invD, const double *__restrict__ wt,
                                                     double *__restrict__ invE, double *__restrict__ s2E,
                                                     int64_t nU, int64_t ld) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e >= ld) return;
    if (e >= nU) {
        invE[e] = 0.0;
        s2E[e] = 0.0;
        return;
    }
    const double E = 1.0 + 1.0 / invD[e];
    invE[e] = 1.0 / E;
    s2E[e] = 1.0 / (wt[e] * E);
}

// u = c / E (the x rows of M g = (c, bhat)).
__global__ __launch_bounds__(kNT) void k_hsde_cu(const double *__restrict__ c, const double *__restrict__ invE,
                                                 double *__restrict__ u, int64_t nU) {
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e < nU) u[e] = c[e] * invE[e];
}

// Constants of the iteration (one workgroup): sc[0] = h^T g = <c, g_x>_w +
// b^T g_y, sc[1] = <c, g_x>_w, sc[2] = ||b||, sc[3] = ||c||_w.
__global__ __launch_bounds__(1024) void k_hsde_consts(const double *__restrict__ c, const double *__restrict__ gx,
                                                      const uint32_t *__restrict__ wbits,
                                                      const double *__restrict__ b, const double *__restrict__ gy,
                                                      int64_t nU, int m, double *__restrict__ sc) {
    __shared__ double red[16];
    double cg = 0.0, cc = 0.0, bg = 0.0, bb = 0.0;
    for (int64_t e = threadIdx.x; e < nU; e += 1024) {
        const double w = entry_weight(wbits, e);
        cg += w * c[e] * gx[e];
        cc += w * c[e] * c[e];
    }
    for (int i = threadIdx.x; i < m; i += 1024) {
        bg += b[i] * gy[i];
        bb += b[i] * b[i];
    }
    cg = block_sum<1024>(cg, red);
    cc = block_sum<1024>(cc, red);
    bg = block_sum<1024>(bg, red);
    bb = block_sum<1024>(bb, red);
    if (threadIdx.x == 0) {
        sc[0] = cg + bg;
        sc[1] = cg;
        sc[2] = sqrt(bb);
        sc[3] = sqrt(cc);
    }
}

// Starting point: u = (0, 0, 0, 1), v = (0, 0, 0, 1).
__global__ __launch_bounds__(kNT) void k_hsde_init(double *__restrict__ x, int64_t nU, double *__restrict__ y, int m,
                                                   float *__restrict__ s, float *__restrict__ z, int64_t nslots,
                                                   double *__restrict__ tk) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (i < nU) x[i] = 0.0;
    if (i < m) y[i] = 0.0;
    if (i < nslots) {
        s[i] = 0.0f;
        z[i] = 0.0f;
    }
    if (i == 0) {
        tk[0] = 1.0;
        tk[1] = 1.0;
    }
}

// p = x + sum_k H_k^T (s_k + z_k), u = p / E; and, for the iterate the last
// iteration produced, the per-block partial sums of ||r_d||_w^2 and
// ||A^T y - sum_k H_k^T z_k||_w^2 with
//   r_d = (x_prev - x) - sum_k H_k^T (s_k - s_k_prev) + (tau - ut) c,
//   A^T y - sum_k H_k^T z_k = r_d - tau c.
// Light blocks give each thread kScatterEPT entries (entry e0 + v kNT), whose
// inverse-map pointers and first slots are loaded before their values, so the
// loads of the entries are in flight together; heavy entries (more than
// kHeavy slots) get a wave each.
__global__ __launch_bounds__(kNT) void k_hsde_scatter(const int32_t *__restrict__ inv_ptr,
                                                      const int32_t *__restrict__ inv_slot,
                                                      const int32_t *__restrict__ heavy, int nheavy,
                                                      int nlight_blocks, const float *__restrict__ s,
                                                      const float *__restrict__ z, const float *__restrict__ dslot,
                                                      const double *__restrict__ x, const double *__restrict__ dx,
                                                      const double *__restrict__ c, const double *__restrict__ invE,
                                                      const uint32_t *__restrict__ wbits,
                                                      const double *__restrict__ sc, const double *__restrict__ tk,
                                                      double *__restrict__ u, double *__restrict__ hpart, int64_t nU,
                                                      const Ctl *ctl) {
    __shared__ double red[kNT / 64];
    if (ctl->stop) return;
    const int lane = threadIdx.x & 63;
    double rd2 = 0.0, at2 = 0.0;
    auto finish = [&](int64_t e, double s_s, double s_z, double s_d) {
        const double ce = c[e];
        u[e] = (x[e] + s_s + s_z) * invE[e];
        const double w = entry_weight(wbits, e);
        const double rd = dx[e] - s_d + sc[5] * ce;
        const double at = rd - tk[0] * ce;
        rd2 += w * rd * rd;
        at2 += w * at * at;
    };
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
        float fs[U], fz[U], fd[U];
#pragma unroll
        for (int v = 0; v < U; ++v) {
            fs[v] = s[sl[v]];
            fz[v] = z[sl[v]];
            fd[v] = dslot[sl[v]];
        }
#pragma unroll
        for (int v = 0; v < U; ++v) {
            const int64_t e = e0 + (int64_t)v * kNT;
            const int32_t D = q1[v] - q0[v];
            if (e >= nU || D > kHeavy) continue;
            double s_s = 0.0, s_z = 0.0, s_d = 0.0;
            if (D > 0) {
                s_s = (double)fs[v];
                s_z = (double)fz[v];
                s_d = (double)fd[v];
            }
            for (int32_t q = q0[v] + 1; q < q1[v]; ++q) {
                const int32_t t = inv_slot[q];
                s_s += (double)s[t];
                s_z += (double)z[t];
                s_d += (double)dslot[t];
            }
            finish(e, s_s, s_z, s_d);
        }
    } else {
        const int hw = ((int)blockIdx.x - nlight_blocks) * (kNT / 64) + (threadIdx.x >> 6);
        if (hw < nheavy) {
            const int64_t e = heavy[hw];
            const int32_t q0 = inv_ptr[e], q1 = inv_ptr[e + 1];
            double s_s = 0.0, s_z = 0.0, s_d = 0.0;
            for (int32_t q = q0 + lane; q < q1; q += 64) {
                const int32_t sl = inv_slot[q];
                s_s += (double)s[sl];
                s_z += (double)z[sl];
                s_d += (double)dslot[sl];
            }
            s_s = wave_sum_d(s_s);
            s_z = wave_sum_d(s_z);
            s_d = wave_sum_d(s_d);
            if (lane == 0) finish(e, s_s, s_z, s_d);
        }
    }
    rd2 = block_sum<kNT>(rd2, red);
    at2 = block_sum<kNT>(at2, red);
    if (threadIdx.x == 0) {
        hpart[2 * (int64_t)blockIdx.x + 0] = rd2;
        hpart[2 * (int64_t)blockIdx.x + 1] = at2;
    }
}

// Partial sums of <c, a>_w, kDotPer * kNT entries per block.
__global__ __launch_bounds__(kNT) void k_hsde_dot(const double *__restrict__ c, const double *__restrict__ a,
                                                  const uint32_t *__restrict__ wbits, double *__restrict__ dpart,
                                                  int64_t nU, const Ctl *ctl) {
    __shared__ double red[kNT / 64];
    if (ctl->stop) return;
    const int64_t e0 = (int64_t)blockIdx.x * (kDotPer * kNT) + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kDotPer; ++r) {
        const int64_t e = e0 + (int64_t)r * kNT;
        if (e < nU) acc += entry_weight(wbits, e) * c[e] * a[e];
    }
    acc = block_sum<kNT>(acc, red);
    if (threadIdx.x == 0) dpart[blockIdx.x] = acc;
}

// The tau row and the y update (one workgroup): ut, y' = yh - ut g_y,
// tau' = max(ut - kappa, 0), kappa' = kappa - ut + tau', and the scalars the
// check of the new iterate needs.
__global__ __launch_bounds__(1024) void k_hsde_tau(const double *__restrict__ dpart, int ndp,
                                                   const double *__restrict__ yh, const double *__restrict__ gy,
                                                   const double *__restrict__ b, double *__restrict__ y, int m,
                                                   double *__restrict__ sc, double *__restrict__ tk, const Ctl *ctl) {
    __shared__ double red[16];
    if (ctl->stop) return;
    const int tid = threadIdx.x;
    double ca = 0.0, byh = 0.0;
    for (int i = tid; i < ndp; i += 1024) ca += dpart[i];
    for (int i = tid; i < m; i += 1024) byh += b[i] * yh[i];
    ca = block_sum<1024>(ca, red);
    byh = block_sum<1024>(byh, red);
    const double tau = tk[0], kappa = tk[1];
    const double ut = (tau + kappa + ca + byh) / (1.0 + sc[0]);
    const double tau1 = fmax(ut - kappa, 0.0);
    double rp = 0.0, ry = 0.0, by = 0.0;
    for (int i = tid; i < m; i += 1024) {
        const double yn = yh[i] - ut * gy[i];
        const double dy = yn - y[i];
        const double bi = b[i];
        const double q1 = dy + (ut - tau1) * bi, q2 = dy + ut * bi;
        rp += q1 * q1;
        ry += q2 * q2;
        by += bi * yn;
        y[i] = yn;
    }
    rp = block_sum<1024>(rp, red);
    ry = block_sum<1024>(ry, red);
    by = block_sum<1024>(by, red);
    if (tid == 0) {
        sc[4] = ut;
        sc[5] = tau1 - ut;
        sc[6] = rp;
        sc[7] = ry;
        sc[8] = by;
        sc[9] = ca - ut * sc[1];
        tk[0] = tau1;
        tk[1] = kappa - ut + tau1;
    }
}

// x' = a - ut g_x, dx = x - x'.
__global__ __launch_bounds__(kNT) void k_hsde_axpy(const double *__restrict__ a, const double *__restrict__ gx,
                                                   const double *__restrict__ sc, double *__restrict__ x,
                                                   double *__restrict__ dx, int64_t nU, const Ctl *ctl) {
    if (ctl->stop) return;
    const int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (e >= nU) return;
    const double ut = sc[4];
    const double xn = a[e] - ut * gx[e];
    dx[e] = x[e] - xn;
    x[e] = xn;
}

// Solution or certificate from the state (which: 0 X = x / tau and
// y_sdp = -y / tau, 1 y / (b^T y), 2 x / (-<c, x>_w)).
__global__ __launch_bounds__(kNT) void k_hsde_solution(int which, const double *__restrict__ x, int64_t nU,
                                                       const double *__restrict__ y, int m,
                                                       const double *__restrict__ sc, const double *__restrict__ tk,
                                                       double *__restrict__ X, double *__restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
    if (which == 0) {
        const double it = 1.0 / tk[0];
        if (i < nU) X[i] = x[i] * it;
        if (i < m) Y[i] = -y[i] * it;
    } else if (which == 1) {
        if (i < m) Y[i] = y[i] / sc[8];
    } else {
        if (i < nU) X[i] = x[i] / (-sc[9]);
    }
}

unsigned nblocks(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int hsde_dot_blocks(const Dev &d) { return (int)nblocks(d.nU, (int64_t)kDotPer * kNT); }

void launch_hsde_scales(const Dev &d, const HsdeDev &hs, hipStream_t s) {
    hipLaunchKernelGGL(k_hsde_scales, dim3(nblocks(d.ldU, kNT)), dim3(kNT), 0, s, (const double *)d.invD,
                       (const double *)d.wt, hs.invE, hs.s2E, d.nU, d.ldU);
}

void launch_hsde_cu(const Dev &d, const HsdeDev &hs, hipStream_t s) {
    hipLaunchKernelGGL(k_hsde_cu, dim3(nblocks(d.nU, kNT)), dim3(kNT), 0, s, (const double *)d.c,
                       (const double *)hs.invE, d.u, d.nU);
}

void launch_hsde_consts(const Dev &d, const HsdeDev &hs, hipStream_t s) {
    hipLaunchKernelGGL(k_hsde_consts, dim3(1), dim3(1024), 0, s, (const double *)d.c, (const double *)hs.gx,
                       (const uint32_t *)d.wbits, (const double *)d.b, (const double *)hs.gy, d.nU, d.m, hs.sc);
}

void launch_hsde_init(const Dev &d, double *x, double *y, float *sl, float *z, double *tk, hipStream_t s) {
    const int64_t n = std::max<int64_t>(std::max<int64_t>(d.nU, d.m), d.nslots);
    hipLaunchKernelGGL(k_hsde_init, dim3(nblocks(n, kNT)), dim3(kNT), 0, s, x, d.nU, y, d.m, sl, z, d.nslots, tk);
}

void launch_hsde_scatter(const Dev &d, const HsdeDev &hs, const float *sl, const float *z, const double *tk,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_hsde_scatter, dim3(pscatter_blocks(d)), dim3(kNT), 0, s, (const int32_t *)d.inv_ptr,
                       (const int32_t *)d.inv_slot, (const int32_t *)d.heavy, d.nheavy, pscatter_light_blocks(d), sl, z,
                       (const float *)d.dslot, (const double *)d.xi, (const double *)hs.dx, (const double *)d.c,
                       (const double *)hs.invE, (const uint32_t *)d.wbits, (const double *)hs.sc, tk, d.u, hs.hpart,
                       d.nU, (const Ctl *)d.ctl);
}

void launch_hsde_tau(const Dev &d, const HsdeDev &hs, double *y, double *tk, hipStream_t s) {
    hipLaunchKernelGGL(k_hsde_dot, dim3((unsigned)hsde_dot_blocks(d)), dim3(kNT), 0, s, (const double *)d.c,
                       (const double *)hs.a, (const uint32_t *)d.wbits, hs.dpart, d.nU, (const Ctl *)d.ctl);
    hipLaunchKernelGGL(k_hsde_tau, dim3(1), dim3(1024), 0, s, (const double *)hs.dpart, hsde_dot_blocks(d),
                       (const double *)hs.yh, (const double *)hs.gy, (const double *)d.b, y, d.m, hs.sc, tk,
                       (const Ctl *)d.ctl);
}

void launch_hsde_axpy(const Dev &d, const HsdeDev &hs, hipStream_t s) {
    hipLaunchKernelGGL(k_hsde_axpy, dim3(nblocks(d.nU, kNT)), dim3(kNT), 0, s, (const double *)hs.a,
                       (const double *)hs.gx, (const double *)hs.sc, d.xi, hs.dx, d.nU, (const Ctl *)d.ctl);
}

void launch_hsde_solution(const Dev &d, const HsdeDev &hs, int which, const double *x, const double *y,
                          const double *tk, double *X, double *Y, hipStream_t s) {
    const int64_t n = std::max<int64_t>(d.nU, d.m);
    hipLaunchKernelGGL(k_hsde_solution, dim3(nblocks(n, kNT)), dim3(kNT), 0, s, which, x, d.nU, y, d.m,
                       (const double *)hs.sc, tk, X, Y);
}

}  // namespace cdcs
