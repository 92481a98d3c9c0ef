// Projections onto the vector cones beside the PSD cliques: the free cone,
// the nonnegative orthant and the second-order cone {(t, z): ||z|| <= t}
// (the cone types other than PSD that CDCS accepts, Sec. IV), fused with the
// same gather and multiplier epilogue as the clique projection kernel.
//
// Work units: blocks of at most kVecChunk slots of one cone, one workgroup
// each.  A second-order cone's projection needs the norm of its whole z part:
// its blocks first write partial sums of z^2 (k_soc_partial), one thread per
// cone adds them in block order and reads t (k_soc_finish), then every block
// projects its slots.  Modes (ProjArgs.mode):
//   PROJ_PRIMAL (Algorithm 1; the HSDE cone step with rho = 1):
//     W = H_k x - lam / rho, x_k = P_K(W), lam += rho (x_k - H_k x), the slot
//     difference x_k(new) - x_k(old), and the three residual partial sums
//     |x_k - H_k x|^2, |H_k x|^2, |x_k|^2 of the block (cpart row cbase + b);
//   PROJ_DUAL (Algorithm 2): z_k = P_K*(v_k - lam / rho) onto the dual cone
//   (free cone: {0}).
// Projections: orthant max(w, 0); second-order cone: w itself if
// ||z|| <= t, 0 if ||z|| <= -t, else ((t + ||z||) / 2) (1, z / ||z||).
// Arithmetic in FP64 from the FP32 state; results rounded to FP32 as the
// clique kernel rounds them.  Deterministic: fixed-order block reductions.
#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kNT = 256;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup (waves added in order), valid in every thread.
__device__ __forceinline__ double block_sum(double v, double *red) {
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

__device__ __forceinline__ double cone_input(const ProjArgs &a, int64_t g) {
    const double l = (double)a.lam[g] * a.inv_rho;
    if (a.mode == PROJ_PRIMAL) return a.x[a.gather[g]] - l;
    return (double)a.v[g] - l;
}

// Partial sums of z^2 over a second-order cone's block (its first slot, t,
// excluded).
__global__ __launch_bounds__(kNT) void k_soc_partial(ProjArgs a, const int32_t *__restrict__ vblk,
                                                     const int32_t *__restrict__ soc, double *__restrict__ part) {
    __shared__ double red[kNT / 64];
    if (a.ctl != nullptr && a.ctl->stop) return;
    const int b = blockIdx.x;
    if (vblk[4 * b + 0] != CDCS_CONE_SOC) return;
    const int64_t first = soc[3 * vblk[4 * b + 3]];
    const int64_t s0 = max<int64_t>(vblk[4 * b + 1], first + 1), s1 = vblk[4 * b + 2];
    double z2 = 0.0;
    for (int64_t g = s0 + threadIdx.x; g < s1; g += kNT) {
        const double w = cone_input(a, g);
        z2 += w * w;
    }
    z2 = block_sum(z2, red);
    if (threadIdx.x == 0) part[b] = z2;
}

// ||z|| and t of every second-order cone (one thread per cone, blocks in order).
__global__ __launch_bounds__(kNT) void k_soc_finish(ProjArgs a, const int32_t *__restrict__ soc, int nsoc,
                                                    const double *__restrict__ part, double *__restrict__ nt) {
    if (a.ctl != nullptr && a.ctl->stop) return;
    const int q = blockIdx.x * kNT + threadIdx.x;
    if (q >= nsoc) return;
    double z2 = 0.0;
    for (int b = soc[3 * q + 1]; b < soc[3 * q + 2]; ++b) z2 += part[b];
    nt[2 * q + 0] = sqrt(z2);
    nt[2 * q + 1] = cone_input(a, soc[3 * q]);
}

__global__ __launch_bounds__(kNT) void k_project_vec(ProjArgs a, const int32_t *__restrict__ vblk,
                                                     const int32_t *__restrict__ soc, const double *__restrict__ nt,
                                                     int cbase) {
    __shared__ double red[kNT / 64];
    if (a.ctl != nullptr && a.ctl->stop) return;
    const int b = blockIdx.x;
    const int kind = vblk[4 * b + 0];
    const int64_t s0 = vblk[4 * b + 1], s1 = vblk[4 * b + 2];
    const int tid = threadIdx.x;
    const bool dual = (a.mode == PROJ_DUAL);
    // second-order cone: ||z|| and t of the whole cone, and its first slot
    double t = 0.0, nz = 0.0;
    int64_t first = -1;
    if (kind == CDCS_CONE_SOC) {
        const int q = vblk[4 * b + 3];
        nz = nt[2 * q + 0];
        t = nt[2 * q + 1];
        first = soc[3 * q];
    }
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int64_t g = s0 + tid; g < s1; g += kNT) {
        const double w = cone_input(a, g);
        double pv;
        if (kind == CDCS_CONE_FREE) {
            pv = dual ? 0.0 : w;
        } else if (kind == CDCS_CONE_ORTHANT) {
            pv = fmax(w, 0.0);
        } else if (nz <= t) {
            pv = w;
        } else if (nz <= -t) {
            pv = 0.0;
        } else {
            const double h = 0.5 * (t + nz);
            pv = (g == first) ? h : (h / nz) * w;
        }
        const float pv32 = (float)pv;
        if (dual) {
            a.blk[g] = pv32;
            continue;
        }
        const double hx = a.x[a.gather[g]];
        const double pr = (double)pv32;
        const float old = a.blk[g];
        a.lam[g] = (float)((double)a.lam[g] + a.rho * (pr - hx));
        a.blk[g] = pv32;
        if (a.dslot != nullptr) a.dslot[g] = (float)(pr - (double)old);
        const double d = pr - hx;
        p0 += d * d;
        p1 += hx * hx;
        p2 += pr * pr;
    }
    if (dual) return;
    p0 = block_sum(p0, red);
    p1 = block_sum(p1, red);
    p2 = block_sum(p2, red);
    if (tid == 0) {
        double *o = a.cpart + 4 * (int64_t)(cbase + b);
        o[0] = p0;
        o[1] = p1;
        o[2] = p2;
    }
}

}  // namespace

void launch_project_vec(const ProjArgs &a, const Dev &d, hipStream_t s) {
    if (d.nvb <= 0 || a.mode == PROJ_STANDALONE) return;
    if (d.nsoc > 0) {
        hipLaunchKernelGGL(k_soc_partial, dim3((unsigned)d.nvb), dim3(kNT), 0, s, a, (const int32_t *)d.vblk,
                           (const int32_t *)d.soc, d.soc_part);
        hipLaunchKernelGGL(k_soc_finish, dim3((unsigned)((d.nsoc + kNT - 1) / kNT)), dim3(kNT), 0, s, a,
                           (const int32_t *)d.soc, d.nsoc, (const double *)d.soc_part, d.soc_nt);
    }
    hipLaunchKernelGGL(k_project_vec, dim3((unsigned)d.nvb), dim3(kNT), 0, s, a, (const int32_t *)d.vblk,
                       (const int32_t *)d.soc, (const double *)d.soc_nt, d.p);
}

}  // namespace cdcs
