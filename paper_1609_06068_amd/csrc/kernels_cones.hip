// Projections onto the vector cones beside the PSD cliques: the free cone,
// the nonnegative orthant and the second-order cone {(t, z): ||z|| <= t}
// (the cone types other than PSD that CDCS accepts, Sec. IV), fused with the
// same gather and multiplier epilogue as the clique projection kernel.
//
// Work units: blocks of at most kVecChunk slots of one cone, one workgroup
// each, in two launches.  A second-order cone's projection needs the norm of
// its whole z part: in the first launch (every block) the free-cone and
// orthant blocks are projected while a second-order cone's blocks write the
// partial sums of z^2 over their slots; in the second (the second-order
// cones' blocks only) every block adds its cone's partial sums, reads t and
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
// clique kernel rounds them.  Deterministic: fixed-order reductions, and every
// block of a cone forms the cone's norm in the same order.
#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kNT = 256;
static_assert(kVecChunk % kNT == 0, "whole slots per thread");

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

// Project slots [s0, s1) of block b (second-order cone: ||z|| = nz, t, and
// the cone's first slot `first`), update the multipliers and write the block's
// residual partial sums.  Called by every thread of the workgroup.
__device__ __forceinline__ void project_block(const ProjArgs &a, int b, int kind, int64_t s0, int64_t s1, double t,
                                              double nz, int64_t first, int cbase, double *red) {
    constexpr int U = kVecChunk / kNT;  // slots per thread
    const int tid = threadIdx.x;
    const bool dual = (a.mode == PROJ_DUAL);
    // the inputs of all of this thread's slots first, so that their loads are
    // in flight together (slots past the block are clamped and not stored)
    double hv[U];
    float lm[U], old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t g = min<int64_t>(s0 + tid + u * kNT, s1 - 1);
        lm[u] = a.lam[g];
        hv[u] = dual ? (double)a.v[g] : a.x[a.gather[g]];
        old[u] = (!dual && a.dslot != nullptr) ? a.blk[g] : 0.0f;
    }
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t g = s0 + tid + u * kNT;
        if (g >= s1) continue;
        const double w = hv[u] - (double)lm[u] * a.inv_rho;
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
        a.blk[g] = pv32;
        if (dual) continue;
        const double hx = hv[u];
        const double pr = (double)pv32;
        a.lam[g] = (float)((double)lm[u] + a.rho * (pr - hx));
        if (a.dslot != nullptr) a.dslot[g] = (float)(pr - (double)old[u]);
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

// First launch, one workgroup per block: free-cone and orthant blocks are
// projected; a second-order cone's block writes the sum of z^2 over its slots
// (the cone's first slot, t, excluded) to part[b].
__global__ __launch_bounds__(kNT) void k_project_vec(ProjArgs a, const int32_t *__restrict__ vblk,
                                                     const int32_t *__restrict__ soc, double *__restrict__ part,
                                                     int cbase) {
    __shared__ double red[kNT / 64];
    if (a.ctl != nullptr && a.ctl->stop) return;
    const int b = blockIdx.x;
    const int kind = vblk[4 * b + 0];
    const int64_t s0 = vblk[4 * b + 1], s1 = vblk[4 * b + 2];
    if (s1 <= s0) return;  // uniform over the workgroup
    if (kind == CDCS_CONE_SOC) {
        const int64_t first = soc[3 * vblk[4 * b + 3]];
        double z2 = 0.0;
        for (int64_t g = max<int64_t>(s0, first + 1) + threadIdx.x; g < s1; g += kNT) {
            const double w = cone_input(a, g);
            z2 += w * w;
        }
        z2 = block_sum(z2, red);
        if (threadIdx.x == 0) part[b] = z2;
        return;
    }
    project_block(a, b, kind, s0, s1, 0.0, 0.0, -1, cbase, red);
}

// Second launch, one workgroup per second-order cone block (list socb): the
// cone's ||z|| from its blocks' partial sums (wave 0: lane-strided sums in
// block order, then a butterfly, the same in every block of the cone) and t,
// then the projection of the block's slots.
__global__ __launch_bounds__(kNT) void k_project_soc(ProjArgs a, const int32_t *__restrict__ vblk,
                                                     const int32_t *__restrict__ socb,
                                                     const int32_t *__restrict__ soc,
                                                     const double *__restrict__ part, int cbase) {
    __shared__ double red[kNT / 64];
    __shared__ double snt[2];
    if (a.ctl != nullptr && a.ctl->stop) return;
    const int b = socb[blockIdx.x];
    const int q = vblk[4 * b + 3];
    const int64_t s0 = vblk[4 * b + 1], s1 = vblk[4 * b + 2];
    if (s1 <= s0) return;  // uniform over the workgroup
    if (threadIdx.x < 64) {
        double z2 = 0.0;
        for (int bb = soc[3 * q + 1] + (int)threadIdx.x; bb < soc[3 * q + 2]; bb += 64) z2 += part[bb];
        z2 = wave_sum_d(z2);
        if (threadIdx.x == 0) {
            snt[0] = sqrt(z2);
            snt[1] = cone_input(a, soc[3 * q]);
        }
    }
    __syncthreads();
    project_block(a, b, CDCS_CONE_SOC, s0, s1, snt[1], snt[0], soc[3 * q], cbase, red);
}

}  // namespace

void launch_project_vec(const ProjArgs &a, const Dev &d, hipStream_t s) {
    if (d.nvb <= 0 || a.mode == PROJ_STANDALONE) return;
    hipLaunchKernelGGL(k_project_vec, dim3((unsigned)d.nvb), dim3(kNT), 0, s, a, (const int32_t *)d.vblk,
                       (const int32_t *)d.soc, d.soc_part, d.p);
    if (d.nsocb > 0)
        hipLaunchKernelGGL(k_project_soc, dim3((unsigned)d.nsocb), dim3(kNT), 0, s, a, (const int32_t *)d.vblk,
                           (const int32_t *)d.socb, (const int32_t *)d.soc, (const double *)d.soc_part, d.p);
}

}  // namespace cdcs
