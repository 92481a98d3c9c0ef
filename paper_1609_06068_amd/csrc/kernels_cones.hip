// Projections onto the vector cones beside the PSD cliques: the free cone,
// the nonnegative orthant and the second-order cone {(t, z): ||z|| <= t}
// (the cone types other than PSD that CDCS accepts, Sec. IV), fused with the
// same gather and multiplier epilogue as the clique projection kernel.
//
// Work units: a block of slots of one cone (orthant and free cones are cut
// into chunks of at most kVecChunk slots, a second-order cone is one block:
// its projection needs the norm of the whole z part).  One workgroup per
// block.  Modes (ProjArgs.mode):
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

__global__ __launch_bounds__(kNT) void k_project_vec(ProjArgs a, const int32_t *__restrict__ vblk, int cbase) {
    __shared__ double red[kNT / 64];
    if (a.ctl != nullptr && a.ctl->stop) return;
    const int b = blockIdx.x;
    const int kind = vblk[4 * b + 0];
    const int64_t s0 = vblk[4 * b + 1], s1 = vblk[4 * b + 2];
    const int tid = threadIdx.x;
    const bool dual = (a.mode == PROJ_DUAL);
    // second-order cone: t and ||z|| of the whole cone first
    double t = 0.0, nz = 0.0;
    if (kind == CDCS_CONE_SOC) {
        // every thread reads t before the reduction's barrier: the epilogue
        // below overwrites the slot's multiplier
        t = cone_input(a, s0);
        double z2 = 0.0;
        for (int64_t g = s0 + 1 + tid; g < s1; g += kNT) {
            const double w = cone_input(a, g);
            z2 += w * w;
        }
        nz = sqrt(block_sum(z2, red));
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
            pv = (g == s0) ? h : (h / nz) * w;
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

void launch_project_vec(const ProjArgs &a, const int32_t *vblk, int nvb, int cbase, hipStream_t s) {
    if (nvb > 0 && a.mode != PROJ_STANDALONE)
        hipLaunchKernelGGL(k_project_vec, dim3((unsigned)nvb), dim3(kNT), 0, s, a, vblk, cbase);
}

}  // namespace cdcs
