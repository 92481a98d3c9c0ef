// Batched projection onto the product of small PSD cones (paper: Sec. III-B.2,
// (E:XkUpdate); Sec. IV-B.2, (E:zkUpdate)), fused with the gather from the
// global vector and, for Algorithm 1, the multiplier update (E:LambdakUpdate)
// and the per-clique residual partial sums.
//
// One workgroup per clique.  The clique matrix W (FP32) is staged in LDS and
// diagonalised by two-sided Jacobi with the round-robin (circle) ordering:
// in each of the kk-1 steps of a sweep the kk/2 disjoint pairs are rotated
// together, so the step is one LDS pass with one barrier between computing
// the rotations and applying them.  The sweep stops when
//   off(A)^2 <= (2^-23)^2 ||W||_F^2.
// FP32 accumulation of the eigenvector matrix loses orthogonality like
// sqrt(#rotations) eps, so one Newton-Schulz step V <- V - V (V^T V - I) / 2
// re-orthonormalises it before the rebuild P = V max(Lambda, 0) V^T.
#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kMaxSweeps = 30;
constexpr float kEps = 1.1920928955078125e-07f;  // 2^-23

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup, result in every thread.  Contains two barriers.
template <int NT, typename T>
__device__ __forceinline__ T block_sum(T v, T *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    T r = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) r += red[i];
    return r;
}

// Max over the workgroup, result in every thread.  Contains two barriers.
template <int NT>
__device__ __forceinline__ float block_max(float v, float *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    float r = red[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) r = fmaxf(r, red[i]);
    return r;
}

// Row a of the packed lower-triangular slot s = a(a+1)/2 + b.
__device__ __forceinline__ int tri_row(int s) {
    int a = (int)((sqrtf(8.0f * (float)s + 1.0f) - 1.0f) * 0.5f);
    while ((a + 1) * (a + 2) / 2 <= s) ++a;
    while (a * (a + 1) / 2 > s) --a;
    return a;
}

template <int S, int NT>
__global__ __launch_bounds__(NT) void k_project(ProjArgs a) {
    constexpr int LD = S + 1;  // odd row stride: column walks hit distinct banks
    __shared__ float sA[S * LD];
    __shared__ float sV[S * LD];
    __shared__ float sX[S * LD];
    __shared__ float sLam[S];
    __shared__ float sLp[S];
    __shared__ int sP[S / 2], sQ[S / 2];
    __shared__ float sC[S / 2], sS[S / 2], sT[S / 2];
    __shared__ float redf[NT / 64];
    __shared__ double redd[NT / 64];

    if (a.ctl != nullptr && a.ctl->stop) return;
    const int bi = blockIdx.x;
    if (bi >= a.nblk) return;
    const int id = a.ids ? a.ids[bi] : bi;
    const int k = a.size[id];
    if (k < 1 || k > S) return;
    const int kk = k + (k & 1);  // padded to even with a zero row/column
    const int np = kk >> 1;
    const int64_t off = a.off[id];
    const int nslot = k * (k + 1) / 2;
    const int tid = threadIdx.x;

    for (int idx = tid; idx < kk * kk; idx += NT) {
        const int i = idx / kk, j = idx - i * kk;
        sA[i * LD + j] = 0.0f;
        sV[i * LD + j] = (i == j) ? 1.0f : 0.0f;
    }
    __syncthreads();

    // Gather W (packed lower triangle) into the full LDS matrix.
    float amax = 0.0f;
    for (int s = tid; s < nslot; s += NT) {
        const int i = tri_row(s), j = s - i * (i + 1) / 2;
        float w;
        if (a.mode == PROJ_STANDALONE) {
            w = a.Win[off + s];
        } else if (a.mode == PROJ_PRIMAL) {
            const double hx = a.x[a.gather[off + s]];
            w = (float)(hx - (double)a.lam[off + s] / a.rho);
        } else {
            w = (float)((double)a.v[off + s] - (double)a.lam[off + s] / a.rho);
        }
        sA[i * LD + j] = w;
        sA[j * LD + i] = w;
        amax = fmaxf(amax, fabsf(w));
    }
    // Scale by a power of two (exact) so that max |w| is in [1, 2): squares
    // neither overflow nor underflow for any finite FP32 input.
    amax = block_max<NT>(amax, redf);
    const int ex = (amax > 0.0f && isfinite(amax)) ? ilogbf(amax) : 0;
    const float scale = ldexpf(1.0f, -ex), unscale = ldexpf(1.0f, ex);
    float fro = 0.0f;
    for (int s = tid; s < nslot; s += NT) {
        const int i = tri_row(s), j = s - i * (i + 1) / 2;
        const float w = sA[i * LD + j] * scale;
        sA[i * LD + j] = w;
        sA[j * LD + i] = w;
        fro += (i == j ? 1.0f : 2.0f) * w * w;
    }
    const float fro2 = block_sum<NT>(fro, redf);
    const float thr = kEps * kEps * fro2;

    for (int sweep = 0;; ++sweep) {
        float o = 0.0f;
        for (int idx = tid; idx < kk * kk; idx += NT) {
            const int i = idx / kk, j = idx - i * kk;
            if (i != j) {
                const float v = sA[i * LD + j];
                o += v * v;
            }
        }
        const float off2 = block_sum<NT>(o, redf);
        if (off2 <= thr) break;
        if (sweep >= kMaxSweeps) {
            if (tid == 0 && a.ctl != nullptr) atomicAdd(&a.ctl->jacobi_cap, 1);
            break;
        }
        for (int r = 0; r < kk - 1; ++r) {
            // Circle ordering: position 0 holds index 0, position j >= 1 holds
            // 1 + (j - 1 + r) mod (kk - 1); pair t joins positions t, kk-1-t.
            if (tid < np) {
                int P = (tid == 0) ? 0 : 1 + (tid - 1 + r) % (kk - 1);
                int Q = 1 + (kk - 2 - tid + r) % (kk - 1);
                if (P > Q) {
                    const int tmp = P;
                    P = Q;
                    Q = tmp;
                }
                const float apq = sA[P * LD + Q];
                float c = 1.0f, s = 0.0f, ta = 0.0f;
                if (apq != 0.0f) {
                    const float app = sA[P * LD + P], aqq = sA[Q * LD + Q];
                    const float tau = (aqq - app) / (2.0f * apq);
                    const float t = copysignf(1.0f, tau) / (fabsf(tau) + sqrtf(1.0f + tau * tau));
                    c = 1.0f / sqrtf(1.0f + t * t);
                    s = t * c;
                    ta = t * apq;
                }
                sP[tid] = P;
                sQ[tid] = Q;
                sC[tid] = c;
                sS[tid] = s;
                sT[tid] = ta;
            }
            __syncthreads();
            // A <- J^T A J by 2x2 blocks (rows of pair I, columns of pair J);
            // every element belongs to exactly one block, so this is in place.
            for (int it = tid; it < np * np; it += NT) {
                const int I = it / np, J = it - I * np;
                const int p1 = sP[I], q1 = sQ[I];
                if (I == J) {
                    const float ta = sT[I];
                    sA[p1 * LD + p1] -= ta;
                    sA[q1 * LD + q1] += ta;
                    sA[p1 * LD + q1] = 0.0f;
                    sA[q1 * LD + p1] = 0.0f;
                } else {
                    const int p2 = sP[J], q2 = sQ[J];
                    const float c1 = sC[I], s1 = sS[I], c2 = sC[J], s2 = sS[J];
                    const float a00 = sA[p1 * LD + p2], a01 = sA[p1 * LD + q2];
                    const float a10 = sA[q1 * LD + p2], a11 = sA[q1 * LD + q2];
                    const float b00 = c1 * a00 - s1 * a10, b01 = c1 * a01 - s1 * a11;
                    const float b10 = s1 * a00 + c1 * a10, b11 = s1 * a01 + c1 * a11;
                    sA[p1 * LD + p2] = c2 * b00 - s2 * b01;
                    sA[p1 * LD + q2] = s2 * b00 + c2 * b01;
                    sA[q1 * LD + p2] = c2 * b10 - s2 * b11;
                    sA[q1 * LD + q2] = s2 * b10 + c2 * b11;
                }
            }
            // V <- V J
            for (int it = tid; it < kk * np; it += NT) {
                const int row = it / np, J = it - row * np;
                const int p2 = sP[J], q2 = sQ[J];
                const float c2 = sC[J], s2 = sS[J];
                const float vp = sV[row * LD + p2], vq = sV[row * LD + q2];
                sV[row * LD + p2] = c2 * vp - s2 * vq;
                sV[row * LD + q2] = s2 * vp + c2 * vq;
            }
            __syncthreads();
        }
    }

    if (tid < kk) {
        const float l = sA[tid * LD + tid] * unscale;
        sLam[tid] = l;
        sLp[tid] = fmaxf(l, 0.0f);
    }
    // E = V^T V - I
    for (int idx = tid; idx < kk * kk; idx += NT) {
        const int i = idx / kk, j = idx - i * kk;
        float acc = 0.0f;
        for (int r = 0; r < kk; ++r) acc += sV[r * LD + i] * sV[r * LD + j];
        sX[i * LD + j] = acc - (i == j ? 1.0f : 0.0f);
    }
    __syncthreads();
    // Vn = V - V E / 2, stored over A (only its diagonal was still needed)
    for (int idx = tid; idx < kk * kk; idx += NT) {
        const int r = idx / kk, j = idx - r * kk;
        float acc = 0.0f;
        for (int i = 0; i < kk; ++i) acc += sV[r * LD + i] * sX[i * LD + j];
        sA[r * LD + j] = sV[r * LD + j] - 0.5f * acc;
    }
    __syncthreads();

    // Rebuild P = Vn max(Lambda, 0) Vn^T on the packed lower triangle.
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int s = tid; s < nslot; s += NT) {
        const int i = tri_row(s), j = s - i * (i + 1) / 2;
        float acc = 0.0f;
        for (int t = 0; t < k; ++t) acc += sA[i * LD + t] * sLp[t] * sA[j * LD + t];
        const int64_t g = off + s;
        if (a.mode == PROJ_STANDALONE) {
            a.Pout[g] = acc;
        } else if (a.mode == PROJ_PRIMAL) {
            const double hx = a.x[a.gather[g]];
            const double pv = (double)acc;
            a.lam[g] = (float)((double)a.lam[g] + a.rho * (pv - hx));
            a.blk[g] = acc;
            const double wgt = (i == j) ? 1.0 : 2.0;
            const double d = pv - hx;
            p0 += wgt * d * d;
            p1 += wgt * hx * hx;
            p2 += wgt * pv * pv;
        } else {
            a.blk[g] = acc;
        }
    }
    if (a.mode == PROJ_PRIMAL) {
        p0 = block_sum<NT>(p0, redd);
        p1 = block_sum<NT>(p1, redd);
        p2 = block_sum<NT>(p2, redd);
        if (tid == 0) {
            a.cpart[4 * (int64_t)id + 0] = p0;
            a.cpart[4 * (int64_t)id + 1] = p1;
            a.cpart[4 * (int64_t)id + 2] = p2;
        }
    }
    if (a.mode == PROJ_STANDALONE) {
        if (a.evals != nullptr)
            for (int t = tid; t < k; t += NT) a.evals[a.eoff[id] + t] = sLam[t];
        if (a.evecs != nullptr)
            for (int idx = tid; idx < k * k; idx += NT) {
                const int i = idx / k, j = idx - i * k;
                a.evecs[a.voff[id] + idx] = sA[i * LD + j];
            }
    }
}

template <int S, int NT>
void launch_t(const ProjArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_project<S, NT>), dim3(a.nblk), dim3(NT), 0, s, a);
}

}  // namespace

void launch_project(const ProjArgs &a, int smax, int nthreads, hipStream_t s) {
    if (a.nblk <= 0) return;
    if (smax <= 32) {
        if (nthreads <= 64) launch_t<32, 64>(a, s);
        else if (nthreads <= 128) launch_t<32, 128>(a, s);
        else launch_t<32, 256>(a, s);
    } else if (smax <= 64) {
        if (nthreads <= 128) launch_t<64, 128>(a, s);
        else launch_t<64, 256>(a, s);
    } else {
        if (nthreads <= 256) launch_t<96, 256>(a, s);
        else launch_t<96, 512>(a, s);
    }
}

}  // namespace cdcs
