// Projection onto the PSD cone for cliques too large for one workgroup's LDS
// (more than 126 vertices; the paper's Table I has cliques of 322 and 323).
//
// P_+(W) = W (I + sign(W)) / 2 (Higham, "Functions of Matrices", ch. 5), so
// the projection needs the matrix sign function, not an eigendecomposition.
// sign(W) comes from the Newton-Schulz iteration
//     X_0 = W / ||W||_F,   X_{t+1} = X_t (3 I - X_t^2) / 2,
// which converges to sign(W) for ||X_0||_2 < sqrt(3) (every step maps an
// eigenvalue s to s (3 - s^2) / 2: quadratically near +-1, by a factor 3/2
// per step while |s| is small).  Every step is two products of k x k FP32
// matrices on the matrix cores, tiled over many workgroups, so a large clique
// is spread across the GPU.  At most kNsSteps = 48 steps take every
// eigenvalue with |lambda| >= 2e-7 ||W||_F to within rounding of +-1; a
// smaller eigenvalue contributes at most |lambda| / 2 to the error of P.  A
// clique stops earlier, after at least kNsMin = 20 steps, once a step changed
// X by at most kNsTol = 3e-5 ||X||_F: then the next step's error is near FP32
// rounding for the eigenvalues near +-1 (the convergence is quadratic there),
// and an eigenvalue still in the linear phase (growing by 3/2 a step) has a
// scaled size below 2 kNsTol sqrt(N) / 1.5^20 <= 3e-7, so it adds at most
// that fraction of ||W||_F to the error of P, as the 48-step bound allows.
// The step at which a clique stopped is recorded (stop[c]); its later
// launches return at once and the final product reads X of that step.
// (The product's FP32 rounding leaves X a few ulps off sign(W); each step
// squares the previous deviation, so it does not accumulate.)  A NaN or Inf
// in W reaches the residual sums, which report it.
//
// Layout: each large clique c has an N x N row-major FP32 block (N = its size
// rounded up to 64, zero padded) in four buffers: W, two iterates and one
// product; launches cover every large clique at once (grid: 64 x 64 tiles x
// cliques), and all reductions are fixed-order (no atomics).  Every matrix of
// the iteration is a polynomial in W, so all of them are symmetric and all
// products commute: a launch computes only the tiles on and below the
// diagonal, T (T + 1) / 2 of the T^2, and writes each off-diagonal tile to
// its mirror position as well (the diagonal tiles keep their lower triangle
// and mirror it), so every matrix of the iteration is exactly symmetric.
#include <cmath>

#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kNT = 256;
constexpr int kTile = 64;
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Workgroup sum in fixed order; the result is valid in thread 0.
__device__ __forceinline__ double block_sum0(double v, double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum_d(v);
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kNT / 64; ++i) r += red[i];
    return r;
}

constexpr int kNsMin = 20;
constexpr double kNsTol2 = 9e-10;  // kNsTol^2

// Lower tile t (row-major over ti >= tj) -> (ti, tj).
__device__ __forceinline__ void lower_tile(int t, int &ti, int &tj) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    ti = i;
    tj = t - i * (i + 1) / 2;
}

__device__ __forceinline__ bool big_skip(const ProjArgs &a, int id) {
    if (a.ctl != nullptr && a.ctl->stop) return true;
    return a.istop != nullptr && a.istop[a.kinst[id]];
}

// Whether clique c's Newton-Schulz iteration has stopped before step `step`:
// at least kNsMin steps done and the last one moved X by at most kNsTol
// ||X||_F (per-tile partial sums of that step, in tile order; the same
// answer in every thread).  Partial sums alternate between two regions by
// step parity, so a launch reads the previous step's while writing its own.
__device__ __forceinline__ bool ns_stopped(const BigCliques &b, int c, int T, int step) {
    if (step < kNsMin) return false;
    const double *q = b.part + 4 * (int64_t)c * b.tmax2 + 2 * ((step - 1) & 1);
    double d2 = 0.0, x2 = 0.0;
    for (int t = 0; t < T * (T + 1) / 2; ++t) {
        d2 += q[4 * t + 0];
        x2 += q[4 * t + 1];
    }
    return d2 <= kNsTol2 * x2;
}

// W of clique c into its N x N block (both triangles, zero padding) from the
// projection's source, and per-tile partial sums of ||W||_F^2.
__global__ __launch_bounds__(kNT) void k_big_gather(ProjArgs a, BigCliques b) {
    __shared__ double red[kNT / 64];
    const int c = blockIdx.y;
    const int id = b.ids[c];
    if (big_skip(a, id)) return;
    const int n = b.n[c], N = b.N[c], T = N / kTile;
    const int t = blockIdx.x;
    if (t >= T * (T + 1) / 2) return;
    int ti, tj;
    lower_tile(t, ti, tj);
    const int64_t off = a.off[id];
    float *W = b.W + b.boff[c];
    double s2 = 0.0;
    for (int e = threadIdx.x; e < kTile * kTile; e += kNT) {
        const int i = ti * kTile + e / kTile, j = tj * kTile + e % kTile;
        float w = 0.0f;
        if (i < n && j < n) {
            const int r = max(i, j), q = min(i, j);
            const int64_t g = off + (int64_t)r * (r + 1) / 2 + q;
            if (a.mode == PROJ_STANDALONE) w = a.Win[g];
            else if (a.mode == PROJ_PRIMAL) w = (float)(a.x[a.gather[g]] - (double)a.lam[g] * a.inv_rho);
            else w = (float)((double)a.v[g] - (double)a.lam[g] * a.inv_rho);
        }
        W[(int64_t)i * N + j] = w;
        if (ti != tj) W[(int64_t)j * N + i] = w;
        s2 += (double)w * (double)w;
    }
    if (t == 0 && threadIdx.x == 0) b.stop[c] = -1;
    s2 = block_sum0(s2, red);
    // an off-diagonal tile stands for its mirror too
    if (threadIdx.x == 0) b.part[(int64_t)c * b.tmax2 + t] = (ti != tj) ? 2.0 * s2 : s2;
}

// ||W||_F from the tile partials (in tile order); 1 / ||W||_F for the scaling.
__global__ __launch_bounds__(64) void k_big_norm(ProjArgs a, BigCliques b) {
    const int c = blockIdx.x;
    if (big_skip(a, b.ids[c])) return;
    const int T = b.N[c] / kTile;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < T * (T + 1) / 2; ++t) s += b.part[(int64_t)c * b.tmax2 + t];
        const double fro = sqrt(s);
        b.inv_norm[c] = fro > 0.0 ? 1.0 / fro : 0.0;
    }
}

// X_0 = W / ||W||_F
__global__ __launch_bounds__(kNT) void k_big_scale(ProjArgs a, BigCliques b) {
    const int c = blockIdx.y;
    if (big_skip(a, b.ids[c])) return;
    const int N = b.N[c];
    const int64_t NN = (int64_t)N * N;
    const float sc = (float)b.inv_norm[c];
    const float *W = b.W + b.boff[c];
    float *X = b.X0 + b.boff[c];
    for (int64_t e = (int64_t)blockIdx.x * kNT + threadIdx.x; e < NN; e += (int64_t)gridDim.x * kNT) X[e] = W[e] * sc;
}

// One 64 x 64 tile (on or below the diagonal) of C = A B for every large
// clique (N x N blocks, N a multiple of 64), on v_mfma_f32_16x16x4_f32: wave
// w computes the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 instruction tiles.
// 32-deep slices of A and B are staged in LDS; the next slice's global loads
// are issued before the current slice's products, so they overlap.  An
// off-diagonal tile is also written to its mirror position.  Epilogue EPI:
// 0: C = A B; 1 (a Newton-Schulz step, A = X, B = X^2): C = 1.5 A - 0.5 A B;
// 2 (the projection, A = W, B = sign(W)): C = (A + A B) / 2.  Operand layout
// of the instruction (lane l): A[l % 16][l / 16], B[l / 16][l % 16]; result
// element r at D[(l / 16) * 4 + r][l % 16].  The upper triangle is written
// as the mirror of the lower one (also inside the diagonal tiles).
constexpr int kK = 32;
template <int EPI>
__global__ __launch_bounds__(kNT) void k_big_gemm(ProjArgs a, BigCliques b, const float *__restrict__ Ab,
                                                  const float *__restrict__ Bb, float *__restrict__ Cb, int step,
                                                  const float *__restrict__ Xalt) {
    __shared__ float As[kTile][kK + 1];
    __shared__ float Bs[kK][kTile + 1];
    __shared__ double red[kNT / 64];
    const int c = blockIdx.y;
    if (big_skip(a, b.ids[c])) return;
    const int N = b.N[c], T = N / kTile;
    const int t = blockIdx.x;
    if (t >= T * (T + 1) / 2) return;
    int ti, tj;
    lower_tile(t, ti, tj);
    const int64_t o = b.boff[c];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int stopped = b.stop[c];  // step at which the clique stopped, or -1
    if (EPI == 0 && stopped < 0 && ns_stopped(b, c, T, step)) {
        if (t == 0 && tid == 0) b.stop[c] = step;  // X of this step (buffer step & 1) is the sign
        return;
    }
    if (EPI != 2 && stopped >= 0) return;
    // the final product reads X of the stopping step (the other buffer when
    // that step had the other parity than kNsSteps)
    const float *A = Ab + o, *B = ((EPI == 2 && stopped >= 0 && ((stopped ^ step) & 1)) ? Xalt : Bb) + o;
    float *C = Cb + o;
    double *np = b.part + 4 * ((int64_t)c * b.tmax2 + t) + 2 * (step & 1);  // this step's partial sums
    const int qr = w >> 1, qc = w & 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni) acc[mi][ni] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int ar = tid >> 2, ac = (tid & 3) * 8;   // A slice: 64 rows x 32 columns, 8 per thread
    const int br = tid >> 3, bc = (tid & 7) * 8;   // B slice: 32 rows x 64 columns, 8 per thread
    const float *pa = A + (int64_t)(ti * kTile + ar) * N + ac;
    const float *pb = B + (int64_t)br * N + tj * kTile + bc;
    f32x4 av0 = *reinterpret_cast<const f32x4 *>(pa), av1 = *reinterpret_cast<const f32x4 *>(pa + 4);
    f32x4 bv0 = *reinterpret_cast<const f32x4 *>(pb), bv1 = *reinterpret_cast<const f32x4 *>(pb + 4);
    for (int k0 = 0; k0 < N; k0 += kK) {
        __syncthreads();  // the previous slice's products are done with LDS
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[ar][ac + q] = av0[q];
            As[ar][ac + 4 + q] = av1[q];
            Bs[br][bc + q] = bv0[q];
            Bs[br][bc + 4 + q] = bv1[q];
        }
        __syncthreads();
        if (k0 + kK < N) {  // next slice in flight during this slice's products
            const float *qa = pa + k0 + kK, *qb = pb + (int64_t)(k0 + kK) * N;
            av0 = *reinterpret_cast<const f32x4 *>(qa);
            av1 = *reinterpret_cast<const f32x4 *>(qa + 4);
            bv0 = *reinterpret_cast<const f32x4 *>(qb);
            bv1 = *reinterpret_cast<const f32x4 *>(qb + 4);
        }
#pragma unroll
        for (int kk = 0; kk < kK; kk += 4) {
            float am[2], bm[2];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) am[mi] = As[qr * 32 + mi * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) bm[ni] = Bs[kk + (lane >> 4)][qc * 32 + ni * 16 + (lane & 15)];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(am[mi], bm[ni], acc[mi][ni], 0, 0, 0);
        }
    }
    double d2 = 0.0, x2 = 0.0;  // EPI 1: ||X_new - X||^2 and ||X_new||^2 of the tile
    // Only the lower triangle is kept and mirrored, the diagonal tiles' too:
    // the computed A B is symmetric only up to rounding, and a matrix whose
    // diagonal tiles kept their own upper triangles next to mirrored
    // off-diagonal tiles is not symmetric; the Newton-Schulz map does not damp
    // an antisymmetric part (it grew to 2e-3 of X over 48 steps in a host
    // emulation of that mix, against 3e-7 for the exactly symmetric one).
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ti * kTile + qr * 32 + mi * 16 + (lane >> 4) * 4 + r;
                const int col = tj * kTile + qc * 32 + ni * 16 + (lane & 15);
                if (row < col) continue;
                const int64_t e = (int64_t)row * N + col;
                const float v = acc[mi][ni][r];
                float out;
                if (EPI == 0) {
                    out = v;
                } else if (EPI == 1) {
                    const float x = A[e];
                    out = 1.5f * x - 0.5f * v;
                    const double wgt = row > col ? 2.0 : 1.0, dd = (double)out - (double)x;
                    d2 += wgt * dd * dd;
                    x2 += wgt * (double)out * (double)out;
                } else {
                    out = 0.5f * (A[e] + v);
                }
                C[e] = out;
                if (row > col) C[(int64_t)col * N + row] = out;
            }
    if (EPI == 1) {
        d2 = block_sum0(d2, red);
        x2 = block_sum0(x2, red);
        if (tid == 0) {
            np[0] = d2;
            np[1] = x2;
            // one Newton-Schulz step of this clique counted with the sweeps
            if (t == 0 && a.ctl != nullptr) atomicAdd(&a.ctl->sweeps, 1);
        }
    }
}

// The projection's epilogue for large cliques, as for the LDS-resident ones:
// P (symmetrised) to the packed outputs, the multiplier update of Algorithm 1
// and per-tile residual partial sums (grid: lower tiles x cliques; the slots
// (i, j), j <= i, of a tile).
__global__ __launch_bounds__(kNT) void k_big_epilogue(ProjArgs a, BigCliques b, const float *__restrict__ Pb) {
    __shared__ double red[kNT / 64];
    const int c = blockIdx.y;
    const int id = b.ids[c];
    if (big_skip(a, id)) return;
    const int n = b.n[c], N = b.N[c], T = N / kTile;
    const int t = blockIdx.x;
    if (t >= T * (T + 1) / 2) return;
    int ti, tj;
    lower_tile(t, ti, tj);
    const float *P = Pb + b.boff[c];
    const int64_t off = a.off[id];
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int e = threadIdx.x; e < kTile * kTile; e += kNT) {
        const int i = ti * kTile + e / kTile, j = tj * kTile + e % kTile;
        if (i >= n || j > i) continue;
        const float pv32 = 0.5f * (P[(int64_t)i * N + j] + P[(int64_t)j * N + i]);
        const int64_t g = off + (int64_t)i * (i + 1) / 2 + j;
        if (a.mode == PROJ_STANDALONE) {
            a.Pout[g] = pv32;
        } else if (a.mode == PROJ_PRIMAL) {
            const double hx = a.x[a.gather[g]];
            const double pv = (double)pv32;
            a.lam[g] = (float)((double)a.lam[g] + a.rho * (pv - hx));
            if (a.dslot != nullptr) a.dslot[g] = (float)(pv - (double)a.blk[g]);
            a.blk[g] = pv32;
            const double wgt = (i == j) ? 1.0 : 2.0;
            const double d = pv - hx;
            p0 += wgt * d * d;
            p1 += wgt * hx * hx;
            p2 += wgt * pv * pv;
        } else {
            a.blk[g] = pv32;
        }
    }
    if (a.mode == PROJ_PRIMAL) {
        p0 = block_sum0(p0, red);
        p1 = block_sum0(p1, red);
        p2 = block_sum0(p2, red);
        if (threadIdx.x == 0) {
            double *q = b.part + 3 * ((int64_t)c * b.tmax2 + t);
            q[0] = p0;
            q[1] = p1;
            q[2] = p2;
        }
    }
}

// The residual partial sums of each large clique from its tiles (tile order).
__global__ __launch_bounds__(64) void k_big_epi_sum(ProjArgs a, BigCliques b) {
    const int c = blockIdx.x;
    const int id = b.ids[c];
    if (big_skip(a, id) || a.mode != PROJ_PRIMAL) return;
    const int T = b.N[c] / kTile;
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int t = 0; t < T * (T + 1) / 2; ++t) {
            const double *q = b.part + 3 * ((int64_t)c * b.tmax2 + t);
            s0 += q[0];
            s1 += q[1];
            s2 += q[2];
        }
        a.cpart[4 * (int64_t)id + 0] = s0;
        a.cpart[4 * (int64_t)id + 1] = s1;
        a.cpart[4 * (int64_t)id + 2] = s2;
    }
}

}  // namespace

void launch_big_projection(const ProjArgs &a, const BigCliques &b, hipStream_t s) {
    if (b.nbig <= 0) return;
    const int tm = (int)std::lround(std::sqrt((double)b.tmax2));
    const dim3 tiles((unsigned)(tm * (tm + 1) / 2), (unsigned)b.nbig);
    hipLaunchKernelGGL(k_big_gather, tiles, dim3(kNT), 0, s, a, b);
    hipLaunchKernelGGL(k_big_norm, dim3((unsigned)b.nbig), dim3(64), 0, s, a, b);
    hipLaunchKernelGGL(k_big_scale, dim3(64, (unsigned)b.nbig), dim3(kNT), 0, s, a, b);
    float *X[2] = {b.X0, b.X1};
    for (int t = 0; t < kNsSteps; ++t) {
        hipLaunchKernelGGL(k_big_gemm<0>, tiles, dim3(kNT), 0, s, a, b, (const float *)X[t & 1],
                           (const float *)X[t & 1], b.Y, t, (const float *)nullptr);
        hipLaunchKernelGGL(k_big_gemm<1>, tiles, dim3(kNT), 0, s, a, b, (const float *)X[t & 1],
                           (const float *)b.Y, X[(t + 1) & 1], t, (const float *)nullptr);
    }
    hipLaunchKernelGGL(k_big_gemm<2>, tiles, dim3(kNT), 0, s, a, b, (const float *)b.W,
                       (const float *)X[kNsSteps & 1], b.Y, kNsSteps, (const float *)X[(kNsSteps + 1) & 1]);
    hipLaunchKernelGGL(k_big_epilogue, tiles, dim3(kNT), 0, s, a, b, (const float *)b.Y);
    hipLaunchKernelGGL(k_big_epi_sum, dim3((unsigned)b.nbig), dim3(64), 0, s, a, b);
}

}  // namespace cdcs
