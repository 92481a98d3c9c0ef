// Batched projection onto the product of small PSD cones (paper: Sec. III-B.2,
// (E:XkUpdate); Sec. IV-B.2, (E:zkUpdate)), fused with the gather from the
// global vector and, for Algorithm 1, the multiplier update (E:LambdakUpdate)
// and the per-clique residual partial sums.
//
// One workgroup per clique.  Every clique of a size bucket is padded to the
// bucket size S (16, 32, ..., 128) with zero rows and columns (a zero pair
// never rotates), so all loops have compile-time trip counts.  Cliques of up
// to kMaxK = 126 vertices fit: the Jacobi runs on K = k rounded up to even
// positions, a wave lane holds two of them, and the odd steps' end pair needs
// one lane more than the K/2 pairs, so K/2 <= 63.  The clique matrix (FP32) lives in LDS
// and is diagonalised by two-sided Jacobi in the odd-even ordering: the
// disjoint pairs of a step are rotated together.  During the sweeps A is
// stored by position, as lower 2x2 pair blocks in four element planes, so a
// thread reads its blocks with unit-stride LDS accesses and writes the rotated
// elements straight to where the step's exchange moves them (two buffers,
// swapped every step); V stays in registers.  A step is two phases separated
// by barriers: one wave computes the rotations (and writes the pairs' new
// diagonal blocks), then every thread applies them to its fixed off-diagonal
// blocks of A and to its rows of V.  Sweeps
// stop when off(A) <= tau ||W||_F: the projection onto the PSD cone is
// 1-Lipschitz in the Frobenius norm, so rebuilding from the diagonal of a
// matrix whose off-diagonal part E remains moves P by at most ||E||_F.  Inside
// the ADMM loop tau = 2^-20 (error <= 1e-6 ||W||_F); when eigenpairs are
// returned (standalone calls with evals/evecs, used by the adjoint) tau = 2^-23.
//
// Warm start (ADMM modes): W changes little between iterations, so the kernel
// keeps each clique's eigenvector matrix V_prev and runs Jacobi on
// V_prev^T W V_prev, accumulating into V_prev.  Any orthogonal start gives the
// same eigendecomposition of W; a good one needs far fewer sweeps.
//
// FP32 accumulation of the eigenvectors loses orthogonality like
// sqrt(#rotations) eps, so one Newton-Schulz step V <- V - V (V^T V - I) / 2
// re-orthonormalises them before P = V max(Lambda, 0) V^T (products on the
// matrix cores for S >= 32, register tiles on the vector ALUs below).
#include <type_traits>

#include "cdcs_internal.h"

namespace cdcs {
namespace {

constexpr int kMaxSweeps = 30;
constexpr int kMaxK = 126;  // largest clique: K / 2 + 1 pairs in one 64-lane wave
constexpr float kTauEig = 1.1920928955078125e-07f;   // 2^-23: eigenpairs returned
constexpr float kTauProj = 9.5367431640625e-07f;     // 2^-20: projection only

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

// A value that is the same in every lane of the wave, moved to a scalar
// register so that branches and loop bounds on it are scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
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
    return uniform(r);
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
    return uniform(r);
}

// Row a of the packed lower-triangular slot s = a(a+1)/2 + b.
__device__ __forceinline__ int tri_row(int s) {
    int a = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)s + 1.0f) - 1.0f) * 0.5f);  // the loops below make it exact
    while ((a + 1) * (a + 2) / 2 <= s) ++a;
    while (a * (a + 1) / 2 > s) --a;
    return a;
}

// Odd-even ordering with swaps on K (even) positions.  Even steps pair
// positions (2i, 2i+1), i < K/2 (tiling 0); odd steps pair (2i-1, 2i), 1 <= i
// < K/2, and put positions 0 and K-1 in the end pairs (ghost, 0) and
// (K-1, ghost) with a ghost position that holds zeros (tiling 1, K/2 + 1
// pairs).  After every rotation the two positions of each pair exchange
// their contents, so over K steps every two positions meet once and the
// order is reversed.  Slot (t, h) is member h of pair t of a tiling.  After
// a step on tiling 0, the content of slot (t, h) sits in slot (t + 1 - h, h)
// of tiling 1; after a step on tiling 1, in slot (t - h, h) of tiling 0,
// except that what the rotation and swap move onto a ghost member, (0, 0) or
// (K/2, 1) of tiling 1, is dropped.

// Element offset (plane * nbs + block) of entry (slot (t1, g1), slot (t2, g2))
// of a symmetric matrix stored as lower 2x2 pair blocks in four planes
// (element e = 2 g_row + g_col of block I (I+1)/2 + J, I >= J).  Entries of an
// upper block are stored transposed; the off-diagonal entry of a diagonal
// block lives in element 2 only.
__device__ __forceinline__ int pair_slot(int t1, int g1, int t2, int g2, int nbs) {
    int I = t1, J = t2, e;
    if (t1 > t2) {
        e = 2 * g1 + g2;
    } else if (t1 < t2) {
        I = t2;
        J = t1;
        e = 2 * g2 + g1;
    } else {
        e = g1 == g2 ? 3 * g1 : 2;
    }
    return e * nbs + I * (I + 1) / 2 + J;
}

// Full-wave lane shifts: lane i receives lane i+1 (shl) or lane i-1 (shr);
// lane 63 of the left shift and lane 0 of the right shift read zero.
__device__ __forceinline__ float wave_shl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float wave_shr0(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}

// Register-tiled S x S products on a GR x GC thread grid (GR = 16 rows of
// threads, GC = NT / 16 columns): thread (ti, tj) owns rows ti*TR .. +TR and
// columns tj*TC .. +TC of the result (TR = S / 16, TC = ceil(S / GC); columns
// past S are computed from clamped loads and never stored).
template <int S, int NT>
struct Tiles {
    static constexpr int GR = 16, GC = NT / 16;
    static constexpr int TR = S / GR, TC = (S + GC - 1) / GC;
};

// mode 0: C = X^T Y   (C[i][j] = sum_q X[q][i] Y[q][j])
// mode 1: C = X Y     (C[i][j] = sum_q X[i][q] Y[q][j])
// mode 2: C = X Y^T   (C[i][j] = sum_q X[i][q] Y[j][q])
// Sums run over q < n (n <= S; the rest of X and Y is zero padding).  With
// lp, the X operand of mode 2 is scaled by lp[q] (C = X diag(lp) Y^T).
template <int S, int NT, int MODE>
__device__ __forceinline__ void tile_product(const float *X, const float *Y,
                                             float (&acc)[Tiles<S, NT>::TR][Tiles<S, NT>::TC], int ti, int tj,
                                             int n = S, const float *lp = nullptr) {
    constexpr int LD = S + 1, TR = Tiles<S, NT>::TR, TC = Tiles<S, NT>::TC;
#pragma unroll
    for (int u = 0; u < TR; ++u)
#pragma unroll
        for (int v = 0; v < TC; ++v) acc[u][v] = 0.0f;
#pragma unroll 4
    for (int q = 0; q < n; ++q) {
        float xa[TR], yb[TC];
#pragma unroll
        for (int u = 0; u < TR; ++u) xa[u] = MODE == 0 ? X[q * LD + ti * TR + u] : X[(ti * TR + u) * LD + q];
        if (lp != nullptr) {
            const float l = lp[q];
#pragma unroll
            for (int u = 0; u < TR; ++u) xa[u] *= l;
        }
#pragma unroll
        for (int v = 0; v < TC; ++v) {
            const int j = min(tj * TC + v, S - 1);
            yb[v] = MODE == 2 ? Y[j * LD + q] : Y[q * LD + j];
        }
#pragma unroll
        for (int u = 0; u < TR; ++u)
#pragma unroll
            for (int v = 0; v < TC; ++v) acc[u][v] += xa[u] * yb[v];
    }
}

// S x S products on FP32 matrix cores (v_mfma_f32_16x16x4_f32), buckets S >=
// 32.  The 16 x 16 output tiles (all T x T, or the T (T+1) / 2 on and below
// the diagonal when only the lower triangle of a symmetric result is needed)
// are dealt to the waves round-robin; a wave keeps the accumulators of its
// tiles and loads one A and one B operand per tile for every 4-deep slice.
// Operand layout of the instruction (lane l): A[l % 16][l / 16] (16 x 4),
// B[l / 16][l % 16] (4 x 16); result element r: D[(l / 16) * 4 + r][l % 16].
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int S, int NT, bool LOWER>
struct MfmaTiles {
    static constexpr int T = S / 16;
    static constexpr int NW = NT / 64;
    static constexpr int NTILE = LOWER ? T * (T + 1) / 2 : T * T;
    static constexpr int PER = (NTILE + NW - 1) / NW;  // tiles per wave, at most
};

// Tile t of the list -> tile row and column (uniform across the wave).
template <int T, bool LOWER>
__device__ __forceinline__ void tile_rc(int t, int &ti, int &tj) {
    if (LOWER) {
        ti = 0;
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = t / T;
        tj = t - ti * T;
    }
}

// C = X^T Y (mode 0), X Y (mode 1) or X diag(lp) Y^T (mode 2) over q < n, on
// this wave's tiles.  With a column list qi (mode 2 only), term q of the sum
// takes column qi[q] of X and Y (and lp[qi[q]]); qi must hold n rounded up to
// 8 entries.
template <int S, int NT, int MODE, bool LOWER>
__device__ __forceinline__ void mfma_product(const float *X, const float *Y, const float *lp, int n, int lane,
                                             int wv, f32x4 (&acc)[MfmaTiles<S, NT, LOWER>::PER],
                                             const int *qi = nullptr) {
    using MT = MfmaTiles<S, NT, LOWER>;
    constexpr int LD = S + 1, PER = MT::PER;
    const int lr = lane & 15, lk = lane >> 4;
    int ra[PER], cb[PER];  // this lane's A row and B column, per tile
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        int ti, tj;
        tile_rc<MT::T, LOWER>(min(wv + r * MT::NW, MT::NTILE - 1), ti, tj);
        ra[r] = ti * 16 + lr;
        cb[r] = tj * 16 + lr;
        acc[r] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    // Two 4-deep slices per iteration (n rounded up to 8 <= S; terms past n
    // are zero), so the second slice's loads overlap the first's products.
    const int n8 = (n + 7) & ~7;
    auto slice = [&](int q0) {
        const int q = (MODE == 2 && qi != nullptr) ? qi[q0 + lk] : q0 + lk;
        const float l = MODE == 2 ? lp[q] : 1.0f;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            if (wv + r * MT::NW >= MT::NTILE) continue;  // uniform
            float av = MODE == 0 ? X[q * LD + ra[r]] : X[ra[r] * LD + q];
            if (MODE == 2) av *= l;
            const float bv = MODE == 2 ? Y[cb[r] * LD + q] : Y[q * LD + cb[r]];
            acc[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[r], 0, 0, 0);
        }
    };
    for (int q0 = 0; q0 < n8; q0 += 8) {
        slice(q0);
        slice(q0 + 4);
    }
}

// Compute an S x S product (matrix cores for S >= 32, register tiles on the
// vector ALUs below), wait until every thread has read its operands, then
// hand each result element to st(row, col, value): the result may overwrite
// an operand.  The caller synchronises before reading what st wrote.  LOWER:
// only elements on and below the diagonal of a symmetric result are needed
// (the matrix-core path then computes only the tiles on and below the
// diagonal and may skip the others; MIRROR also hands over their transposes).
template <int S, int NT, int MODE, bool LOWER = false, bool MIRROR = false, typename Store>
__device__ __forceinline__ void product_store(const float *X, const float *Y, const float *lp, int n, int tid,
                                              Store st, const int *qi = nullptr) {
    if constexpr (S >= 32) {
        using MT = MfmaTiles<S, NT, LOWER>;
        const int lane = tid & 63, wv = uniform(tid >> 6);
        f32x4 acc[MT::PER];
        mfma_product<S, NT, MODE, LOWER>(X, Y, lp, n, lane, wv, acc, qi);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < MT::PER; ++r) {
            const int t = wv + r * MT::NW;
            if (t >= MT::NTILE) continue;
            int ti, tj;
            tile_rc<MT::T, LOWER>(t, ti, tj);
            const int col = tj * 16 + (lane & 15);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int row = ti * 16 + (lane >> 4) * 4 + rr;
                st(row, col, acc[r][rr]);
                if (MIRROR && ti != tj) st(col, row, acc[r][rr]);
            }
        }
    } else {
        using TL = Tiles<S, NT>;
        const int ti = tid / TL::GC, tj = tid % TL::GC;
        float acc[TL::TR][TL::TC];
        tile_product<S, NT, MODE>(X, Y, acc, ti, tj, n, MODE == 2 ? lp : nullptr);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < TL::TR; ++u)
#pragma unroll
            for (int v = 0; v < TL::TC; ++v)
                if (tj * TL::TC + v < S) st(ti * TL::TR + u, tj * TL::TC + v, acc[u][v]);
    }
}

// Small per-workgroup LDS of the projection (sized for the largest bucket).
struct ProjSmall {
    union {
        float2 cst[64];          // rotations of one step: (c, s) of pair t (8-byte stride: the reads of
                                 // consecutive pairs fall in distinct bank pairs)
        int pidx[128];           // after the sweeps: indices of the positive eigenvalues, then the others
    };
    int npos[2];                 // positive eigenvalues counted by waves 0 and 1
    float lam[128], lp[128];     // eigenvalues, clamped eigenvalues
    float redf[8];
    double redd[24];             // three FP64 partial sums per wave
    int zero;                    // 0; read as volatile (see project_one)
};

// Projection of clique `id` by one workgroup of NT threads, cliques padded to
// S.  sA and sV are S x (S+1) FP32 LDS arrays.
template <int S, int NT>
__device__ __forceinline__ void project_one(const ProjArgs &a, int id, float *__restrict__ sA,
                                            float *__restrict__ sV, ProjSmall &sm) {
    static_assert(S % 16 == 0 && S <= 128, "bucket size");
    static_assert(NT == 64 || NT == 256 || NT == 512, "workgroup size");
    constexpr int LD = S + 1;                    // odd row stride
    constexpr int HMAX = S / 2;                  // pairs per step, at most
    constexpr int NBS = (HMAX + 1) * (HMAX + 2) / 2;           // 2x2 blocks of a tiling, at most
    constexpr int NA = (NBS + NT - 1) / NT;                    // blocks per thread, at most
    constexpr int NW = NT / 64;                  // waves
    constexpr int RPW = (S + NW - 1) / NW;       // rows of V per wave, at most

    if (a.istop != nullptr && a.istop[a.kinst[id]]) return;  // instance already stopped
    const int k = uniform(a.size[id]);
    if (k < 1 || k > S || k > kMaxK) return;
    const int64_t off = a.off[id];
    const int nslot = k * (k + 1) / 2;
    // The thread index goes through a volatile LDS zero so that the compiler
    // cannot hoist the per-thread work tables out of a queue launch's clique
    // loop (which would keep them live across all cliques and buckets).
    const int tid = threadIdx.x + *(volatile int *)&sm.zero;
    const bool warm = a.vwarm != nullptr;
    float *vw = warm ? a.vwarm + a.vwoff[id] : nullptr;

    // A <- 0; V <- V_prev (warm start) or I, padded with the identity.  All
    // of a thread's V_prev loads are issued before its first store.
    constexpr int NI = (S * S + NT - 1) / NT;
    float vv[NI];
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        const int idx = tid + r * NT, i = idx / S, j = idx % S;
        vv[r] = (i == j) ? 1.0f : 0.0f;
        if (warm && idx < S * S && i < k && j < k) vv[r] = vw[i * k + j];
    }
#pragma unroll
    for (int r = 0; r < NI; ++r) {
        const int idx = tid + r * NT, i = idx / S, j = idx % S;
        if (idx < S * S) {
            sA[i * LD + j] = 0.0f;
            sV[i * LD + j] = vv[r];
        }
    }
    __syncthreads();

    // Gather W (packed lower triangle of the k x k block).  Each thread
    // loads GU slots before storing any, so their memory latencies overlap
    // (indices past the block are clamped for the loads and not stored).
    constexpr int GU = 4;
    float amax = 0.0f;
    for (int s0 = tid; s0 < nslot; s0 += GU * NT) {
        float w[GU];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int64_t g = off + min(s0 + u * NT, nslot - 1);
            if (a.mode == PROJ_STANDALONE) {
                w[u] = a.Win[g];
            } else if (a.mode == PROJ_PRIMAL) {
                const double hx = a.x[a.gather[g]];
                w[u] = (float)(hx - (double)a.lam[g] * a.inv_rho);
            } else {
                w[u] = (float)((double)a.v[g] - (double)a.lam[g] * a.inv_rho);
            }
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int s = s0 + u * NT;
            if (s < nslot) {
                const int i = tri_row(s), j = s - i * (i + 1) / 2;
                sA[i * LD + j] = w[u];
                sA[j * LD + i] = w[u];
                amax = fmaxf(amax, fabsf(w[u]));
            }
        }
    }
    // Scale by a power of two (exact) so that max |w| lies in [1, 2): squares
    // neither overflow nor underflow for any finite FP32 input.
    amax = block_max<NT>(amax, sm.redf);
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
    const float fro2 = block_sum<NT>(fro, sm.redf);
    // standalone calls that return eigenpairs converge them to 2^-23; the
    // ADMM modes keep the loop's rule also when they save eigenpairs (for the
    // adjoint of an unrolled iteration), so that iteration is the loop's own
    const float tau = (a.mode == PROJ_STANDALONE && (a.evals != nullptr || a.evecs != nullptr)) ? kTauEig : kTauProj;
    const float thr = tau * tau * fro2;

    const int Kw = k + (k & 1);  // products run over the active size
    auto to_sA = [&](int i, int j, float v) { sA[i * LD + j] = v; };
    if (warm) {
        // A <- V^T W V (V = V_prev, orthonormal to FP32 accuracy); the
        // eigensolver reads only its lower triangle.
        product_store<S, NT, 1>(sA, sV, nullptr, Kw, tid, to_sA);        // W V
        __syncthreads();
        product_store<S, NT, 0, true>(sV, sA, nullptr, Kw, tid, to_sA);  // V^T (W V)
        __syncthreads();
    }

    // Jacobi on the K = k rounded up to even leading indices (one zero
    // padding row and column for odd k; the rest of the bucket is not
    // touched), in the odd-even ordering: a sweep is K steps, even steps on
    // tiling 0 and odd steps on tiling 1.  The end pairs of tiling 1 hold a
    // ghost position and rotate by (c, s) = (0, -1) and (0, 1): with the swap
    // that leaves the real position as it is and the ghost at zero.  A is
    // kept by position as the lower 2x2 pair blocks of the current tiling in
    // four element planes; a step reads one buffer and writes each rotated
    // element straight to its slot of the other tiling in the other buffer
    // (ghost entries go to a dummy slot).  Those addresses are set once per
    // eigensolve.  V is kept by position in registers (lane i: positions 2i
    // and 2i+1).  After an odd number of sweeps position p holds index K-1-p.
    const int K = k + (k & 1);
    const int HK = K >> 1;
    const int nblk0 = HK * (HK + 1) / 2, nblk1 = (HK + 1) * (HK + 2) / 2;
    constexpr int PL = NBS * 4;          // plane stride in bytes
    constexpr int DUMMY = 4 * NBS * 4;   // write-only slot for ghost entries
    static_assert(4 * NBS + 1 <= S * LD, "a pair-block buffer fits in an S x (S+1) array");
    // Byte offset in tiling 1-T of element e (= 2 h_row + h_col) of block
    // (I, J) of tiling T after the rotation and the swap.
    auto move_to = [&](int T, int I, int J, int e) {
        const int h1 = e >> 1, h2 = e & 1;  // members of the row and the column
        if (T == 0) return pair_slot(I + 1 - h1, h1, J + 1 - h2, h2, NBS) * 4;
        // ghost members of the end pairs (their contents come from the ghost)
        if ((I == 0 && h1 == 1) || (I == HK && h1 == 0) || (J == 0 && h2 == 1) || (J == HK && h2 == 0)) return DUMMY;
        return pair_slot(I - h1, h1, J - h2, h2, NBS) * 4;
    };
    // Blocks of this thread (the same lower-triangle numbering in both
    // tilings): pair indices and, per tiling, where the four rotated
    // elements go.  The diagonal block of a real pair is written by the
    // thread that computes that pair's rotation (thread t: pair t), with the
    // targets in dgo; element 1 of a diagonal block is not kept (it equals
    // element 2; in tiling 1 the ghost pairs' element 1 stays zero).
    int bI[NA], bJ[NA], dst[2][NA][4], dgo[2][3];
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int b = tid + q * NT;
        const int bc = min(b, nblk1 - 1);
        const int I = tri_row(bc), J = bc - I * (I + 1) / 2;
        bI[q] = (b < nblk1) ? I : -1;
        bJ[q] = J;
#pragma unroll
        for (int T = 0; T < 2; ++T)
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[T][q][e] = move_to(T, I, J, e);
    }
    {
        const int t = min(tid, HK);
#pragma unroll
        for (int T = 0; T < 2; ++T) {
            dgo[T][0] = move_to(T, t, t, 0);
            dgo[T][1] = move_to(T, t, t, 2);
            dgo[T][2] = move_to(T, t, t, 3);
        }
    }
    // V in registers: the lane for pair i holds, for its rows (wave w: rows
    // w, w + NW, ...), the columns at positions 2i ("top") and 2i+1.  Buckets
    // up to 48 use at most 25 lanes per row, so a register carries two rows:
    // lanes 0-31 and 32-63 (lane 31 is never a pair's lane, so nothing a lane
    // shift carries across the halves reaches one; lane 32 is the ghost pair
    // of its row, which ignores what it receives).
    constexpr bool PACK = S <= 48;
    static_assert(!PACK || HMAX + 1 < 32, "two rows per register need a spare lane between them");
    constexpr int RV = PACK ? (RPW + 1) / 2 : RPW;  // V registers per wave
    const int lane = tid & 63, wv = uniform(tid >> 6);
    const int pi = PACK ? (lane & 31) : lane;  // pair of this lane
    const int half = PACK ? (lane >> 5) : 0;
    auto vrow = [&](int j) { return wv + (PACK ? 2 * j + half : j) * NW; };
    const bool vlane = pi < HK;
    float vt[RV], vb[RV];
#pragma unroll
    for (int j = 0; j < RV; ++j) {
        const int row = vrow(j);
        const bool ok = vlane && row < K;
        vt[j] = ok ? sV[row * LD + 2 * pi] : 0.0f;
        vb[j] = ok ? sV[row * LD + 2 * pi + 1] : 0.0f;
    }
    __syncthreads();  // sV is free: it becomes pair-block buffer 0
    char *const B0 = reinterpret_cast<char *>(sV);
    char *const B1 = reinterpret_cast<char *>(sA);
#define LF(ptr, off) (*reinterpret_cast<const float *>((ptr) + (off)))
#define SF(ptr, off) (*reinterpret_cast<float *>((ptr) + (off)))
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int b = tid + q * NT;
        if (b >= nblk0) continue;
        const int r = 2 * bI[q], c = 2 * bJ[q], b4 = b * 4;  // positions are indices at the start
        SF(B0, b4) = sA[r * LD + c];
        SF(B0, PL + b4) = sA[r * LD + c + 1];
        SF(B0, 2 * PL + b4) = sA[(r + 1) * LD + c];
        SF(B0, 3 * PL + b4) = sA[(r + 1) * LD + c + 1];
    }
    __syncthreads();
    for (int idx = tid; idx < 4 * NBS; idx += NT) SF(B1, idx * 4) = 0.0f;  // ghost slots of tiling 1 stay zero
    __syncthreads();

    // One rotation step on tiling T, from buffer `cur` into buffer `nxt`.
    auto step = [&](auto tiling, const char *__restrict__ cur, char *__restrict__ nxt) {
        constexpr int T = decltype(tiling)::value;
        const int npair = HK + T;
        if (tid < npair) {
            float c = 1.0f, s = 0.0f;
            if (T == 1 && (tid == 0 || tid == HK)) {
                c = 0.0f;
                s = tid == 0 ? -1.0f : 1.0f;
            } else {
                // Jacobi rotation of pair t; the new diagonal block (exact zero
                // off the diagonal) goes straight to the other tiling.
                const int bd = tid * (tid + 3) * 2;  // block (t, t), bytes
                const float app = LF(cur, bd), apq = LF(cur, 2 * PL + bd), aqq = LF(cur, 3 * PL + bd);
                float ta = 0.0f;
                if (fabsf(apq) > 1e-30f) {  // entries are scaled to max |a| ~ 1
                    // hardware rcp / sqrt / rsq (about 1 ulp): the step needs
                    // c^2 + s^2 = 1 to rounding, which c = rsq(1 + t^2) and
                    // s = t c give for any t, not a correctly rounded t
                    const float tau = 0.5f * (aqq - app) * __builtin_amdgcn_rcpf(apq);
                    const float t = copysignf(
                        __builtin_amdgcn_rcpf(fabsf(tau) + __builtin_amdgcn_sqrtf(1.0f + tau * tau)), tau);
                    c = __builtin_amdgcn_rsqf(1.0f + t * t);
                    s = t * c;
                    ta = t * apq;
                }
                SF(nxt, dgo[T][0]) = app - ta;
                SF(nxt, dgo[T][1]) = 0.0f;
                SF(nxt, dgo[T][2]) = aqq + ta;
            }
            sm.cst[tid] = make_float2(c, s);
        }
        __syncthreads();
        // A <- J^T A J on this thread's off-diagonal blocks (and the ghost
        // pairs' diagonal blocks, exact for their (0, +-1) rotations), swapped
        // and stored in the other tiling.
        const int nblk = T == 0 ? nblk0 : nblk1;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const int I = bI[q], J = bJ[q];
            if (tid + q * NT >= nblk || (I == J && (T == 0 || (I != 0 && I != HK)))) continue;
            const int b4 = (tid + q * NT) * 4;
            const float a00 = LF(cur, b4), a01 = LF(cur, PL + b4);
            const float a10 = LF(cur, 2 * PL + b4), a11 = LF(cur, 3 * PL + b4);
            const float2 cs1 = sm.cst[I];
            const float2 cs2 = sm.cst[J];
            const float c1 = cs1.x, s1 = cs1.y, c2 = cs2.x, s2 = cs2.y;
            const float b00 = c1 * a00 - s1 * a10, b01 = c1 * a01 - s1 * a11;
            const float b10 = s1 * a00 + c1 * a10, b11 = s1 * a01 + c1 * a11;
            SF(nxt, dst[T][q][0]) = c2 * b00 - s2 * b01;
            SF(nxt, dst[T][q][1]) = s2 * b00 + c2 * b01;
            SF(nxt, dst[T][q][2]) = c2 * b10 - s2 * b11;
            SF(nxt, dst[T][q][3]) = s2 * b10 + c2 * b11;
        }
        // V <- V J, swapped.  Even steps: a lane's own two columns.  Odd
        // steps: lane i pairs position 2i-1 (bottom of lane i-1) with its top;
        // the new position 2i-1 goes back to lane i-1.  Lanes past the pairs
        // rotate by the identity and keep zeros.
        const bool pl = pi < npair;
        const float2 csl = sm.cst[pl ? pi : 0];
        const float c = pl ? csl.x : 1.0f, sg = pl ? csl.y : 0.0f;
#pragma unroll
        for (int j = 0; j < RV; ++j) {
            if (T == 0) {
                const float t0 = vt[j];
                vt[j] = sg * t0 + c * vb[j];
                vb[j] = c * t0 - sg * vb[j];
            } else {
                const float x = wave_shr0(vb[j]);  // bottom of lane - 1 (lane 0: ghost)
                const float z = sg * x + c * vt[j];
                vt[j] = c * x - sg * vt[j];
                vb[j] = wave_shl1(z);
            }
        }
        __syncthreads();
    };

    int sweep = 0;
    for (;; ++sweep) {
        // off(A)^2 = 2 x (squares of the lower off-diagonal entries), tiling 0
        float o = 0.0f;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            if (tid + q * NT >= nblk0) continue;
            const int b4 = (tid + q * NT) * 4;
            const float a10 = LF(B0, 2 * PL + b4);
            if (bI[q] == bJ[q]) {
                o += 2.0f * a10 * a10;
            } else {
                const float a00 = LF(B0, b4), a01v = LF(B0, PL + b4), a11 = LF(B0, 3 * PL + b4);
                o += 2.0f * (a00 * a00 + a01v * a01v + a10 * a10 + a11 * a11);
            }
        }
        const float off2 = block_sum<NT>(o, sm.redf);
        if (off2 <= thr) break;
        if (sweep >= kMaxSweeps) {
            if (tid == 0 && a.ctl != nullptr) atomicAdd(&a.ctl->jacobi_cap, 1);
            break;
        }
#pragma unroll 1
        for (int r = 0; r < K; r += 2) {
            step(std::integral_constant<int, 0>{}, B0, B1);
            step(std::integral_constant<int, 1>{}, B1, B0);
        }
    }
    if (tid == 0 && a.ctl != nullptr) atomicAdd(&a.ctl->sweeps, sweep);
    const bool rev = sweep & 1;  // position p holds index K-1-p

    // Eigenvalues from the diagonal blocks of tiling 0; indices past K are
    // padding.
    if (tid < S) {
        float l = 0.0f;
        if (tid < K) {
            const int p = rev ? K - 1 - tid : tid;
            const int t = p >> 1;
            l = LF(B0, ((p & 1) ? 3 * PL : 0) + t * (t + 3) * 2) * unscale;
        }
        sm.lam[tid] = l;
        sm.lp[tid] = fmaxf(l, 0.0f);
    }
#undef LF
#undef SF
    __syncthreads();  // buffers are read; sV takes V back
    // registers -> sV; outside the leading K x K block the identity, so that
    // the products below see exact zeros there
    for (int idx = tid; idx < S * S; idx += NT) {
        const int i = idx / S, j = idx % S;
        if (i >= K || j >= K) sV[i * LD + j] = (i == j) ? 1.0f : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < RV; ++j) {
        const int row = vrow(j);
        if (vlane && row < K) {
            const int c0 = rev ? K - 1 - 2 * pi : 2 * pi, c1 = rev ? K - 2 - 2 * pi : 2 * pi + 1;
            sV[row * LD + c0] = vt[j];
            sV[row * LD + c1] = vb[j];
        }
    }
    __syncthreads();

    // Re-orthonormalisation, only after rotations: without a sweep V is the
    // start matrix as it came in (the identity, or eigenvectors that were
    // re-orthonormalised when they were made).
    if (sweep > 0) {
        // E = V^T V - I  -> sA (A's eigenvalues are in sm.lam)
        product_store<S, NT, 0, true, true>(
            sV, sV, nullptr, K, tid, [&](int i, int j, float v) { sA[i * LD + j] = v - (i == j ? 1.0f : 0.0f); });
        __syncthreads();
        // Vn = V - V E / 2  -> sV
        product_store<S, NT, 1>(sV, sA, nullptr, K, tid,
                                [&](int i, int j, float v) { sV[i * LD + j] -= 0.5f * v; });
        __syncthreads();
    }
    // P = Vn diag(max(Lambda, 0)) Vn^T  -> sA (lower triangle; only it is
    // read).  On the matrix cores the sum runs over the columns of the
    // positive eigenvalues only: they are listed first in sm.pidx (the others
    // follow, so the list is padded with columns whose clamped eigenvalue is
    // zero), and the sum has their number rounded up to 8 terms instead of K.
    if constexpr (S >= 32) {
        static_assert(NT >= S, "one thread per column");
        const int lane = tid & 63;
        bool pos = false;
        unsigned long long m = 0ull;
        if (tid < S) {
            pos = sm.lp[tid] > 0.0f;
            m = __ballot(pos);
            if (lane == 0) sm.npos[tid >> 6] = __popcll(m);
        }
        __syncthreads();
        const int r = uniform(sm.npos[0] + (S > 64 ? sm.npos[1] : 0));
        if (tid < S) {
            const int before = (tid >= 64 ? sm.npos[0] : 0) + __popcll(m & ((1ull << lane) - 1ull));
            sm.pidx[pos ? before : r + tid - before] = tid;
        }
        __syncthreads();
        product_store<S, NT, 2, true>(sV, sV, sm.lp, r, tid, to_sA, sm.pidx);
    } else {
        product_store<S, NT, 2, true>(sV, sV, sm.lp, K, tid, to_sA);
    }
    __syncthreads();

    // eigenvectors out row by row (a wave per row, lanes along it)
    if (warm && a.warm_store)
        for (int i = wv; i < k; i += NW)
            for (int j = lane; j < k; j += 64) vw[i * k + j] = sV[i * LD + j];

    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    for (int s0 = tid; s0 < nslot; s0 += GU * NT) {
        double hx[GU];
        float lm[GU], bo[GU];
        if (a.mode == PROJ_PRIMAL) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int64_t g = off + min(s0 + u * NT, nslot - 1);
                hx[u] = a.x[a.gather[g]];
                lm[u] = a.lam[g];
                bo[u] = a.dslot != nullptr ? a.blk[g] : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int s = s0 + u * NT;
            if (s >= nslot) continue;
            const int i = tri_row(s), j = s - i * (i + 1) / 2;
            const float pv32 = sA[i * LD + j];
            const int64_t g = off + s;
            if (a.mode == PROJ_STANDALONE) {
                a.Pout[g] = pv32;
            } else if (a.mode == PROJ_PRIMAL) {
                const double pv = (double)pv32;
                a.lam[g] = (float)((double)lm[u] + a.rho * (pv - hx[u]));
                a.blk[g] = pv32;
                if (a.dslot != nullptr) a.dslot[g] = (float)(pv - (double)bo[u]);
                const double wgt = (i == j) ? 1.0 : 2.0;
                const double d = pv - hx[u];
                p0 += wgt * d * d;
                p1 += wgt * hx[u] * hx[u];
                p2 += wgt * pv * pv;
            } else {
                a.blk[g] = pv32;
            }
        }
    }
    if (a.mode == PROJ_PRIMAL) {
        // the three residual partial sums in one workgroup reduction (waves
        // added in order, as block_sum does); only thread 0 reads the result
        p0 = wave_sum(p0);
        p1 = wave_sum(p1);
        p2 = wave_sum(p2);
        if ((tid & 63) == 0) {
            const int w = tid >> 6;
            sm.redd[3 * w + 0] = p0;
            sm.redd[3 * w + 1] = p1;
            sm.redd[3 * w + 2] = p2;
        }
        __syncthreads();
        if (tid == 0) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int i = 0; i < NT / 64; ++i) {
                s0 += sm.redd[3 * i + 0];
                s1 += sm.redd[3 * i + 1];
                s2 += sm.redd[3 * i + 2];
            }
            a.cpart[4 * (int64_t)id + 0] = s0;
            a.cpart[4 * (int64_t)id + 1] = s1;
            a.cpart[4 * (int64_t)id + 2] = s2;
        }
    }
    // eigenpairs of the k x k block: Lambda and the re-orthonormalised V
    if (a.evals != nullptr)
        for (int t = tid; t < k; t += NT) a.evals[a.eoff[id] + t] = sm.lam[t];
    if (a.evecs != nullptr)
        for (int i = wv; i < k; i += NW)
            for (int j = lane; j < k; j += 64) a.evecs[a.voff[id] + i * k + j] = sV[i * LD + j];
    __syncthreads();  // LDS is reused by the next clique of a queue launch
}

// Waves per SIMD that the LDS of one workgroup (2 S x (S+1) FP32 buffers
// and the small arrays) allows on a CU of 160 KB, capped at 4: the register
// budget the compiler is asked to meet (512 / waves registers per lane).
constexpr int proj_waves_per_eu(int S, int NT) {
    const int lds = 2 * S * (S + 1) * 4 + 2048;
    const int wg = 163840 / lds;
    const int w = wg * (NT / 64) / 4;
    const int cap = NT == 64 ? 2 : 4;  // one-wave workgroups hold all of V in registers
    return w < 1 ? 1 : (w > cap ? cap : w);
}

// One launch per size bucket: workgroup b projects clique ids[b] (or b).
template <int S, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(proj_waves_per_eu(S, NT))))
void k_project(ProjArgs a) {
    __shared__ float sbuf[2 * S * (S + 1)];
    __shared__ ProjSmall sm;
    if (a.ctl != nullptr && a.ctl->stop) return;
    const int bi = blockIdx.x;
    if (bi >= a.nblk) return;
    if (threadIdx.x == 0) sm.zero = 0;
    __syncthreads();
    project_one<S, NT>(a, a.ids ? a.ids[bi] : bi, sbuf, sbuf + S * (S + 1), sm);
}

__device__ __forceinline__ int bucket_of(int k) {
    return k <= 16 ? 16 : k <= 32 ? 32 : k <= 48 ? 48 : k <= 64 ? 64 : k <= 80 ? 80 : k <= 96 ? 96 : k <= 112 ? 112 : 128;
}

// Draw the next queue ticket for the workgroup (two barriers).
__device__ __forceinline__ int draw_item(unsigned long long *ticket, unsigned long long period, int *s_item) {
    if (threadIdx.x == 0) *s_item = (int)(atomicAdd(ticket, 1ull) % period);
    __syncthreads();
    const int item = *s_item;
    __syncthreads();
    return item;
}

// Drain the queue while it hands out cliques of bucket S.  Tickets of one
// workgroup only increase and ids are in decreasing size, so a workgroup
// passes through the buckets in order; each bucket's loop-invariant state
// (work tables of the rotation steps) is live only inside its own loop.
template <int S, int NT>
__device__ __forceinline__ int drain_bucket(const ProjArgs &a, int item, float *sbuf, ProjSmall &sm,
                                            unsigned long long *ticket, unsigned long long period, int *s_item) {
    while (item < a.nblk) {
        const int id = a.ids[item];
        if (bucket_of(a.size[id]) != S) break;
        project_one<S, NT>(a, id, sbuf, sbuf + S * (S + 1), sm);
        item = draw_item(ticket, period, s_item);
    }
    return item;
}

// One persistent launch over every clique (all size buckets up to SB): each
// workgroup repeatedly draws a ticket from a 64-bit counter and projects
// clique ids[ticket mod period] (ids in decreasing size: largest first), until
// its ticket falls past nblk.  A launch of G workgroups draws exactly
// nblk + G = period tickets (every workgroup ends on one failing draw), so
// launch L owns tickets [L period, (L+1) period) and the counter never needs a
// reset between stream-ordered launches of the same configuration.
template <int SB, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(proj_waves_per_eu(SB, NT))))
void k_project_queue(ProjArgs a, unsigned long long *ticket,
                                                      unsigned long long period) {
    __shared__ float sbuf[2 * SB * (SB + 1)];
    __shared__ ProjSmall sm;
    __shared__ int s_item;
    if (a.ctl != nullptr && a.ctl->stop) return;
    if (threadIdx.x == 0) sm.zero = 0;  // published by draw_item's barriers
    int item = draw_item(ticket, period, &s_item);
    if constexpr (SB >= 128) item = drain_bucket<128, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    if constexpr (SB >= 112) item = drain_bucket<112, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    if constexpr (SB >= 96) item = drain_bucket<96, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    if constexpr (SB >= 80) item = drain_bucket<80, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    if constexpr (SB >= 64) item = drain_bucket<64, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    if constexpr (SB >= 48) item = drain_bucket<48, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    if constexpr (SB >= 32) item = drain_bucket<32, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    item = drain_bucket<16, NT>(a, item, sbuf, sm, ticket, period, &s_item);
    // every clique's bucket is <= SB, so the queue is exhausted here
}

// Adjoint of the projection (Daleckii-Krein): for W = V diag(lambda) V^T and a
// cotangent G of P(W) (symmetric), Wbar = V (Gamma o (V^T G V)) V^T with
// Gamma_ij the first divided difference of max(., 0) at (lambda_i, lambda_j)
// (1 if both positive, 0 if both <= 0, else (l_i+ - l_j+) / (l_i - l_j)).
// Packed coordinates: an off-diagonal packed cotangent stands for both
// triangles, so G gets half of it on each side and Wbar's two triangles add up.
template <int S, int NT>
__global__ __launch_bounds__(NT) void k_project_vjp(VjpArgs a) {
    static_assert(S % 16 == 0 && S <= 128, "bucket size");
    constexpr int LD = S + 1;
    __shared__ float sA[S * LD];
    __shared__ float sV[S * LD];
    __shared__ float sLam[S], sOne[S];
    const int bi = blockIdx.x;
    if (bi >= a.nblk) return;
    const int k = a.size[bi];
    if (k < 1 || k > S) return;
    const int64_t off = a.off[bi], eo = a.eoff[bi], vo = a.voff[bi];
    const int nslot = k * (k + 1) / 2;
    const int tid = threadIdx.x;
    // V (identity past k: harmless, every product pairs it with zeros) and
    // G (zero past k)
    for (int idx = tid; idx < S * S; idx += NT) {
        const int i = idx / S, j = idx % S;
        sA[i * LD + j] = 0.0f;
        sV[i * LD + j] = (i < k && j < k) ? a.evecs[vo + i * k + j] : (i == j ? 1.0f : 0.0f);
    }
    if (tid < S) {
        sLam[tid] = tid < k ? a.evals[eo + tid] : 0.0f;
        sOne[tid] = 1.0f;
    }
    __syncthreads();
    for (int s = tid; s < nslot; s += NT) {
        const int i = tri_row(s), j = s - i * (i + 1) / 2;
        const float g = a.gP[off + s];
        if (i == j) {
            sA[i * LD + i] = g;
        } else {
            sA[i * LD + j] = 0.5f * g;
            sA[j * LD + i] = 0.5f * g;
        }
    }
    __syncthreads();
    // Each product keeps its result in registers until every thread has read
    // its operands, so it may overwrite one (matrix cores for S >= 32).
    auto to_sA = [&](int i, int j, float v) { sA[i * LD + j] = v; };
    product_store<S, NT, 1>(sA, sV, nullptr, k, tid, to_sA);  // G V
    __syncthreads();
    product_store<S, NT, 0>(sV, sA, nullptr, k, tid, [&](int i, int j, float v) {  // Gamma o (V^T G V)
        const float li = sLam[i], lj = sLam[j];
        float gam;
        if (li > 0.0f && lj > 0.0f) gam = 1.0f;
        else if (li <= 0.0f && lj <= 0.0f) gam = 0.0f;
        else gam = (fmaxf(li, 0.0f) - fmaxf(lj, 0.0f)) / (li - lj);
        sA[i * LD + j] = gam * v;
    });
    __syncthreads();
    product_store<S, NT, 1>(sV, sA, nullptr, k, tid, to_sA);  // V (Gamma o B)
    __syncthreads();
    // (V (Gamma o B)) V^T is symmetric: its lower triangle suffices
    product_store<S, NT, 2, true>(sA, sV, sOne, k, tid, to_sA);
    __syncthreads();
    for (int s = tid; s < nslot; s += NT) {
        const int i = tri_row(s), j = s - i * (i + 1) / 2;
        a.gW[off + s] = (i == j) ? sA[i * LD + i] : 2.0f * sA[i * LD + j];
    }
}

template <int S, int NT>
void launch_vjp_t(const VjpArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_project_vjp<S, NT>), dim3(a.nblk), dim3(NT), 0, s, a);
}

template <int S, int NT>
void launch_t(const ProjArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_project<S, NT>), dim3(a.nblk), dim3(NT), 0, s, a);
}

template <int SB, int NT>
void launch_queue_t(const ProjArgs &a, int grid, unsigned long long *ticket, hipStream_t s) {
    hipLaunchKernelGGL((k_project_queue<SB, NT>), dim3(grid), dim3(NT), 0, s, a, ticket,
                       (unsigned long long)(a.nblk + grid));
}

template <int SB, int NT>
int queue_occ_t() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_project_queue<SB, NT>, NT, 0) != hipSuccess) return 0;
    return nb;
}

// Autotuning input: for each clique a symmetric k x k block with distinct
// diagonal values in (-1, 1) and off-diagonal values of size 1e-3 from an
// integer hash, i.e. the nearly diagonal matrices a warm-started eigensolve
// sees inside the ADMM loop.
__global__ void k_tune_blocks(const int32_t *__restrict__ size, const int64_t *__restrict__ off, int p,
                              float *__restrict__ W) {
    const int id = blockIdx.x;
    if (id >= p) return;
    const int k = size[id];
    const int nslot = k * (k + 1) / 2;
    for (int s = threadIdx.x; s < nslot; s += blockDim.x) {
        const int i = tri_row(s), j = s - i * (i + 1) / 2;
        uint32_t h = (uint32_t)id * 0x9E3779B1u ^ (uint32_t)s * 0x85EBCA77u;
        h ^= h >> 15;
        h *= 0x2C1B3C6Du;
        h ^= h >> 12;
        const float u = (float)(h & 0xFFFFFF) * (2.0f / 16777216.0f) - 1.0f;
        W[off[id] + s] = (i == j) ? (float)(2 * i - k + 1) / (float)k : 1e-3f * u;
    }
}

__global__ void k_identity_blocks(const int32_t *__restrict__ size, const int64_t *__restrict__ voff, int p,
                                  float *__restrict__ V) {
    const int id = blockIdx.x;
    if (id >= p) return;
    const int k = size[id];
    for (int idx = threadIdx.x; idx < k * k; idx += blockDim.x) V[voff[id] + idx] = (idx / k == idx % k) ? 1.0f : 0.0f;
}

}  // namespace

int proj_bucket(int smax) {
    if (smax <= 16) return 16;
    if (smax <= 32) return 32;
    if (smax <= 48) return 48;
    if (smax <= 64) return 64;
    if (smax <= 80) return 80;
    if (smax <= 96) return 96;
    if (smax <= 112) return 112;
    return 128;
}

bool proj_threads_ok(int S, int nthreads) {
    if (nthreads == 256 || nthreads == 512) return true;
    if (nthreads == 64) return S <= 32;
    return false;
}

void launch_project(const ProjArgs &a, int smax, int nthreads, hipStream_t s) {
    if (a.nblk <= 0) return;
    const int S = proj_bucket(smax);
    const int nt = proj_threads_ok(S, nthreads) ? nthreads : 256;
    switch (S) {
    case 16: nt == 64 ? launch_t<16, 64>(a, s) : nt == 512 ? launch_t<16, 512>(a, s) : launch_t<16, 256>(a, s); break;
    case 32: nt == 64 ? launch_t<32, 64>(a, s) : nt == 512 ? launch_t<32, 512>(a, s) : launch_t<32, 256>(a, s); break;
    case 48: nt == 512 ? launch_t<48, 512>(a, s) : launch_t<48, 256>(a, s); break;
    case 64: nt == 512 ? launch_t<64, 512>(a, s) : launch_t<64, 256>(a, s); break;
    case 80: nt == 512 ? launch_t<80, 512>(a, s) : launch_t<80, 256>(a, s); break;
    case 96: nt == 512 ? launch_t<96, 512>(a, s) : launch_t<96, 256>(a, s); break;
    case 112: nt == 512 ? launch_t<112, 512>(a, s) : launch_t<112, 256>(a, s); break;
    default: nt == 512 ? launch_t<128, 512>(a, s) : launch_t<128, 256>(a, s); break;
    }
}

int project_queue_occupancy(int smax, int nthreads) {
    const bool w = nthreads == 512;
    if (!w && proj_bucket(smax) > 96) return 0;  // queue launches over buckets 112 and 128 use 512 threads
    switch (proj_bucket(smax)) {
    case 16: return w ? queue_occ_t<16, 512>() : queue_occ_t<16, 256>();
    case 32: return w ? queue_occ_t<32, 512>() : queue_occ_t<32, 256>();
    case 48: return w ? queue_occ_t<48, 512>() : queue_occ_t<48, 256>();
    case 64: return w ? queue_occ_t<64, 512>() : queue_occ_t<64, 256>();
    case 80: return w ? queue_occ_t<80, 512>() : queue_occ_t<80, 256>();
    case 96: return w ? queue_occ_t<96, 512>() : queue_occ_t<96, 256>();
    case 112: return queue_occ_t<112, 512>();
    default: return queue_occ_t<128, 512>();
    }
}

void launch_project_queue(const ProjArgs &a, int smax, int nthreads, int grid, unsigned long long *ticket,
                          hipStream_t s) {
    if (a.nblk <= 0 || grid <= 0) return;
    const bool w = nthreads == 512;
    // Buckets 112 and 128 are drained by 512-thread workgroups only: with 256
    // threads every thread holds twice the eigenvector rows, and the kernel
    // that drains all eight buckets exceeds the architected registers (the
    // 256-thread build gave wrong results in its bucket-96 loop).
    if (!w && proj_bucket(smax) > 96) return;
    switch (proj_bucket(smax)) {
    case 16: w ? launch_queue_t<16, 512>(a, grid, ticket, s) : launch_queue_t<16, 256>(a, grid, ticket, s); break;
    case 32: w ? launch_queue_t<32, 512>(a, grid, ticket, s) : launch_queue_t<32, 256>(a, grid, ticket, s); break;
    case 48: w ? launch_queue_t<48, 512>(a, grid, ticket, s) : launch_queue_t<48, 256>(a, grid, ticket, s); break;
    case 64: w ? launch_queue_t<64, 512>(a, grid, ticket, s) : launch_queue_t<64, 256>(a, grid, ticket, s); break;
    case 80: w ? launch_queue_t<80, 512>(a, grid, ticket, s) : launch_queue_t<80, 256>(a, grid, ticket, s); break;
    case 96: w ? launch_queue_t<96, 512>(a, grid, ticket, s) : launch_queue_t<96, 256>(a, grid, ticket, s); break;
    case 112: launch_queue_t<112, 512>(a, grid, ticket, s); break;
    default: launch_queue_t<128, 512>(a, grid, ticket, s); break;
    }
}

void launch_project_vjp(const VjpArgs &a, int smax, hipStream_t s) {
    if (a.nblk <= 0) return;
    switch (proj_bucket(smax)) {
    case 16: launch_vjp_t<16, 256>(a, s); break;
    case 32: launch_vjp_t<32, 256>(a, s); break;
    case 48: launch_vjp_t<48, 256>(a, s); break;
    case 64: launch_vjp_t<64, 256>(a, s); break;
    case 80: launch_vjp_t<80, 256>(a, s); break;
    case 96: launch_vjp_t<96, 256>(a, s); break;
    case 112: launch_vjp_t<112, 256>(a, s); break;
    default: launch_vjp_t<128, 256>(a, s); break;
    }
}

void launch_tune_blocks(const int32_t *size, const int64_t *off, int p, float *W, hipStream_t s) {
    if (p > 0) hipLaunchKernelGGL(k_tune_blocks, dim3(p), dim3(256), 0, s, size, off, p, W);
}

void launch_identity_blocks(const int32_t *size, const int64_t *voff, int p, float *V, hipStream_t s) {
    if (p > 0) hipLaunchKernelGGL(k_identity_blocks, dim3(p), dim3(256), 0, s, size, voff, p, V);
}

}  // namespace cdcs
