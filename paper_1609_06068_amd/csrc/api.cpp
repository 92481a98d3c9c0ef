// C-ABI entry points: setup (validation, chordal-decomposition maps, upload,
// KKT factorisation), the batched projection, the affine projection and the
// ADMM driver with HIP-graph capture of whole iterations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "cdcs_internal.h"

using namespace cdcs;

namespace {

thread_local std::string g_err;

cdcs_status fail(cdcs_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIP_OK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? CDCS_E_NOMEM : CDCS_E_DEVICE,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)

int64_t round_up(int64_t v, int64_t q) { return (v + q - 1) / q * q; }


// Internal form of the HSDE iteration (graphs and enqueue), beside CDCS_PRIMAL / CDCS_DUAL.
constexpr int kFormHsde = 2;

struct GraphKey {
    int form;
    int K;
    double rho;
    const void *x, *y, *blk, *lam, *v, *vw, *tk;
    bool operator<(const GraphKey &o) const {
        return std::tie(form, K, rho, x, y, blk, lam, v, vw, tk) <
               std::tie(o.form, o.K, o.rho, o.x, o.y, o.blk, o.lam, o.v, o.vw, o.tk);
    }
};

// The inverse-factor fields of Dev (Algorithm 1/2's factor or the HSDE one).
struct FactorFields {
    double *Linv = nullptr, *LinvT = nullptr, *Minv = nullptr;
    int32_t sparse_linv = 0, spchol = 0;
    int64_t nnz_linv = 0, nnz_l = 0;
    int32_t *li_ptr = nullptr, *li_col = nullptr, *lt_ptr = nullptr, *lt_col = nullptr;
    double *li_val = nullptr, *lt_val = nullptr;
};

FactorFields get_factor(const Dev &d) {
    FactorFields f;
    f.Linv = d.Linv;
    f.LinvT = d.LinvT;
    f.Minv = d.Minv;
    f.sparse_linv = d.sparse_linv;
    f.spchol = d.spchol;
    f.nnz_linv = d.nnz_linv;
    f.nnz_l = d.nnz_l;
    f.li_ptr = d.li_ptr;
    f.li_col = d.li_col;
    f.li_val = d.li_val;
    f.lt_ptr = d.lt_ptr;
    f.lt_col = d.lt_col;
    f.lt_val = d.lt_val;
    return f;
}

void set_factor(Dev &d, const FactorFields &f) {
    d.Linv = f.Linv;
    d.LinvT = f.LinvT;
    d.Minv = f.Minv;
    d.sparse_linv = f.sparse_linv;
    d.spchol = f.spchol;
    d.nnz_linv = f.nnz_linv;
    d.nnz_l = f.nnz_l;
    d.li_ptr = f.li_ptr;
    d.li_col = f.li_col;
    d.li_val = f.li_val;
    d.lt_ptr = f.lt_ptr;
    d.lt_col = f.lt_col;
    d.lt_val = f.lt_val;
}

struct Bucket {
    int smax;
    int count;
    int32_t *ids;  // device
    int nt = 256;  // workgroup size (autotuned)
    float us = -1.0f;  // tuned launch time
};

// How the projection of every clique is launched: one persistent queue launch
// over all cliques, or one launch per size bucket.  Chosen at setup by timing
// the candidates on this handle's cliques.
struct ProjPlan {
    bool queue = false;
    bool parallel = false;  // per-bucket launches on parallel streams (not queue)
    int nt = 256;      // queue workgroup size
    int grid = 0;      // queue workgroups
    float queue_us = -1.0f, buckets_us = -1.0f, parallel_us = -1.0f;
};

constexpr int kSideStreams = 3;  // streams besides the caller's for the size buckets' launches

}  // namespace

struct cdcs_handle {
    int device = 0;
    Dev d;
    std::vector<void *> allocs;
    std::vector<int64_t> off_host;
    std::vector<Bucket> buckets;
    ProjPlan plan;
    unsigned long long *ticket = nullptr;  // device counter of the queue launch
    hipStream_t cap_stream = nullptr;
    // the size buckets' launches of the parallel plan: forked from the
    // caller's stream by fork_ev, joined back by join_ev (default priority)
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kSideStreams] = {};
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<hipGraph_t> graph_defs;
    std::unique_ptr<Batch> batch_host;
    int last_iters = 0;
    double last_rho = 1.0;
    int last_form = CDCS_PRIMAL;
    // differentiation (allocated at the first call that needs them)
    struct Diff {
        double *c = nullptr;       // [ldU] caller's c in internal entry order
        int64_t *eoff = nullptr;   // [p+1] offsets of each clique's eigenvalues (prefix sums of s_k)
        float *gP = nullptr, *gW = nullptr;  // [nslots] projection adjoint in/out
        double *hbar = nullptr;    // [nslots]
        double *x = nullptr;       // [ldU] solve output, then r1bar
        double *y = nullptr;       // [ldM]
    } diff;
    float *save_evals = nullptr;  // set while an unrolled step runs: the projection
    float *save_evecs = nullptr;  // writes its eigenpairs here
    // sparse A: the symbolic input of the factor (touched entries' rows, host;
    // touched-entry index of each coefficient, device), kept for the HSDE factor
    std::vector<int32_t> sym_tcp, sym_tcr;
    int32_t *sym_tid = nullptr;
    // homogeneous self-dual embedding (built at the first HSDE call)
    HsdeDev hs;
    FactorFields hs_fac;
    bool hs_ready = false;
    double *hs_tk = nullptr;      // tau, kappa of the state the HSDE graphs were captured for

    template <typename T>
    cdcs_status alloc(T **p, int64_t count) {
        *p = nullptr;
        if (count <= 0) count = 1;
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, (size_t)count * sizeof(T));
        if (e != hipSuccess) return fail(CDCS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(q);
        *p = static_cast<T *>(q);
        return CDCS_OK;
    }

    ~cdcs_handle() {
        for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
        for (auto g : graph_defs) (void)hipGraphDestroy(g);
        for (void *p : allocs) (void)hipFree(p);
        if (d.ctl_host) (void)hipHostFree(d.ctl_host);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (int i = 0; i < kSideStreams; ++i) {
            if (side[i]) (void)hipStreamDestroy(side[i]);
            if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
        }
        if (fork_ev) (void)hipEventDestroy(fork_ev);
    }
};

namespace {

#define CK(expr)                          \
    do {                                  \
        cdcs_status s_ = (expr);          \
        if (s_ != CDCS_OK) return s_;     \
    } while (0)

cdcs_status tune_projection(cdcs_handle *h, hipStream_t s);

cdcs_status compress_factors(cdcs_handle *h, hipStream_t s);

template <typename T>
cdcs_status upload(cdcs_handle *h, T **dst, const std::vector<T> &src, hipStream_t s) {
    CK(h->alloc(dst, (int64_t)src.size()));
    (void)s;
    // Synchronous copy: the host vectors die when setup returns, also on error paths.
    if (!src.empty()) HIP_OK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return CDCS_OK;
}

// One SDP validated and decomposed on the host, in its own (local) indices.
struct HostProblem {
    int32_t n = 0, m = 0, p = 0, smax = 0;
    int64_t nU = 0, nslots = 0, ld = 0;
    std::vector<int32_t> size;       // [p] clique sizes
    std::vector<int64_t> off;        // [p+1] packed slot offsets
    std::vector<int32_t> gather;     // [nslots] internal entry of each packed slot (H_k)
    std::vector<int32_t> perm;       // [nU] pattern position of each internal entry
    std::vector<int32_t> cnt;        // [nU] D_e = number of cliques covering e
    std::vector<double> wt, invD, s2, c, b;
    std::vector<float> Aw;           // [m * ld] w-scaled A, row-major, zero padded (dense path)
    bool sparse = false;             // CSR path: rows sorted by entry, duplicates summed
    std::vector<int32_t> sp_ptr, sp_col;
    std::vector<double> sp_val;      // w_e * A_ie
    int64_t nslots_psd = 0;          // clique slots; the vector cones' slots follow
    int32_t nvc = 0;                 // vector cones
    std::vector<int32_t> vblk;       // [nvb * 4] (kind, s0, s1, cone) work blocks of the vector cones
    std::vector<int32_t> soc;        // [nsoc * 3] (first slot, first block, end block) per second-order cone
    std::vector<int32_t> socb;       // indices of the second-order cones' work blocks
};

// A CSR input is kept sparse when a dense FP32 copy would be read at more
// than five times the bytes of the coefficients.
bool keep_sparse(int64_t nnz, int64_t m, int64_t nU) { return nnz * 5 < m * nU; }

cdcs_status host_problem(const cdcs_pattern *pat, const cdcs_constraints *A, const double *b, const double *c,
                         const cdcs_cliques *cl, const cdcs_vcones *cones, int64_t align, bool allow_sparse,
                         HostProblem &P) {
    if (!pat || !A || !b || !c || !cl) return fail(CDCS_E_ARG, "NULL argument");
    if (pat->n < 1 || pat->nnz < 1 || !pat->i || !pat->j) return fail(CDCS_E_ARG, "empty or NULL pattern");
    if (A->m < 1 || !A->val) return fail(CDCS_E_ARG, "no constraints");
    const int32_t nvc = cones ? cones->ncones : 0;
    if (nvc < 0 || (nvc > 0 && (!cones->kind || !cones->ptr || !cones->vert)))
        return fail(CDCS_E_ARG, "bad vector cone arrays");
    if (cl->p < 0 || (cl->p == 0 && nvc == 0) || (cl->p > 0 && (!cl->ptr || !cl->vert)))
        return fail(CDCS_E_ARG, "no cliques");
    const int32_t n = pat->n;
    const int64_t nU = pat->nnz;
    const int32_t m = A->m;
    const int32_t p = cl->p;
    if (nU >= (int64_t)1 << 31) return fail(CDCS_E_ARG, "pattern too large");

    // Pattern: lower triangular, in range, distinct.
    std::vector<std::pair<int64_t, int32_t>> keys((size_t)nU);
    for (int64_t e = 0; e < nU; ++e) {
        const int32_t i = pat->i[e], j = pat->j[e];
        if (j < 0 || i < j || i >= n)
            return fail(CDCS_E_PATTERN, "pattern entry " + std::to_string(e) + " not lower triangular / out of range");
        keys[(size_t)e] = {(int64_t)i * n + j, (int32_t)e};
    }
    std::sort(keys.begin(), keys.end());
    for (size_t q = 1; q < keys.size(); ++q)
        if (keys[q].first == keys[q - 1].first) return fail(CDCS_E_PATTERN, "duplicate pattern entry");
    auto find = [&](int32_t i, int32_t j) -> int32_t {
        const int64_t key = (int64_t)std::max(i, j) * n + std::min(i, j);
        auto it = std::lower_bound(keys.begin(), keys.end(), std::make_pair(key, (int32_t)-1));
        if (it == keys.end() || it->first != key) return -1;
        return it->second;
    };

    // Cliques: E_k with vertices in increasing order (Sec. II-B); gather map H_k.
    if (p > 0 && cl->ptr[0] != 0) return fail(CDCS_E_PATTERN, "clique ptr[0] != 0");
    P.n = n;
    P.m = m;
    P.p = p;
    P.nU = nU;
    P.smax = 0;
    P.off.assign((size_t)p + 1, 0);
    P.size.resize((size_t)p);
    for (int32_t k = 0; k < p; ++k) {
        const int64_t a0 = cl->ptr[k], a1 = cl->ptr[k + 1];
        const int64_t sk = a1 - a0;
        if (sk < 1 || sk > CDCS_MAX_CLIQUE)
            return fail(sk < 1 ? CDCS_E_PATTERN : CDCS_E_ARG,
                        "clique " + std::to_string(k) + " size " + std::to_string(sk) + " outside 1.." +
                            std::to_string(CDCS_MAX_CLIQUE));
        for (int64_t q = a0; q < a1; ++q) {
            const int32_t v = cl->vert[q];
            if (v < 0 || v >= n) return fail(CDCS_E_PATTERN, "clique vertex out of range");
            if (q > a0 && v <= cl->vert[q - 1])
                return fail(CDCS_E_PATTERN, "clique " + std::to_string(k) + " not strictly increasing");
        }
        P.size[(size_t)k] = (int32_t)sk;
        P.smax = std::max<int32_t>(P.smax, (int32_t)sk);
        P.off[(size_t)k + 1] = P.off[(size_t)k] + sk * (sk + 1) / 2;
    }
    P.nslots_psd = P.off[(size_t)p];
    // vector cones: one slot per vertex (its diagonal entry), after the cliques
    int64_t nvs = 0;
    if (nvc > 0) {
        if (cones->ptr[0] != 0) return fail(CDCS_E_PATTERN, "cone ptr[0] != 0");
        for (int32_t q = 0; q < nvc; ++q) {
            const int64_t sz = cones->ptr[q + 1] - cones->ptr[q];
            const int32_t kind = cones->kind[q];
            if (kind != CDCS_CONE_FREE && kind != CDCS_CONE_ORTHANT && kind != CDCS_CONE_SOC)
                return fail(CDCS_E_ARG, "vector cone " + std::to_string(q) + ": unknown kind");
            if (sz < (kind == CDCS_CONE_SOC ? 2 : 1))
                return fail(CDCS_E_PATTERN, "vector cone " + std::to_string(q) + " too small");
            nvs += sz;
        }
    }
    P.nvc = nvc;
    P.nslots = P.nslots_psd + nvs;
    if (P.nslots >= (int64_t)1 << 31) return fail(CDCS_E_ARG, "too many clique slots");
    P.gather.resize((size_t)P.nslots);
    P.cnt.assign((size_t)nU, 0);
    for (int32_t k = 0; k < p; ++k) {
        const int32_t *cv = cl->vert + cl->ptr[k];
        const int sk = P.size[(size_t)k];
        int64_t g = P.off[(size_t)k];
        for (int a = 0; a < sk; ++a)
            for (int bb = 0; bb <= a; ++bb, ++g) {
                const int32_t e = find(cv[a], cv[bb]);
                if (e < 0) return fail(CDCS_E_PATTERN, "clique " + std::to_string(k) + " pair missing from the pattern");
                P.gather[(size_t)g] = e;
                ++P.cnt[(size_t)e];
            }
    }
    if (nvc > 0) {
        // a cone vertex: in no clique and no other cone, only its diagonal entry
        std::vector<char> taken((size_t)n, 0);
        for (int32_t k = 0; k < p; ++k)
            for (int64_t q = cl->ptr[k]; q < cl->ptr[k + 1]; ++q) taken[(size_t)cl->vert[q]] = 1;
        std::vector<char> offd((size_t)n, 0);
        for (int64_t e = 0; e < nU; ++e)
            if (pat->i[e] != pat->j[e]) offd[(size_t)pat->i[e]] = offd[(size_t)pat->j[e]] = 1;
        int64_t g = P.nslots_psd;
        for (int32_t q = 0; q < nvc; ++q) {
            const int32_t kind = cones->kind[q];
            const int64_t s0 = g;
            for (int64_t t = cones->ptr[q]; t < cones->ptr[q + 1]; ++t, ++g) {
                const int32_t v = cones->vert[t];
                if (v < 0 || v >= n) return fail(CDCS_E_PATTERN, "cone vertex out of range");
                if (taken[(size_t)v] || offd[(size_t)v])
                    return fail(CDCS_E_PATTERN, "cone vertex " + std::to_string(v) +
                                                    " in a clique, in another cone or with off-diagonal entries");
                taken[(size_t)v] = 1;
                const int32_t e = find(v, v);
                if (e < 0) return fail(CDCS_E_PATTERN, "cone vertex " + std::to_string(v) + " without diagonal entry");
                P.gather[(size_t)g] = e;
                ++P.cnt[(size_t)e];
            }
            // work blocks of at most kVecChunk slots; a second-order cone's
            // blocks carry its index among the second-order cones
            const int32_t b0 = (int32_t)(P.vblk.size() / 4);
            const int32_t si = (int32_t)(P.soc.size() / 3);
            for (int64_t a = s0; a < g; a += kVecChunk) {
                P.vblk.push_back(kind);
                P.vblk.push_back((int32_t)a);
                P.vblk.push_back((int32_t)std::min<int64_t>(g, a + kVecChunk));
                P.vblk.push_back(kind == CDCS_CONE_SOC ? si : q);
            }
            if (kind == CDCS_CONE_SOC) {
                P.soc.push_back((int32_t)s0);
                P.soc.push_back(b0);
                P.soc.push_back((int32_t)(P.vblk.size() / 4));
                for (int32_t b = b0; b < (int32_t)(P.vblk.size() / 4); ++b) P.socb.push_back(b);
            }
        }
    }
    for (int64_t e = 0; e < nU; ++e)
        if (P.cnt[(size_t)e] == 0)
            return fail(CDCS_E_PATTERN, "pattern entry " + std::to_string(e) + " lies in no clique or cone");
    // Internal entry order: first appearance in the packed slots, clique by
    // clique.  An entry's value then sits where its (first) clique's slots
    // sit, so the gather of x into the blocks and the scatter back read
    // consecutive addresses; only entries shared by several cliques are read
    // out of order.  Entry-space vectors cross the interface in pattern order.
    std::vector<int32_t> inv((size_t)nU, -1);
    P.perm.resize((size_t)nU);
    {
        int32_t nxt = 0;
        for (int64_t g = 0; g < P.nslots; ++g) {
            int32_t &ie = inv[(size_t)P.gather[(size_t)g]];
            if (ie < 0) {
                ie = nxt;
                P.perm[(size_t)nxt++] = P.gather[(size_t)g];
            }
            P.gather[(size_t)g] = ie;
        }
    }
    // D = sum_k H_k^T H_k: overlap count of each entry (Sec. III-B.1).
    std::vector<int32_t> cnt_pat;
    cnt_pat.swap(P.cnt);
    P.cnt.resize((size_t)nU);
    P.wt.resize((size_t)nU);
    P.invD.resize((size_t)nU);
    P.s2.resize((size_t)nU);
    P.c.resize((size_t)nU);
    P.b.assign(b, b + m);
    for (int64_t e = 0; e < nU; ++e) {
        const size_t ie = (size_t)inv[(size_t)e];
        const double w = (pat->i[e] == pat->j[e]) ? 1.0 : 2.0;
        const double D = (double)cnt_pat[(size_t)e];
        P.cnt[ie] = cnt_pat[(size_t)e];
        P.wt[ie] = w;
        P.invD[ie] = 1.0 / D;
        P.s2[ie] = 1.0 / (w * D);
        P.c[ie] = c[e];
    }
    P.ld = round_up(nU, align);
    if (!A->dense) {
        if (!A->ptr || !A->idx) return fail(CDCS_E_ARG, "CSR A without ptr/idx");
        if (A->ptr[0] != 0) return fail(CDCS_E_ARG, "CSR A ptr[0] != 0");
        for (int32_t i = 0; i < m; ++i)
            if (A->ptr[i + 1] < A->ptr[i]) return fail(CDCS_E_ARG, "CSR A ptr not monotone");
        for (int64_t q = 0; q < A->ptr[m]; ++q)
            if (A->idx[q] < 0 || A->idx[q] >= nU) return fail(CDCS_E_PATTERN, "A entry index out of range");
    }
    if (!A->dense && allow_sparse && keep_sparse(A->ptr[m], m, nU)) {
        // Sparse path: w A in FP64, each row sorted by entry with duplicates summed.
        if (A->ptr[m] >= (int64_t)1 << 31) return fail(CDCS_E_ARG, "too many A coefficients");
        P.sparse = true;
        P.sp_ptr.assign((size_t)m + 1, 0);
        std::vector<std::pair<int32_t, double>> row;
        for (int32_t i = 0; i < m; ++i) {
            row.clear();
            for (int64_t q = A->ptr[i]; q < A->ptr[i + 1]; ++q) row.push_back({inv[(size_t)A->idx[q]], A->val[q]});
            std::sort(row.begin(), row.end(),
                      [](const std::pair<int32_t, double> &x, const std::pair<int32_t, double> &y) {
                          return x.first < y.first;
                      });
            for (size_t q = 0; q < row.size(); ++q) {
                if (q > 0 && row[q].first == row[q - 1].first) {
                    P.sp_val.back() += P.wt[(size_t)row[q].first] * row[q].second;
                    continue;
                }
                P.sp_col.push_back(row[q].first);
                P.sp_val.push_back(P.wt[(size_t)row[q].first] * row[q].second);
            }
            P.sp_ptr[(size_t)i + 1] = (int32_t)P.sp_col.size();
        }
        return CDCS_OK;
    }
    // Constraint matrix, w A in FP32 (exact for FP32-representable A).
    const int64_t dense_elems = (int64_t)m * P.ld;
    if (dense_elems > ((int64_t)1 << 33)) return fail(CDCS_E_ARG, "dense A too large (sparse A path not built)");
    P.Aw.assign((size_t)dense_elems, 0.0f);
    if (A->dense) {
        for (int32_t i = 0; i < m; ++i)
            for (int64_t e = 0; e < nU; ++e) {
                const int64_t ie = inv[(size_t)e];
                P.Aw[(size_t)(i * P.ld + ie)] = (float)(P.wt[(size_t)ie] * A->val[(size_t)i * nU + e]);
            }
    } else {
        std::vector<double> row((size_t)nU);
        for (int32_t i = 0; i < m; ++i) {
            std::fill(row.begin(), row.end(), 0.0);
            for (int64_t q = A->ptr[i]; q < A->ptr[i + 1]; ++q) row[(size_t)inv[(size_t)A->idx[q]]] += A->val[q];
            for (int64_t e = 0; e < nU; ++e) P.Aw[(size_t)(i * P.ld + e)] = (float)(P.wt[(size_t)e] * row[(size_t)e]);
        }
    }
    return CDCS_OK;
}

// Inverse of the gather map as CSR (entry -> its slots, in slot order), and
// the entries whose lists are long enough to be summed by a whole wave.
void inverse_map(const std::vector<int32_t> &gather, const std::vector<int32_t> &cnt, int heavy_above,
                 std::vector<int32_t> &inv_ptr, std::vector<int32_t> &inv_slot, std::vector<int32_t> &heavy) {
    const int64_t nU = (int64_t)cnt.size();
    inv_ptr.assign((size_t)nU + 1, 0);
    for (int64_t e = 0; e < nU; ++e) inv_ptr[(size_t)e + 1] = inv_ptr[(size_t)e] + cnt[(size_t)e];
    heavy.clear();
    for (int64_t e = 0; e < nU; ++e)
        if (cnt[(size_t)e] > heavy_above) heavy.push_back((int32_t)e);
    inv_slot.resize(gather.size());
    std::vector<int32_t> fillp(inv_ptr.begin(), inv_ptr.end() - 1);
    for (size_t g = 0; g < gather.size(); ++g) inv_slot[(size_t)fillp[(size_t)gather[g]]++] = (int32_t)g;
}

// Common device state: maps, per-entry scalars, buckets, work buffers.
cdcs_status upload_common(cdcs_handle *h, const std::vector<int32_t> &size, const std::vector<int32_t> &gather,
                          const std::vector<int32_t> &cnt, const std::vector<double> &wt,
                          const std::vector<double> &invD, const std::vector<double> &s2,
                          const std::vector<double> &c, const std::vector<double> &b,
                          const std::vector<int32_t> &perm, int heavy_above, hipStream_t s) {
    Dev &d = h->d;
    const int32_t p = d.p;
    std::vector<int32_t> inv_ptr, inv_slot, heavy;
    inverse_map(gather, cnt, heavy_above, inv_ptr, inv_slot, heavy);
    d.nheavy = (int32_t)heavy.size();
    // Cliques by decreasing size: those that fit a workgroup's LDS split into
    // size buckets, the larger ones projected by the Newton-Schulz path.
    std::vector<int32_t> order, big;
    for (int32_t k = 0; k < p; ++k) (size[(size_t)k] > kMaxLdsClique ? big : order).push_back(k);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t bq) { return size[(size_t)a] > size[(size_t)bq]; });
    d.p_lds = (int32_t)order.size();
    d.smax_lds = order.empty() ? 1 : size[(size_t)order.front()];
    constexpr int NBK = 8;
    const int bmax[NBK] = {16, 32, 48, 64, 80, 96, 112, 128};
    std::vector<std::vector<int32_t>> bl(NBK);
    for (int32_t k : order) {
        const int S = proj_bucket(size[(size_t)k]);
        for (int q = 0; q < NBK; ++q)
            if (bmax[q] == S) bl[(size_t)q].push_back(k);
    }
    if (!big.empty()) {
        BigCliques &B = d.big;
        std::vector<int32_t> bn, bN;
        std::vector<int64_t> boff(1, 0);
        int32_t tmax = 0;
        for (int32_t k : big) {
            const int32_t sk = size[(size_t)k], Nk = (sk + 63) / 64 * 64;
            bn.push_back(sk);
            bN.push_back(Nk);
            boff.push_back(boff.back() + (int64_t)Nk * Nk);
            tmax = std::max(tmax, Nk / 64);
        }
        B.nbig = (int32_t)big.size();
        B.tmax2 = tmax * tmax;
        int32_t *ids_d = nullptr, *n_d = nullptr, *N_d = nullptr;
        int64_t *boff_d = nullptr;
        CK(upload(h, &ids_d, big, s));
        CK(upload(h, &n_d, bn, s));
        CK(upload(h, &N_d, bN, s));
        CK(upload(h, &boff_d, boff, s));
        B.ids = ids_d;
        B.n = n_d;
        B.N = N_d;
        B.boff = boff_d;
        CK(h->alloc(&B.W, boff.back()));
        CK(h->alloc(&B.X0, boff.back()));
        CK(h->alloc(&B.X1, boff.back()));
        CK(h->alloc(&B.Y, boff.back()));
        CK(h->alloc(&B.part, 4 * (int64_t)B.nbig * B.tmax2));
        CK(h->alloc(&B.inv_norm, B.nbig));
        CK(h->alloc(&B.stop, B.nbig));
    }
    CK(upload(h, &d.clq_size, size, s));
    CK(upload(h, &d.clq_off, h->off_host, s));
    CK(upload(h, &d.gather, gather, s));
    CK(upload(h, &d.perm, perm, s));
    CK(h->alloc(&d.xi, d.ldU));
    CK(h->alloc(&d.xtmp, d.ldU));
    HIP_OK(hipMemsetAsync(d.xi, 0, (size_t)d.ldU * sizeof(double), s));
    HIP_OK(hipMemsetAsync(d.xtmp, 0, (size_t)d.ldU * sizeof(double), s));
    CK(upload(h, &d.inv_ptr, inv_ptr, s));
    CK(upload(h, &d.inv_slot, inv_slot, s));
    CK(upload(h, &d.heavy, heavy, s));
    CK(upload(h, &d.invD, invD, s));
    CK(upload(h, &d.s2, s2, s));
    CK(upload(h, &d.wt, wt, s));
    CK(upload(h, &d.c, c, s));
    CK(upload(h, &d.b, b, s));
    CK(upload(h, &d.order, order, s));
    std::vector<int64_t> vwoff((size_t)p + 1, 0);
    for (int32_t k = 0; k < p; ++k)
        vwoff[(size_t)k + 1] = vwoff[(size_t)k] + (int64_t)size[(size_t)k] * size[(size_t)k];
    CK(upload(h, &d.vwoff, vwoff, s));
    CK(h->alloc(&d.vwarm, vwoff[(size_t)p]));
    d.nwarm = vwoff[(size_t)p];
    launch_identity_blocks(d.clq_size, d.vwoff, p, d.vwarm, s);
    for (int q = 0; q < NBK; ++q) {
        if (bl[(size_t)q].empty()) continue;
        Bucket bk{bmax[q], (int)bl[(size_t)q].size(), nullptr};
        CK(upload(h, &bk.ids, bl[(size_t)q], s));
        h->buckets.push_back(bk);
    }
    CK(h->alloc(&d.t, d.ldM));
    CK(h->alloc(&d.tpart, 8 * d.ldM));
    CK(h->alloc(&d.y1, d.ldM));
    CK(h->alloc(&d.dslot, d.nslots));
    HIP_OK(hipMemsetAsync(d.dslot, 0, (size_t)d.nslots * sizeof(float), s));
    {
        std::vector<uint32_t> bits((size_t)((d.nU + 31) / 32), 0u);
        for (int64_t e = 0; e < d.nU; ++e)
            if (wt[(size_t)e] == 2.0) bits[(size_t)(e >> 5)] |= 1u << (e & 31);
        CK(upload(h, &d.wbits, bits, s));
    }
    CK(h->alloc(&d.cpart, 4 * (int64_t)(p + d.nvb)));
    HIP_OK(hipMemsetAsync(d.cpart, 0, (size_t)(4 * (p + d.nvb)) * sizeof(double), s));
    CK(h->alloc(&d.vpart, 5 * (int64_t)vupdate_blocks(d)));
    CK(h->alloc(&d.obj, 2));
    CK(h->alloc(&d.opart, objective_partials()));
    CK(h->alloc(&d.info, 4));
    HIP_OK(hipMemsetAsync(d.info, 0, 4 * sizeof(int32_t), s));
    CK(h->alloc(&d.ctl, 1));
    CK(h->alloc(&h->ticket, 1));
    HIP_OK(hipMemsetAsync(h->ticket, 0, sizeof(unsigned long long), s));
    HIP_OK(hipHostMalloc((void **)&d.ctl_host, sizeof(Ctl), hipHostMallocDefault));
    d.hist_cap = 0;
    return CDCS_OK;
}

// Keep the inverse factors as CSR when L^-1 holds under an eighth of the
// entries of a triangle (nearly diagonal M, e.g. sparse constraints that
// rarely share an entry): the two triangular products then read their
// nonzeros only.  The dense copies are released.
cdcs_status compress_factors(cdcs_handle *h, hipStream_t s) {
    Dev &d = h->d;
    const int m = d.m;
    std::vector<int32_t> cnt((size_t)m);
    int32_t *cnt_d = nullptr;
    HIP_OK(hipMalloc(&cnt_d, (size_t)m * sizeof(int32_t)));
    launch_tri_count(d.Linv, m, 0, cnt_d, s);
    hipError_t e = hipMemcpyAsync(cnt.data(), cnt_d, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(cnt_d);
        return fail(CDCS_E_DEVICE, std::string("factor nonzero count: ") + hipGetErrorString(e));
    }
    int64_t nnz = 0;
    for (int32_t c : cnt) nnz += c;
    const int64_t tri = (int64_t)m * (m + 1) / 2;
    if (nnz * 8 >= tri || nnz >= ((int64_t)1 << 31)) {
        (void)hipFree(cnt_d);
        return CDCS_OK;
    }
    // CSR of L^-1; L^-T's rows are L^-1's columns, counted from the dense transpose
    std::vector<int32_t> ptr((size_t)m + 1, 0), tcnt((size_t)m), tptr((size_t)m + 1, 0);
    for (int i = 0; i < m; ++i) ptr[(size_t)i + 1] = ptr[(size_t)i] + cnt[(size_t)i];
    launch_tri_count(d.LinvT, m, 1, cnt_d, s);
    e = hipMemcpyAsync(tcnt.data(), cnt_d, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(cnt_d);
    if (e != hipSuccess) return fail(CDCS_E_DEVICE, std::string("factor nonzero count: ") + hipGetErrorString(e));
    for (int i = 0; i < m; ++i) tptr[(size_t)i + 1] = tptr[(size_t)i] + tcnt[(size_t)i];
    if (tptr[(size_t)m] != nnz) return fail(CDCS_E_NUMERIC, "inverse factor and its transpose differ in nonzeros");
    CK(upload(h, &d.li_ptr, ptr, s));
    CK(upload(h, &d.lt_ptr, tptr, s));
    CK(h->alloc(&d.li_col, nnz));
    CK(h->alloc(&d.li_val, nnz));
    CK(h->alloc(&d.lt_col, nnz));
    CK(h->alloc(&d.lt_val, nnz));
    launch_tri_compress(d.Linv, m, 0, d.li_ptr, d.li_col, d.li_val, s);
    launch_tri_compress(d.LinvT, m, 1, d.lt_ptr, d.lt_col, d.lt_val, s);
    HIP_OK(hipStreamSynchronize(s));
    // drop the dense copies
    for (double *p : {d.Linv, d.LinvT}) {
        h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), (void *)p), h->allocs.end());
        (void)hipFree(p);
    }
    d.Linv = nullptr;
    d.LinvT = nullptr;
    d.sparse_linv = 1;
    d.nnz_linv = nnz;
    return CDCS_OK;
}

// Symbolic sparse Cholesky of M = A D^-1 A^T (host, integer work).  The graph
// of M joins two constraints that share a pattern entry; its elimination
// order (perfect when the graph is chordal, else minimum degree) gives the
// structure of every column of L (factor order), the elimination tree
// (parent = first row below the diagonal), its levels (a column's
// descendants are in lower levels), the row lists (columns k < j with
// L_jk != 0 and where row j sits in column k) and the structure of
// X = L^-1: column j is nonzero on the tree path from j to its root.
// Returns false when a path is longer than max_path or X would hold more
// than max_x entries (then the dense factor is used).
struct SpSym {
    std::vector<int32_t> order, pinv, cp, ri, rk_ptr, rk_col, rk_pos, level_cols, level_off, xr;
    std::vector<int64_t> xp;
};

bool sp_symbolic(int32_t m, const std::vector<int32_t> &tcp, const std::vector<int32_t> &tcr, int max_path,
                 int64_t max_x, SpSym &S) {
    std::vector<std::vector<int32_t>> adj((size_t)m);
    for (size_t t = 0; t + 1 < tcp.size(); ++t)
        for (int32_t a = tcp[t]; a < tcp[t + 1]; ++a)
            for (int32_t b2 = tcp[t]; b2 < a; ++b2) {
                adj[(size_t)tcr[(size_t)a]].push_back(tcr[(size_t)b2]);
                adj[(size_t)tcr[(size_t)b2]].push_back(tcr[(size_t)a]);
            }
    for (auto &l : adj) {
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
    }
    std::vector<char> used((size_t)m, 1);
    std::vector<std::vector<int32_t>> later;
    elimination_order(m, adj, used, S.order, later);
    if ((int32_t)S.order.size() != m) return false;
    S.pinv.assign((size_t)m, 0);
    for (int32_t j = 0; j < m; ++j) S.pinv[(size_t)S.order[(size_t)j]] = j;
    S.cp.assign(1, 0);
    std::vector<int32_t> parent((size_t)m, -1), col;
    for (int32_t j = 0; j < m; ++j) {
        col.assign(1, j);
        for (int32_t u : later[(size_t)S.order[(size_t)j]]) col.push_back(S.pinv[(size_t)u]);
        std::sort(col.begin() + 1, col.end());
        if (col.size() > 1) parent[(size_t)j] = col[1];
        S.ri.insert(S.ri.end(), col.begin(), col.end());
        S.cp.push_back((int32_t)S.ri.size());
    }
    // levels: a column after all of its descendants
    std::vector<int32_t> lev((size_t)m, 0);
    int32_t nlev = 0;
    for (int32_t j = 0; j < m; ++j) {
        nlev = std::max(nlev, lev[(size_t)j] + 1);
        if (parent[(size_t)j] >= 0)
            lev[(size_t)parent[(size_t)j]] = std::max(lev[(size_t)parent[(size_t)j]], lev[(size_t)j] + 1);
    }
    S.level_off.assign((size_t)nlev + 1, 0);
    for (int32_t j = 0; j < m; ++j) ++S.level_off[(size_t)lev[(size_t)j] + 1];
    for (int32_t l = 0; l < nlev; ++l) S.level_off[(size_t)l + 1] += S.level_off[(size_t)l];
    S.level_cols.assign((size_t)m, 0);
    {
        std::vector<int32_t> fp(S.level_off.begin(), S.level_off.end() - 1);
        for (int32_t j = 0; j < m; ++j) S.level_cols[(size_t)fp[(size_t)lev[(size_t)j]]++] = j;
    }
    // row lists (k increasing)
    std::vector<int32_t> rcount((size_t)m, 0);
    for (int32_t k = 0; k < m; ++k)
        for (int32_t q = S.cp[(size_t)k] + 1; q < S.cp[(size_t)k + 1]; ++q) ++rcount[(size_t)S.ri[(size_t)q]];
    S.rk_ptr.assign((size_t)m + 1, 0);
    for (int32_t j = 0; j < m; ++j) S.rk_ptr[(size_t)j + 1] = S.rk_ptr[(size_t)j] + rcount[(size_t)j];
    S.rk_col.resize((size_t)S.rk_ptr[(size_t)m]);
    S.rk_pos.resize((size_t)S.rk_ptr[(size_t)m]);
    {
        std::vector<int32_t> fp(S.rk_ptr.begin(), S.rk_ptr.end() - 1);
        for (int32_t k = 0; k < m; ++k)
            for (int32_t q = S.cp[(size_t)k] + 1; q < S.cp[(size_t)k + 1]; ++q) {
                const int32_t i = S.ri[(size_t)q];
                S.rk_col[(size_t)fp[(size_t)i]] = k;
                S.rk_pos[(size_t)fp[(size_t)i]++] = q - S.cp[(size_t)k];
            }
    }
    // X = L^-1 by columns: the tree paths
    std::vector<int32_t> plen((size_t)m, 1);
    int64_t nx = 0;
    for (int32_t j = m - 1; j >= 0; --j) {
        if (parent[(size_t)j] >= 0) plen[(size_t)j] = 1 + plen[(size_t)parent[(size_t)j]];
        if (plen[(size_t)j] > max_path) return false;
        nx += plen[(size_t)j];
    }
    if (nx > max_x) return false;
    S.xp.assign(1, 0);
    S.xr.reserve((size_t)nx);
    for (int32_t j = 0; j < m; ++j) {
        for (int32_t v = j; v >= 0; v = parent[(size_t)v]) S.xr.push_back(v);
        S.xp.push_back((int64_t)S.xr.size());
    }
    return true;
}

// Numeric sparse factor on the device from the symbolic step, then the CSR
// copies the affine step multiplies by: y1 = L^-1 (P t) with the columns
// labelled by the original rows, and y = P^T L^-T y1 with the rows labelled
// by the original rows (P M P^T = L L^T, so M^-1 = P^T L^-T L^-1 P).
cdcs_status sparse_factor(cdcs_handle *h, const SpSym &S, const int32_t *tid_d, double shift, hipStream_t s) {
    Dev &d = h->d;
    const int32_t m = d.m;
    SpFactor f;
    int32_t *order_d, *pinv_d, *cp_d, *ri_d, *rkp_d, *rkc_d, *rkq_d, *lc_d, *xr_d;
    int64_t *xp_d;
    CK(upload(h, &order_d, S.order, s));
    CK(upload(h, &pinv_d, S.pinv, s));
    CK(upload(h, &cp_d, S.cp, s));
    CK(upload(h, &ri_d, S.ri, s));
    CK(upload(h, &rkp_d, S.rk_ptr, s));
    CK(upload(h, &rkc_d, S.rk_col, s));
    CK(upload(h, &rkq_d, S.rk_pos, s));
    CK(upload(h, &lc_d, S.level_cols, s));
    CK(upload(h, &xp_d, S.xp, s));
    CK(upload(h, &xr_d, S.xr, s));
    f.order = order_d;
    f.pinv = pinv_d;
    f.cp = cp_d;
    f.ri = ri_d;
    f.rk_ptr = rkp_d;
    f.rk_col = rkc_d;
    f.rk_pos = rkq_d;
    f.level_cols = lc_d;
    f.xp = xp_d;
    f.xr = xr_d;
    const int64_t nnzL = (int64_t)S.ri.size(), nnzX = (int64_t)S.xr.size();
    CK(h->alloc(&f.Lv, nnzL));
    CK(h->alloc(&f.diag0, m));
    CK(h->alloc(&f.xv, nnzX));
    launch_spchol_fill(d, f, tid_d, shift, s);
    launch_spchol(d, f, S.level_off, d.info, s);
    // CSR copies: rows of X (columns relabelled to original rows) and rows of
    // P^T X^T (= columns of X, in original row order)
    std::vector<int32_t> li_ptr((size_t)m + 1, 0), li_col((size_t)nnzX), lt_ptr((size_t)m + 1, 0),
        lt_col((size_t)nnzX);
    std::vector<int64_t> li_idx((size_t)nnzX), lt_idx((size_t)nnzX);
    for (int64_t q = 0; q < nnzX; ++q) ++li_ptr[(size_t)S.xr[(size_t)q] + 1];
    for (int32_t r = 0; r < m; ++r) li_ptr[(size_t)r + 1] += li_ptr[(size_t)r];
    {
        std::vector<int32_t> fp(li_ptr.begin(), li_ptr.end() - 1);
        for (int32_t cidx = 0; cidx < m; ++cidx)  // columns increasing: each row's columns increase
            for (int64_t q = S.xp[(size_t)cidx]; q < S.xp[(size_t)cidx + 1]; ++q) {
                const int32_t r = S.xr[(size_t)q];
                li_col[(size_t)fp[(size_t)r]] = S.order[(size_t)cidx];
                li_idx[(size_t)fp[(size_t)r]++] = q;
            }
    }
    for (int32_t i = 0; i < m; ++i) {
        const int32_t cidx = S.pinv[(size_t)i];
        lt_ptr[(size_t)i + 1] = lt_ptr[(size_t)i] + (int32_t)(S.xp[(size_t)cidx + 1] - S.xp[(size_t)cidx]);
        int64_t o = lt_ptr[(size_t)i];
        for (int64_t q = S.xp[(size_t)cidx]; q < S.xp[(size_t)cidx + 1]; ++q, ++o) {
            lt_col[(size_t)o] = S.xr[(size_t)q];
            lt_idx[(size_t)o] = q;
        }
    }
    int64_t *li_idx_d = nullptr, *lt_idx_d = nullptr;
    CK(upload(h, &d.li_ptr, li_ptr, s));
    CK(upload(h, &d.li_col, li_col, s));
    CK(upload(h, &d.lt_ptr, lt_ptr, s));
    CK(upload(h, &d.lt_col, lt_col, s));
    CK(upload(h, &li_idx_d, li_idx, s));
    CK(upload(h, &lt_idx_d, lt_idx, s));
    CK(h->alloc(&d.li_val, nnzX));
    CK(h->alloc(&d.lt_val, nnzX));
    launch_gather_vals(f.xv, li_idx_d, d.li_val, nnzX, s);
    launch_gather_vals(f.xv, lt_idx_d, d.lt_val, nnzX, s);
    int32_t info_h[4] = {0, 0, 0, 0};
    HIP_OK(hipMemcpyAsync(info_h, d.info, sizeof(info_h), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (info_h[0] != 0)
        return fail(CDCS_E_RANK,
                    "A D^-1 A^T is not positive definite (pivot " + std::to_string(info_h[1]) + "): A is rank deficient");
    d.sparse_linv = 1;
    d.spchol = 1;
    d.nnz_linv = nnzX;
    d.nnz_l = nnzL;
    return CDCS_OK;
}

// KKT factor of M = Aw diag(s2) Aw^T + shift I with s2 = d.s2, into d's
// factor fields: sparse when A is kept sparse and the factor's inverse stays
// sparse (the symbolic step decides); otherwise M dense, Cholesky, inverse
// factors (kept as CSR when sparse enough).
cdcs_status factor_into(cdcs_handle *h, double shift, hipStream_t s) {
    Dev &d = h->d;
    const int64_t m = d.m;
    if (d.sparse) {
        SpSym S;
        if (sp_symbolic((int32_t)m, h->sym_tcp, h->sym_tcr, spinv_max_path(), (int64_t)m * (m + 1) / 2 / 8, S))
            return sparse_factor(h, S, h->sym_tid, shift, s);
    }
    if (m > 8192) return fail(CDCS_E_ARG, "m > 8192 is not supported by the dense factor");
    double *M = nullptr, *diag0 = nullptr;
    HIP_OK(hipMalloc(&M, (size_t)m * m * sizeof(double)));
    hipError_t e1 = hipMalloc(&diag0, (size_t)m * sizeof(double));
    if (e1 != hipSuccess) {
        (void)hipFree(M);
        return fail(CDCS_E_NOMEM, "hipMalloc diag");
    }
    CK(h->alloc(&d.Linv, m * m));
    CK(h->alloc(&d.LinvT, m * m));
    if (d.sparse) launch_sp_syrk(d, h->sym_tid, M, s);
    else launch_syrk(d.Aw, d.ldU, d.s2, (int)m, M, s);
    if (shift != 0.0) launch_add_diag(M, (int)m, shift, s);
    launch_potrf(M, (int)m, diag0, d.info, s);
    launch_trtri(M, (int)m, d.LinvT, d.Linv, s);
    int32_t info_h[4] = {0, 0, 0, 0};
    hipError_t e2 = hipMemcpyAsync(info_h, d.info, sizeof(info_h), hipMemcpyDeviceToHost, s);
    hipError_t e3 = hipStreamSynchronize(s);
    (void)hipFree(M);
    (void)hipFree(diag0);
    if (e2 != hipSuccess || e3 != hipSuccess)
        return fail(CDCS_E_DEVICE, std::string("setup kernels: ") + hipGetErrorString(e2 != hipSuccess ? e2 : e3));
    if (info_h[0] != 0)
        return fail(CDCS_E_RANK,
                    "A D^-1 A^T is not positive definite (pivot " + std::to_string(info_h[1]) + "): A is rank deficient");
    CK(compress_factors(h, s));
    if (d.sparse_linv) return CDCS_OK;
    // dense inverse factor: keep M^-1 = L^-T L^-1 instead, so each solve is one product
    CK(h->alloc(&d.Minv, m * m));
    launch_inv_product(d.LinvT, (int)m, d.Minv, s);
    HIP_OK(hipStreamSynchronize(s));
    for (double *p : {d.Linv, d.LinvT}) {
        h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), (void *)p), h->allocs.end());
        (void)hipFree(p);
    }
    d.Linv = nullptr;
    d.LinvT = nullptr;
    return CDCS_OK;
}

cdcs_status create_side_streams(cdcs_handle *h) {
    for (int i = 0; i < kSideStreams; ++i) {
        HIP_OK(hipStreamCreateWithFlags(&h->side[i], hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&h->join_ev[i], hipEventDisableTiming));
    }
    HIP_OK(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
    return CDCS_OK;
}

cdcs_status build(cdcs_handle *h, const cdcs_pattern *pat, const cdcs_constraints *A, const double *b,
                  const double *c, const cdcs_cliques *cl, const cdcs_vcones *cones, hipStream_t s) {
    Dev &d = h->d;
    HostProblem P;
    CK(host_problem(pat, A, b, c, cl, cones, 64, true, P));
    d.n = P.n;
    d.m = P.m;
    d.p = P.p;
    d.nU = P.nU;
    d.smax = P.smax;
    d.nslots = P.nslots;
    d.nslots_psd = P.nslots_psd;
    d.nvc = P.nvc;
    d.nvb = (int32_t)(P.vblk.size() / 4);
    if (d.nvb > 0) CK(upload(h, &d.vblk, P.vblk, s));
    d.nsoc = (int32_t)(P.soc.size() / 3);
    if (d.nsoc > 0) {
        CK(upload(h, &d.soc, P.soc, s));
        d.nsocb = (int32_t)P.socb.size();
        CK(upload(h, &d.socb, P.socb, s));
        CK(h->alloc(&d.soc_part, d.nvb));
    }
    d.ldU = P.ld;
    d.ldM = round_up(P.m, 32);  // rows of A^T start on 128-byte lines
    h->off_host = P.off;
    // u is padded to ldU (the A u kernel reads whole 4-wide groups)
    std::vector<double> pad_invD(P.invD), pad_s2(P.s2), pad_wt(P.wt);
    pad_invD.resize((size_t)d.ldU, 0.0);
    pad_s2.resize((size_t)d.ldU, 0.0);
    pad_wt.resize((size_t)d.ldU, 0.0);
    CK(upload_common(h, P.size, P.gather, P.cnt, pad_wt, pad_invD, pad_s2, P.c, P.b, P.perm, heavy_threshold(), s));
    CK(h->alloc(&d.spart, 2 * (int64_t)scatter_blocks(d)));
    CK(h->alloc(&d.u, d.ldU));
    HIP_OK(hipMemsetAsync(d.u, 0, (size_t)d.ldU * sizeof(double), s));
    const int64_t nU = P.nU, m = P.m;
    std::vector<int32_t> tid;  // touched-entry index of each coefficient (sparse setup only)
    std::vector<int32_t> tcp_h, tcr_h;  // the touched entries' constraint rows (sparse setup only)
    if (P.sparse) {
        // Coefficients by touched entry (the columns of A that are not zero).
        d.sparse = 1;
        d.nnzA = (int64_t)P.sp_col.size();
        std::vector<int32_t> ccount((size_t)nU, 0), tc_of((size_t)nU, -1), tc_e, tc_ptr(1, 0), tc_row;
        std::vector<double> tc_val;
        for (int32_t e : P.sp_col) ++ccount[(size_t)e];
        for (int64_t e = 0; e < nU; ++e)
            if (ccount[(size_t)e] > 0) {
                tc_of[(size_t)e] = (int32_t)tc_e.size();
                tc_e.push_back((int32_t)e);
                tc_ptr.push_back(tc_ptr.back() + ccount[(size_t)e]);
            }
        d.ntc = (int32_t)tc_e.size();
        tc_row.resize((size_t)d.nnzA);
        tc_val.resize((size_t)d.nnzA);
        tid.resize((size_t)d.nnzA);
        std::vector<int32_t> fillp(tc_ptr.begin(), tc_ptr.end() - 1);
        for (int32_t i = 0; i < (int32_t)m; ++i)
            for (int32_t q = P.sp_ptr[(size_t)i]; q < P.sp_ptr[(size_t)i + 1]; ++q) {
                const int32_t t = tc_of[(size_t)P.sp_col[(size_t)q]];
                tid[(size_t)q] = t;
                tc_row[(size_t)fillp[(size_t)t]] = i;
                tc_val[(size_t)fillp[(size_t)t]++] = P.sp_val[(size_t)q];
            }
        CK(upload(h, &d.sp_ptr, P.sp_ptr, s));
        CK(upload(h, &d.sp_col, P.sp_col, s));
        CK(upload(h, &d.sp_val, P.sp_val, s));
        CK(upload(h, &d.tc_e, tc_e, s));
        CK(upload(h, &d.tc_ptr, tc_ptr, s));
        CK(upload(h, &d.tc_row, tc_row, s));
        CK(upload(h, &d.tc_val, tc_val, s));
        tcp_h.swap(tc_ptr);
        tcr_h.swap(tc_row);
    } else {
        // A (w-scaled, FP32) row-major and transposed.
        std::vector<float> AwT((size_t)(nU * d.ldM), 0.0f);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t e = 0; e < nU; ++e) AwT[(size_t)(e * d.ldM + i)] = P.Aw[(size_t)(i * d.ldU + e)];
        CK(upload(h, &d.Aw, P.Aw, s));
        CK(upload(h, &d.AwT, AwT, s));
    }

    if (d.sparse) {
        h->sym_tcp.swap(tcp_h);
        h->sym_tcr.swap(tcr_h);
        CK(upload(h, &h->sym_tid, tid, s));
    }
    CK(factor_into(h, 0.0, s));
    CK(create_side_streams(h));
    CK(tune_projection(h, s));
    HIP_OK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    return CDCS_OK;
}

// Many SDPs: concatenate every instance's entries, cliques, slots and rows.
cdcs_status build_batch(cdcs_handle *h, int32_t nprob, const cdcs_problem *probs, hipStream_t s) {
    Dev &d = h->d;
    if (nprob < 1 || !probs) return fail(CDCS_E_ARG, "no problems");
    h->batch_host.reset(new Batch());
    d.batch = h->batch_host.get();
    Batch &B = *d.batch;
    B.nprob = nprob;
    std::vector<int64_t> U_off(1, 0), A_off, F_off;
    std::vector<int32_t> m_off(1, 0), k_off(1, 0), A_ld, einst, rinst, kinst;
    std::vector<int32_t> size, gather, cnt, perm;
    std::vector<double> wt, invD, s2, c, b;
    std::vector<float> Aw;
    std::vector<int32_t> sblk, sblk_off(1, 0), vblk, vblk_off(1, 0), syrk_jobs, trtri_jobs, rjobs, ejobs, nch;
    std::vector<int64_t> p_off;
    int64_t ptot = 0;
    h->off_host.assign(1, 0);
    int64_t Atot = 0, Ftot = 0;
    d.smax = 0;
    d.n = 0;
    for (int32_t q = 0; q < nprob; ++q) {
        HostProblem P;
        const cdcs_problem &pr = probs[q];
        cdcs_status st = host_problem(pr.pattern, pr.A, pr.b, pr.c, pr.cliques, nullptr, 4, false, P);
        if (st != CDCS_OK) return fail(st, "problem " + std::to_string(q) + ": " + g_err);
        if (P.m > 256) return fail(CDCS_E_ARG, "problem " + std::to_string(q) + ": batched factors need m <= 256");
        if (P.smax > kMaxLdsClique)
            return fail(CDCS_E_ARG, "problem " + std::to_string(q) + ": batch handles take cliques of at most " +
                                        std::to_string(kMaxLdsClique) + " vertices");
        const int64_t u0 = U_off.back();
        const int64_t slot0 = h->off_host.back();
        for (int32_t k = 0; k < P.p; ++k) {
            size.push_back(P.size[(size_t)k]);
            h->off_host.push_back(slot0 + P.off[(size_t)k + 1]);
            kinst.push_back(q);
        }
        for (int32_t g : P.gather) gather.push_back((int32_t)(u0 + g));
        for (int32_t e : P.perm) perm.push_back((int32_t)(u0 + e));
        cnt.insert(cnt.end(), P.cnt.begin(), P.cnt.end());
        wt.insert(wt.end(), P.wt.begin(), P.wt.end());
        invD.insert(invD.end(), P.invD.begin(), P.invD.end());
        s2.insert(s2.end(), P.s2.begin(), P.s2.end());
        c.insert(c.end(), P.c.begin(), P.c.end());
        b.insert(b.end(), P.b.begin(), P.b.end());
        for (int64_t e = 0; e < P.nU; ++e) einst.push_back(q);
        for (int32_t i = 0; i < P.m; ++i) rinst.push_back(q);
        // rows of A_q start on 128-byte lines (leading dimension a multiple of
        // 32 floats), so the column blocks of the A^T y product touch no
        // straddled line
        const int64_t ldq = round_up(P.nU, 32);
        A_off.push_back(Atot);
        A_ld.push_back((int32_t)ldq);
        Aw.resize((size_t)(Atot + P.m * ldq), 0.0f);
        for (int32_t i = 0; i < P.m; ++i)
            std::copy(P.Aw.begin() + (size_t)i * P.ld, P.Aw.begin() + (size_t)i * P.ld + P.nU,
                      Aw.begin() + (size_t)(Atot + i * ldq));
        Atot += P.m * ldq;
        F_off.push_back(Ftot);
        Ftot += (int64_t)P.m * P.m;
        // scatter blocks of <= 256 entries inside the instance
        for (int64_t e0 = 0; e0 < P.nU; e0 += 256) {
            sblk.push_back(q);
            sblk.push_back((int32_t)(u0 + e0));
            sblk.push_back((int32_t)(u0 + std::min<int64_t>(P.nU, e0 + 256)));
            sblk.push_back(0);
        }
        sblk_off.push_back((int32_t)(sblk.size() / 4));
        // Alg. 2 epilogue blocks of <= 256 slots inside the instance
        for (int64_t s0 = 0; s0 < P.nslots; s0 += 256) {
            vblk.push_back(q);
            vblk.push_back((int32_t)(slot0 + s0));
            vblk.push_back((int32_t)(slot0 + std::min<int64_t>(P.nslots, s0 + 256)));
            vblk.push_back(0);
        }
        vblk_off.push_back((int32_t)(vblk.size() / 4));
        const int T = (P.m + 31) / 32;
        for (int I = 0; I < T; ++I)
            for (int J = 0; J <= I; ++J) {
                syrk_jobs.push_back(q);
                syrk_jobs.push_back(I);
                syrk_jobs.push_back(J);
                syrk_jobs.push_back(0);
            }
        for (int32_t j = 0; j < P.m; ++j) {
            trtri_jobs.push_back(q);
            trtri_jobs.push_back(j);
        }
        const int32_t nc = (int32_t)((P.nU + kBatchAuChunk - 1) / kBatchAuChunk);
        nch.push_back(nc);
        p_off.push_back(ptot);
        if (nc > 1) ptot += (int64_t)P.m * nc;
        // chunk-major: the row groups that share one u chunk are consecutive
        for (int32_t c = 0; c < nc; ++c)
            for (int32_t r = 0; r < P.m; r += 4) {
                rjobs.push_back(q);
                rjobs.push_back(m_off.back() + r);
                rjobs.push_back(std::min<int32_t>(4, P.m - r));
                rjobs.push_back(c);
            }
        for (int64_t e0 = 0; e0 < P.nU; e0 += 1024) {
            ejobs.push_back(q);
            ejobs.push_back((int32_t)e0);
        }
        U_off.push_back(u0 + P.nU);
        m_off.push_back(m_off.back() + P.m);
        k_off.push_back(k_off.back() + P.p);
        d.smax = std::max(d.smax, P.smax);
        d.n += P.n;
    }
    d.nU = U_off.back();
    d.m = m_off.back();
    d.p = k_off.back();
    d.nslots = h->off_host.back();
    d.nslots_psd = d.nslots;
    if (d.nU >= (int64_t)1 << 31 || d.nslots >= (int64_t)1 << 31) return fail(CDCS_E_ARG, "batch too large");
    d.ldU = d.nU;
    d.ldM = round_up(d.m, 4);
    CK(upload_common(h, size, gather, cnt, wt, invD, s2, c, b, perm, 1 << 30, s));
    CK(h->alloc(&d.u, d.nU));
    CK(upload(h, &d.Aw, Aw, s));
    CK(upload(h, &B.U_off, U_off, s));
    CK(upload(h, &B.m_off, m_off, s));
    CK(upload(h, &B.k_off, k_off, s));
    CK(upload(h, &B.A_off, A_off, s));
    CK(upload(h, &B.A_ld, A_ld, s));
    CK(upload(h, &B.F_off, F_off, s));
    CK(upload(h, &B.einst, einst, s));
    CK(upload(h, &B.rinst, rinst, s));
    CK(upload(h, &B.kinst, kinst, s));
    CK(upload(h, &B.sblk, sblk, s));
    CK(upload(h, &B.sblk_off, sblk_off, s));
    CK(upload(h, &B.syrk_jobs, syrk_jobs, s));
    CK(upload(h, &B.trtri_jobs, trtri_jobs, s));
    // A u jobs by XCD: workgroups are handed to the 8 XCDs round robin
    // (workgroup b to XCD b mod 8), each with its own L2.  The job list (in
    // instance, chunk, row-group order) is cut into 8 contiguous segments of
    // equal work and workgroup b takes the next 4 jobs of segment b mod 8, so
    // the waves that share a u chunk run on one XCD, mostly on one CU.  Unused
    // slots hold rows = 0.  The order only affects speed: every row's chunk
    // partials are summed in chunk order.
    {
        const size_t nj = rjobs.size() / 4;
        std::vector<int64_t> wsum(nj + 1, 0);
        for (size_t t = 0; t < nj; ++t) {
            const int32_t q = rjobs[t * 4];
            const int64_t nUq = U_off[(size_t)q + 1] - U_off[(size_t)q];
            const int64_t c0 = (int64_t)rjobs[t * 4 + 3] * kBatchAuChunk;
            wsum[t + 1] = wsum[t] + std::min<int64_t>(kBatchAuChunk, nUq - c0) * rjobs[t * 4 + 2];
        }
        size_t bnd[kXcds + 1];
        for (int x = 0; x <= kXcds; ++x)
            bnd[x] = (size_t)(std::lower_bound(wsum.begin(), wsum.end(), wsum[nj] * x / kXcds) - wsum.begin());
        bnd[kXcds] = nj;
        size_t wg = 0;
        for (int x = 0; x < kXcds; ++x) wg = std::max(wg, (bnd[x + 1] - bnd[x] + 3) / 4);
        std::vector<int32_t> slots(wg * kXcds * 4 * 4, 0);
        for (int x = 0; x < kXcds; ++x)
            for (size_t k = 0; k < bnd[x + 1] - bnd[x]; ++k) {
                const size_t slot = ((k / 4) * kXcds + (size_t)x) * 4 + k % 4;
                std::copy(rjobs.begin() + (bnd[x] + k) * 4, rjobs.begin() + (bnd[x] + k) * 4 + 4,
                          slots.begin() + slot * 4);
            }
        rjobs.swap(slots);
    }
    // A^T y blocks of the instances with the most constraints first, so no long
    // job starts last
    {
        std::vector<int32_t> eorder((size_t)(ejobs.size() / 2));
        for (size_t t = 0; t < eorder.size(); ++t) eorder[t] = (int32_t)t;
        auto ework = [&](int32_t t) {
            const int32_t q = ejobs[(size_t)t * 2];
            return m_off[(size_t)q + 1] - m_off[(size_t)q];
        };
        std::stable_sort(eorder.begin(), eorder.end(), [&](int32_t a, int32_t b) { return ework(a) > ework(b); });
        std::vector<int32_t> esorted;
        esorted.reserve(ejobs.size());
        for (int32_t t : eorder) esorted.insert(esorted.end(), ejobs.begin() + (size_t)t * 2, ejobs.begin() + (size_t)t * 2 + 2);
        ejobs.swap(esorted);
    }
    CK(upload(h, &B.rjobs, rjobs, s));
    CK(upload(h, &B.ejobs, ejobs, s));
    CK(upload(h, &B.nch, nch, s));
    CK(upload(h, &B.p_off, p_off, s));
    B.split = ptot > 0;
    CK(h->alloc(&B.tpart, std::max<int64_t>(ptot, 1)));
    B.nrjobs = (int32_t)(rjobs.size() / 4);
    B.nejobs = (int32_t)(ejobs.size() / 2);
    B.nsblk = (int32_t)(sblk.size() / 4);
    B.nsyrk = (int32_t)(syrk_jobs.size() / 4);
    CK(h->alloc(&d.spart, 2 * (int64_t)B.nsblk));
    CK(upload(h, &B.vblk, vblk, s));
    CK(upload(h, &B.vblk_off, vblk_off, s));
    B.nvblk = (int32_t)(vblk.size() / 4);
    CK(h->alloc(&d.vpart, 5 * (int64_t)B.nvblk));  // per slot block (the single-SDP layout is per 256 slots)
    CK(h->alloc(&B.istop, nprob));
    HIP_OK(hipMemsetAsync(B.istop, 0, (size_t)nprob * sizeof(int32_t), s));
    CK(h->alloc(&B.iiters, nprob));
    CK(h->alloc(&B.itime, nprob));
    CK(h->alloc(&B.t0, 1));
    CK(h->alloc(&B.ieps, 2 * (int64_t)nprob));
    HIP_OK(hipMemsetAsync(B.ieps, 0, (size_t)(2 * nprob) * sizeof(double), s));
    CK(h->alloc(&B.iobj, 2 * (int64_t)nprob));
    CK(h->alloc(&B.nrunning, 1));
    CK(h->alloc(&B.finfo, nprob));
    HIP_OK(hipMemsetAsync(B.finfo, 0, (size_t)nprob * sizeof(int32_t), s));
    // per-instance KKT factors
    double *M = nullptr;
    HIP_OK(hipMalloc(&M, (size_t)std::max<int64_t>(Ftot, 1) * sizeof(double)));
    CK(h->alloc(&d.Linv, Ftot));
    CK(h->alloc(&d.LinvT, Ftot));
    launch_bsetup(d, M, s);
    std::vector<int32_t> finfo((size_t)nprob, 0);
    hipError_t e2 = hipMemcpyAsync(finfo.data(), B.finfo, (size_t)nprob * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    hipError_t e3 = hipStreamSynchronize(s);
    (void)hipFree(M);
    if (e2 != hipSuccess || e3 != hipSuccess)
        return fail(CDCS_E_DEVICE, std::string("batch setup kernels: ") + hipGetErrorString(e2 != hipSuccess ? e2 : e3));
    for (int32_t q = 0; q < nprob; ++q)
        if (finfo[(size_t)q] != 0)
            return fail(CDCS_E_RANK, "problem " + std::to_string(q) + ": A D^-1 A^T is not positive definite (pivot " +
                                         std::to_string(finfo[(size_t)q] - 1) + ")");
    CK(create_side_streams(h));
    CK(tune_projection(h, s));
    HIP_OK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    return CDCS_OK;
}

ProjArgs proj_args(const cdcs_handle *h, int mode, const cdcs_state *st, double rho) {
    const Dev &d = h->d;
    ProjArgs a{};
    a.mode = mode;
    a.size = d.clq_size;
    a.off = d.clq_off;
    a.gather = d.gather;
    if (st) {
        a.x = st->x;
        a.blk = st->blk;
        a.lam = st->lam;
        a.v = st->v;
    }
    a.rho = rho;
    a.inv_rho = 1.0 / rho;
    a.kinst = d.batch ? d.batch->kinst : nullptr;
    a.istop = d.batch ? d.batch->istop : nullptr;
    a.vwarm = (st && st->vw) ? st->vw : d.vwarm;
    a.vwoff = d.vwoff;
    a.warm_store = 1;
    a.cpart = d.cpart;
    a.ctl = d.ctl;
    a.dslot = mode == PROJ_PRIMAL ? d.dslot : nullptr;
    if (h->save_evals || h->save_evecs) {
        a.evals = h->save_evals;
        a.eoff = h->diff.eoff;
        a.evecs = h->save_evecs;
        a.voff = d.vwoff;
    }
    return a;
}

// Buffers of the differentiation entry points, allocated once per handle.
cdcs_status diff_buffers(cdcs_handle *h) {
    cdcs_handle::Diff &f = h->diff;
    if (f.c) return CDCS_OK;
    const Dev &d = h->d;
    std::vector<int64_t> eoff((size_t)d.p + 1, 0);
    for (int32_t k = 0; k < d.p; ++k) {
        const int64_t pk = h->off_host[(size_t)k + 1] - h->off_host[(size_t)k];  // s (s + 1) / 2
        const int64_t sk = (int64_t)((std::sqrt(8.0 * (double)pk + 1.0) - 1.0) / 2.0 + 0.5);
        eoff[(size_t)k + 1] = eoff[(size_t)k] + sk;
    }
    CK(upload(h, &f.eoff, eoff, nullptr));
    CK(h->alloc(&f.gP, d.nslots));
    CK(h->alloc(&f.gW, d.nslots));
    CK(h->alloc(&f.hbar, d.nslots));
    CK(h->alloc(&f.x, d.ldU));
    CK(h->alloc(&f.y, d.ldM));
    CK(h->alloc(&f.c, d.ldU));  // last: marks the set as complete
    return CDCS_OK;
}

// The projection of every clique with the handle's plan.
// One launch per size bucket, in stream order on s or (parallel) forked onto
// the side streams and joined back into s: bucket 0 on s, bucket i >= 1 on
// side stream (i - 1) mod kSideStreams.  Each clique is projected by the same
// kernel either way, so both give the same bits.
void launch_buckets(cdcs_handle *h, ProjArgs a, hipStream_t s, bool parallel) {
    const int nb = (int)h->buckets.size();
    const int ns = std::min(nb - 1, kSideStreams);
    if (parallel && ns > 0) {
        (void)hipEventRecord(h->fork_ev, s);
        for (int j = 0; j < ns; ++j) (void)hipStreamWaitEvent(h->side[j], h->fork_ev, 0);
    }
    for (int i = 0; i < nb; ++i) {
        const Bucket &bk = h->buckets[(size_t)i];
        a.nblk = bk.count;
        a.ids = bk.ids;
        launch_project(a, bk.smax, bk.nt, (parallel && i > 0) ? h->side[(i - 1) % kSideStreams] : s);
    }
    if (parallel && ns > 0)
        for (int j = 0; j < ns; ++j) {
            (void)hipEventRecord(h->join_ev[j], h->side[j]);
            (void)hipStreamWaitEvent(s, h->join_ev[j], 0);
        }
}

void launch_plan(cdcs_handle *h, ProjArgs a, hipStream_t s) {
    const Dev &d = h->d;
    launch_big_projection(a, d.big, s);  // cliques above the LDS limit, if any
    if (h->plan.queue) {
        a.nblk = d.p_lds;
        a.ids = d.order;
        launch_project_queue(a, d.smax_lds, h->plan.nt, h->plan.grid, h->ticket, s);
        return;
    }
    launch_buckets(h, a, s, h->plan.parallel);
}

void launch_projection(cdcs_handle *h, int mode, const cdcs_state *st, double rho, hipStream_t s) {
    const ProjArgs a = proj_args(h, mode, st, rho);
    launch_plan(h, a, s);
    launch_project_vec(a, h->d, s);  // vector cones, if any
}

int device_cus(cdcs_handle *h) {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || ncu < 1)
        ncu = 256;
    return ncu;
}

int queue_grid(cdcs_handle *h, int nt) {
    if (h->d.p_lds < 1) return 0;
    const int occ = project_queue_occupancy(h->d.smax_lds, nt);
    return occ < 1 ? 0 : std::min(h->d.p_lds, occ * device_cus(h));
}

// Autotuner: time every candidate launch form of the projection on this
// handle's cliques (generated nearly diagonal blocks, warm-start products on,
// outputs to scratch) and keep the fastest: per size bucket the best
// workgroup size, against the persistent queue launch at 256 or 512 threads.
cdcs_status tune_projection(cdcs_handle *h, hipStream_t s) {
    Dev &d = h->d;
    float *W = nullptr, *P = nullptr, *Vt = nullptr;
    int64_t vtot = 0;
    HIP_OK(hipMemcpy(&vtot, d.vwoff + d.p, sizeof(int64_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMalloc(&W, (size_t)std::max<int64_t>(d.nslots, 1) * sizeof(float)));
    hipError_t e = hipMalloc(&P, (size_t)std::max<int64_t>(d.nslots, 1) * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&Vt, (size_t)std::max<int64_t>(vtot, 1) * sizeof(float));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(W);
        (void)hipFree(P);
        (void)hipFree(Vt);
    };
    if (e != hipSuccess) {
        cleanup();
        return fail(CDCS_E_NOMEM, "autotuner scratch");
    }
    launch_tune_blocks(d.clq_size, d.clq_off, d.p, W, s);
    launch_identity_blocks(d.clq_size, d.vwoff, d.p, Vt, s);
    ProjArgs a = proj_args(h, PROJ_STANDALONE, nullptr, 1.0);
    a.Win = W;
    a.Pout = P;
    a.vwarm = Vt;
    a.warm_store = 0;
    a.kinst = nullptr;
    a.istop = nullptr;
    a.ctl = nullptr;
    constexpr int REPS = 3;
    auto time_us = [&](auto &&launch) -> float {
        launch();  // warm
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < REPS; ++r) launch();
        (void)hipEventRecord(e1, s);
        float ms = -1.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1e30f;
        return ms * 1e3f / REPS;
    };
    // per-bucket launches
    float bsum = 0.0f;
    for (Bucket &bk : h->buckets) {
        float best = 1e30f;
        for (int nt : {64, 256, 512}) {
            if (!proj_threads_ok(proj_bucket(bk.smax), nt)) continue;
            ProjArgs b = a;
            b.nblk = bk.count;
            b.ids = bk.ids;
            const float us = time_us([&]() { launch_project(b, bk.smax, nt, s); });
            if (us < best) {
                best = us;
                bk.nt = nt;
            }
        }
        bk.us = best;
        bsum += best;
    }
    h->plan.buckets_us = bsum;
    // the same launches with the buckets on parallel streams
    float psum = 1e30f;
    if (h->buckets.size() > 1) psum = time_us([&]() { launch_buckets(h, a, s, true); });
    h->plan.parallel_us = psum < 1e29f ? psum : -1.0f;
    // persistent queue launch
    float qbest = 1e30f;
    for (int nt : {256, 512}) {
        const int grid = queue_grid(h, nt);
        if (grid < 1) continue;
        HIP_OK(hipMemsetAsync(h->ticket, 0, sizeof(unsigned long long), s));
        ProjArgs b = a;
        b.nblk = d.p_lds;
        b.ids = d.order;
        const float us = time_us([&]() { launch_project_queue(b, d.smax_lds, nt, grid, h->ticket, s); });
        if (us < qbest) {
            qbest = us;
            h->plan.nt = nt;
            h->plan.grid = grid;
        }
    }
    h->plan.queue_us = qbest < 1e29f ? qbest : -1.0f;
    h->plan.queue = qbest < std::min(bsum, psum);
    h->plan.parallel = !h->plan.queue && psum < bsum;
    HIP_OK(hipMemsetAsync(h->ticket, 0, sizeof(unsigned long long), s));
    e = hipStreamSynchronize(s);
    cleanup();
    if (e != hipSuccess) return fail(CDCS_E_DEVICE, std::string("autotuner: ") + hipGetErrorString(e));
    return CDCS_OK;
}

// HIP events around the kernels of eager iterations (cdcs_admm_solve_timed):
// a pool for kGroup iterations, read back and summed per cdcs_kernel kind
// after each group's stream synchronisation.
struct IterTimer {
    static constexpr int kGroup = 64;
    static constexpr int kPerIter = 5;
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;  // of each recorded pair
    double ms[kPerIter] = {0.0, 0.0, 0.0, 0.0, 0.0};
    int64_t n[kPerIter] = {0, 0, 0, 0, 0};
    hipError_t init() {
        ev.assign((size_t)2 * kGroup * kPerIter, nullptr);
        for (hipEvent_t &e : ev) {
            // no system-scope fence at the events: they only time device work
            const hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    ~IterTimer() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    // launch `fn` on stream s between two events of the pool
    template <class F>
    void around(int k, hipStream_t s, F &&fn) {
        const size_t i = 2 * kind.size();
        (void)hipEventRecord(ev[i], s);
        fn();
        (void)hipEventRecord(ev[i + 1], s);
        kind.push_back(k);
    }
    // after a synchronisation of the stream: add up the recorded pairs
    hipError_t collect() {
        for (size_t p = 0; p < kind.size(); ++p) {
            float t = 0.0f;
            const hipError_t r = hipEventElapsedTime(&t, ev[2 * p], ev[2 * p + 1]);
            if (r != hipSuccess) return r;
            ms[kind[p]] += (double)t;
            n[kind[p]] += 1;
        }
        kind.clear();
        return hipSuccess;
    }
};

// One ADMM iteration.  With a timer (eager launches only) each kernel kind is
// bracketed by events; the launches are the same either way.
// Dev as the HSDE linear step sees it: 1 / E, 1 / (w E) and the factor of
// I + A diag(w / E) A^T in place of Algorithm 1's.
Dev hsde_dev(const cdcs_handle *h) {
    Dev dh = h->d;
    dh.invD = h->hs.invE;
    dh.s2 = h->hs.s2E;
    set_factor(dh, h->hs_fac);
    return dh;
}

void enqueue_iteration(cdcs_handle *h, const cdcs_state *st, int form, double rho, hipStream_t s,
                       IterTimer *tm = nullptr) {
    Dev &d = h->d;
    auto timed = [&](int k, auto &&fn) {
        if (tm) tm->around(k, s, fn);
        else fn();
    };
    if (form == kFormHsde) {  // st: x = u_x (internal order), y = u_y, blk = s, lam = z
        const Dev dh = hsde_dev(h);
        HsdeDev &hs = h->hs;
        double *tk = h->hs_tk;
        timed(CDCS_K_SCATTER, [&] { launch_hsde_scatter(d, hs, st->blk, st->lam, tk, s); });
        if (check_in_au(d)) {  // the check runs in the A u launch's first workgroup
            timed(CDCS_K_GEMV_AU, [&] { launch_au_with_hsde_check(dh, d, hs, tk, st->y, -1.0, d.ctl, s); });
        } else {
            launch_hsde_check(d, hs, tk, s);
            timed(CDCS_K_GEMV_AU, [&] { launch_affine_part(dh, 0, st->y, -1.0, hs.a, hs.yh, d.ctl, s); });
        }
        launch_affine_part(dh, 3, st->y, -1.0, hs.a, hs.yh, d.ctl, s);
        timed(CDCS_K_TRMV, [&] { launch_affine_part(dh, 1, st->y, -1.0, hs.a, hs.yh, d.ctl, s); });
        timed(CDCS_K_GEMV_ATY, [&] { launch_affine_part(dh, 2, st->y, -1.0, hs.a, hs.yh, d.ctl, s); });
        launch_hsde_tau(d, hs, st->y, tk, s);
        launch_hsde_axpy(d, hs, s);
        timed(CDCS_K_PROJECT, [&] { launch_projection(h, PROJ_PRIMAL, st, 1.0, s); });
        return;
    }
    if (d.batch && form == CDCS_PRIMAL) {  // Algorithm 1, per-instance stopping
        timed(CDCS_K_SCATTER, [&] { launch_bscatter_primal(d, st->blk, st->lam, rho, s); });
        launch_bcheck_primal(d, rho, s);
        timed(CDCS_K_GEMV_AU, [&] { launch_baffine(d, d.b, 1.0, st->x, st->y, d.ctl, d.batch->istop, s); });
        timed(CDCS_K_PROJECT, [&] { launch_projection(h, PROJ_PRIMAL, st, rho, s); });
        return;
    }
    if (d.batch) {  // Algorithm 2, per-instance stopping
        timed(CDCS_K_PROJECT, [&] { launch_projection(h, PROJ_DUAL, st, rho, s); });
        timed(CDCS_K_SCATTER, [&] { launch_bscatter_dual(d, st->blk, st->lam, rho, s); });
        timed(CDCS_K_GEMV_AU,
              [&] { launch_baffine(d, d.b, -1.0 / rho, st->x, st->y, d.ctl, d.batch->istop, s); });
        launch_bvupdate(d, st->x, st->blk, st->lam, st->v, rho, s);
        launch_bcheck_dual(d, rho, s);
        return;
    }
    // the affine step (t, then y = L^-T L^-1 t, then x) part by part; with
    // check_au, Algorithm 1's residual check runs in the A u launch
    auto affine = [&](double r2scale, bool check_au) {
        if (check_au) timed(CDCS_K_GEMV_AU, [&] { launch_au_with_check(d, d.b, r2scale, rho, d.ctl, s); });
        else timed(CDCS_K_GEMV_AU, [&] { launch_affine_part(d, 0, d.b, r2scale, st->x, st->y, d.ctl, s); });
        launch_affine_part(d, 3, d.b, r2scale, st->x, st->y, d.ctl, s);
        timed(CDCS_K_TRMV, [&] { launch_affine_part(d, 1, d.b, r2scale, st->x, st->y, d.ctl, s); });
        timed(CDCS_K_GEMV_ATY, [&] { launch_affine_part(d, 2, d.b, r2scale, st->x, st->y, d.ctl, s); });
    };
    if (form == CDCS_PRIMAL) {
        timed(CDCS_K_SCATTER, [&] { launch_scatter_primal(d, st->blk, st->lam, rho, s); });
        const bool check_au = check_in_au(d);
        if (!check_au) launch_check_primal(d, rho, s);
        affine(1.0, check_au);
        timed(CDCS_K_PROJECT, [&] { launch_projection(h, PROJ_PRIMAL, st, rho, s); });
    } else {
        timed(CDCS_K_PROJECT, [&] { launch_projection(h, PROJ_DUAL, st, rho, s); });
        timed(CDCS_K_SCATTER, [&] { launch_scatter_dual(d, st->blk, st->lam, rho, s); });
        affine(-1.0 / rho, false);
        launch_vupdate(d, st->x, st->blk, st->lam, st->v, rho, s);
        launch_check_dual(d, rho, s);
    }
}

cdcs_status get_graph(cdcs_handle *h, const cdcs_state *st, int form, int K, double rho, hipGraphExec_t *out) {
    GraphKey key{form, K, rho, st->x, st->y, st->blk, st->lam, st->v, st->vw,
                 form == kFormHsde ? (const void *)h->hs_tk : nullptr};
    auto it = h->graphs.find(key);
    if (it != h->graphs.end()) {
        *out = it->second;
        return CDCS_OK;
    }
    HIP_OK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < K; ++i) enqueue_iteration(h, st, form, rho, h->cap_stream);
    hipGraph_t g = nullptr;
    HIP_OK(hipStreamEndCapture(h->cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(CDCS_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    h->graph_defs.push_back(g);
    h->graphs[key] = ex;
    *out = ex;
    return CDCS_OK;
}

}  // namespace

namespace cdcs {

cdcs_status set_error(cdcs_status st, const std::string &msg) { return fail(st, msg); }

void handle_dims(const cdcs_handle *h, int64_t *ldU, int64_t *ldM) {
    *ldU = h->d.ldU;
    *ldM = h->d.ldM;
}

// The affine adjoint with the solve's x and y staged in xs [ldU] and ys [ldM]
// (device): r1bar = w F(xbar / w, 0), r2bar = that solve's y.  Every element
// of xs and ys is written before it is read.
cdcs_status affine_adjoint_into(cdcs_handle *h, const double *xbar, double *r1bar, double *r2bar, double *xs,
                                double *ys, hipStream_t stream) {
    Dev &d = h->d;
    launch_adjoint_scatter(d, nullptr, xbar, stream);
    if (d.batch) launch_baffine(d, d.b, 0.0, xs, ys, nullptr, nullptr, stream);
    else launch_affine(d, d.b, 0.0, xs, ys, nullptr, stream);
    launch_adjoint_post(d, xs, r1bar, 1.0, 0, stream);
    launch_add_to(ys, r2bar, d.m, 0, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

}  // namespace cdcs

extern "C" {

const char *cdcs_last_error(void) { return g_err.c_str(); }

cdcs_status cdcs_chordal_extension(const cdcs_pattern *pattern, int64_t *nfill, int32_t *p, int64_t *nvert,
                                   int32_t *fill_i, int32_t *fill_j, int64_t *clique_ptr, int32_t *clique_vert) {
    if (!pattern || !nfill || !p || !nvert) return fail(CDCS_E_ARG, "NULL argument");
    ChordalExt ext;
    std::string err;
    const cdcs_status st = chordal_extension(pattern->n, pattern->nnz, pattern->i, pattern->j, ext, err);
    if (st != CDCS_OK) return fail(st, err);
    *nfill = (int64_t)ext.fill_i.size();
    *p = (int32_t)(ext.ptr.size() - 1);
    *nvert = ext.ptr.back();
    if (fill_i && fill_j) {
        std::copy(ext.fill_i.begin(), ext.fill_i.end(), fill_i);
        std::copy(ext.fill_j.begin(), ext.fill_j.end(), fill_j);
    }
    if (clique_ptr) std::copy(ext.ptr.begin(), ext.ptr.end(), clique_ptr);
    if (clique_vert) std::copy(ext.vert.begin(), ext.vert.end(), clique_vert);
    return CDCS_OK;
}

cdcs_status cdcs_setup_cones(const cdcs_pattern *pattern, const cdcs_constraints *A, const double *b,
                             const double *c, const cdcs_cliques *cliques, const cdcs_vcones *cones,
                             const cdcs_options *opts, hipStream_t stream, cdcs_handle **out) {
    (void)opts;
    if (!out) return fail(CDCS_E_ARG, "out is NULL");
    *out = nullptr;
    g_err.clear();
    if (cones && cones->ncones == 0) cones = nullptr;
    if (!cliques) {
        // chordal decomposition of an arbitrary pattern: the extension's fill
        // entries follow the caller's entries, with zero data (C and every A_i
        // vanish on them); the vector cones' vertices stay out of it
        if (!pattern || !A || !b || !c || !A->val) return fail(CDCS_E_ARG, "NULL argument");
        if (pattern->n < 1 || pattern->nnz < 1 || !pattern->i || !pattern->j)
            return fail(CDCS_E_ARG, "empty or NULL pattern");
        const int32_t *ei = pattern->i, *ej = pattern->j;
        int64_t next = pattern->nnz;
        std::vector<int32_t> fi, fj;
        if (cones) {
            if (cones->ncones < 0 || !cones->ptr || !cones->vert || cones->ptr[0] != 0)
                return fail(CDCS_E_ARG, "bad vector cone arrays");
            std::vector<char> isc((size_t)pattern->n, 0);
            for (int64_t t = 0; t < cones->ptr[cones->ncones]; ++t) {
                const int32_t v = cones->vert[t];
                if (v < 0 || v >= pattern->n) return fail(CDCS_E_PATTERN, "cone vertex out of range");
                isc[(size_t)v] = 1;
            }
            for (int64_t e = 0; e < pattern->nnz; ++e) {
                const int32_t i = pattern->i[e], j = pattern->j[e];
                if (i < 0 || j < 0 || i >= pattern->n || j >= pattern->n)
                    return fail(CDCS_E_PATTERN, "pattern entry " + std::to_string(e) + " out of range");
                if (isc[(size_t)i] || isc[(size_t)j]) continue;
                fi.push_back(i);
                fj.push_back(j);
            }
            ei = fi.data();
            ej = fj.data();
            next = (int64_t)fi.size();
        }
        ChordalExt ext;
        ext.ptr.assign(1, 0);
        if (next > 0) {
            std::string err;
            const cdcs_status st = chordal_extension(pattern->n, next, ei, ej, ext, err);
            if (st != CDCS_OK) return fail(st, err);
        }
        const int64_t nu = pattern->nnz, nf = (int64_t)ext.fill_i.size(), ne = nu + nf;
        std::vector<int32_t> pi(pattern->i, pattern->i + nu), pj(pattern->j, pattern->j + nu);
        pi.insert(pi.end(), ext.fill_i.begin(), ext.fill_i.end());
        pj.insert(pj.end(), ext.fill_j.begin(), ext.fill_j.end());
        std::vector<double> cx(c, c + nu);
        cx.resize((size_t)ne, 0.0);
        std::vector<double> ax;
        cdcs_constraints Ax = *A;
        if (A->dense && nf > 0) {
            ax.assign((size_t)(A->m * ne), 0.0);
            for (int32_t r = 0; r < A->m; ++r)
                std::copy(A->val + (size_t)r * nu, A->val + (size_t)(r + 1) * nu, ax.begin() + (size_t)r * ne);
            Ax.val = ax.data();
        }
        const cdcs_pattern px{pattern->n, ne, pi.data(), pj.data()};
        const cdcs_cliques cx_cl{(int32_t)(ext.ptr.size() - 1), ext.ptr.data(), ext.vert.data()};
        return cdcs_setup_cones(&px, &Ax, b, cx.data(), &cx_cl, cones, opts, stream, out);
    }
    cdcs_handle *h = new (std::nothrow) cdcs_handle();
    if (!h) return fail(CDCS_E_NOMEM, "host allocation");
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return fail(CDCS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    cdcs_status st = build(h, pattern, A, b, c, cliques, cones, stream);
    if (st != CDCS_OK) {
        (void)hipStreamSynchronize(stream);
        delete h;
        return st;
    }
    *out = h;
    return CDCS_OK;
}

cdcs_status cdcs_setup(const cdcs_pattern *pattern, const cdcs_constraints *A, const double *b, const double *c,
                       const cdcs_cliques *cliques, const cdcs_options *opts, hipStream_t stream,
                       cdcs_handle **out) {
    return cdcs_setup_cones(pattern, A, b, c, cliques, nullptr, opts, stream, out);
}

cdcs_status cdcs_setup_batch(int32_t nprob, const cdcs_problem *probs, const cdcs_options *opts, hipStream_t stream,
                             cdcs_handle **out) {
    (void)opts;
    if (!out) return fail(CDCS_E_ARG, "out is NULL");
    *out = nullptr;
    g_err.clear();
    cdcs_handle *h = new (std::nothrow) cdcs_handle();
    if (!h) return fail(CDCS_E_NOMEM, "host allocation");
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return fail(CDCS_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    cdcs_status st = build_batch(h, nprob, probs, stream);
    if (st != CDCS_OK) {
        (void)hipStreamSynchronize(stream);
        delete h;
        return st;
    }
    *out = h;
    return CDCS_OK;
}

cdcs_status cdcs_batch_info(const cdcs_handle *h, int32_t nprob, cdcs_instance_info *out_host) {
    if (!h || !out_host) return fail(CDCS_E_ARG, "NULL argument");
    const Batch *B = h->d.batch;
    if (!B) return fail(CDCS_E_ARG, "not a batch handle");
    if (nprob != B->nprob) return fail(CDCS_E_ARG, "nprob does not match the handle");
    std::vector<int32_t> stp((size_t)nprob), its((size_t)nprob);
    std::vector<uint64_t> tim((size_t)nprob);
    std::vector<double> eps((size_t)(2 * nprob)), obj((size_t)(2 * nprob));
    uint64_t t0 = 0;
    HIP_OK(hipMemcpy(stp.data(), B->istop, stp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(its.data(), B->iiters, its.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(tim.data(), B->itime, tim.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(eps.data(), B->ieps, eps.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(obj.data(), B->iobj, obj.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&t0, B->t0, sizeof(uint64_t), hipMemcpyDeviceToHost));
    int rate_khz = 0;
    HIP_OK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, h->device));
    const double rho = h->last_rho;
    for (int32_t q = 0; q < nprob; ++q) {
        cdcs_instance_info &o = out_host[q];
        o.iters = stp[(size_t)q] ? its[(size_t)q] : h->last_iters;
        o.status = stp[(size_t)q] == 1 ? CDCS_OK : stp[(size_t)q] == 3 ? CDCS_E_NUMERIC : CDCS_E_NOT_CONVERGED;
        o.eps_p = eps[(size_t)(2 * q)];
        o.eps_d = eps[(size_t)(2 * q + 1)];
        if (h->last_form == CDCS_PRIMAL) {
            o.obj_primal = obj[(size_t)(2 * q)];
            o.obj_dual = -rho * obj[(size_t)(2 * q + 1)];
        } else {  // Algorithm 2: X_sdp = -rho x, y_sdp = y
            o.obj_primal = -rho * obj[(size_t)(2 * q)];
            o.obj_dual = obj[(size_t)(2 * q + 1)];
        }
        o.time_to_tol_s = (stp[(size_t)q] && rate_khz > 0) ? (double)(tim[(size_t)q] - t0) / (1e3 * rate_khz) : -1.0;
    }
    return CDCS_OK;
}

cdcs_status cdcs_get_sizes(const cdcs_handle *h, cdcs_sizes *out) {
    if (!h || !out) return fail(CDCS_E_ARG, "NULL argument");
    out->n = h->d.n;
    out->m = h->d.m;
    out->p = h->d.p;
    out->smax = h->d.smax;
    out->nnz = h->d.nU;
    out->nslots = h->d.nslots;
    out->sparse_a = h->d.sparse;
    out->sparse_factor = h->d.sparse_linv;
    out->nnz_a = h->d.sparse ? h->d.nnzA : (int64_t)h->d.m * h->d.nU;
    out->nnz_factor = h->d.sparse_linv ? h->d.nnz_linv : (int64_t)h->d.m * (h->d.m + 1) / 2;
    out->nwarm = h->d.nwarm;
    out->nnz_l = h->d.spchol ? h->d.nnz_l : 0;
    out->nvcones = h->d.nvc;
    out->pad_ = 0;
    out->nslots_psd = h->d.nvc > 0 ? h->d.nslots_psd : h->d.nslots;
    return CDCS_OK;
}

cdcs_status cdcs_warm_reset(const cdcs_handle *h, float *vw, hipStream_t stream) {
    if (!h || !vw) return fail(CDCS_E_ARG, "NULL argument");
    const Dev &d = h->d;
    launch_identity_blocks(d.clq_size, d.vwoff, d.p, vw, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_clique_offsets(const cdcs_handle *h, int64_t *off_host) {
    if (!h || !off_host) return fail(CDCS_E_ARG, "NULL argument");
    std::memcpy(off_host, h->off_host.data(), h->off_host.size() * sizeof(int64_t));
    return CDCS_OK;
}

cdcs_status cdcs_psd_project_batched(int32_t nb, int32_t smax, const int32_t *sizes, const int64_t *off,
                                     const float *W, float *P, float *evals, const int64_t *eoff, float *evecs,
                                     const int64_t *voff, hipStream_t stream) {
    if (nb <= 0) return CDCS_OK;
    if (smax < 1 || smax > CDCS_MAX_BATCHED_CLIQUE) return fail(CDCS_E_ARG, "smax outside 1..CDCS_MAX_BATCHED_CLIQUE");
    if (!sizes || !off || !W || !P) return fail(CDCS_E_ARG, "NULL device pointer");
    if ((evals && !eoff) || (evecs && !voff)) return fail(CDCS_E_ARG, "evals/evecs need eoff/voff");
    ProjArgs a{};
    a.mode = PROJ_STANDALONE;
    a.nblk = nb;
    a.size = sizes;
    a.off = off;
    a.Win = W;
    a.Pout = P;
    a.evals = evals;
    a.eoff = eoff;
    a.evecs = evecs;
    a.voff = voff;
    launch_project(a, proj_bucket(smax), 256, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_psd_project_cliques(cdcs_handle *h, const float *W, float *P, hipStream_t stream) {
    if (!h || !W || !P) return fail(CDCS_E_ARG, "NULL argument");
    ProjArgs a = proj_args(h, PROJ_STANDALONE, nullptr, 1.0);
    a.Win = W;
    a.Pout = P;
    a.vwarm = nullptr;  // cold start: Jacobi from the identity
    a.warm_store = 0;
    a.kinst = nullptr;
    a.istop = nullptr;
    a.ctl = nullptr;
    launch_plan(h, a, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_psd_project_vjp(int32_t nb, int32_t smax, const int32_t *sizes, const int64_t *off,
                                 const float *evals, const int64_t *eoff, const float *evecs, const int64_t *voff,
                                 const float *gP, float *gW, hipStream_t stream) {
    if (nb <= 0) return CDCS_OK;
    if (smax < 1 || smax > CDCS_MAX_BATCHED_CLIQUE) return fail(CDCS_E_ARG, "smax outside 1..CDCS_MAX_BATCHED_CLIQUE");
    if (!sizes || !off || !evals || !eoff || !evecs || !voff || !gP || !gW)
        return fail(CDCS_E_ARG, "NULL device pointer");
    VjpArgs a{};
    a.nblk = nb;
    a.size = sizes;
    a.off = off;
    a.evals = evals;
    a.eoff = eoff;
    a.evecs = evecs;
    a.voff = voff;
    a.gP = gP;
    a.gW = gW;
    launch_project_vjp(a, smax, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_gather(const cdcs_handle *h, const double *x, double *packed, hipStream_t stream) {
    if (!h || !x || !packed) return fail(CDCS_E_ARG, "NULL argument");
    launch_perm_in(h->d, x, h->d.xtmp, stream);
    launch_gather_f64(h->d, h->d.xtmp, packed, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_scatter(const cdcs_handle *h, const double *packed, double *out, hipStream_t stream) {
    if (!h || !packed || !out) return fail(CDCS_E_ARG, "NULL argument");
    launch_scatter_f64(h->d, packed, h->d.xtmp, stream);
    launch_perm_out(h->d, h->d.xtmp, out, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_affine_project(const cdcs_handle *h, const double *r1, const double *r2, double *x, double *y,
                                hipStream_t stream) {
    if (!h || !r1 || !r2 || !x || !y) return fail(CDCS_E_ARG, "NULL argument");
    const Dev &d = h->d;
    launch_perm_in(d, r1, d.xtmp, stream);
    launch_scale_u(d, d.xtmp, stream);
    if (d.batch) launch_baffine(d, r2, 1.0, d.xi, y, nullptr, nullptr, stream);
    else launch_affine(d, r2, 1.0, d.xi, y, nullptr, stream);
    launch_perm_out(d, d.xi, x, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

namespace {
// Validation shared by the solve entry points, and the residual history
// buffer sized for max_iter (allocating it drops the captured graphs, which
// hold the old pointer).
cdcs_status solve_check(cdcs_handle *h, const cdcs_state *st_user, const cdcs_options *opts, hipStream_t stream) {
    if (!h || !st_user || !opts) return fail(CDCS_E_ARG, "NULL argument");
    if (!st_user->x || !st_user->y || !st_user->blk || !st_user->lam) return fail(CDCS_E_ARG, "state has NULL buffers");
    const int form = opts->form;
    if (form != CDCS_PRIMAL && form != CDCS_DUAL) return fail(CDCS_E_ARG, "bad form");
    if (form == CDCS_DUAL && !st_user->v) return fail(CDCS_E_ARG, "dual form needs state.v");
    if (!(opts->rho > 0.0) || !(opts->tol >= 0.0) || opts->max_iter < 1 || opts->check_every < 0)
        return fail(CDCS_E_ARG, "need rho > 0, tol >= 0, max_iter >= 1, check_every >= 0");
    Dev &d = h->d;
    if (d.hist_cap < opts->max_iter) {
        if (d.hist) {
            HIP_OK(hipStreamSynchronize(stream));
            (void)hipFree(d.hist);
            h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), (void *)d.hist), h->allocs.end());
            d.hist = nullptr;
        }
        CK(h->alloc(&d.hist, 2 * (int64_t)opts->max_iter));
        d.hist_cap = opts->max_iter;
        // captured graphs hold the old history pointer
        for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
        h->graphs.clear();
    }
    return CDCS_OK;
}

// The graphs a solve launches: max_iter / check_every launches of a graph of
// check_every iterations, then one of the remaining max_iter % check_every.
cdcs_status solve_graphs(cdcs_handle *h, const cdcs_state *st, const cdcs_options *opts, hipGraphExec_t *full,
                         hipGraphExec_t *tail) {
    const int K = opts->check_every;
    *full = nullptr;
    *tail = nullptr;
    if (opts->max_iter >= K) CK(get_graph(h, st, opts->form, K, opts->rho, full));
    if (opts->max_iter % K) CK(get_graph(h, st, opts->form, opts->max_iter % K, opts->rho, tail));
    return CDCS_OK;
}

cdcs_status solve_impl(cdcs_handle *h, const cdcs_state *st_user, const cdcs_options *opts, cdcs_info *info,
                       hipStream_t stream, IterTimer *tm) {
    CK(solve_check(h, st_user, opts, stream));
    // the iteration runs on x in internal entry order
    cdcs_state st_int = *st_user;
    st_int.x = h->d.xi;
    const cdcs_state *st = &st_int;
    const int form = opts->form;
    Dev &d = h->d;
    const double rho = opts->rho;
    h->last_rho = rho;
    h->last_form = form;
    launch_reset_ctl(d, opts->max_iter, opts->tol, stream);
    if (d.batch) launch_breset(d, stream);
    // a solve is a function of (problem, state, options) only: without a
    // warm-start buffer in the state the handle's copy restarts at identity
    if (!st_user->vw) launch_identity_blocks(d.clq_size, d.vwoff, d.p, d.vwarm, stream);
    launch_perm_in(d, st_user->x, d.xi, stream);
    HIP_OK(hipGetLastError());
    auto t0 = std::chrono::steady_clock::now();
    const int K = tm ? 0 : opts->check_every;
    if (K > 0) {
        hipGraphExec_t full = nullptr, tail = nullptr;
        CK(solve_graphs(h, st, opts, &full, &tail));
        for (int done = 0; done < opts->max_iter;) {
            const int n = std::min(K, opts->max_iter - done);
            HIP_OK(hipGraphLaunch(n == K ? full : tail, stream));
            done += n;
            HIP_OK(hipMemcpyAsync(d.ctl_host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
            HIP_OK(hipStreamSynchronize(stream));
            if (d.ctl_host->stop) break;
        }
    } else {
        const int group = tm ? IterTimer::kGroup : 16;
        for (int it = 0; it < opts->max_iter; ++it) {
            enqueue_iteration(h, st, form, rho, stream, tm);
            HIP_OK(hipGetLastError());
            if ((it + 1) % group == 0 || (tm && it + 1 == opts->max_iter)) {
                HIP_OK(hipMemcpyAsync(d.ctl_host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
                HIP_OK(hipStreamSynchronize(stream));
                if (tm) HIP_OK(tm->collect());
                if (d.ctl_host->stop) break;
            }
        }
    }
    if (d.batch) {
        if (form == CDCS_PRIMAL) {
            launch_bscatter_primal(d, st->blk, st->lam, rho, stream);
            launch_bcheck_primal(d, rho, stream);
        }
        launch_bobjectives(d, st->x, st->y, d.batch->iobj, stream);
    } else if (form == CDCS_PRIMAL) {
        // residuals of the last iteration need the next right-hand side's scatter
        // (it writes u only; x keeps the last iterate)
        launch_scatter_primal(d, st->blk, st->lam, rho, stream);
        launch_check_primal(d, rho, stream);
    }
    launch_objectives(d, st->x, st->y, stream);
    launch_perm_out(d, d.xi, st_user->x, stream);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(d.ctl_host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    double obj[2] = {0.0, 0.0};
    HIP_OK(hipMemcpyAsync(obj, d.obj, sizeof(obj), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    auto t1 = std::chrono::steady_clock::now();
    const Ctl c = *d.ctl_host;
    h->last_iters = c.iter;
    cdcs_status status = CDCS_OK;
    int converged = (c.stop == 1);
    if (d.batch) {
        std::vector<int32_t> stp((size_t)d.batch->nprob);
        HIP_OK(hipMemcpy(stp.data(), d.batch->istop, stp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        converged = std::all_of(stp.begin(), stp.end(), [](int32_t v) { return v == 1; });
    }
    bool nonfinite = c.stop == 3;
    if (d.batch) {
        std::vector<int32_t> stp((size_t)d.batch->nprob);
        HIP_OK(hipMemcpy(stp.data(), d.batch->istop, stp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        nonfinite = std::any_of(stp.begin(), stp.end(), [](int32_t v) { return v == 3; });
    }
    if (c.jacobi_cap > 0 || nonfinite) status = CDCS_E_NUMERIC;
    else if (!converged && opts->tol > 0.0) status = CDCS_E_NOT_CONVERGED;
    if (info) {
        info->iters = c.iter;
        info->status = status;
        info->converged = converged;
        info->jacobi_cap_hits = c.jacobi_cap;
        info->eps_p = c.eps_p;
        info->eps_d = c.eps_d;
        if (form == CDCS_PRIMAL) {
            info->obj_primal = obj[0];
            info->obj_dual = -rho * obj[1];
        } else {
            info->obj_primal = -rho * obj[0];
            info->obj_dual = obj[1];
        }
        info->loop_s = std::chrono::duration<double>(t1 - t0).count();
        info->jacobi_sweeps = c.sweeps;
    }
    if (status != CDCS_OK)
        g_err = nonfinite                     ? "NaN or Inf in the iterate (residuals not finite)"
                : status == CDCS_E_NUMERIC ? "an eigensolve hit its sweep cap"
                                           : "iteration cap reached";
    return status;
}
}  // namespace

namespace {
// HSDE data of a handle: 1 / E and 1 / (w E), the factor of
// I + A diag(w / E) A^T (the Algorithm-1 factor code with those scales and a
// unit diagonal shift), g = M^-1 (c, bhat) and the constants.
cdcs_status hsde_prepare(cdcs_handle *h, hipStream_t s) {
    if (h->hs_ready) return CDCS_OK;
    Dev &d = h->d;
    HsdeDev &hs = h->hs;
    if (!hs.invE) {
        CK(h->alloc(&hs.invE, d.ldU));
        CK(h->alloc(&hs.s2E, d.ldU));
        CK(h->alloc(&hs.gx, d.ldU));
        CK(h->alloc(&hs.gy, d.ldM));
        CK(h->alloc(&hs.a, d.ldU));
        CK(h->alloc(&hs.yh, d.ldM));
        CK(h->alloc(&hs.dx, d.ldU));
        CK(h->alloc(&hs.sc, 16));
        CK(h->alloc(&hs.hpart, 2 * (int64_t)scatter_blocks(d)));
        CK(h->alloc(&hs.dpart, hsde_dot_blocks(d)));
        for (double *q : {hs.a, hs.dx, hs.gx})
            HIP_OK(hipMemsetAsync(q, 0, (size_t)d.ldU * sizeof(double), s));
        HIP_OK(hipMemsetAsync(hs.sc, 0, 16 * sizeof(double), s));
    }
    launch_hsde_scales(d, hs, s);
    HIP_OK(hipGetLastError());
    const FactorFields keep = get_factor(d);
    double *s2keep = d.s2;
    set_factor(d, FactorFields());
    d.s2 = hs.s2E;
    const cdcs_status st = factor_into(h, 1.0, s);
    h->hs_fac = get_factor(d);
    set_factor(d, keep);
    d.s2 = s2keep;
    CK(st);
    // g: u = c / E, t = A(w u) + b, g_y = M'^-1 t, g_x = u - (A^T g_y) / E
    const Dev dh = hsde_dev(h);
    launch_hsde_cu(d, hs, s);
    launch_affine(dh, d.b, -1.0, hs.gx, hs.gy, nullptr, s);
    launch_hsde_consts(d, hs, s);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    h->hs_ready = true;
    return CDCS_OK;
}

cdcs_status hsde_check_state(const cdcs_handle *h, const cdcs_hsde_state *st) {
    if (!h || !st) return fail(CDCS_E_ARG, "NULL argument");
    if (!st->x || !st->y || !st->s || !st->z || !st->tk) return fail(CDCS_E_ARG, "HSDE state has NULL buffers");
    if (h->d.batch) return fail(CDCS_E_ARG, "the HSDE solver runs on single-SDP handles");
    return CDCS_OK;
}
}  // namespace

cdcs_status cdcs_hsde_init(cdcs_handle *h, const cdcs_hsde_state *st, hipStream_t stream) {
    CK(hsde_check_state(h, st));
    const Dev &d = h->d;
    launch_hsde_init(d, st->x, st->y, st->s, st->z, st->tk, stream);
    if (st->vw) launch_identity_blocks(d.clq_size, d.vwoff, d.p, st->vw, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

namespace {
cdcs_status hsde_solve_impl(cdcs_handle *h, const cdcs_hsde_state *st, const cdcs_options *opts,
                            cdcs_hsde_info *info, hipStream_t stream, IterTimer *tm) {
    CK(hsde_check_state(h, st));
    if (!opts) return fail(CDCS_E_ARG, "NULL argument");
    if (!(opts->tol >= 0.0) || opts->max_iter < 1 || opts->check_every < 0)
        return fail(CDCS_E_ARG, "need tol >= 0, max_iter >= 1, check_every >= 0");
    CK(hsde_prepare(h, stream));
    Dev &d = h->d;
    HsdeDev &hs = h->hs;
    if (hs.hist_cap < opts->max_iter) {
        if (hs.hist) {
            HIP_OK(hipStreamSynchronize(stream));
            (void)hipFree(hs.hist);
            h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), (void *)hs.hist), h->allocs.end());
            hs.hist = nullptr;
        }
        CK(h->alloc(&hs.hist, 3 * (int64_t)opts->max_iter));
        hs.hist_cap = opts->max_iter;
        for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
        h->graphs.clear();
    }
    // the iteration runs on x in internal entry order; s and z take the
    // places of x_k and lambda_k
    cdcs_state sti{d.xi, st->y, st->s, st->z, nullptr, st->vw};
    h->hs_tk = st->tk;
    launch_reset_ctl(d, opts->max_iter, opts->tol, stream);
    if (!st->vw) launch_identity_blocks(d.clq_size, d.vwoff, d.p, d.vwarm, stream);
    launch_perm_in(d, st->x, d.xi, stream);
    HIP_OK(hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    const int K = tm ? 0 : opts->check_every;
    if (K > 0) {
        hipGraphExec_t full = nullptr, tail = nullptr;
        if (opts->max_iter >= K) CK(get_graph(h, &sti, kFormHsde, K, 1.0, &full));
        if (opts->max_iter % K) CK(get_graph(h, &sti, kFormHsde, opts->max_iter % K, 1.0, &tail));
        for (int done = 0; done < opts->max_iter;) {
            const int n = std::min(K, opts->max_iter - done);
            HIP_OK(hipGraphLaunch(n == K ? full : tail, stream));
            done += n;
            HIP_OK(hipMemcpyAsync(d.ctl_host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
            HIP_OK(hipStreamSynchronize(stream));
            if (d.ctl_host->stop) break;
        }
    } else {
        const int group = tm ? IterTimer::kGroup : 16;
        for (int it = 0; it < opts->max_iter; ++it) {
            enqueue_iteration(h, &sti, kFormHsde, 1.0, stream, tm);
            HIP_OK(hipGetLastError());
            if ((it + 1) % group == 0 || (tm && it + 1 == opts->max_iter)) {
                HIP_OK(hipMemcpyAsync(d.ctl_host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
                HIP_OK(hipStreamSynchronize(stream));
                if (tm) HIP_OK(tm->collect());
                if (d.ctl_host->stop) break;
            }
        }
    }
    // the last iterate's check needs the next iteration's scatter
    launch_hsde_scatter(d, hs, sti.blk, sti.lam, st->tk, stream);
    launch_hsde_check(d, hs, st->tk, stream);
    launch_perm_out(d, d.xi, st->x, stream);
    HIP_OK(hipGetLastError());
    double sc[16], tk[2];
    HIP_OK(hipMemcpyAsync(d.ctl_host, d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(sc, hs.sc, sizeof(sc), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipMemcpyAsync(tk, st->tk, sizeof(tk), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));
    const auto t1 = std::chrono::steady_clock::now();
    const Ctl c = *d.ctl_host;
    h->last_iters = c.iter;
    cdcs_status status = CDCS_OK;
    if (c.stop == 3 || c.jacobi_cap > 0) status = CDCS_E_NUMERIC;
    else if (c.stop == 4) status = CDCS_PRIMAL_INFEASIBLE;
    else if (c.stop == 5) status = CDCS_DUAL_INFEASIBLE;
    else if (c.stop != 1 && opts->tol > 0.0) status = CDCS_E_NOT_CONVERGED;
    if (info) {
        info->iters = c.iter;
        info->status = status;
        info->jacobi_cap_hits = c.jacobi_cap;
        info->pad_ = 0;
        info->res_pri = sc[10];
        info->res_dual = sc[11];
        info->gap = sc[12];
        const double nan = std::nan("");
        info->obj_primal = tk[0] > 0.0 ? sc[9] / tk[0] : nan;
        info->obj_dual = tk[0] > 0.0 ? -sc[8] / tk[0] : nan;
        info->tau = tk[0];
        info->kappa = tk[1];
        info->loop_s = std::chrono::duration<double>(t1 - t0).count();
        info->jacobi_sweeps = c.sweeps;
    }
    if (status == CDCS_E_NUMERIC)
        g_err = c.stop == 3 ? "NaN or Inf in the iterate (residuals not finite)" : "an eigensolve hit its sweep cap";
    else if (status == CDCS_E_NOT_CONVERGED)
        g_err = "iteration cap reached";
    else if (status == CDCS_PRIMAL_INFEASIBLE)
        g_err = "primal infeasible (certificate in y)";
    else if (status == CDCS_DUAL_INFEASIBLE)
        g_err = "dual infeasible (certificate in x)";
    return status;
}
}  // namespace

cdcs_status cdcs_hsde_solve(cdcs_handle *h, const cdcs_hsde_state *st, const cdcs_options *opts, cdcs_hsde_info *info,
                            hipStream_t stream) {
    return hsde_solve_impl(h, st, opts, info, stream, nullptr);
}

cdcs_status cdcs_hsde_solve_timed(cdcs_handle *h, const cdcs_hsde_state *st, const cdcs_options *opts,
                                  cdcs_hsde_info *info, double *kernel_ms, int64_t *launches, hipStream_t stream) {
    if (!kernel_ms || !launches) return fail(CDCS_E_ARG, "NULL kernel_ms or launches");
    IterTimer tm;
    HIP_OK(tm.init());
    const cdcs_status r = hsde_solve_impl(h, st, opts, info, stream, &tm);
    for (int k = 0; k < IterTimer::kPerIter; ++k) {
        kernel_ms[k] = tm.ms[k];
        launches[k] = tm.n[k];
    }
    return r;
}

cdcs_status cdcs_hsde_solution(cdcs_handle *h, const cdcs_hsde_state *st, int32_t which, double *X_out,
                               double *y_out, hipStream_t stream) {
    CK(hsde_check_state(h, st));
    if (which < 0 || which > 2) return fail(CDCS_E_ARG, "which must be 0, 1 or 2");
    if ((which != 1 && !X_out) || (which != 2 && !y_out)) return fail(CDCS_E_ARG, "NULL output");
    if (!h->hs_ready) return fail(CDCS_E_ARG, "no HSDE solve on this handle yet");
    launch_hsde_solution(h->d, h->hs, which, st->x, st->y, st->tk, X_out, y_out, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_admm_solve(cdcs_handle *h, const cdcs_state *st, const cdcs_options *opts, cdcs_info *info,
                            hipStream_t stream) {
    return solve_impl(h, st, opts, info, stream, nullptr);
}

cdcs_status cdcs_admm_prepare(cdcs_handle *h, const cdcs_state *st_user, const cdcs_options *opts,
                              hipStream_t stream) {
    CK(solve_check(h, st_user, opts, stream));
    if (opts->check_every == 0) return CDCS_OK;
    cdcs_state st_int = *st_user;
    st_int.x = h->d.xi;
    hipGraphExec_t full = nullptr, tail = nullptr;
    CK(solve_graphs(h, &st_int, opts, &full, &tail));
    return CDCS_OK;
}

cdcs_status cdcs_unrolled_step(cdcs_handle *h, const cdcs_state *st, const double *c, const double *b, double rho,
                               float *evals, float *evecs, hipStream_t stream) {
    if (!h || !st || !c || !b) return fail(CDCS_E_ARG, "NULL argument");
    if (h->d.batch) return fail(CDCS_E_ARG, "unrolled steps run on single-SDP handles");
    if (h->d.nvc > 0) return fail(CDCS_E_ARG, "unrolled steps run on handles without vector cones");
    if (h->d.big.nbig > 0)
        return fail(CDCS_E_ARG, "unrolled steps need eigenpairs: cliques of at most " +
                                    std::to_string(kMaxLdsClique) + " vertices");
    CK(diff_buffers(h));
    Dev &d = h->d;
    launch_perm_in(d, c, h->diff.c, stream);
    double *c0 = d.c, *b0 = d.b;
    d.c = h->diff.c;
    d.b = const_cast<double *>(b);
    h->save_evals = evals;
    h->save_evecs = evecs;
    cdcs_options o{};
    o.rho = rho;
    o.tol = 0.0;
    o.max_iter = 1;
    o.form = CDCS_PRIMAL;
    o.check_every = 0;
    const cdcs_status r = cdcs_admm_solve(h, st, &o, nullptr, stream);
    d.c = c0;
    d.b = b0;
    h->save_evals = nullptr;
    h->save_evecs = nullptr;
    return r;
}

cdcs_status cdcs_unrolled_step_vjp(cdcs_handle *h, double rho, const float *evals, const float *evecs,
                                   const double *xbar, double *blkbar, double *lambar, double *cbar, double *bbar,
                                   hipStream_t stream) {
    if (!h || !evals || !evecs || !blkbar || !lambar || !cbar || !bbar) return fail(CDCS_E_ARG, "NULL argument");
    if (!(rho > 0.0)) return fail(CDCS_E_ARG, "need rho > 0");
    if (h->d.batch) return fail(CDCS_E_ARG, "unrolled steps run on single-SDP handles");
    if (h->d.nvc > 0) return fail(CDCS_E_ARG, "unrolled steps run on handles without vector cones");
    if (h->d.big.nbig > 0)
        return fail(CDCS_E_ARG, "unrolled steps need eigenpairs: cliques of at most " +
                                    std::to_string(kMaxLdsClique) + " vertices");
    CK(diff_buffers(h));
    Dev &d = h->d;
    cdcs_handle::Diff &f = h->diff;
    launch_adjoint_in(d, blkbar, lambar, rho, f.gP, stream);
    VjpArgs a{};
    a.nblk = d.p;
    a.size = d.clq_size;
    a.off = d.clq_off;
    a.evals = evals;
    a.eoff = f.eoff;
    a.evecs = evecs;
    a.voff = d.vwoff;
    a.gP = f.gP;
    a.gW = f.gW;
    launch_project_vjp(a, d.smax, stream);
    launch_adjoint_mid(d, f.gW, lambar, rho, f.hbar, stream);
    launch_adjoint_scatter(d, f.hbar, xbar, stream);
    launch_affine(d, d.b, 0.0, f.x, f.y, nullptr, stream);
    launch_adjoint_post(d, f.x, cbar, -1.0 / rho, 1, stream);
    launch_adjoint_slots(d, f.x, blkbar, lambar, rho, stream);
    launch_add_to(f.y, bbar, d.m, 1, stream);
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_affine_project_adjoint(cdcs_handle *h, const double *xbar, double *r1bar, double *bbar,
                                        hipStream_t stream) {
    if (!h || !xbar || !r1bar || !bbar) return fail(CDCS_E_ARG, "NULL argument");
    CK(diff_buffers(h));
    return cdcs::affine_adjoint_into(h, xbar, r1bar, bbar, h->diff.x, h->diff.y, stream);
}

cdcs_status cdcs_admm_solve_timed(cdcs_handle *h, const cdcs_state *st, const cdcs_options *opts, cdcs_info *info,
                                  double *kernel_ms, int64_t *launches, hipStream_t stream) {
    if (!kernel_ms || !launches) return fail(CDCS_E_ARG, "NULL kernel_ms or launches");
    IterTimer tm;
    HIP_OK(tm.init());
    const cdcs_status r = solve_impl(h, st, opts, info, stream, &tm);
    for (int k = 0; k < IterTimer::kPerIter; ++k) {
        kernel_ms[k] = tm.ms[k];
        launches[k] = tm.n[k];
    }
    return r;
}

cdcs_status cdcs_admm_step(cdcs_handle *h, const cdcs_state *st, int32_t form, double rho, hipStream_t stream) {
    cdcs_options o{};
    o.rho = rho;
    o.tol = 0.0;
    o.max_iter = 1;
    o.form = form;
    o.check_every = 0;
    return cdcs_admm_solve(h, st, &o, nullptr, stream);
}

cdcs_status cdcs_profile_kernel(cdcs_handle *h, const cdcs_state *st_user, int32_t form, double rho,
                                int32_t kernel, int32_t reps, hipStream_t stream) {
    if (!h || !st_user || !st_user->x || !st_user->y || !st_user->blk || !st_user->lam)
        return fail(CDCS_E_ARG, "NULL argument");
    if (form != CDCS_PRIMAL && form != CDCS_DUAL) return fail(CDCS_E_ARG, "bad form");
    if (form == CDCS_DUAL && !st_user->v) return fail(CDCS_E_ARG, "dual form needs state.v");
    if (reps < 1 || !(rho > 0.0)) return fail(CDCS_E_ARG, "need reps >= 1, rho > 0");
    Dev &d = h->d;
    // x is the handle's copy of the iterate (internal entry order), so that
    // only the named kernel runs between the caller's events
    cdcs_state st_int = *st_user;
    st_int.x = d.xi;
    const cdcs_state *st = &st_int;
    launch_reset_ctl(d, 1 << 30, 0.0, stream);
    if (d.batch) {
        launch_breset(d, stream);
        const bool primal = form == CDCS_PRIMAL;
        for (int r = 0; r < reps; ++r) {
            if (kernel == CDCS_K_PROJECT) launch_projection(h, primal ? PROJ_PRIMAL : PROJ_DUAL, st, rho, stream);
            else if (kernel == CDCS_K_SCATTER)
                primal ? launch_bscatter_primal(d, st->blk, st->lam, rho, stream)
                       : launch_bscatter_dual(d, st->blk, st->lam, rho, stream);
            else if (kernel == CDCS_K_GEMV_AU)
                launch_baffine(d, d.b, primal ? 1.0 : -1.0 / rho, st->x, st->y, d.ctl, nullptr, stream);
            else return fail(CDCS_E_ARG, "batch handles profile CDCS_K_PROJECT, CDCS_K_SCATTER, CDCS_K_GEMV_AU");
        }
        HIP_OK(hipGetLastError());
        return CDCS_OK;
    }
    for (int r = 0; r < reps; ++r) {
        switch (kernel) {
        case CDCS_K_PROJECT:
            launch_projection(h, form == CDCS_PRIMAL ? PROJ_PRIMAL : PROJ_DUAL, st, rho, stream);
            break;
        case CDCS_K_GEMV_AU:
            launch_affine_part(d, 0, d.b, form == CDCS_PRIMAL ? 1.0 : -1.0 / rho, st->x, st->y, d.ctl, stream);
            break;
        case CDCS_K_TRMV:
            launch_affine_part(d, 1, d.b, 1.0, st->x, st->y, d.ctl, stream);
            break;
        case CDCS_K_GEMV_ATY:
            launch_affine_part(d, 2, d.b, 1.0, st->x, st->y, d.ctl, stream);
            break;
        case CDCS_K_SCATTER:
            if (form == CDCS_PRIMAL) launch_scatter_primal(d, st->blk, st->lam, rho, stream);
            else launch_scatter_dual(d, st->blk, st->lam, rho, stream);
            break;
        default:
            return fail(CDCS_E_ARG, "unknown kernel id");
        }
    }
    HIP_OK(hipGetLastError());
    return CDCS_OK;
}

cdcs_status cdcs_get_tuning(const cdcs_handle *h, cdcs_tuning *out) {
    if (!h || !out) return fail(CDCS_E_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->persistent = h->plan.queue ? 1 : h->plan.parallel ? 2 : 0;
    out->threads = h->plan.nt;
    out->grid = h->plan.grid;
    out->nbuckets = (int32_t)std::min<size_t>(h->buckets.size(), 8);
    for (int q = 0; q < out->nbuckets; ++q) {
        out->bucket_size[q] = h->buckets[(size_t)q].smax;
        out->bucket_threads[q] = h->buckets[(size_t)q].nt;
        out->bucket_count[q] = h->buckets[(size_t)q].count;
        out->bucket_us[q] = h->buckets[(size_t)q].us;
    }
    out->queue_us = h->plan.queue_us;
    out->buckets_us = h->plan.buckets_us;
    out->parallel_us = h->plan.parallel_us;
    return CDCS_OK;
}

cdcs_status cdcs_set_projection_plan(cdcs_handle *h, int32_t persistent, int32_t threads, int32_t grid_req) {
    if (!h) return fail(CDCS_E_ARG, "NULL handle");
    if (persistent < 0 || persistent > 2) return fail(CDCS_E_ARG, "persistent must be 0, 1 or 2");
    if (persistent == 1) {
        if (threads != 256 && threads != 512) return fail(CDCS_E_ARG, "queue launches use 256 or 512 threads");
        const int grid_max = queue_grid(h, threads);
        if (grid_max < 1)
            return fail(CDCS_E_ARG, h->d.p_lds < 1 ? "no cliques for the queue launch"
                                                    : "queue launches over cliques above 96 vertices use 512 threads");
        if (grid_req < 0 || grid_req > grid_max)
            return fail(CDCS_E_ARG, "grid outside 0.." + std::to_string(grid_max) + " (resident workgroups)");
        const int grid = grid_req > 0 ? grid_req : grid_max;
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMemset(h->ticket, 0, sizeof(unsigned long long)));
        h->plan.queue = true;
        h->plan.parallel = false;
        h->plan.nt = threads;
        h->plan.grid = grid;
    } else {
        if (threads != 0 && threads != 64 && threads != 256 && threads != 512)
            return fail(CDCS_E_ARG, "threads must be 0, 64, 256 or 512");
        h->plan.queue = false;
        h->plan.parallel = persistent == 2;
        if (threads != 0)
            for (Bucket &bk : h->buckets) bk.nt = proj_threads_ok(proj_bucket(bk.smax), threads) ? threads : 256;
    }
    // captured graphs hold the old launches
    HIP_OK(hipDeviceSynchronize());
    for (auto &kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    return CDCS_OK;
}

cdcs_status cdcs_hsde_history(const cdcs_handle *h, double *hist_host, int32_t n_host) {
    if (!h || (!hist_host && n_host > 0)) return fail(CDCS_E_ARG, "NULL argument");
    const int n = std::min<int>(n_host, std::min(h->last_iters, h->hs.hist_cap));
    if (n <= 0) return CDCS_OK;
    HIP_OK(hipMemcpy(hist_host, h->hs.hist, (size_t)n * 3 * sizeof(double), hipMemcpyDeviceToHost));
    return CDCS_OK;
}

cdcs_status cdcs_residual_history(const cdcs_handle *h, double *hist_host, int32_t n_host) {
    if (!h || (!hist_host && n_host > 0)) return fail(CDCS_E_ARG, "NULL argument");
    const int n = std::min<int>(n_host, std::min(h->last_iters, h->d.hist_cap));
    if (n <= 0) return CDCS_OK;
    HIP_OK(hipMemcpy(hist_host, h->d.hist, (size_t)n * 2 * sizeof(double), hipMemcpyDeviceToHost));
    return CDCS_OK;
}

cdcs_status cdcs_destroy(cdcs_handle *h) {
    if (!h) return CDCS_OK;
    (void)hipDeviceSynchronize();
    delete h;
    return CDCS_OK;
}

}  // extern "C"
