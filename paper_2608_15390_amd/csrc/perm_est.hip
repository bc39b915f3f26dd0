// perm_est.hip -- host side of the C ABI declared in include/perm_est.h.
//
// create : validate CSR/CSC on the host, upload, build the CSC->CSR edge
//          map on the device.
// run    : (once per initial-DM / K0 setting) initial support filter and
//          compaction of the kept entries, K0 outer SK iterations,
//          degree / min-tree templates; then the persistent trajectory
//          kernel and the FP64 statistics reduction on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "perm_est.h"
#include "prep.hpp"
#include "reduce.hpp"

using namespace pe;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define PE_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(PE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline unsigned blocks_for(int64_t n, int threads = 256) {
    return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads);
}

template <typename T>
int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) return fail(PE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    return PE_OK;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

struct Prepared {
    int32_t initial_dm = -1, K0 = -1;
    int32_t ok = 1;
    bool own = false;  // filtered copy (else aliases the input matrix)
    int64_t m = 0;
    int32_t dmax = 0;
    int32_t *row_ptr = nullptr, *col_idx = nullptr, *col_ptr = nullptr, *row_idx = nullptr,
            *csc2csr = nullptr, *edge_row = nullptr;
    float *val = nullptr, *val_csc = nullptr;
    float *r0 = nullptr, *c0 = nullptr;
    int32_t *mate_r = nullptr, *mate_c = nullptr;  // perfect matching found by the initial filter
    uint16_t *deg0 = nullptr;
    uint32_t *tree0 = nullptr;
    int32_t n_leaf = 0;
    TreeLayout tree{};

    void release() {
        if (own) {
            dfree(row_ptr); dfree(col_idx); dfree(col_ptr); dfree(row_idx); dfree(csc2csr);
            dfree(val); dfree(val_csc); dfree(edge_row);
        }
        dfree(r0); dfree(c0); dfree(deg0); dfree(tree0); dfree(mate_r); dfree(mate_c);
    }
};

}  // namespace

struct perm_est {
    int device = 0;
    uint32_t opt_flags = 0;
    int32_t n = 0;
    int64_t m = 0;
    bool weighted = false;
    int32_t dmax = 0;
    int32_t *row_ptr = nullptr, *col_idx = nullptr, *col_ptr = nullptr, *row_idx = nullptr,
            *csc2csr = nullptr, *edge_row = nullptr;
    float *val = nullptr, *val_csc = nullptr;
    std::vector<Prepared> preps;
    int cu_count = 256;
    // reusable run buffers
    char *hbm_state = nullptr;
    size_t hbm_bytes = 0;
    uint32_t *work = nullptr;
    unsigned long long *work_totals = nullptr;
    DevStats *stats = nullptr;
    int64_t *seg = nullptr;
    int32_t *flags = nullptr;  // small scratch integers for preprocessing loops
    double *tmp_logw = nullptr;
    uint8_t *tmp_alive = nullptr;
    int32_t *tmp_counters = nullptr;
    int64_t tmp_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

int check_lists(int32_t n, int64_t nnz, const int32_t *ptr, const int32_t *idx, const char *what) {
    if (!ptr) return fail(PE_EINVAL, std::string(what) + ": null pointer array");
    if (ptr[0] != 0 || (int64_t)ptr[n] != nnz)
        return fail(PE_EINVAL, std::string(what) + ": ptr[0] must be 0 and ptr[n] == nnz");
    for (int32_t a = 0; a < n; ++a) {
        if (ptr[a + 1] < ptr[a]) return fail(PE_EINVAL, std::string(what) + ": ptr not monotone");
        if (ptr[a + 1] - ptr[a] > 65534)
            return fail(PE_ENOTSUP, std::string(what) + ": a list has more than 65534 entries");
        for (int32_t p = ptr[a]; p < ptr[a + 1]; ++p) {
            if (idx[p] < 0 || idx[p] >= n) return fail(PE_EINVAL, std::string(what) + ": index out of range");
            if (p > ptr[a] && idx[p] <= idx[p - 1])
                return fail(PE_EINVAL, std::string(what) + ": indices not strictly ascending");
        }
    }
    return PE_OK;
}

int read_flag(const int32_t *dflag, int32_t *host, hipStream_t s) {
    PE_HIP(hipMemcpyAsync(host, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    return PE_OK;
}

int zero_flag(int32_t *dflag, hipStream_t s) {
    k_fill_i32<<<1, 64, 0, s>>>(1, dflag, 0);
    PE_HIP(hipGetLastError());
    return PE_OK;
}

// Initial support filter of the whole input: maximum matching by greedy
// rounds plus multi-source BFS augmentation, strongly connected components
// of the contracted alternating digraph by trimming and max-label colouring,
// then keep[e].  Returns ok = 0 when no perfect matching exists.
int initial_filter(perm_est *h, uint8_t *keep, int32_t *ok, int32_t *out_mate_r, int32_t *out_mate_c,
                   hipStream_t s) {
    const int32_t n = h->n;
    int32_t *mate_r, *mate_c, *root, *level, *claim, *path_end, *scc, *color, *mark;
    int rc;
    if ((rc = dalloc(&mate_r, n)) || (rc = dalloc(&mate_c, n)) || (rc = dalloc(&root, n)) ||
        (rc = dalloc(&level, n)) || (rc = dalloc(&claim, n)) || (rc = dalloc(&path_end, n)) ||
        (rc = dalloc(&scc, n)) || (rc = dalloc(&color, n)) || (rc = dalloc(&mark, n)))
        return rc;
    auto cleanup = [&]() {
        dfree(mate_r); dfree(mate_c); dfree(root); dfree(level); dfree(claim);
        dfree(path_end); dfree(scc); dfree(color); dfree(mark);
    };
    const unsigned gb = blocks_for(n);
    int32_t flag = 0;
    int32_t *f = h->flags;
    auto run = [&]() -> int {
        k_fill_i32<<<gb, 256, 0, s>>>(n, mate_r, -1);
        k_fill_i32<<<gb, 256, 0, s>>>(n, mate_c, -1);
        for (int it = 0; it < 64; ++it) {
            if ((rc = zero_flag(f, s))) return rc;
            k_greedy<<<gb, 256, 0, s>>>(n, h->row_ptr, h->col_idx, mate_r, mate_c, f);
            if ((rc = read_flag(f, &flag, s))) return rc;
            if (!flag) break;
        }
        for (;;) {
            if ((rc = zero_flag(f, s))) return rc;
            k_aug_init<<<gb, 256, 0, s>>>(n, mate_r, root, level, claim, path_end, f);
            if ((rc = read_flag(f, &flag, s))) return rc;
            if (flag == 0) break;  // perfect matching
            for (int32_t cur = 0;; ++cur) {
                if ((rc = zero_flag(f + 1, s))) return rc;
                k_aug_level<<<gb, 256, 0, s>>>(n, h->row_ptr, h->col_idx, mate_c, root, level, claim,
                                               path_end, cur, f + 1);
                if ((rc = read_flag(f + 1, &flag, s))) return rc;
                if (!flag) break;
            }
            if ((rc = zero_flag(f + 2, s))) return rc;
            k_aug_flip<<<gb, 256, 0, s>>>(n, claim, path_end, mate_r, mate_c, f + 2);
            if ((rc = read_flag(f + 2, &flag, s))) return rc;
            if (flag == 0) break;  // maximum, not perfect
        }
        if ((rc = zero_flag(f, s))) return rc;
        k_count_matched<<<gb, 256, 0, s>>>(n, mate_r, f);
        if ((rc = read_flag(f, &flag, s))) return rc;
        if (flag != n) { *ok = 0; return PE_OK; }
        *ok = 1;
        k_fill_i32<<<gb, 256, 0, s>>>(n, scc, -1);
        for (;;) {
            for (;;) {
                if ((rc = zero_flag(f, s))) return rc;
                k_scc_trim<<<gb, 256, 0, s>>>(n, h->row_ptr, h->col_idx, h->col_ptr, h->row_idx, mate_r,
                                              mate_c, scc, f);
                if ((rc = read_flag(f, &flag, s))) return rc;
                if (!flag) break;
            }
            if ((rc = zero_flag(f, s))) return rc;
            k_scc_unassigned<<<gb, 256, 0, s>>>(n, scc, f);
            if ((rc = read_flag(f, &flag, s))) return rc;
            if (flag == 0) break;
            k_scc_color_init<<<gb, 256, 0, s>>>(n, scc, color);
            for (;;) {
                if ((rc = zero_flag(f, s))) return rc;
                k_scc_color_prop<<<gb, 256, 0, s>>>(n, h->row_ptr, h->col_idx, mate_r, mate_c, scc, color, f);
                if ((rc = read_flag(f, &flag, s))) return rc;
                if (!flag) break;
            }
            k_scc_roots<<<gb, 256, 0, s>>>(n, color, scc, mark);
            for (;;) {
                if ((rc = zero_flag(f, s))) return rc;
                k_scc_back<<<gb, 256, 0, s>>>(n, h->col_ptr, h->row_idx, mate_r, color, scc, mark, f);
                if ((rc = read_flag(f, &flag, s))) return rc;
                if (!flag) break;
            }
        }
        k_keep_edges<<<gb, 256, 0, s>>>(n, h->row_ptr, h->col_idx, mate_r, mate_c, scc, keep);
        PE_HIP(hipGetLastError());
        PE_HIP(hipMemcpyAsync(out_mate_r, mate_r, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        PE_HIP(hipMemcpyAsync(out_mate_c, mate_c, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        PE_HIP(hipStreamSynchronize(s));
        return PE_OK;
    };
    rc = run();
    cleanup();
    return rc;
}

int build_prepared(perm_est *h, int32_t initial_dm, int32_t K0, hipStream_t s, Prepared &P) {
    const int32_t n = h->n;
    int rc;
    P.initial_dm = initial_dm;
    P.K0 = K0;
    P.ok = 1;
    P.own = false;
    P.m = h->m;
    P.row_ptr = h->row_ptr; P.col_idx = h->col_idx; P.col_ptr = h->col_ptr;
    P.row_idx = h->row_idx; P.csc2csr = h->csc2csr; P.val = h->val; P.val_csc = h->val_csc;
    P.edge_row = h->edge_row;
    P.dmax = h->dmax;
    if (initial_dm && h->m > 0) {
        uint8_t *keep;
        if ((rc = dalloc(&keep, (size_t)h->m))) return rc;
        int32_t ok = 0;
        if ((rc = dalloc(&P.mate_r, n)) || (rc = dalloc(&P.mate_c, n))) { dfree(keep); return rc; }
        rc = initial_filter(h, keep, &ok, P.mate_r, P.mate_c, s);
        if (rc) { dfree(keep); return rc; }
        P.ok = ok;
        if (ok) {
            int32_t *len, *new_id;
            if ((rc = dalloc(&len, n)) || (rc = dalloc(&new_id, (size_t)h->m)) ||
                (rc = dalloc(&P.row_ptr, n + 1)) || (rc = dalloc(&P.col_ptr, n + 1))) {
                dfree(keep);
                return rc;
            }
            P.own = true;
            P.col_idx = P.row_idx = P.csc2csr = P.edge_row = nullptr;
            P.val = P.val_csc = nullptr;
            const unsigned gb = blocks_for(n);
            k_row_keep_count<<<gb, 256, 0, s>>>(n, h->row_ptr, keep, len);
            k_scan_excl<<<1, 1024, 0, s>>>(n, len, P.row_ptr);
            int32_t m2 = 0;
            PE_HIP(hipMemcpyAsync(&m2, P.row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            PE_HIP(hipStreamSynchronize(s));
            P.m = m2;
            if ((rc = dalloc(&P.col_idx, m2)) || (rc = dalloc(&P.row_idx, m2)) ||
                (rc = dalloc(&P.csc2csr, m2)) || (rc = dalloc(&P.edge_row, m2)))
                return rc;
            if (h->val && ((rc = dalloc(&P.val, m2)) || (rc = dalloc(&P.val_csc, m2)))) return rc;
            k_row_scatter<<<gb, 256, 0, s>>>(n, h->row_ptr, h->col_idx, h->val, keep, P.row_ptr,
                                             P.col_idx, P.val, new_id);
            k_col_keep_count<<<gb, 256, 0, s>>>(n, h->col_ptr, h->csc2csr, keep, len);
            k_scan_excl<<<1, 1024, 0, s>>>(n, len, P.col_ptr);
            k_col_scatter<<<gb, 256, 0, s>>>(n, h->col_ptr, h->row_idx, h->csc2csr, keep, new_id,
                                             P.col_ptr, P.row_idx, P.csc2csr);
            if (h->val) k_gather_f32<<<blocks_for(m2), 256, 0, s>>>(m2, P.val, P.csc2csr, P.val_csc);
            k_edge_row<<<gb, 256, 0, s>>>(n, P.row_ptr, P.edge_row);
            PE_HIP(hipGetLastError());
            // maximum degree of the filtered matrix
            std::vector<int32_t> rp(n + 1), cp(n + 1);
            PE_HIP(hipMemcpyAsync(rp.data(), P.row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
            PE_HIP(hipMemcpyAsync(cp.data(), P.col_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
            PE_HIP(hipStreamSynchronize(s));
            int32_t dm = 1;
            for (int32_t a = 0; a < n; ++a) dm = std::max({dm, rp[a + 1] - rp[a], cp[a + 1] - cp[a]});
            P.dmax = dm;
            dfree(len);
            dfree(new_id);
        }
        dfree(keep);
    }
    if (K0 > 0) {
        if ((rc = dalloc(&P.r0, n)) || (rc = dalloc(&P.c0, n))) return rc;
        const unsigned gb = blocks_for(n);
        k_fill_f32<<<gb, 256, 0, s>>>(n, P.r0, 1.0f);
        k_fill_f32<<<gb, 256, 0, s>>>(n, P.c0, 1.0f);
        if (P.ok) {
            for (int32_t it = 0; it < K0; ++it) {
                k_sk_cols<<<gb, 256, 0, s>>>(n, P.col_ptr, P.row_idx, P.val_csc, P.r0, P.c0);
                k_sk_rows<<<gb, 256, 0, s>>>(n, P.row_ptr, P.col_idx, P.val, P.r0, P.c0);
            }
        }
        PE_HIP(hipGetLastError());
    }
    // degree leaves and min-tree templates
    P.n_leaf = (int32_t)(((int64_t)2 * n + 255) / 256 * 256);
    const int32_t g1 = P.n_leaf / 256;
    TreeLayout T{};
    T.size[0] = g1;
    T.levels = 1;
    while (T.size[T.levels - 1] > 64) {
        if (T.levels == 3) return fail(PE_ENOTSUP, "matrix order too large for the min-tree");
        T.size[T.levels] = (T.size[T.levels - 1] + 63) / 64;
        T.levels += 1;
    }
    int32_t off = 0;
    for (int k = 0; k < T.levels; ++k) { T.off[k] = off; off += T.size[k]; }
    T.total = (off + 3) / 4 * 4;
    P.tree = T;
    if ((rc = dalloc(&P.deg0, P.n_leaf)) || (rc = dalloc(&P.tree0, T.total))) return rc;
    k_deg_template<<<blocks_for(P.n_leaf), 256, 0, s>>>(n, P.n_leaf, P.row_ptr, P.col_ptr, P.deg0);
    k_tree_leaves<<<blocks_for(g1), 256, 0, s>>>(g1, P.deg0, P.tree0 + T.off[0]);
    for (int k = 1; k < T.levels; ++k)
        k_tree_up<<<blocks_for(T.size[k]), 256, 0, s>>>(T.size[k - 1], P.tree0 + T.off[k - 1], T.size[k],
                                                        P.tree0 + T.off[k]);
    PE_HIP(hipGetLastError());
    PE_HIP(hipStreamSynchronize(s));
    return PE_OK;
}

int get_prepared(perm_est *h, int32_t initial_dm, int32_t K0, hipStream_t s, Prepared **out) {
    for (auto &P : h->preps)
        if (P.initial_dm == initial_dm && P.K0 == K0) { *out = &P; return PE_OK; }
    Prepared P;
    int rc = build_prepared(h, initial_dm, K0, s, P);
    if (rc) { P.release(); return rc; }
    h->preps.push_back(P);
    *out = &h->preps.back();
    return PE_OK;
}

uint32_t align_up(uint64_t x, uint64_t a) { return (uint32_t)((x + a - 1) / a * a); }

template <int SK, bool DM>
void launch_w(bool wt, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s, const TrajArgs &a) {
    if (wt) traj_kernel<SK, DM, true><<<blocks, threads, shmem, s>>>(a);
    else traj_kernel<SK, DM, false><<<blocks, threads, shmem, s>>>(a);
}

template <int SK>
void launch_dm(bool dm, bool wt, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s,
               const TrajArgs &a) {
    if (dm) launch_w<SK, true>(wt, blocks, threads, shmem, s, a);
    else launch_w<SK, false>(wt, blocks, threads, shmem, s, a);
}

void launch_traj(int sk, bool dm, bool wt, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s,
                 const TrajArgs &a) {
    switch (sk) {
        case PE_SK_NONE: launch_dm<kSkNone>(dm, wt, blocks, threads, shmem, s, a); break;
        case PE_SK_FIXED: launch_dm<kSkFixed>(dm, wt, blocks, threads, shmem, s, a); break;
        case PE_SK_ADAPTIVE: launch_dm<kSkAdaptive>(dm, wt, blocks, threads, shmem, s, a); break;
        default: launch_dm<kSkLocal>(dm, wt, blocks, threads, shmem, s, a); break;
    }
}

int check_schedule(const perm_est_schedule *s) {
    if (!s) return fail(PE_EINVAL, "schedule is NULL");
    if (s->vertex_rule < 0 || s->vertex_rule > 1) return fail(PE_EINVAL, "bad vertex_rule");
    if (s->sk_policy < 0 || s->sk_policy > 3) return fail(PE_EINVAL, "bad sk_policy");
    if (s->dm_policy < 0 || s->dm_policy > 3) return fail(PE_EINVAL, "bad dm_policy");
    if (s->initial_dm < 0 || s->initial_dm > 1) return fail(PE_EINVAL, "bad initial_dm");
    if (s->K0 < 0 || s->K < 0) return fail(PE_EINVAL, "K0 and K must be >= 0");
    if (!std::isfinite(s->theta_th) || !std::isfinite(s->theta_tr)) return fail(PE_EINVAL, "bad thresholds");
    for (int i = 0; i < 4; ++i)
        if (s->reserved[i] != 0) return fail(PE_EINVAL, "reserved schedule fields must be 0");
    return PE_OK;
}

}  // namespace

extern "C" {

const char *perm_est_last_error(void) { return g_err.c_str(); }

int perm_est_schedule_preset(const char *name, perm_est_schedule *out) {
    if (!name || !out) return fail(PE_EINVAL, "null argument");
    perm_est_schedule s;
    std::memset(&s, 0, sizeof(s));
    s.vertex_rule = PE_VR_MD;
    s.K = 10;
    s.theta_th = 0.33;
    s.theta_tr = 0.33;
    const std::string nm(name);
    auto paper = [&](int sk, int dm) {
        s.sk_policy = sk; s.dm_policy = dm; s.initial_dm = 1; s.K0 = 100; s.K = 10;
    };
    if (nm == "plain") {
    } else if (nm == "rasmussen") {
        s.vertex_rule = PE_VR_ROW_ORDER;
    } else if (nm == "fixed_all") {
        paper(PE_SK_FIXED, PE_DM_ALL);
    } else if (nm == "adaptive_threshold") {
        paper(PE_SK_ADAPTIVE, PE_DM_THRS);
    } else if (nm == "local_threshold") {
        paper(PE_SK_LOCAL, PE_DM_THRS);
    } else if (nm == "adaptive_tracked") {
        paper(PE_SK_ADAPTIVE, PE_DM_TRCK);
    } else if (nm == "local_tracked") {
        paper(PE_SK_LOCAL, PE_DM_TRCK);
    } else if (nm == "local_nodm") {
        paper(PE_SK_LOCAL, PE_DM_NONE);
    } else {
        return fail(PE_EINVAL, "unknown preset '" + nm + "'");
    }
    *out = s;
    return PE_OK;
}

int perm_est_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                    const int32_t *col_ptr, const int32_t *row_idx, const float *values,
                    const perm_est_options *opts, perm_est_t **out) {
    if (!out) return fail(PE_EINVAL, "out is NULL");
    *out = nullptr;
    if (n <= 0) return fail(PE_EINVAL, "n must be positive");
    if (nnz < 0 || nnz >= (int64_t)1 << 31) return fail(PE_EINVAL, "nnz out of range");
    if (nnz > 0 && (!col_idx || !row_idx)) return fail(PE_EINVAL, "null index array");
    if (opts && (opts->flags & ~PE_FLAG_FORCE_HBM) != 0) return fail(PE_EINVAL, "unknown option flags");
    int rc;
    if ((rc = check_lists(n, nnz, row_ptr, col_idx, "CSR"))) return rc;
    if ((rc = check_lists(n, nnz, col_ptr, row_idx, "CSC"))) return rc;
    if (values)
        for (int64_t p = 0; p < nnz; ++p)
            if (!(values[p] > 0.0f) || !std::isfinite(values[p])) return fail(PE_EINVAL, "values must be finite and > 0");
    perm_est *h = new (std::nothrow) perm_est();
    if (!h) return fail(PE_ENOMEM, "host allocation failed");
    h->device = opts ? opts->device : 0;
    h->opt_flags = opts ? opts->flags : 0;
    h->n = n;
    h->m = nnz;
    h->weighted = values != nullptr;
    int32_t dm = 1;
    for (int32_t a = 0; a < n; ++a) dm = std::max({dm, row_ptr[a + 1] - row_ptr[a], col_ptr[a + 1] - col_ptr[a]});
    h->dmax = dm;
    auto bail = [&](int code) { perm_est_destroy(h); return code; };
    if (hipSetDevice(h->device) != hipSuccess) return bail(fail(PE_EDEVICE, "hipSetDevice failed"));
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
        h->cu_count = cus;
    if ((rc = dalloc(&h->row_ptr, n + 1)) || (rc = dalloc(&h->col_ptr, n + 1)) ||
        (rc = dalloc(&h->col_idx, nnz)) || (rc = dalloc(&h->row_idx, nnz)) ||
        (rc = dalloc(&h->csc2csr, nnz)) || (rc = dalloc(&h->edge_row, nnz)) || (rc = dalloc(&h->work, 2)) || (rc = dalloc(&h->work_totals, 5)) || (rc = dalloc(&h->stats, 1)) ||
        (rc = dalloc(&h->seg, 2)) || (rc = dalloc(&h->flags, 8)))
        return bail(rc);
    if (values && ((rc = dalloc(&h->val, nnz)) || (rc = dalloc(&h->val_csc, nnz)))) return bail(rc);
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
        return bail(fail(PE_EDEVICE, "hipEventCreate failed"));
    auto up = [&](void *d, const void *s, size_t bytes) {
        return bytes == 0 || hipMemcpy(d, s, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(h->row_ptr, row_ptr, sizeof(int32_t) * (n + 1)) || !up(h->col_ptr, col_ptr, sizeof(int32_t) * (n + 1)) ||
        !up(h->col_idx, col_idx, sizeof(int32_t) * nnz) || !up(h->row_idx, row_idx, sizeof(int32_t) * nnz) ||
        (values && !up(h->val, values, sizeof(float) * nnz)))
        return bail(fail(PE_EDEVICE, "upload failed"));
    int32_t err = 0;
    if (hipMemset(h->flags, 0, sizeof(int32_t)) != hipSuccess) return bail(fail(PE_EDEVICE, "hipMemset failed"));
    k_csc2csr<<<blocks_for(n), 256>>>(n, h->row_ptr, h->col_idx, h->col_ptr, h->row_idx, h->csc2csr, h->flags);
    k_edge_row<<<blocks_for(n), 256>>>(n, h->row_ptr, h->edge_row);
    if (values) k_gather_f32<<<blocks_for(nnz), 256>>>(nnz, h->val, h->csc2csr, h->val_csc);
    if (hipGetLastError() != hipSuccess || hipMemcpy(&err, h->flags, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return bail(fail(PE_EDEVICE, "edge map kernel failed"));
    if (err) return bail(fail(PE_EINVAL, "CSR and CSC hold different entries"));
    *out = h;
    return PE_OK;
}

void perm_est_destroy(perm_est_t *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    for (auto &P : h->preps) P.release();
    dfree(h->row_ptr); dfree(h->col_idx); dfree(h->col_ptr); dfree(h->row_idx); dfree(h->csc2csr);
    dfree(h->edge_row); dfree(h->val); dfree(h->val_csc);
    dfree(h->hbm_state); dfree(h->work); dfree(h->work_totals); dfree(h->stats); dfree(h->seg); dfree(h->flags);
    dfree(h->tmp_logw); dfree(h->tmp_alive); dfree(h->tmp_counters);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

int perm_est_run_range(perm_est_t *h, int64_t first, int64_t count, uint64_t seed,
                       const perm_est_schedule *sched, perm_est_result *res, double *logw,
                       uint8_t *alive, uint64_t *path_hash, int32_t *path, int32_t *counters,
                       void *stream) {
    if (!h || !res) return fail(PE_EINVAL, "null handle or result");
    if (count < 1 || first < 0 || first + count > ((int64_t)1 << 32))
        return fail(PE_EINVAL, "trajectory range must lie in [0, 2^32) and be non-empty");
    int rc;
    if ((rc = check_schedule(sched))) return rc;
    PE_HIP(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    Prepared *P;
    if ((rc = get_prepared(h, sched->initial_dm, sched->K0, s, &P))) return rc;
    const int32_t n = h->n;

    // ---- buffers for outputs the caller did not ask for
    if (!logw || !alive || !counters) {
        if (h->tmp_cap < count) {
            dfree(h->tmp_logw); dfree(h->tmp_alive); dfree(h->tmp_counters);
            h->tmp_cap = 0;
            if ((rc = dalloc(&h->tmp_logw, count)) || (rc = dalloc(&h->tmp_alive, count)) ||
                (rc = dalloc(&h->tmp_counters, 4 * count)))
                return rc;
            h->tmp_cap = count;
        }
    }
    double *lw = logw ? logw : h->tmp_logw;
    uint8_t *al = alive ? alive : h->tmp_alive;
    int32_t *cn = counters ? counters : h->tmp_counters;

    // ---- per-trajectory state layout
    const bool own_rc = sched->sk_policy != PE_SK_NONE;
    const bool local = sched->sk_policy == PE_SK_LOCAL;
    const bool dm = sched->dm_policy != PE_DM_NONE;
    StateLayout L{};
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) { uint32_t at = align_up(o, 16); o = (uint64_t)at + bytes; return at; };
    L.deg = take((uint64_t)P->n_leaf * 2);
    L.rec = take(own_rc ? 16ull * n : 0);
    L.lst_a = take(4ull * P->dmax);
    L.lst_b = take(4ull * P->dmax);
    L.loc_r = take(local ? 4ull * n : 0);
    L.loc_c = take(local ? 4ull * n : 0);
    L.new_v = take(local ? 8ull * n : 0);
    L.rem = take(dm ? 4ull * ((P->m + 31) / 32) : 0);
    L.mate_r = take(dm ? 4ull * n : 0);
    L.mate_c = take(dm ? 4ull * n : 0);
    L.ws = take(dm ? 24ull * n : 0);
    L.bytes = align_up(o, 256);
    if (o >= (1ull << 32)) return fail(PE_ENOTSUP, "per-trajectory state exceeds 4 GiB");

    TrajArgs a{};
    a.A = DevMat{n, (int32_t)P->m, P->row_ptr, P->col_idx, P->col_ptr, P->row_idx, P->csc2csr,
                 P->edge_row, P->val, P->val_csc};
    a.r0 = P->r0;
    a.c0 = P->c0;
    a.deg0 = P->deg0;
    a.tree0 = P->tree0;
    a.mate0_r = P->mate_r;
    a.mate0_c = P->mate_c;
    a.n_leaf = P->n_leaf;
    a.tree = P->tree;
    a.st = L;
    a.ok0 = P->ok;
    a.vertex_rule = sched->vertex_rule;
    a.sk_policy = sched->sk_policy;
    a.dm_policy = sched->dm_policy;
    a.K = sched->K;
    a.scaled = (P->r0 != nullptr) || own_rc;
    a.theta_th = sched->theta_th;
    a.theta_tr = sched->theta_tr;
    a.seed = seed;
    a.b = 0;
    a.first = first;
    a.count = count;
    a.logw = lw;
    a.alive = al;
    a.path_hash = path_hash;
    a.path = path;
    a.counters = cn;
    a.work_next = h->work;
    a.err = h->work + 1;
    a.work_totals = h->work_totals;

    // ---- tier and launch shape
    const size_t tree_bytes = (size_t)P->tree.total * 4;
    const size_t lds_wave = tree_bytes + L.bytes;
    const size_t kLdsBlock = 64 * 1024, kLdsCU = 160 * 1024;
    int wpb;
    unsigned blocks;
    size_t shmem;
    if (lds_wave <= 32 * 1024 && !(h->opt_flags & PE_FLAG_FORCE_HBM)) {
        a.hbm_state = nullptr;
        a.lds_state_bytes = (int32_t)L.bytes;
        wpb = (int)std::max<size_t>(1, std::min<size_t>(4, kLdsBlock / lds_wave));
        shmem = (size_t)wpb * lds_wave;
        const size_t per_cu = std::max<size_t>(1, std::min<size_t>(16 / wpb, kLdsCU / shmem));
        blocks = (unsigned)std::min<int64_t>((count + wpb - 1) / wpb, (int64_t)h->cu_count * per_cu);
    } else {
        wpb = 4;
        a.lds_state_bytes = 0;
        shmem = (size_t)wpb * tree_bytes;
        const size_t per_cu = std::max<size_t>(1, std::min<size_t>(4, kLdsCU / std::max<size_t>(shmem, 1)));
        blocks = (unsigned)std::min<int64_t>((count + wpb - 1) / wpb, (int64_t)h->cu_count * per_cu);
        const size_t need = (size_t)blocks * wpb * L.bytes;
        if (h->hbm_bytes < need) {
            dfree(h->hbm_state);
            h->hbm_bytes = 0;
            if ((rc = dalloc(&h->hbm_state, need))) return rc;
            h->hbm_bytes = need;
        }
        a.hbm_state = h->hbm_state;
        a.hbm_stride = L.bytes;
    }
    a.waves_per_block = wpb;

    int64_t seg_host[2] = {0, count};
    PE_HIP(hipMemcpyAsync(h->seg, seg_host, sizeof(seg_host), hipMemcpyHostToDevice, s));
    k_set_u32<<<1, 1, 0, s>>>(h->work, 0u);
    k_set_u32<<<1, 1, 0, s>>>(h->work + 1, 0u);
    k_fill_i32<<<1, 64, 0, s>>>(10, reinterpret_cast<int32_t *>(h->work_totals), 0);
    PE_HIP(hipEventRecord(h->ev0, s));
    launch_traj(sched->sk_policy, dm, P->val != nullptr, blocks, wpb * kWave, shmem, s, a);
    PE_HIP(hipGetLastError());
    k_reduce_stats<<<1, 1024, 0, s>>>(lw, al, cn, h->seg, h->stats);
    PE_HIP(hipGetLastError());
    PE_HIP(hipEventRecord(h->ev1, s));
    DevStats st;
    uint32_t err_bits = 0;
    unsigned long long wt[5];
    PE_HIP(hipMemcpyAsync(&st, h->stats, sizeof(st), hipMemcpyDeviceToHost, s));
    PE_HIP(hipMemcpyAsync(wt, h->work_totals, sizeof(wt), hipMemcpyDeviceToHost, s));
    PE_HIP(hipMemcpyAsync(&err_bits, h->work + 1, sizeof(err_bits), hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    if (err_bits) return fail(PE_EDEVICE, "trajectory kernel reported an internal inconsistency (bits " +
                                              std::to_string(err_bits) + ")");
    float ms = 0.0f;
    PE_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    res->log_estimate = st.log_estimate;
    res->p_match = st.p_match;
    res->rel_spread = st.rel_spread;
    res->rse = st.rse;
    res->ess = st.ess;
    res->var_logw = st.var_logw;
    res->max_logw = st.max_logw;
    res->n_traj = st.n_traj;
    res->n_alive = st.n_alive;
    res->n_dm = st.n_dm;
    res->n_full_sk = st.n_full_sk;
    res->n_local_sk = st.n_local_sk;
    res->n_steps = st.n_steps;
    res->seconds = ms * 1e-3;
    res->n_entries_scanned = (int64_t)wt[0];
    res->n_decrements = (int64_t)wt[1];
    res->n_local_entries = (int64_t)wt[2];
    res->n_local_values = (int64_t)wt[3];
    return PE_OK;
}

int perm_est_run(perm_est_t *h, int64_t n_traj, uint64_t seed, const perm_est_schedule *sched,
                 perm_est_result *res, double *logw, uint8_t *alive, uint64_t *path_hash,
                 void *stream) {
    return perm_est_run_range(h, 0, n_traj, seed, sched, res, logw, alive, path_hash, nullptr, nullptr,
                              stream);
}

}  // extern "C"
