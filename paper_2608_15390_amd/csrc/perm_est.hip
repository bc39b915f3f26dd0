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
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "perm_est.h"
#include "consensus.hpp"
#include "prep.hpp"
#include "reduce.hpp"
#include "rows.hpp"
#include "rows_learned.hpp"

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
    uint32_t *tree0a = nullptr;  // tree0 with level 1 packed as (degree << 8 | position)
    int32_t n_leaf = 0;
    TreeLayout tree{};

    void release() {
        if (own) {
            dfree(row_ptr); dfree(col_idx); dfree(col_ptr); dfree(row_idx); dfree(csc2csr);
            dfree(val); dfree(val_csc); dfree(edge_row);
        }
        dfree(r0); dfree(c0); dfree(deg0); dfree(tree0); dfree(tree0a); dfree(mate_r); dfree(mate_c);
    }
};

// one input matrix on the device, plus its preprocessed variants
struct MatData {
    int32_t n = 0;
    int64_t m = 0;
    bool weighted = false;
    int32_t dmax = 0;
    int32_t *row_ptr = nullptr, *col_idx = nullptr, *col_ptr = nullptr, *row_idx = nullptr,
            *csc2csr = nullptr, *edge_row = nullptr;
    float *val = nullptr, *val_csc = nullptr;
    std::vector<Prepared> preps;
    int32_t *flags = nullptr;  // borrowed: the handle's small scratch integers

    void release() {
        for (auto &P : preps) P.release();
        preps.clear();
        dfree(row_ptr); dfree(col_idx); dfree(col_ptr); dfree(row_idx); dfree(csc2csr);
        dfree(edge_row); dfree(val); dfree(val_csc);
    }
};

// launch shape chosen for a (schedule, tier) pair
struct Tune {
    int32_t sk = -1, dm = -1, force_hbm = -1;
    int32_t wpb = 4;      // waves per block
    int32_t per_cu = 4;   // blocks per CU in the persistent grid
};

}  // namespace

constexpr int kWorkTotals = 12;
// bytes of a min-tree's lowest internal level above which it lives in the
// trajectory's state slot (one trajectory per wave, HBM tier); 1024 nodes
// = 2^18 leaves, i.e. n above 131072
constexpr size_t kTreeLevel0LdsMax = 4096;  // launch-wide work counters, see BatchArgs::work_totals

// Scratch of perm_est_run_range_noalloc: one array per GPU the library runs
// on, held until the process ends.  Host code never uses this name as an
// address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device (noalloc_scratch).
constexpr size_t kScratchBytes = (size_t)PE_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on `dev` (the current device), looked up
// the first time a handle is created on that device
int noalloc_scratch(int dev, char **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(PE_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return PE_OK;
}
}  // namespace

struct perm_est {
    int device = 0;
    uint32_t opt_flags = 0;
    int cu_count = 256;
    double wall_hz = 0.0;  // rate of the device wall clock the kernels read
    size_t lds_block = 64 * 1024;  // LDS one workgroup may allocate (queried)
    size_t lds_cu = 160 * 1024;    // LDS of one compute unit
    std::vector<MatData> mats;
    std::vector<Tune> tunes;
    // reusable run buffers
    char *hbm_state = nullptr;
    size_t hbm_bytes = 0;
    uint32_t *work = nullptr;  // [0] item counter, [1] error bits
    unsigned long long *work_totals = nullptr;
    int32_t *flags = nullptr;  // small scratch integers for preprocessing loops
    TrajArgs *args_dev = nullptr;
    BatchArgs *batch_dev = nullptr;
    int32_t *order_dev = nullptr;
    int64_t *item_off_dev = nullptr;
    ReduceSeg *seg_dev = nullptr;
    DevStats *stats = nullptr;
    size_t cap_mats = 0;
    double *tmp_logw = nullptr;
    uint8_t *tmp_alive = nullptr;
    int32_t *tmp_counters = nullptr;
    int64_t tmp_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evk0 = nullptr, evk1 = nullptr;  // the trajectory kernel alone (eager launches)
    // learned proposal: snapped network parameters and the softmax table
    float *mlp = nullptr;
    int64_t *etab = nullptr;
    double mix_alpha = 0.05;
    bool has_model = false;
    unsigned long long *rec_ctr = nullptr;  // [0] claimed, [1] written (records << 32 | groups)
    // captured launch sequence (counter fills, trajectory kernel, reduction);
    // its kernels read every per-run value from device memory uploaded before
    // each replay, so one capture serves every run with the same launch shape
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const void *graph_fn = nullptr;
    unsigned graph_blocks = 0, graph_threads = 0;
    size_t graph_shmem = 0;
    bool graph_res = false;
    // host copies the async uploads read from
    std::vector<TrajArgs> args_host;
    BatchArgs batch_host{};
    std::vector<int32_t> order_host;
    std::vector<int64_t> item_off_host;
    std::vector<ReduceSeg> seg_host;
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
int initial_filter(MatData *h, uint8_t *keep, int32_t *ok, int32_t *out_mate_r, int32_t *out_mate_c,
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

int build_prepared(MatData *h, int32_t initial_dm, int32_t K0, hipStream_t s, Prepared &P) {
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
    if ((rc = dalloc(&P.deg0, P.n_leaf)) || (rc = dalloc(&P.tree0, T.total)) || (rc = dalloc(&P.tree0a, T.total)))
        return rc;
    k_deg_template<<<blocks_for(P.n_leaf), 256, 0, s>>>(n, P.n_leaf, P.row_ptr, P.col_ptr, P.deg0);
    k_tree_leaves<<<blocks_for(g1), 256, 0, s>>>(g1, P.deg0, P.tree0 + T.off[0]);
    for (int k = 1; k < T.levels; ++k)
        k_tree_up<<<blocks_for(T.size[k]), 256, 0, s>>>(T.size[k - 1], P.tree0 + T.off[k - 1], T.size[k],
                                                        P.tree0 + T.off[k]);
    k_tree_leaves_argmin<<<blocks_for(g1), 256, 0, s>>>(g1, P.deg0, P.tree0a + T.off[0]);
    if (T.levels > 1)
        PE_HIP(hipMemcpyAsync(P.tree0a + T.off[1], P.tree0 + T.off[1], sizeof(uint32_t) * (T.total - T.off[1]),
                              hipMemcpyDeviceToDevice, s));
    PE_HIP(hipGetLastError());
    PE_HIP(hipStreamSynchronize(s));
    return PE_OK;
}

// the preprocessed variant for (initial_dm, K0) if it exists (never builds one)
int find_prepared(MatData *h, int32_t initial_dm, int32_t K0, Prepared **out) {
    for (auto &P : h->preps)
        if (P.initial_dm == initial_dm && P.K0 == K0) { *out = &P; return PE_OK; }
    return fail(PE_EINVAL, "this schedule's preprocessing (initial_dm, K0) has not run on the handle; "
                           "run it once with an allocating entry point first");
}

int get_prepared(MatData *h, int32_t initial_dm, int32_t K0, hipStream_t s, Prepared **out) {
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
void launch_w(bool wt, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s, const BatchArgs *b) {
    if (wt) traj_kernel<SK, DM, true><<<blocks, threads, shmem, s>>>(b);
    else traj_kernel<SK, DM, false><<<blocks, threads, shmem, s>>>(b);
}

template <int SK>
void launch_dm(bool dm, bool wt, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s,
               const BatchArgs *b) {
    if (dm) launch_w<SK, true>(wt, blocks, threads, shmem, s, b);
    else launch_w<SK, false>(wt, blocks, threads, shmem, s, b);
}

void launch_traj(int sk, bool dm, bool wt, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s,
                 const BatchArgs *b) {
    switch (sk) {
        case PE_SK_NONE: launch_dm<kSkNone>(dm, wt, blocks, threads, shmem, s, b); break;
        case PE_SK_FIXED: launch_dm<kSkFixed>(dm, wt, blocks, threads, shmem, s, b); break;
        case PE_SK_ADAPTIVE: launch_dm<kSkAdaptive>(dm, wt, blocks, threads, shmem, s, b); break;
        case PE_SK_LOCAL: launch_dm<kSkLocal>(dm, wt, blocks, threads, shmem, s, b); break;
        case kSkLearnedGated: launch_dm<kSkLearnedGated>(dm, wt, blocks, threads, shmem, s, b); break;
        default: launch_dm<kSkLearned>(dm, wt, blocks, threads, shmem, s, b); break;
    }
}

template <int SK>
const void *kernel_dm(bool dm, bool wt) {
    if (dm) return wt ? (const void *)&traj_kernel<SK, true, true> : (const void *)&traj_kernel<SK, true, false>;
    return wt ? (const void *)&traj_kernel<SK, false, true> : (const void *)&traj_kernel<SK, false, false>;
}

// the trajectory kernel instance a launch uses (for occupancy queries)
const void *traj_kernel_fn(int sk, bool dm, bool wt) {
    switch (sk) {
        case PE_SK_NONE: return kernel_dm<kSkNone>(dm, wt);
        case PE_SK_FIXED: return kernel_dm<kSkFixed>(dm, wt);
        case PE_SK_ADAPTIVE: return kernel_dm<kSkAdaptive>(dm, wt);
        case PE_SK_LOCAL: return kernel_dm<kSkLocal>(dm, wt);
        case kSkLearnedGated: return kernel_dm<kSkLearnedGated>(dm, wt);
        default: return kernel_dm<kSkLearned>(dm, wt);
    }
}

// four-trajectories-per-wave kernel (plain estimator)
const void *rows_kernel_fn(bool wt) {
    return wt ? (const void *)&traj_rows_kernel<true> : (const void *)&traj_rows_kernel<false>;
}

void launch_rows(bool wt, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s, const BatchArgs *b) {
    if (wt) traj_rows_kernel<true><<<blocks, threads, shmem, s>>>(b);
    else traj_rows_kernel<false><<<blocks, threads, shmem, s>>>(b);
}

// four-trajectories-per-wave kernel of the learned proposal
// l0g: the min-tree's lowest level in the state slot (TrajArgs::l0_state)
const void *rows_learned_kernel_fn(bool wt, bool l0g) {
    if (l0g)
        return wt ? (const void *)&traj_rows_learned_kernel<true, kAsGlobal>
                  : (const void *)&traj_rows_learned_kernel<false, kAsGlobal>;
    return wt ? (const void *)&traj_rows_learned_kernel<true, kAsLds>
              : (const void *)&traj_rows_learned_kernel<false, kAsLds>;
}

void launch_rows_learned(bool wt, bool l0g, unsigned blocks, unsigned threads, size_t shmem, hipStream_t s,
                         const BatchArgs *b) {
    if (l0g) {
        if (wt) traj_rows_learned_kernel<true, kAsGlobal><<<blocks, threads, shmem, s>>>(b);
        else traj_rows_learned_kernel<false, kAsGlobal><<<blocks, threads, shmem, s>>>(b);
    } else {
        if (wt) traj_rows_learned_kernel<true, kAsLds><<<blocks, threads, shmem, s>>>(b);
        else traj_rows_learned_kernel<false, kAsLds><<<blocks, threads, shmem, s>>>(b);
    }
}

// upper bound on resident trajectory waves per CU for the default launch shape
#ifndef PE_MAX_WAVES_PER_CU
#define PE_MAX_WAVES_PER_CU 32
#endif

int check_schedule(const perm_est_schedule *s) {
    if (!s) return fail(PE_EINVAL, "schedule is NULL");
    if (s->vertex_rule < 0 || s->vertex_rule > 1) return fail(PE_EINVAL, "bad vertex_rule");
    if (s->sk_policy < 0 || s->sk_policy > 4) return fail(PE_EINVAL, "bad sk_policy");
    if (s->dm_policy < 0 || s->dm_policy > 3) return fail(PE_EINVAL, "bad dm_policy");
    if (s->initial_dm < 0 || s->initial_dm > 1) return fail(PE_EINVAL, "bad initial_dm");
    if (s->K0 < 0 || s->K < 0) return fail(PE_EINVAL, "K0 and K must be >= 0");
    if (!std::isfinite(s->theta_th) || !std::isfinite(s->theta_tr)) return fail(PE_EINVAL, "bad thresholds");
    if (s->local_gate < 0 || s->local_gate > 1) return fail(PE_EINVAL, "bad local_gate");
    if (s->local_gate && s->sk_policy != PE_SK_LEARNED)
        return fail(PE_EINVAL, "local_gate applies to the learned proposal only");
    if (s->local_cap < 0 || s->local_cap > 65535) return fail(PE_EINVAL, "local_cap must lie in [0, 65535]");
    if (s->local_cap && !(s->sk_policy == PE_SK_LOCAL || (s->sk_policy == PE_SK_LEARNED && s->local_gate)))
        return fail(PE_EINVAL, "local_cap applies to the local repair only");
    for (int i = 0; i < 2; ++i)
        if (s->reserved[i] != 0) return fail(PE_EINVAL, "reserved schedule fields must be 0");
    return PE_OK;
}

// validate one CSR/CSC pair on the host and move it to the device
int make_matrix(perm_est *h, int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                const int32_t *col_ptr, const int32_t *row_idx, const float *values, MatData &M) {
    if (n <= 0) return fail(PE_EINVAL, "n must be positive");
    if (nnz < 0 || nnz >= (int64_t)1 << 31) return fail(PE_EINVAL, "nnz out of range");
    if (nnz > 0 && (!col_idx || !row_idx)) return fail(PE_EINVAL, "null index array");
    int rc;
    if ((rc = check_lists(n, nnz, row_ptr, col_idx, "CSR"))) return rc;
    if ((rc = check_lists(n, nnz, col_ptr, row_idx, "CSC"))) return rc;
    if (values)
        for (int64_t p = 0; p < nnz; ++p)
            if (!(values[p] > 0.0f) || !std::isfinite(values[p]))
                return fail(PE_EINVAL, "values must be finite and > 0");
    M.n = n;
    M.m = nnz;
    M.weighted = values != nullptr;
    M.flags = h->flags;
    int32_t dm = 1;
    for (int32_t a = 0; a < n; ++a) dm = std::max({dm, row_ptr[a + 1] - row_ptr[a], col_ptr[a + 1] - col_ptr[a]});
    M.dmax = dm;
    if ((rc = dalloc(&M.row_ptr, n + 1)) || (rc = dalloc(&M.col_ptr, n + 1)) || (rc = dalloc(&M.col_idx, nnz)) ||
        (rc = dalloc(&M.row_idx, nnz)) || (rc = dalloc(&M.csc2csr, nnz)) || (rc = dalloc(&M.edge_row, nnz)))
        return rc;
    if (values && ((rc = dalloc(&M.val, nnz)) || (rc = dalloc(&M.val_csc, nnz)))) return rc;
    auto up = [&](void *d, const void *src, size_t bytes) {
        return bytes == 0 || hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(M.row_ptr, row_ptr, sizeof(int32_t) * (n + 1)) || !up(M.col_ptr, col_ptr, sizeof(int32_t) * (n + 1)) ||
        !up(M.col_idx, col_idx, sizeof(int32_t) * nnz) || !up(M.row_idx, row_idx, sizeof(int32_t) * nnz) ||
        (values && !up(M.val, values, sizeof(float) * nnz)))
        return fail(PE_EDEVICE, "upload failed");
    int32_t err = 0;
    if (hipMemset(h->flags, 0, sizeof(int32_t)) != hipSuccess) return fail(PE_EDEVICE, "hipMemset failed");
    k_csc2csr<<<blocks_for(n), 256>>>(n, M.row_ptr, M.col_idx, M.col_ptr, M.row_idx, M.csc2csr, h->flags);
    k_edge_row<<<blocks_for(n), 256>>>(n, M.row_ptr, M.edge_row);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpy(&err, h->flags, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(PE_EDEVICE, "edge map kernel failed");
    // the map has an entry for every CSC position only when both forms agree;
    // the value gather reads through it, so it runs after the check
    if (err) return fail(PE_EINVAL, "CSR and CSC hold different entries");
    if (values) {
        k_gather_f32<<<blocks_for(nnz), 256>>>(nnz, M.val, M.csc2csr, M.val_csc);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
            return fail(PE_EDEVICE, "value gather kernel failed");
    }
    return PE_OK;
}

int new_handle(const perm_est_options *opts, perm_est **out) {
    if (opts && (opts->flags & ~(PE_FLAG_FORCE_HBM | PE_FLAG_WAVE_PER_TRAJECTORY)) != 0)
        return fail(PE_EINVAL, "unknown option flags");
    perm_est *h = new (std::nothrow) perm_est();
    if (!h) return fail(PE_ENOMEM, "host allocation failed");
    h->device = opts ? opts->device : 0;
    h->opt_flags = opts ? opts->flags : 0;
    *out = h;
    if (hipSetDevice(h->device) != hipSuccess) return fail(PE_EDEVICE, "hipSetDevice failed");
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && cus > 0)
        h->cu_count = cus;
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, h->device) == hipSuccess && wall_khz > 0)
        h->wall_hz = 1e3 * (double)wall_khz;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess && lds > 0)
        h->lds_block = (size_t)lds;
    h->lds_cu = std::max(h->lds_cu, h->lds_block);
    char *scr = nullptr;
    if (int rc0 = noalloc_scratch(h->device, &scr)) return rc0;
    int rc;
    if ((rc = dalloc(&h->work, 3)) || (rc = dalloc(&h->work_totals, kWorkTotals)) || (rc = dalloc(&h->flags, 8)) ||
        (rc = dalloc(&h->batch_dev, 1)) || (rc = dalloc(&h->rec_ctr, 2)))
        return rc;
    if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
        hipEventCreate(&h->evk0) != hipSuccess || hipEventCreate(&h->evk1) != hipSuccess)
        return fail(PE_EDEVICE, "hipEventCreate failed");
    return PE_OK;
}

// outputs of one matrix's share of a launch
struct RunPart {
    int64_t first = 0, count = 0;
    double *logw = nullptr;
    uint8_t *alive = nullptr;
    uint64_t *path_hash = nullptr;
    int32_t *path = nullptr;
    int32_t *counters = nullptr;
};

int grow_tmp(perm_est *h, int64_t total) {
    if (h->tmp_cap >= total) return PE_OK;
    dfree(h->tmp_logw); dfree(h->tmp_alive); dfree(h->tmp_counters);
    h->tmp_cap = 0;
    int rc;
    if ((rc = dalloc(&h->tmp_logw, total)) || (rc = dalloc(&h->tmp_alive, total)) ||
        (rc = dalloc(&h->tmp_counters, 4 * total)))
        return rc;
    h->tmp_cap = total;
    return PE_OK;
}

int grow_mats(perm_est *h, size_t count) {
    if (h->cap_mats >= count) return PE_OK;
    dfree(h->args_dev); dfree(h->order_dev); dfree(h->item_off_dev); dfree(h->seg_dev); dfree(h->stats);
    h->cap_mats = 0;
    int rc;
    if ((rc = dalloc(&h->args_dev, count)) || (rc = dalloc(&h->order_dev, count)) ||
        (rc = dalloc(&h->item_off_dev, count + 1)) || (rc = dalloc(&h->seg_dev, count)) ||
        (rc = dalloc(&h->stats, count)))
        return rc;
    h->cap_mats = count;
    return PE_OK;
}

// Device buffers one launch writes besides its outputs: the handle's own
// (grown on demand) or, for the no-alloc entry point, regions of the
// library's static scratch array (fixed capacities, nothing is allocated).
struct LaunchBufs {
    uint32_t *work = nullptr;                   // [2] item counter, error bits
    unsigned long long *work_totals = nullptr;  // [kWorkTotals]
    TrajArgs *args = nullptr;                   // [count]
    BatchArgs *batch = nullptr;                 // [1]
    int32_t *order = nullptr;                   // [count]
    int64_t *item_off = nullptr;                // [count + 1]
    ReduceSeg *seg = nullptr;                   // [count]
    DevStats *stats = nullptr;                  // [count]
    double *tmp_logw = nullptr;                 // outputs the caller did not ask for
    uint8_t *tmp_alive = nullptr;
    int32_t *tmp_counters = nullptr;
    char *hbm_state = nullptr;                  // per-wave HBM slots
    size_t hbm_bytes = 0;                       // their capacity in bytes
};

// one persistent launch over every matrix's trajectories + per-matrix
// reductions.  res == nullptr: only time the launch shape (wpb, per_cu);
// outputs go to scratch buffers.  rec: training-pair recording, or nullptr.
int launch(perm_est *h, const perm_est_schedule *sched, uint64_t seed, std::vector<RunPart> &parts,
           perm_est_result *res, hipStream_t s, int wpb_req, int per_cu_req, double *elapsed_ms,
           const perm_est_record_buffers *rec = nullptr, bool graph = false, const LaunchBufs *fixed = nullptr) {
    const size_t count = h->mats.size();
    int rc;
    if (!fixed && (rc = grow_mats(h, count))) return rc;
    LaunchBufs lb;
    if (fixed) {
        lb = *fixed;
    } else {
        lb.work = h->work; lb.work_totals = h->work_totals; lb.args = h->args_dev; lb.batch = h->batch_dev;
        lb.order = h->order_dev; lb.item_off = h->item_off_dev; lb.seg = h->seg_dev; lb.stats = h->stats;
    }
    const bool learned = sched->sk_policy == PE_SK_LEARNED;
    if (learned && !h->has_model) return fail(PE_EINVAL, "PE_SK_LEARNED needs perm_est_set_model first");
    // the gated fallback keeps its own scaling values and repairs them locally
    const bool gated = learned && sched->local_gate;
    const int sk_kind = gated ? kSkLearnedGated : sched->sk_policy;
    const bool own_rc = (sched->sk_policy != PE_SK_NONE && !learned) || gated;
    const bool local = sched->sk_policy == PE_SK_LOCAL || gated;
    const bool dm = sched->dm_policy != PE_DM_NONE;
    const bool wt = h->mats[0].weighted;
    for (auto &M : h->mats)
        if (M.weighted != wt) return fail(PE_EINVAL, "a batch must be all 0/1 or all weighted");

    // ---- per-matrix preprocessing and state layout (slots sized for the largest)
    std::vector<Prepared *> prep(count);
    int64_t total = 0;
    uint64_t state_bytes = 0;
    int32_t tree_total = 0;
    std::vector<uint64_t> mat_bytes(count, 0);
    for (size_t b = 0; b < count; ++b) {
        if ((rc = fixed ? find_prepared(&h->mats[b], sched->initial_dm, sched->K0, &prep[b])
                        : get_prepared(&h->mats[b], sched->initial_dm, sched->K0, s, &prep[b])))
            return rc;
        total += parts[b].count;
        tree_total = std::max(tree_total, prep[b]->tree.total);
    }
    if (total > ((int64_t)1 << 32) - 1) return fail(PE_EINVAL, "too many trajectories in one launch");
    bool need_tmp = false;
    for (auto &pt : parts) need_tmp = need_tmp || !pt.logw || !pt.alive || !pt.counters;
    if (need_tmp && !fixed) {
        if ((rc = grow_tmp(h, total))) return rc;
        lb.tmp_logw = h->tmp_logw; lb.tmp_alive = h->tmp_alive; lb.tmp_counters = h->tmp_counters;
    }

    h->args_host.assign(count, TrajArgs{});
    int64_t tmp_off = 0;
    for (size_t b = 0; b < count; ++b) {
        const MatData &M = h->mats[b];
        const Prepared *P = prep[b];
        const int32_t n = M.n;
        StateLayout L{};
        uint64_t o = 0;
        auto take = [&](uint64_t bytes) {
            const uint64_t at = (o + 15) / 16 * 16;
            o = at + bytes;
            return (uint32_t)at;
        };
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
        L.bytes = (uint32_t)((o + 255) / 256 * 256);
        if (o >= (1ull << 32)) return fail(PE_ENOTSUP, "per-trajectory state exceeds 4 GiB");
        state_bytes = std::max<uint64_t>(state_bytes, L.bytes);
        mat_bytes[b] = L.bytes;

        TrajArgs &a = h->args_host[b];
        a.A = DevMat{n, (int32_t)P->m, P->row_ptr, P->col_idx, P->col_ptr, P->row_idx, P->csc2csr,
                     P->edge_row, P->val, P->val_csc};
        a.r0 = P->r0;
        a.c0 = P->c0;
        a.deg0 = P->deg0;
        a.tree0 = P->tree0;
        a.tree0a = P->tree0a;
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
        a.local_cap = sched->local_cap;
        a.scaled = gated || (!learned && ((P->r0 != nullptr) || own_rc));
        a.theta_th = sched->theta_th;
        a.theta_tr = sched->theta_tr;
        a.seed = seed;
        a.b = (uint32_t)b;
        a.first = parts[b].first;
        a.count = parts[b].count;
        a.logw = parts[b].logw ? parts[b].logw : lb.tmp_logw + tmp_off;
        a.alive = parts[b].alive ? parts[b].alive : lb.tmp_alive + tmp_off;
        a.counters = parts[b].counters ? parts[b].counters : lb.tmp_counters + 4 * tmp_off;
        a.path_hash = parts[b].path_hash;
        a.path = parts[b].path;
        a.err = lb.work + 1;
        a.mlp = learned ? h->mlp : nullptr;
        a.etab = learned ? h->etab : nullptr;
        a.mix_alpha = h->mix_alpha;
        if (rec) {
            a.rec_x = rec->x;
            a.rec_y = rec->y;
            a.rec_gstart = rec->gstart;
            a.rec_ginfo = rec->ginfo;
            a.rec_counter = h->rec_ctr;
            a.rec_written = h->rec_ctr + 1;
            a.rec_cap = rec->rec_cap;
            a.rec_gcap = rec->group_cap;
            a.rec_stride = rec->stride;
        }
        tmp_off += parts[b].count;
    }
    // processing order: most expensive matrices first (n * m per trajectory)
    h->order_host.resize(count);
    for (size_t b = 0; b < count; ++b) h->order_host[b] = (int32_t)b;
    std::stable_sort(h->order_host.begin(), h->order_host.end(), [&](int32_t x, int32_t y) {
        return (double)prep[x]->m * h->mats[x].n > (double)prep[y]->m * h->mats[y].n;
    });
    h->item_off_host.assign(count + 1, 0);
    for (size_t i = 0; i < count; ++i) h->item_off_host[i + 1] = h->item_off_host[i] + parts[h->order_host[i]].count;
    // each matrix reduces its own slice: segment (0, count_b) per matrix
    h->seg_host.resize(count);
    for (size_t b = 0; b < count; ++b) {
        const TrajArgs &a = h->args_host[b];
        h->seg_host[b] = ReduceSeg{a.logw, a.alive, a.counters, a.count};
    }

    // ---- tier and launch shape
    size_t tree_bytes = ((size_t)tree_total * 4 + 15) / 16 * 16;
    const size_t kLdsBlock = h->lds_block, kLdsCU = h->lds_cu;
    // per-matrix tier: a matrix whose state fits beside the tree in 32 KB runs
    // in LDS, unless such matrices carry under half of the launch's work (then
    // reserving their LDS would only cost the others occupancy)
    double work_lds = 0.0, work_all = 0.0;
    uint64_t lds_cap = 0, hbm_cap = 0;
    std::vector<int32_t> tier(count, 0);
    for (size_t b = 0; b < count; ++b) {
        const double wgt = (double)prep[b]->m * h->mats[b].n * (double)parts[b].count;
        work_all += wgt;
        if (tree_bytes + mat_bytes[b] <= 32 * 1024 && !(h->opt_flags & PE_FLAG_FORCE_HBM)) {
            tier[b] = 1;
            work_lds += wgt;
        }
    }
    if (work_lds < 0.5 * work_all) std::fill(tier.begin(), tier.end(), 0);
    for (size_t b = 0; b < count; ++b) {
        if (tier[b]) lds_cap = std::max<uint64_t>(lds_cap, mat_bytes[b]);
        else hbm_cap = std::max<uint64_t>(hbm_cap, mat_bytes[b]);
        h->args_host[b].lds_tier = tier[b];
    }
    static_assert(kMlpBlockBytes % 16 == 0 && kMlpWaveBytes % 16 == 0, "LDS carve-outs keep 16-byte alignment");
    BatchArgs &B = h->batch_host;
    B = BatchArgs{};
    B.mats = lb.args;
    B.order = lb.order;
    B.item_off = lb.item_off;
    B.count = (int32_t)count;
    B.total = total;
    B.work_next = lb.work;
    B.work_totals = lb.work_totals;
    B.lds_tree_bytes = (int32_t)tree_bytes;
    B.lds_mlp_bytes = learned ? kMlpWaveBytes : 0;
    B.mlp = learned ? h->mlp : nullptr;
    B.etab = learned ? h->etab : nullptr;
    // four trajectories per wave (16-lane rows) for a single large matrix
    // under the plain or the learned proposal: short candidate lists leave
    // most of a wave idle, so rows give 4x the parallelism per wave
    const size_t block_fixed = learned ? (size_t)kMlpBlockBytes : 0;
    // (a wave of rows holds four trees; when even one such wave does not fit
    // a block's LDS, the matrix runs one trajectory per wave instead)
    const bool rows_ok = count == 1 && !rec && !dm && sched->vertex_rule == PE_VR_MD && hbm_cap > 0 &&
                         !parts[0].path && !(h->opt_flags & PE_FLAG_WAVE_PER_TRAJECTORY);
    // Rows only while four of their waves (sixteen trajectories) fit a CU's
    // LDS: a wave of rows holds four trees, so at large n the rows would
    // run fewer trajectories per CU than whole waves, whose lowest tree
    // level then moves to the state slot (below).
    const size_t lds4 = std::min(kLdsBlock, kLdsCU);
    // the tree's lowest level, moved to a trajectory's state slot: LDS then
    // holds only the levels above it (offsets from 0)
    auto relocate_l0 = [&](size_t b) -> int {
        TrajArgs &a = h->args_host[b];
        const TreeLayout &full = prep[b]->tree;
        const uint64_t at = (mat_bytes[b] + 255) / 256 * 256;
        const uint64_t end = (at + 4ull * full.size[0] + 255) / 256 * 256;
        if (end >= (1ull << 32)) return fail(PE_ENOTSUP, "per-trajectory state exceeds 4 GiB");
        a.st.lvl0 = (uint32_t)at;
        a.st.bytes = (uint32_t)end;
        mat_bytes[b] = end;
        hbm_cap = std::max<uint64_t>(hbm_cap, end);
        a.l0_state = 1;
        a.tree_l1_src = full.off[1];
        TreeLayout up = full;
        int32_t o = 0;
        up.off[0] = 0;
        for (int k = 1; k < full.levels; ++k) { up.off[k] = o; o += full.size[k]; }
        up.total = (o + 3) / 4 * 4;
        a.tree = up;
        return PE_OK;
    };
    // learned rows: when four whole trees per wave would let fewer blocks
    // share a CU's LDS than the kernel's registers allow, the lowest tree
    // level goes to the row's state slot (one more dependent load per
    // selection, more waves in flight)
    const bool learned_rows_cand = rows_ok && learned && !gated;
    bool l0_rows = false;
    size_t row_tree_bytes = tree_bytes;
    int reg_blocks = 0;  // resident 4-wave blocks per CU as registers allow
    if (learned_rows_cand &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(&reg_blocks, rows_learned_kernel_fn(wt, false), 4 * kWave,
                                                      0) != hipSuccess ||
         reg_blocks < 1)) {
        (void)hipGetLastError();
        reg_blocks = 3;
    }
    if (learned_rows_cand && prep[0]->tree.levels >= 2 &&
        kLdsCU / (block_fixed + 4 * (4 * tree_bytes + (size_t)kRowNetScratchBytes)) < (size_t)reg_blocks) {
        const TreeLayout &full = prep[0]->tree;
        int32_t up = 0;
        for (int k = 1; k < full.levels; ++k) up += full.size[k];
        row_tree_bytes = ((size_t)((up + 3) / 4 * 4) * 4 + 15) / 16 * 16;
        l0_rows = true;
    }
    const bool rows_learned = learned_rows_cand &&
                              block_fixed + 4 * (4 * row_tree_bytes + (size_t)kRowNetScratchBytes) <= lds4;
    if (rows_learned && l0_rows) {
        if ((rc = relocate_l0(0))) return rc;
        tree_bytes = row_tree_bytes;
        B.lds_tree_bytes = (int32_t)tree_bytes;
    }
    const bool rows = rows_learned || (rows_ok && sched->sk_policy == PE_SK_NONE &&
                                       block_fixed + 4 * (4 * tree_bytes + (size_t)lds_cap) <= lds4);
    const bool l0g = rows_learned && l0_rows;  // learned rows with level 0 in the state slot
    const void *rows_fn = rows_learned ? rows_learned_kernel_fn(wt, l0g) : rows_kernel_fn(wt);
    const int tpw = rows ? 4 : 1;  // trajectories per wave
    // One trajectory per wave: a large matrix keeps the lowest internal level
    // of its min-tree (one node per 256 leaves, the bulk of the tree) in its
    // state slot and only the levels above in LDS, so the LDS a wave reserves
    // no longer grows with n and large orders keep their occupancy.
    if (!rows) {
        int32_t lds_total = 0;
        for (size_t b = 0; b < count; ++b) {
            TrajArgs &a = h->args_host[b];
            const TreeLayout &full = prep[b]->tree;
            if (!a.lds_tier && full.levels >= 2 && (size_t)full.size[0] * 4 > kTreeLevel0LdsMax)
                if ((rc = relocate_l0(b))) return rc;
            lds_total = std::max(lds_total, a.tree.total);
        }
        tree_bytes = ((size_t)lds_total * 4 + 15) / 16 * 16;
        B.lds_tree_bytes = (int32_t)tree_bytes;
    }
    size_t per_wave = rows_learned ? 4 * tree_bytes + (size_t)kRowNetScratchBytes
                                   : (size_t)tpw * tree_bytes + (size_t)B.lds_mlp_bytes + (size_t)lds_cap;
    int wpb = wpb_req > 0 ? wpb_req : 4;
    if (rows && wpb_req <= 0) {
        // the row kernels' LDS (four trees per wave) limits residency: take the
        // block size that keeps the most of this launch's waves resident and
        // spreads them over the most CUs (ties: the larger block)
        const int64_t need = (total + tpw - 1) / tpw;
        int64_t best_run = -1, best_cus = -1;
        for (int w : {8, 4, 2, 1}) {
            if (!rows_learned && w > 4) continue;
            const size_t sm = block_fixed + (size_t)w * per_wave;
            if (sm > kLdsBlock) continue;
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, rows_fn, w * kWave, sm) != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            nb = std::min<int>(nb, (int)(kLdsCU / sm));
            if (nb < 1) continue;
            const int resident = std::min(nb * w, PE_MAX_WAVES_PER_CU);
            const int64_t cap = (int64_t)resident * h->cu_count;
            const int64_t run = std::min(need, cap);
            const int64_t blocks_w = std::min<int64_t>((run + w - 1) / w, (int64_t)h->cu_count * nb);
            const int64_t cus = std::min<int64_t>(blocks_w, h->cu_count);
            if (run > best_run || (run == best_run && cus > best_cus)) {
                best_run = run;
                best_cus = cus;
                wpb = w;
            }
        }
    }
    wpb = (int)std::max<size_t>(1, std::min<size_t>(wpb, (kLdsBlock - block_fixed) / std::max<size_t>(per_wave, 1)));
    const size_t shmem = block_fixed + (size_t)wpb * per_wave;
    if (shmem > kLdsBlock) return fail(PE_ENOTSUP, "per-trajectory LDS need exceeds one block's LDS");
    size_t per_cu;
    if (per_cu_req > 0) {
        per_cu = (size_t)per_cu_req;
    } else {
        // as many resident blocks as registers and LDS allow, up to the cap
        int nb = 0;
        const void *kfn = rows ? rows_fn : traj_kernel_fn(sk_kind, dm, wt);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kfn, wpb * kWave, shmem) != hipSuccess || nb < 1) {
            (void)hipGetLastError();
            nb = std::max(1, 16 / wpb);
        }
        per_cu = (size_t)std::max(1, std::min(nb, PE_MAX_WAVES_PER_CU / wpb));
    }
    per_cu = std::max<size_t>(1, std::min<size_t>(per_cu, kLdsCU / std::max<size_t>(shmem, 1)));
    unsigned blocks = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((total + (int64_t)wpb * tpw - 1) / ((int64_t)wpb * tpw), (int64_t)h->cu_count * (int64_t)per_cu));
    B.waves_per_block = wpb;
    B.lds_state_bytes = (int32_t)lds_cap;
    B.hbm_state = nullptr;
    if (hbm_cap > 0) {
        const size_t per_block = (size_t)wpb * tpw * hbm_cap;
        if (fixed) {
            // as many resident blocks as the fixed slot region holds
            const size_t fit = lb.hbm_bytes / per_block;
            if (fit < 1)
                return fail(PE_ENOTSUP, "per-trajectory state of one block (" + std::to_string(per_block) +
                                            " B) exceeds the scratch left for it (" + std::to_string(lb.hbm_bytes) +
                                            " B)");
            blocks = (unsigned)std::min<size_t>(blocks, fit);
        } else {
            const size_t need = (size_t)blocks * per_block;
            if (h->hbm_bytes < need) {
                dfree(h->hbm_state);
                h->hbm_bytes = 0;
                if ((rc = dalloc(&h->hbm_state, need))) return rc;
                h->hbm_bytes = need;
            }
            lb.hbm_state = h->hbm_state;
        }
        B.hbm_state = lb.hbm_state;
        B.hbm_stride = hbm_cap;
    }

    PE_HIP(hipMemcpyAsync(lb.args, h->args_host.data(), sizeof(TrajArgs) * count, hipMemcpyHostToDevice, s));
    PE_HIP(hipMemcpyAsync(lb.order, h->order_host.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, s));
    PE_HIP(hipMemcpyAsync(lb.item_off, h->item_off_host.data(), sizeof(int64_t) * (count + 1),
                          hipMemcpyHostToDevice, s));
    PE_HIP(hipMemcpyAsync(lb.seg, h->seg_host.data(), sizeof(ReduceSeg) * count, hipMemcpyHostToDevice, s));
    // the learned row kernel reduces its statistics in its last block: at
    // its register use no other wave fits beside three of its own on a SIMD,
    // so a separate reduction would wait for one of them to end
    const bool fused_stats = rows_learned && res != nullptr;
    B.seg = fused_stats ? lb.seg : nullptr;
    B.stats = fused_stats ? lb.stats : nullptr;
    B.blocks_done = lb.work + 2;
    PE_HIP(hipMemcpyAsync(lb.batch, &B, sizeof(BatchArgs), hipMemcpyHostToDevice, s));
    // the launch sequence; counters are cleared by kernels (no memset nodes):
    // work[0] item counter, [1] error bits, [2] finished blocks
    auto enqueue = [&](hipStream_t q, bool kernel_events) -> int {
        k_fill_i32<<<1, 64, 0, q>>>(3, reinterpret_cast<int32_t *>(lb.work), 0);
        k_fill_i32<<<1, 64, 0, q>>>(2 * kWorkTotals, reinterpret_cast<int32_t *>(lb.work_totals), 0);
        if (rec) k_fill_i32<<<1, 64, 0, q>>>(4, reinterpret_cast<int32_t *>(h->rec_ctr), 0);
        if (kernel_events) PE_HIP(hipEventRecord(h->evk0, q));
        if (rows_learned) launch_rows_learned(wt, l0g, blocks, wpb * kWave, shmem, q, lb.batch);
        else if (rows) launch_rows(wt, blocks, wpb * kWave, shmem, q, lb.batch);
        else launch_traj(sk_kind, dm, wt, blocks, wpb * kWave, shmem, q, lb.batch);
        PE_HIP(hipGetLastError());
        if (kernel_events) PE_HIP(hipEventRecord(h->evk1, q));
        // per-matrix statistics over each matrix's slice of the outputs
        if (res && !fused_stats) k_reduce_stats<<<(unsigned)count, kWave, 0, q>>>(lb.seg, lb.stats);
        PE_HIP(hipGetLastError());
        return PE_OK;
    };
    if (graph && !rec && !fixed) {
        const void *fn = rows ? rows_fn : traj_kernel_fn(sk_kind, dm, wt);
        const bool same = h->graph_exec && h->graph_fn == fn && h->graph_blocks == blocks &&
                          h->graph_threads == (unsigned)(wpb * kWave) && h->graph_shmem == shmem &&
                          h->graph_res == (res != nullptr);
        if (!same) {
            if (h->graph_exec) { (void)hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
            if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
            if (!h->cap_stream) PE_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
            PE_HIP(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            const int erc = enqueue(h->cap_stream, false);
            hipGraph_t g = nullptr;
            const hipError_t ce = hipStreamEndCapture(h->cap_stream, &g);
            if (erc) { if (g) (void)hipGraphDestroy(g); return erc; }
            if (ce != hipSuccess) return fail(PE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
            h->graph = g;
            PE_HIP(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
            h->graph_fn = fn;
            h->graph_blocks = blocks;
            h->graph_threads = (unsigned)(wpb * kWave);
            h->graph_shmem = shmem;
            h->graph_res = res != nullptr;
        }
        PE_HIP(hipEventRecord(h->ev0, s));
        PE_HIP(hipGraphLaunch(h->graph_exec, s));
    } else {
        PE_HIP(hipEventRecord(h->ev0, s));
        if ((rc = enqueue(s, true))) return rc;
    }
    PE_HIP(hipEventRecord(h->ev1, s));
    std::vector<DevStats> st(count);
    uint32_t err_bits = 0;
    unsigned long long wt_tot[kWorkTotals];
    if (res) PE_HIP(hipMemcpyAsync(st.data(), lb.stats, sizeof(DevStats) * count, hipMemcpyDeviceToHost, s));
    PE_HIP(hipMemcpyAsync(wt_tot, lb.work_totals, sizeof(wt_tot), hipMemcpyDeviceToHost, s));
    PE_HIP(hipMemcpyAsync(&err_bits, lb.work + 1, sizeof(err_bits), hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    float ms = 0.0f, kms = 0.0f;
    PE_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    if (graph && !rec && !fixed) kms = ms;  // a replayed graph is timed as a whole
    else PE_HIP(hipEventElapsedTime(&kms, h->evk0, h->evk1));
    if (elapsed_ms) *elapsed_ms = ms;
    if (err_bits)
        return fail(PE_EDEVICE, "trajectory kernel reported an internal inconsistency (bits " +
                                    std::to_string(err_bits) + ")");
    if (res) {
        for (size_t b = 0; b < count; ++b) {
            perm_est_result &r = res[b];
            r.log_estimate = st[b].log_estimate;
            r.p_match = st[b].p_match;
            r.rel_spread = st[b].rel_spread;
            r.rse = st[b].rse;
            r.ess = st[b].ess;
            r.var_logw = st[b].var_logw;
            r.max_logw = st[b].max_logw;
            r.n_traj = st[b].n_traj;
            r.n_alive = st[b].n_alive;
            r.n_dm = st[b].n_dm;
            r.n_full_sk = st[b].n_full_sk;
            r.n_local_sk = st[b].n_local_sk;
            r.n_steps = st[b].n_steps;
            r.seconds = ms * 1e-3;  // the whole launch
            // work units are per launch; reported on every matrix of the batch
            r.n_entries_scanned = (int64_t)wt_tot[0];
            r.n_decrements = (int64_t)wt_tot[1];
            r.n_local_entries = (int64_t)wt_tot[2];
            r.n_local_values = (int64_t)wt_tot[3];
            r.n_mlp_tiles = (int64_t)wt_tot[5];
            r.n_entries_scanned_v = (int64_t)wt_tot[6];
            const double tick = h->wall_hz > 0 ? 1.0 / h->wall_hz : 0.0;
            r.wave_seconds = (double)wt_tot[7] * tick;
            r.wave_seconds_full_sk = (double)wt_tot[8] * tick;
            r.wave_seconds_dm = (double)wt_tot[9] * tick;
            r.wave_seconds_local = (double)wt_tot[10] * tick;
            r.n_dm_entries = (int64_t)wt_tot[11];
            r.launch_blocks = (int32_t)blocks;
            r.launch_waves_per_block = wpb;
            r.launch_trajectories_per_wave = tpw;
            r.launch_blocks_per_cu = (int32_t)per_cu;
            r.kernel_seconds = kms * 1e-3;
        }
    }
    return PE_OK;
}

// Launch-shape autotuner: run candidate (waves per block, blocks per CU)
// pairs on a probe range of trajectories (results are identical for every
// shape) and keep the best per (schedule kind, tier).  A probe's elapsed
// time is set by its longest trajectories (large matrices run 1e6 steps),
// which favours low occupancy; so where the kernel reports its waves' device
// time, a shape is scored by its steady-state rate instead: the waves it
// keeps resident (up to the probe's size) over the mean wave time per step.
int tuned_shape(perm_est *h, const perm_est_schedule *sched, uint64_t seed, const std::vector<RunPart> &parts,
                hipStream_t s, int *wpb, int *per_cu) {
    const int force = (h->opt_flags & PE_FLAG_FORCE_HBM) ? 1 : 0;
    const int sk_kind = (sched->sk_policy == PE_SK_LEARNED && sched->local_gate) ? kSkLearnedGated : sched->sk_policy;
    for (auto &t : h->tunes)
        if (t.sk == sk_kind && t.dm == (sched->dm_policy != 0) && t.force_hbm == force) {
            *wpb = t.wpb; *per_cu = t.per_cu;
            return PE_OK;
        }
    // probe: a slice of every matrix (at least a few waves' worth per CU)
    std::vector<RunPart> probe(parts.size());
    int64_t total = 0;
    for (auto &p : parts) total += p.count;
    const int64_t want = std::min<int64_t>(total, (int64_t)h->cu_count * 16);
    for (size_t b = 0; b < parts.size(); ++b) {
        probe[b].first = parts[b].first;
        probe[b].count = std::max<int64_t>(1, parts[b].count * want / std::max<int64_t>(total, 1));
    }
    const int cand_wpb[] = {1, 2, 4};
    const int cand_cu[] = {4, 8, 16};
    double best = 1e300;
    Tune tb;
    tb.sk = sk_kind; tb.dm = sched->dm_policy != 0; tb.force_hbm = force;
    int64_t probe_items = 0;
    for (auto &p : probe) probe_items += p.count;
    std::vector<perm_est_result> rr(parts.size());
    for (int w : cand_wpb)
        for (int c : cand_cu) {
            const int per_cu_blocks = std::max(1, c / w);
            double ms = 0;
            int rc = launch(h, sched, seed, probe, rr.data(), s, w, per_cu_blocks, &ms);
            if (rc) return rc;
            int64_t steps = 0;
            for (auto &r : rr) steps += r.n_steps;
            const perm_est_result &r0 = rr[0];
            double score = ms;
            if (r0.wave_seconds > 0.0 && steps > 0) {
                const int64_t tpw = std::max(1, r0.launch_trajectories_per_wave);
                const int64_t capacity = (int64_t)h->cu_count * r0.launch_blocks_per_cu * r0.launch_waves_per_block;
                const int64_t resident = std::max<int64_t>(1, std::min(capacity, (probe_items + tpw - 1) / tpw));
                score = r0.wave_seconds / (double)steps / (double)resident;
            }
            if (score < best) { best = score; tb.wpb = w; tb.per_cu = per_cu_blocks; }
        }
    h->tunes.push_back(tb);
    *wpb = tb.wpb;
    *per_cu = tb.per_cu;
    return PE_OK;
}

// true when p is device (or managed) memory of the current device
bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    const hipError_t e = hipPointerGetAttributes(&at, p);
    (void)hipGetLastError();  // a host pointer leaves an error behind: clear it
    if (e != hipSuccess) return false;
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace

// trainer of the proposal network (declared opaque in the header)
struct perm_est_mlp {
    int device = 0;
    float *P = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    float *logits = nullptr, *dl = nullptr, *parts = nullptr;
    int64_t ws_cap = 0;
    double *loss = nullptr;
    int64_t step = 0;
};

namespace {

constexpr int kMlpMaxWaves = 1024;  // backward: one parameter-sized partial per wave

int mlp_grow(perm_est_mlp *t, int64_t n) {
    if (t->ws_cap >= n) return PE_OK;
    dfree(t->logits); dfree(t->dl);
    t->ws_cap = 0;
    int rc;
    const int64_t cap = std::max<int64_t>(n, 4096);
    if ((rc = dalloc(&t->logits, cap)) || (rc = dalloc(&t->dl, cap))) return rc;
    t->ws_cap = cap;
    return PE_OK;
}

__global__ void k_sum_parts(const float *parts, int nparts, float *grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParam) return;
    float acc = 0.0f;
    for (int w = 0; w < nparts; ++w) acc += parts[(size_t)w * kNParam + i];
    grad[i] = acc;
}

// loss (added to *loss_dev) and gradient (into grad) of groups [g0, g1)
// whose records are [r0, r0 + n)
int mlp_window(perm_est_mlp *t, const float *x, const float *y, const int64_t *gstart, const int32_t *ginfo,
               int64_t g0, int64_t g1, int64_t r0, int64_t n, float *grad, hipStream_t s) {
    int rc;
    if ((rc = mlp_grow(t, n))) return rc;
    const float *xw = x + r0 * kIn;
    const int64_t tiles = (n + 15) / 16;
    const unsigned fblocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 1024));
    k_mlp_forward<<<fblocks, 256, 0, s>>>(t->P, xw, n, t->logits);
    k_softmax_xent<<<blocks_for(g1 - g0), 256, 0, s>>>(t->logits, y, gstart, ginfo, g0, g1, t->dl, t->loss);
    const int64_t waves = std::max<int64_t>(1, std::min<int64_t>(tiles, kMlpMaxWaves));
    const unsigned bblocks = (unsigned)((waves + 3) / 4);
    k_mlp_backward<<<bblocks, 256, 0, s>>>(t->P, xw, t->dl, n, t->parts);
    k_sum_parts<<<blocks_for(kNParam), 256, 0, s>>>(t->parts, (int)bblocks * 4, grad);
    PE_HIP(hipGetLastError());
    return PE_OK;
}

// copy the group table [g0, g1) to the host and check that the groups are
// non-empty and tile one contiguous range of records
int load_groups(const int64_t *gstart, const int32_t *ginfo, int64_t g0, int64_t g1, hipStream_t s,
                std::vector<int64_t> &gs, std::vector<int32_t> &gi) {
    const int64_t G = g1 - g0;
    gs.resize(G);
    gi.resize(4 * G);
    PE_HIP(hipMemcpyAsync(gs.data(), gstart + g0, sizeof(int64_t) * G, hipMemcpyDeviceToHost, s));
    PE_HIP(hipMemcpyAsync(gi.data(), ginfo + 4 * g0, sizeof(int32_t) * 4 * G, hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    if (gs[0] < 0) return fail(PE_EINVAL, "negative record offset");
    for (int64_t g = 0; g < G; ++g) {
        if (gi[4 * g] < 1) return fail(PE_EINVAL, "empty group");
        if (g > 0 && gs[g] != gs[g - 1] + gi[4 * (g - 1)])
            return fail(PE_EINVAL, "groups are not contiguous records");
    }
    return PE_OK;
}

// out[i] = in[src[i]] for records (8 features and one target each)
__global__ void k_gather_records(const float *x, const float *y, const int64_t *src, int64_t n, float *xo,
                                 float *yo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = src[i];
#pragma unroll
    for (int f = 0; f < kIn; ++f) xo[i * kIn + f] = x[r * kIn + f];
    yo[i] = y[r];
}

// device buffers freed on every return path
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

int mlp_adam(perm_est_mlp *t, double lr, hipStream_t s) {
    t->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, (double)t->step));
    const float c2 = (float)(1.0 - std::pow(b2, (double)t->step));
    k_adam<<<blocks_for(kNParam), 256, 0, s>>>(t->P, t->grad, t->m, t->v, kNParam, (float)lr, (float)b1, (float)b2,
                                               1e-8f, c1, c2);
    PE_HIP(hipGetLastError());
    return PE_OK;
}

// the training loop over windows of a recording in canonical group order
int mlp_train_windows(perm_est_mlp *t, const float *x, const float *y, const int64_t *gstart,
                      const int32_t *ginfo, const std::vector<int64_t> &gs, const std::vector<int32_t> &gi,
                      int64_t n_groups, int32_t epochs, int64_t batch_groups, double lr, uint64_t seed,
                      double *loss_per_epoch, hipStream_t s) {
    int rc;
    const int64_t nwin = (n_groups + batch_groups - 1) / batch_groups;
    std::vector<int64_t> order(nwin);
    for (int64_t w = 0; w < nwin; ++w) order[w] = w;
    uint64_t rs = seed;
    auto next = [&]() {  // SplitMix64 stream for the window shuffle
        uint64_t z = (rs += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int32_t ep = 0; ep < epochs; ++ep) {
        for (int64_t w = nwin - 1; w > 0; --w) std::swap(order[w], order[(int64_t)(next() % (uint64_t)(w + 1))]);
        k_fill_f32n<<<1, 64, 0, s>>>(2, reinterpret_cast<float *>(t->loss), 0.0f);
        for (int64_t w : order) {
            const int64_t g0 = w * batch_groups, g1 = std::min<int64_t>(n_groups, g0 + batch_groups);
            const int64_t r0 = gs[g0], n = gs[g1 - 1] + gi[4 * (g1 - 1)] - r0;
            if ((rc = mlp_window(t, x, y, gstart, ginfo, g0, g1, r0, n, t->grad, s))) return rc;
            if ((rc = mlp_adam(t, lr, s))) return rc;
        }
        double ls = 0.0;
        PE_HIP(hipMemcpyAsync(&ls, t->loss, sizeof(double), hipMemcpyDeviceToHost, s));
        PE_HIP(hipStreamSynchronize(s));
        if (loss_per_epoch) loss_per_epoch[ep] = ls / (double)nwin;
    }
    PE_HIP(hipStreamSynchronize(s));
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
    } else if (nm == "learned") {
        paper(PE_SK_LEARNED, PE_DM_NONE);
    } else if (nm == "learned_threshold") {
        paper(PE_SK_LEARNED, PE_DM_THRS);
    } else if (nm == "learned_gated") {
        paper(PE_SK_LEARNED, PE_DM_NONE);
        s.local_gate = 1;
    } else if (nm == "learned_threshold_gated") {
        paper(PE_SK_LEARNED, PE_DM_THRS);
        s.local_gate = 1;
    } else {
        return fail(PE_EINVAL, "unknown preset '" + nm + "'");
    }
    *out = s;
    return PE_OK;
}

int perm_est_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                    const int32_t *col_ptr, const int32_t *row_idx, const float *values,
                    const perm_est_options *opts, perm_est_t **out) {
    const int32_t nn[1] = {n};
    const int64_t zz[1] = {nnz};
    return perm_est_create_batch(1, nn, zz, &row_ptr, &col_idx, &col_ptr, &row_idx, values ? &values : nullptr,
                                 opts, out);
}

int perm_est_create_batch(int32_t count, const int32_t *n, const int64_t *nnz,
                          const int32_t *const *row_ptr, const int32_t *const *col_idx,
                          const int32_t *const *col_ptr, const int32_t *const *row_idx,
                          const float *const *values, const perm_est_options *opts, perm_est_t **out) {
    if (!out) return fail(PE_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !n || !nnz || !row_ptr || !col_idx || !col_ptr || !row_idx)
        return fail(PE_EINVAL, "count must be >= 1 and the array-of-arrays arguments non-NULL");
    // host-side validation first: no device work for malformed input
    for (int32_t b = 0; b < count; ++b) {
        if (n[b] <= 0) return fail(PE_EINVAL, "n must be positive");
        if (nnz[b] < 0 || nnz[b] >= (int64_t)1 << 31) return fail(PE_EINVAL, "nnz out of range");
        if (nnz[b] > 0 && (!col_idx[b] || !row_idx[b])) return fail(PE_EINVAL, "null index array");
        int rc;
        if ((rc = check_lists(n[b], nnz[b], row_ptr[b], col_idx[b], "CSR"))) return rc;
        if ((rc = check_lists(n[b], nnz[b], col_ptr[b], row_idx[b], "CSC"))) return rc;
        if (values && values[b])
            for (int64_t p = 0; p < nnz[b]; ++p)
                if (!(values[b][p] > 0.0f) || !std::isfinite(values[b][p]))
                    return fail(PE_EINVAL, "values must be finite and > 0");
        if (values && !values[b] && nnz[b] > 0) return fail(PE_EINVAL, "values[b] is NULL in a weighted batch");
    }
    perm_est *h = nullptr;
    int rc = new_handle(opts, &h);
    if (rc) { perm_est_destroy(h); return rc; }
    h->mats.resize(count);
    for (int32_t b = 0; b < count; ++b) {
        rc = make_matrix(h, n[b], nnz[b], row_ptr[b], col_idx[b], col_ptr[b], row_idx[b],
                         values ? values[b] : nullptr, h->mats[b]);
        if (rc) { perm_est_destroy(h); return rc; }
    }
    *out = h;
    return PE_OK;
}

void perm_est_destroy(perm_est_t *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    for (auto &M : h->mats) M.release();
    dfree(h->hbm_state); dfree(h->work); dfree(h->work_totals); dfree(h->flags); dfree(h->batch_dev);
    dfree(h->args_dev); dfree(h->order_dev); dfree(h->item_off_dev); dfree(h->seg_dev); dfree(h->stats);
    dfree(h->tmp_logw); dfree(h->tmp_alive); dfree(h->tmp_counters);
    dfree(h->mlp); dfree(h->etab); dfree(h->rec_ctr);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->evk0) (void)hipEventDestroy(h->evk0);
    if (h->evk1) (void)hipEventDestroy(h->evk1);
    delete h;
}

int perm_est_run_range(perm_est_t *h, int64_t first, int64_t count, uint64_t seed,
                       const perm_est_schedule *sched, perm_est_result *res, double *logw,
                       uint8_t *alive, uint64_t *path_hash, int32_t *path, int32_t *counters,
                       void *stream) {
    if (!h || !res) return fail(PE_EINVAL, "null handle or result");
    if (h->mats.size() != 1) return fail(PE_EINVAL, "handle holds a batch: use perm_est_run_batch");
    if (count < 1 || first < 0 || first + count > ((int64_t)1 << 32))
        return fail(PE_EINVAL, "trajectory range must lie in [0, 2^32) and be non-empty");
    int rc;
    if ((rc = check_schedule(sched))) return rc;
    PE_HIP(hipSetDevice(h->device));
    std::vector<RunPart> parts(1);
    parts[0] = RunPart{first, count, logw, alive, path_hash, path, counters};
    return launch(h, sched, seed, parts, res, (hipStream_t)stream, 0, 0, nullptr);
}

int perm_est_run(perm_est_t *h, int64_t n_traj, uint64_t seed, const perm_est_schedule *sched,
                 perm_est_result *res, double *logw, uint8_t *alive, uint64_t *path_hash,
                 void *stream) {
    return perm_est_run_range(h, 0, n_traj, seed, sched, res, logw, alive, path_hash, nullptr, nullptr,
                              stream);
}

int perm_est_run_range_noalloc(perm_est_t *h, int64_t first, int64_t count, uint64_t seed,
                               const perm_est_schedule *sched, perm_est_result *res, double *logw,
                               uint8_t *alive, uint64_t *path_hash, int32_t *path, int32_t *counters,
                               void *stream) {
    if (!h || !res) return fail(PE_EINVAL, "null handle or result");
    if (h->mats.size() != 1) return fail(PE_EINVAL, "handle holds a batch: no-alloc runs take one matrix");
    if (count < 1 || first < 0 || first + count > ((int64_t)1 << 32))
        return fail(PE_EINVAL, "trajectory range must lie in [0, 2^32) and be non-empty");
    int rc;
    if ((rc = check_schedule(sched))) return rc;
    PE_HIP(hipSetDevice(h->device));
    char *base = nullptr;
    if ((rc = noalloc_scratch(h->device, &base))) return rc;
    // carve the scratch: launch bookkeeping, the outputs the caller left
    // NULL, then per-wave state slots in what remains
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off = (off + bytes + 255) / 256 * 256;
        return p;
    };
    LaunchBufs lb;
    lb.work = reinterpret_cast<uint32_t *>(take(3 * sizeof(uint32_t)));
    lb.work_totals = reinterpret_cast<unsigned long long *>(take(kWorkTotals * sizeof(unsigned long long)));
    lb.args = reinterpret_cast<TrajArgs *>(take(sizeof(TrajArgs)));
    lb.batch = reinterpret_cast<BatchArgs *>(take(sizeof(BatchArgs)));
    lb.order = reinterpret_cast<int32_t *>(take(sizeof(int32_t)));
    lb.item_off = reinterpret_cast<int64_t *>(take(2 * sizeof(int64_t)));
    lb.seg = reinterpret_cast<ReduceSeg *>(take(sizeof(ReduceSeg)));
    lb.stats = reinterpret_cast<DevStats *>(take(sizeof(DevStats)));
    const size_t tmp_need = (logw ? 0 : 8 * (size_t)count + 256) + (alive ? 0 : (size_t)count + 256) +
                            (counters ? 0 : 16 * (size_t)count + 256);
    if (off + tmp_need > kScratchBytes)
        return fail(PE_ENOTSUP, std::to_string(count) + " trajectories need more than the no-alloc scratch of " +
                                    std::to_string(kScratchBytes) + " bytes for the outputs left NULL");
    if (!logw) lb.tmp_logw = reinterpret_cast<double *>(take(8 * (size_t)count));
    if (!alive) lb.tmp_alive = reinterpret_cast<uint8_t *>(take((size_t)count));
    if (!counters) lb.tmp_counters = reinterpret_cast<int32_t *>(take(16 * (size_t)count));
    lb.hbm_state = base + off;
    lb.hbm_bytes = off < kScratchBytes ? kScratchBytes - off : 0;
    std::vector<RunPart> parts(1);
    parts[0] = RunPart{first, count, logw, alive, path_hash, path, counters};
    return launch(h, sched, seed, parts, res, (hipStream_t)stream, 0, 0, nullptr, nullptr, false, &lb);
}

int perm_est_run_batch(perm_est_t *h, const int64_t *n_traj, uint64_t seed, const perm_est_schedule *sched,
                       perm_est_result *res, double *logw, uint8_t *alive, uint64_t *path_hash,
                       int32_t flags, void *stream) {
    if (!h || !res || !n_traj) return fail(PE_EINVAL, "null handle, result or n_traj");
    if (flags & ~(PE_RUN_AUTOTUNE | PE_RUN_GRAPH)) return fail(PE_EINVAL, "unknown run flags");
    int rc;
    if ((rc = check_schedule(sched))) return rc;
    PE_HIP(hipSetDevice(h->device));
    const size_t count = h->mats.size();
    std::vector<RunPart> parts(count);
    int64_t off = 0;
    for (size_t b = 0; b < count; ++b) {
        if (n_traj[b] < 1 || n_traj[b] >= ((int64_t)1 << 32))
            return fail(PE_EINVAL, "every matrix needs 1 <= n_traj < 2^32");
        parts[b].count = n_traj[b];
        parts[b].logw = logw ? logw + off : nullptr;
        parts[b].alive = alive ? alive + off : nullptr;
        parts[b].path_hash = path_hash ? path_hash + off : nullptr;
        off += n_traj[b];
    }
    int wpb = 0, per_cu = 0;
    hipStream_t s = (hipStream_t)stream;
    if (flags & PE_RUN_AUTOTUNE)
        if ((rc = tuned_shape(h, sched, seed, parts, s, &wpb, &per_cu))) return rc;
    return launch(h, sched, seed, parts, res, s, wpb, per_cu, nullptr, nullptr, (flags & PE_RUN_GRAPH) != 0);
}

int perm_est_set_model(perm_est_t *h, const float *params, double mix_alpha, void *stream) {
    if (!h) return fail(PE_EINVAL, "null handle");
    if (!(mix_alpha >= 0.0 && mix_alpha <= 1.0)) return fail(PE_EINVAL, "mix_alpha must lie in [0, 1]");
    PE_HIP(hipSetDevice(h->device));
    if (!is_device_ptr(params)) return fail(PE_EINVAL, "params must be device memory");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (!h->mlp && (rc = dalloc(&h->mlp, kNParam))) return rc;
    if (!h->etab && (rc = dalloc(&h->etab, kEtabN))) return rc;
    if ((rc = zero_flag(h->flags, s))) return rc;
    k_quantize_params<<<blocks_for(kNParam), 256, 0, s>>>(params, h->mlp, kNParam, h->flags);
    k_etab<<<blocks_for(kEtabN), 256, 0, s>>>(h->etab);
    PE_HIP(hipGetLastError());
    int32_t bad = 0;
    if ((rc = read_flag(h->flags, &bad, s))) return rc;
    if (bad) {
        h->has_model = false;
        return fail(PE_EINVAL, "params hold a non-finite value");
    }
    h->mix_alpha = mix_alpha;
    h->has_model = true;
    return PE_OK;
}

// ---- model files: "PEMLP001", u32 parameter count, u32 0, f64 alpha,
// f32 parameters, u64 FNV-1a of everything before it (all little-endian)
namespace {
constexpr char kModelMagic[8] = {'P', 'E', 'M', 'L', 'P', '0', '0', '1'};
constexpr size_t kModelBytes = 8 + 4 + 4 + 8 + 4 * (size_t)kNParam;

uint64_t fnv1a64(const unsigned char *p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}
}  // namespace

int perm_est_consensus(int32_t n_variants, int32_t n_seeds, const perm_est_result *runs, double alpha,
                       perm_est_consensus_result *out, double *log_ybar, double *rel_e) {
    if (!runs || !out) return fail(PE_EINVAL, "consensus: NULL runs or out");
    if (n_variants < 2 || n_seeds < 2) return fail(PE_EINVAL, "consensus: needs at least 2 variants and 2 seeds");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(PE_EINVAL, "consensus: alpha must lie in (0, 1)");
    return pe::consensus::run(n_variants, n_seeds, runs, alpha, out, log_ybar, rel_e);
}

int perm_est_model_save(const char *path, const float *params, double mix_alpha) {
    if (!path || !params) return fail(PE_EINVAL, "null path or params");
    if (!(mix_alpha >= 0.0 && mix_alpha <= 1.0)) return fail(PE_EINVAL, "mix_alpha must lie in [0, 1]");
    for (int i = 0; i < kNParam; ++i)
        if (!std::isfinite(params[i])) return fail(PE_EINVAL, "params hold a non-finite value");
    std::vector<unsigned char> buf(kModelBytes + 8);
    unsigned char *q = buf.data();
    const uint32_t np = (uint32_t)kNParam, zero = 0;
    std::memcpy(q, kModelMagic, 8);
    std::memcpy(q + 8, &np, 4);
    std::memcpy(q + 12, &zero, 4);
    std::memcpy(q + 16, &mix_alpha, 8);
    std::memcpy(q + 24, params, 4 * (size_t)kNParam);
    const uint64_t h = fnv1a64(q, kModelBytes);
    std::memcpy(q + kModelBytes, &h, 8);
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(PE_EIO, std::string("cannot open for writing: ") + path);
    const bool ok = std::fwrite(q, 1, buf.size(), f) == buf.size();
    if (std::fclose(f) != 0 || !ok) return fail(PE_EIO, std::string("write failed: ") + path);
    return PE_OK;
}

int perm_est_model_load(const char *path, float *params, double *mix_alpha) {
    if (!path || !params || !mix_alpha) return fail(PE_EINVAL, "null path, params or mix_alpha");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(PE_EIO, std::string("cannot open for reading: ") + path);
    std::vector<unsigned char> buf(kModelBytes + 9);
    const size_t got = std::fread(buf.data(), 1, buf.size(), f);
    std::fclose(f);
    if (got != kModelBytes + 8) return fail(PE_EINVAL, "model file has the wrong size");
    const unsigned char *q = buf.data();
    uint32_t np = 0, zero = 1;
    uint64_t h = 0;
    double alpha = 0.0;
    std::memcpy(&np, q + 8, 4);
    std::memcpy(&zero, q + 12, 4);
    std::memcpy(&alpha, q + 16, 8);
    std::memcpy(&h, q + kModelBytes, 8);
    if (std::memcmp(q, kModelMagic, 8) != 0 || np != (uint32_t)kNParam || zero != 0)
        return fail(PE_EINVAL, "not a model file of this network");
    if (fnv1a64(q, kModelBytes) != h) return fail(PE_EINVAL, "model file checksum mismatch");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(PE_EINVAL, "model file holds a bad mix_alpha");
    std::vector<float> p(kNParam);
    std::memcpy(p.data(), q + 24, 4 * (size_t)kNParam);
    for (int i = 0; i < kNParam; ++i)
        if (!std::isfinite(p[i])) return fail(PE_EINVAL, "model file holds a non-finite value");
    std::memcpy(params, p.data(), 4 * (size_t)kNParam);
    *mix_alpha = alpha;
    return PE_OK;
}

int perm_est_record(perm_est_t *h, const int64_t *n_traj, uint64_t seed, const perm_est_schedule *sched,
                    const perm_est_record_buffers *buf, perm_est_result *res, int64_t *n_records,
                    int64_t *n_groups, void *stream) {
    if (!h || !res || !n_traj || !buf || !n_records || !n_groups)
        return fail(PE_EINVAL, "null handle, n_traj, buffers, result or count outputs");
    int rc;
    if ((rc = check_schedule(sched))) return rc;
    if (sched->sk_policy == PE_SK_LEARNED) return fail(PE_EINVAL, "recording needs a scaling-based schedule");
    if (buf->rec_cap < 2 || buf->rec_cap >= ((int64_t)1 << 31) || buf->group_cap < 1 ||
        buf->group_cap >= ((int64_t)1 << 31) || buf->stride < 1 || buf->reserved != 0)
        return fail(PE_EINVAL, "bad record capacities or stride");
    if ((reinterpret_cast<uintptr_t>(buf->x) & 15) != 0) return fail(PE_EINVAL, "x must be 16-byte aligned");
    PE_HIP(hipSetDevice(h->device));
    if (!is_device_ptr(buf->x) || !is_device_ptr(buf->y) || !is_device_ptr(buf->gstart) ||
        !is_device_ptr(buf->ginfo))
        return fail(PE_EINVAL, "record buffers must be device memory");
    const size_t count = h->mats.size();
    std::vector<RunPart> parts(count);
    for (size_t b = 0; b < count; ++b) {
        if (n_traj[b] < 1 || n_traj[b] >= ((int64_t)1 << 32))
            return fail(PE_EINVAL, "every matrix needs 1 <= n_traj < 2^32");
        parts[b].count = n_traj[b];
    }
    hipStream_t s = (hipStream_t)stream;
    if ((rc = launch(h, sched, seed, parts, res, s, 0, 0, nullptr, buf))) return rc;
    unsigned long long written = 0;
    PE_HIP(hipMemcpyAsync(&written, h->rec_ctr + 1, sizeof(written), hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    *n_records = (int64_t)(written >> 32);
    *n_groups = (int64_t)(written & 0xFFFFFFFFull);
    return PE_OK;
}

int perm_est_mlp_create(int32_t device, const float *params, perm_est_mlp_t **out) {
    if (!out) return fail(PE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params) return fail(PE_EINVAL, "params is NULL");
    for (int i = 0; i < kNParam; ++i)
        if (!std::isfinite(params[i])) return fail(PE_EINVAL, "params hold a non-finite value");
    perm_est_mlp *t = new (std::nothrow) perm_est_mlp();
    if (!t) return fail(PE_ENOMEM, "host allocation failed");
    t->device = device;
    int rc = PE_OK;
    auto setup = [&]() -> int {
        PE_HIP(hipSetDevice(device));
        int r;
        if ((r = dalloc(&t->P, kNParam)) || (r = dalloc(&t->m, kNParam)) || (r = dalloc(&t->v, kNParam)) ||
            (r = dalloc(&t->grad, kNParam)) || (r = dalloc(&t->loss, 1)) ||
            (r = dalloc(&t->parts, (size_t)kMlpMaxWaves * kNParam)))
            return r;
        PE_HIP(hipMemcpy(t->P, params, sizeof(float) * kNParam, hipMemcpyHostToDevice));
        PE_HIP(hipMemset(t->m, 0, sizeof(float) * kNParam));
        PE_HIP(hipMemset(t->v, 0, sizeof(float) * kNParam));
        return PE_OK;
    };
    if ((rc = setup())) { perm_est_mlp_destroy(t); return rc; }
    *out = t;
    return PE_OK;
}

int perm_est_mlp_get_params(perm_est_mlp_t *t, float *out, void *stream) {
    if (!t || !out) return fail(PE_EINVAL, "null trainer or output");
    PE_HIP(hipSetDevice(t->device));
    hipStream_t s = (hipStream_t)stream;
    PE_HIP(hipMemcpyAsync(out, t->P, sizeof(float) * kNParam, hipMemcpyDefault, s));
    PE_HIP(hipStreamSynchronize(s));
    return PE_OK;
}

int perm_est_mlp_forward(perm_est_mlp_t *t, const float *x, int64_t n, float *logits, void *stream) {
    if (!t || n < 0 || (n > 0 && (!x || !logits))) return fail(PE_EINVAL, "bad trainer, n or pointers");
    if (n == 0) return PE_OK;
    PE_HIP(hipSetDevice(t->device));
    if (!is_device_ptr(x) || !is_device_ptr(logits)) return fail(PE_EINVAL, "x and logits must be device memory");
    hipStream_t s = (hipStream_t)stream;
    const int64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 1024));
    k_mlp_forward<<<blocks, 256, 0, s>>>(t->P, x, n, logits);
    PE_HIP(hipGetLastError());
    PE_HIP(hipStreamSynchronize(s));
    return PE_OK;
}

int perm_est_mlp_loss_grad(perm_est_mlp_t *t, const float *x, const float *y, const int64_t *gstart,
                           const int32_t *ginfo, int64_t g0, int64_t g1, double *loss, float *grad,
                           void *stream) {
    if (!t || !x || !y || !gstart || !ginfo || !loss) return fail(PE_EINVAL, "null argument");
    if (g0 < 0 || g1 <= g0) return fail(PE_EINVAL, "empty or negative group window");
    PE_HIP(hipSetDevice(t->device));
    if (!is_device_ptr(x) || !is_device_ptr(y) || !is_device_ptr(gstart) || !is_device_ptr(ginfo) ||
        (grad && !is_device_ptr(grad)))
        return fail(PE_EINVAL, "recording arrays and grad must be device memory");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> gs;
    std::vector<int32_t> gi;
    int rc;
    if ((rc = load_groups(gstart, ginfo, g0, g1, s, gs, gi))) return rc;
    const int64_t first = gs.front(), n = gs.back() + gi[gi.size() - 4] - first;
    k_fill_f32n<<<1, 64, 0, s>>>(2, reinterpret_cast<float *>(t->loss), 0.0f);
    if ((rc = mlp_window(t, x, y, gstart, ginfo, g0, g1, first, n, grad ? grad : t->grad, s))) return rc;
    PE_HIP(hipMemcpyAsync(loss, t->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    PE_HIP(hipStreamSynchronize(s));
    return PE_OK;
}

int perm_est_mlp_train(perm_est_mlp_t *t, const float *x, const float *y, const int64_t *gstart,
                       const int32_t *ginfo, int64_t n_groups, int32_t epochs, int64_t batch_groups,
                       double lr, uint64_t seed, double *loss_per_epoch, void *stream) {
    if (!t || !x || !y || !gstart || !ginfo) return fail(PE_EINVAL, "null argument");
    if (n_groups < 1 || epochs < 0 || batch_groups < 1 || !(lr > 0.0) || !std::isfinite(lr))
        return fail(PE_EINVAL, "bad n_groups, epochs, batch_groups or lr");
    PE_HIP(hipSetDevice(t->device));
    if (!is_device_ptr(x) || !is_device_ptr(y) || !is_device_ptr(gstart) || !is_device_ptr(ginfo))
        return fail(PE_EINVAL, "recording arrays must be device memory");
    hipStream_t s = (hipStream_t)stream;
    // window bounds from the group table (one copy)
    std::vector<int64_t> gs;
    std::vector<int32_t> gi;
    int rc;
    if ((rc = load_groups(gstart, ginfo, 0, n_groups, s, gs, gi))) return rc;
    // canonical order of the groups: (matrix, trajectory, step)
    {
        std::vector<int64_t> perm((size_t)n_groups);
        for (int64_t g = 0; g < n_groups; ++g) perm[(size_t)g] = g;
        std::sort(perm.begin(), perm.end(), [&](int64_t p, int64_t q) {
            for (int f = 1; f < 4; ++f)
                if (gi[4 * p + f] != gi[4 * q + f]) return gi[4 * p + f] < gi[4 * q + f];
            return p < q;
        });
        const int64_t n_rec = gs.back() + gi[4 * (n_groups - 1)] - gs.front();
        std::vector<int64_t> src;
        src.reserve((size_t)n_rec);
        std::vector<int64_t> gs2((size_t)n_groups);
        std::vector<int32_t> gi2(4 * (size_t)n_groups);
        int64_t pos = 0;
        for (int64_t i = 0; i < n_groups; ++i) {
            const int64_t g = perm[(size_t)i];
            gs2[(size_t)i] = pos;
            for (int f = 0; f < 4; ++f) gi2[4 * (size_t)i + f] = gi[4 * g + f];
            for (int32_t r = 0; r < gi[4 * g]; ++r) src.push_back(gs[g] + r);
            pos += gi[4 * g];
        }
        gs.swap(gs2);
        gi.swap(gi2);
        DevBuf b_src, b_x, b_y, b_gs, b_gi;
        int64_t *d_src;
        float *d_x, *d_y;
        int64_t *d_gs;
        int32_t *d_gi;
        if ((rc = dalloc(&d_src, (size_t)n_rec))) return rc;
        b_src.p = d_src;
        if ((rc = dalloc(&d_x, (size_t)n_rec * kIn))) return rc;
        b_x.p = d_x;
        if ((rc = dalloc(&d_y, (size_t)n_rec))) return rc;
        b_y.p = d_y;
        if ((rc = dalloc(&d_gs, (size_t)n_groups))) return rc;
        b_gs.p = d_gs;
        if ((rc = dalloc(&d_gi, 4 * (size_t)n_groups))) return rc;
        b_gi.p = d_gi;
        PE_HIP(hipMemcpyAsync(d_src, src.data(), sizeof(int64_t) * (size_t)n_rec, hipMemcpyHostToDevice, s));
        PE_HIP(hipMemcpyAsync(d_gs, gs.data(), sizeof(int64_t) * (size_t)n_groups, hipMemcpyHostToDevice, s));
        PE_HIP(hipMemcpyAsync(d_gi, gi.data(), sizeof(int32_t) * 4 * (size_t)n_groups, hipMemcpyHostToDevice, s));
        k_gather_records<<<blocks_for(n_rec), 256, 0, s>>>(x, y, d_src, n_rec, d_x, d_y);
        PE_HIP(hipGetLastError());
        rc = mlp_train_windows(t, d_x, d_y, d_gs, d_gi, gs, gi, n_groups, epochs, batch_groups, lr, seed,
                               loss_per_epoch, s);
        // the copies are freed when this block ends; wait for the last use
        hipError_t e = hipStreamSynchronize(s);
        if (rc == PE_OK && e != hipSuccess) return fail(PE_EDEVICE, hipGetErrorString(e));
        return rc;
    }
}


void perm_est_mlp_destroy(perm_est_mlp_t *t) {
    if (!t) return;
    (void)hipSetDevice(t->device);
    dfree(t->P); dfree(t->m); dfree(t->v); dfree(t->grad); dfree(t->logits); dfree(t->dl); dfree(t->parts);
    dfree(t->loss);
    delete t;
}

}  // extern "C"
