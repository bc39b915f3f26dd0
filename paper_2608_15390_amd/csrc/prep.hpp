// prep.hpp -- kernels of the shared preprocessing of Alg. 2: the initial
// support filter (Sec. 2, "Support filtering with DM"), the outer
// Sinkhorn-Knopp iterations (Sec. 3.1) and the per-trajectory templates.
#pragma once
#include "traj.hpp"

namespace pe {

// csc2csr[p] = CSR position of the CSC entry p; err = 1 if an entry of the
// CSC has no CSR twin
__global__ void k_csc2csr(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          const int32_t *col_ptr, const int32_t *row_idx, int32_t *csc2csr,
                          int32_t *err) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int32_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
        const int32_t i = row_idx[p];
        int32_t lo = row_ptr[i], hi = row_ptr[i + 1];
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col_idx[mid] < j) lo = mid + 1; else hi = mid;
        }
        if (lo < row_ptr[i + 1] && col_idx[lo] == j) csc2csr[p] = lo;
        else { csc2csr[p] = -1; *err = 1; }
    }
}

__global__ void k_edge_row(int32_t n, const int32_t *row_ptr, int32_t *edge_row) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) edge_row[e] = i;
}

__global__ void k_gather_f32(int64_t m, const float *src, const int32_t *idx, float *dst) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < m) {
        const int32_t q = idx[p];
        if (q >= 0) dst[p] = src[q];
    }
}

__global__ void k_fill_i32(int64_t cnt, int32_t *p, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

__global__ void k_fill_f32(int64_t cnt, float *p, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

// ------------------------------------------------------------ matching
// greedy rounds: every unmatched row claims its first unclaimed column
__global__ void k_greedy(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                         int32_t *mate_r, int32_t *mate_c, int32_t *changed) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || mate_r[i] >= 0) return;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int32_t j = col_idx[e];
        if (__hip_atomic_load(&mate_c[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) continue;
        if (atomicCAS(&mate_c[j], -1, i) == -1) {
            mate_r[i] = j;
            *changed = 1;
            return;
        }
    }
}

// start of an augmentation phase: every free row roots its own BFS tree
__global__ void k_aug_init(int32_t n, const int32_t *mate_r, int32_t *root, int32_t *level,
                           int32_t *claim, int32_t *path_end, int32_t *nfree) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool fr = mate_r[i] < 0;
    root[i] = fr ? i : -1;
    level[i] = fr ? 0 : -1;
    path_end[i] = -1;
    claim[i] = -1;
    if (fr) atomicAdd(nfree, 1);
}

// one BFS level of all trees at once: a column is claimed by exactly one
// row (so trees stay vertex disjoint); a free column ends its tree's path
__global__ void k_aug_level(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                            const int32_t *mate_c, int32_t *root, int32_t *level, int32_t *claim,
                            int32_t *path_end, int32_t cur, int32_t *grew) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || level[i] != cur) return;
    const int32_t r = root[i];
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        if (__hip_atomic_load(&path_end[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) return;
        const int32_t j = col_idx[e];
        if (__hip_atomic_load(&claim[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) continue;
        if (atomicCAS(&claim[j], -1, i) != -1) continue;
        const int32_t i2 = mate_c[j];
        if (i2 < 0) {
            atomicCAS(&path_end[r], -1, j);
        } else {
            root[i2] = r;
            level[i2] = cur + 1;
            *grew = 1;
        }
    }
}

// flip every found path (paths of different trees share no vertex)
__global__ void k_aug_flip(int32_t n, const int32_t *claim, const int32_t *path_end,
                           int32_t *mate_r, int32_t *mate_c, int32_t *found) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int32_t j = path_end[r];
    if (j < 0) return;
    atomicAdd(found, 1);
    for (;;) {
        const int32_t i = claim[j];
        const int32_t next = mate_r[i];
        mate_r[i] = j;
        mate_c[j] = i;
        if (i == r) break;
        j = next;
    }
}

__global__ void k_count_matched(int32_t n, const int32_t *mate_r, int32_t *cnt) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && mate_r[i] >= 0) atomicAdd(cnt, 1);
}

// ------------------------------------------------------------------ SCC
// Alternating digraph with every matched pair (row i, column mate_r[i])
// contracted into node i: a non-matching entry (i, j) gives the arc
// mate_c[j] -> i.  Out-arcs of node x: rows of column mate_r[x]'s list
// other than x; in-arcs of node x: mate_c[j] for the columns j of row x's
// list other than mate_r[x].
__global__ void k_scc_trim(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                           const int32_t *col_ptr, const int32_t *row_idx, const int32_t *mate_r,
                           const int32_t *mate_c, int32_t *scc, int32_t *changed) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n || scc[x] >= 0) return;
    bool has_in = false, has_out = false;
    for (int32_t e = row_ptr[x]; e < row_ptr[x + 1] && !has_in; ++e) {
        const int32_t j = col_idx[e];
        if (j == mate_r[x]) continue;
        const int32_t a = mate_c[j];
        if (scc[a] < 0) has_in = true;
    }
    const int32_t jm = mate_r[x];
    for (int32_t p = col_ptr[jm]; p < col_ptr[jm + 1] && !has_out; ++p) {
        const int32_t b = row_idx[p];
        if (b != x && scc[b] < 0) has_out = true;
    }
    if (!has_in || !has_out) { scc[x] = x; *changed = 1; }
}

__global__ void k_scc_color_init(int32_t n, const int32_t *scc, int32_t *color) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) color[x] = scc[x] < 0 ? x : -1;
}

// color[x] <- max color over in-neighbours (monotone, converges to the
// largest node id that reaches x)
__global__ void k_scc_color_prop(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                 const int32_t *mate_r, const int32_t *mate_c, const int32_t *scc,
                                 int32_t *color, int32_t *changed) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n || scc[x] >= 0) return;
    int32_t best = __hip_atomic_load(&color[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t mine = best;
    for (int32_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e) {
        const int32_t j = col_idx[e];
        if (j == mate_r[x]) continue;
        const int32_t a = mate_c[j];
        if (scc[a] >= 0) continue;
        const int32_t ca = __hip_atomic_load(&color[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        best = ca > best ? ca : best;
    }
    if (best > mine) {
        atomicMax(&color[x], best);
        *changed = 1;
    }
}

// roots of this round: nodes that kept their own color
__global__ void k_scc_roots(int32_t n, const int32_t *color, int32_t *scc, int32_t *round_mark) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n || scc[x] >= 0) return;
    round_mark[x] = 0;
    if (color[x] == x) { scc[x] = x; round_mark[x] = 1; }
}

// backward closure inside a color class: x joins its root's component if
// one of its out-neighbours already did in this round
__global__ void k_scc_back(int32_t n, const int32_t *col_ptr, const int32_t *row_idx,
                           const int32_t *mate_r, const int32_t *color, int32_t *scc,
                           int32_t *round_mark, int32_t *changed) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n || __hip_atomic_load(&scc[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= 0) return;
    const int32_t cx = color[x];
    const int32_t jm = mate_r[x];
    for (int32_t p = col_ptr[jm]; p < col_ptr[jm + 1]; ++p) {
        const int32_t b = row_idx[p];
        if (b == x) continue;
        if (__hip_atomic_load(&round_mark[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1 &&
            color[b] == cx) {
            scc[x] = cx;
            __hip_atomic_store(&round_mark[x], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *changed = 1;
            return;
        }
    }
}

__global__ void k_scc_unassigned(int32_t n, const int32_t *scc, int32_t *cnt) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n && scc[x] < 0) atomicAdd(cnt, 1);
}

// keep[e] = 1 iff entry e lies in some perfect matching
__global__ void k_keep_edges(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                             const int32_t *mate_r, const int32_t *mate_c, const int32_t *scc,
                             uint8_t *keep) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int32_t j = col_idx[e];
        keep[e] = (mate_r[i] == j || scc[mate_c[j]] == scc[i]) ? 1 : 0;
    }
}

// ----------------------------------------------------------- compaction
__global__ void k_row_keep_count(int32_t n, const int32_t *row_ptr, const uint8_t *keep, int32_t *len) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = 0;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) c += keep[e];
    len[i] = c;
}

__global__ void k_col_keep_count(int32_t n, const int32_t *col_ptr, const int32_t *csc2csr,
                                 const uint8_t *keep, int32_t *len) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t c = 0;
    for (int32_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) c += keep[csc2csr[p]];
    len[j] = c;
}

// exclusive scan of len[0..n) into out[0..n], one block of 1024 threads
__global__ void __launch_bounds__(1024) k_scan_excl(int32_t n, const int32_t *len, int32_t *out) {
    __shared__ int32_t part[1024];
    const int32_t t = threadIdx.x;
    const int32_t chunk = (n + 1023) / 1024;
    const int32_t lo = min(n, t * chunk), hi = min(n, lo + chunk);
    int32_t s = 0;
    for (int32_t i = lo; i < hi; ++i) s += len[i];
    part[t] = s;
    __syncthreads();
    for (int32_t o = 1; o < 1024; o <<= 1) {
        const int32_t v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;
    for (int32_t i = lo; i < hi; ++i) { out[i] = run; run += len[i]; }
    if (t == 1023) out[n] = part[1023];
}

__global__ void k_row_scatter(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              const float *val, const uint8_t *keep, const int32_t *new_ptr,
                              int32_t *new_col, float *new_val, int32_t *new_id) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t o = new_ptr[i];
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        if (!keep[e]) { new_id[e] = -1; continue; }
        new_col[o] = col_idx[e];
        if (val) new_val[o] = val[e];
        new_id[e] = o;
        ++o;
    }
}

__global__ void k_col_scatter(int32_t n, const int32_t *col_ptr, const int32_t *row_idx,
                              const int32_t *csc2csr, const uint8_t *keep, const int32_t *new_id,
                              const int32_t *new_ptr, int32_t *new_row, int32_t *new_map) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int32_t o = new_ptr[j];
    for (int32_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
        const int32_t e = csc2csr[p];
        if (!keep[e]) continue;
        new_row[o] = row_idx[p];
        new_map[o] = new_id[e];
        ++o;
    }
}

// ------------------------------------------------------------ outer SK
// Sec. 3.3 iteration on the whole (filtered) matrix: columns with the old
// r, then rows with the new c; sequential binary32 sums in list order.
__global__ void k_sk_cols(int32_t n, const int32_t *col_ptr, const int32_t *row_idx,
                          const float *val_csc, const float *r, float *c) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float acc = 0.0f;
    for (int32_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
        const float bv = val_csc ? val_csc[p] : 1.0f;
        const float prod = bv * r[row_idx[p]];
        acc = acc + prod;
    }
    if (acc != 0.0f) c[j] = 1.0f / acc;
}

__global__ void k_sk_rows(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          const float *val, float *r, const float *c) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float acc = 0.0f;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const float bv = val ? val[e] : 1.0f;
        const float prod = bv * c[col_idx[e]];
        acc = acc + prod;
    }
    if (acc != 0.0f) r[i] = 1.0f / acc;
}

// ------------------------------------------------------------ templates
__global__ void k_deg_template(int32_t n, int32_t n_leaf, const int32_t *row_ptr,
                               const int32_t *col_ptr, uint16_t *deg0) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n_leaf) return;
    uint16_t d = kRetired;
    if (x < n) d = (uint16_t)(row_ptr[x + 1] - row_ptr[x]);
    else if (x < 2 * n) d = (uint16_t)(col_ptr[x - n + 1] - col_ptr[x - n]);
    deg0[x] = d;
}

__global__ void k_tree_leaves(int32_t groups, const uint16_t *deg0, uint32_t *lvl) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= groups) return;
    uint32_t m = 0xFFFFFFFFu;
    for (int32_t i = 0; i < 256; ++i) m = min(m, (uint32_t)deg0[256 * g + i]);
    lvl[g] = m;
}

// the same level with each node packed as (minimum << 8 | position of the
// first leaf of that minimum within the group)
__global__ void k_tree_leaves_argmin(int32_t groups, const uint16_t *deg0, uint32_t *lvl) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= groups) return;
    uint32_t m = 0xFFFFFFFFu;
    for (int32_t i = 0; i < 256; ++i) m = min(m, ((uint32_t)deg0[256 * g + i] << 8) | (uint32_t)i);
    lvl[g] = m;
}

__global__ void k_tree_up(int32_t n_in, const uint32_t *in, int32_t n_out, uint32_t *out) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_out) return;
    uint32_t m = 0xFFFFFFFFu;
    for (int32_t i = 64 * g; i < min(n_in, 64 * g + 64); ++i) m = min(m, in[i]);
    out[g] = m;
}

__global__ void k_set_u32(uint32_t *p, uint32_t v) { *p = v; }

}  // namespace pe
