// traj.hpp -- the trajectory kernel: one wave64 runs one trajectory of the
// generic estimator (Alg. 2) at a time and pulls trajectory ids from a
// global counter until the range is exhausted.
//
// Per-trajectory state (one block per wave, in LDS for small n or in an HBM
// scratch slot for large n):
//   deg    u16[n_leaf]  residual degree of every vertex (rows 0..n-1,
//                       columns n..2n-1), 0xFFFF once matched; padded with
//                       0xFFFF to a multiple of 256
//   r, c   f32[n]       scaling vectors when a policy changes them
//   stamp  i32[2n]      set-membership marks of the local repair
//   lst_a  i32[dmax]    N_t(v): the candidates of the selected vertex
//   lst_b  i32[dmax]    N_t(u) \ {v}
//   loc_r, loc_c i32[n] R_loc, C_loc of Eq. (local)
//   new_r, new_c f32[n] staged values of the Jacobi repair
//   rem    u32[m/32]    edges removed by inner DM (CSR edge ids)
// Minimum-degree selection uses a min-tree whose internal nodes are u32 in
// LDS: level-1 node g is the minimum of leaves [256g, 256g+256), higher
// levels have fan-out 64, the top level has at most 64 nodes.  The leftmost
// minimum is followed down, so the selected vertex is the active vertex of
// minimum degree with the smallest id.
#pragma once
#include "device.hpp"

namespace pe {

struct DevMat {
    int32_t n, m;
    const int32_t *row_ptr, *col_idx, *col_ptr, *row_idx, *csc2csr;
    const float *val;      // CSR order, nullptr = 0/1
    const float *val_csc;  // CSC order, nullptr = 0/1
};

struct TreeLayout {
    int32_t levels;   // internal levels, 1..3
    int32_t size[3];  // nodes per level (level 1 first)
    int32_t off[3];   // u32 offset of each level within the tree block
    int32_t total;    // u32 count of the tree block
};

struct StateLayout {  // byte offsets in one trajectory's state block
    uint32_t deg, r, c, stamp, lst_a, lst_b, loc_r, loc_c, new_r, new_c, rem, dm;
    uint32_t bytes;
};

enum : int32_t { kSkNone = 0, kSkFixed = 1, kSkAdaptive = 2, kSkLocal = 3 };
enum : int32_t { kDmNone = 0, kDmAll = 1, kDmThrs = 2, kDmTrck = 3 };

struct TrajArgs {
    DevMat A;
    const float *r0, *c0;      // shared outer scaling, nullptr = all ones
    const uint16_t *deg0;      // leaf template [n_leaf]
    const uint32_t *tree0;     // internal-node template [tree.total]
    int32_t n_leaf;
    TreeLayout tree;
    StateLayout st;
    int32_t ok0;               // 0: the input has no perfect matching
    int32_t vertex_rule, sk_policy, dm_policy, K;
    int32_t scaled;            // proposal uses r/c
    int32_t own_rc;            // per-trajectory r/c copies
    double theta_th, theta_tr;
    uint64_t seed;
    uint32_t b;
    int64_t first, count;
    double *logw;
    uint8_t *alive;
    uint64_t *path_hash;
    int32_t *path;             // [count][2n] or nullptr
    int32_t *counters;         // [count][4] or nullptr
    uint32_t *work_next;       // work counter (zeroed before launch)
    uint32_t *err;             // internal-consistency error bits (zeroed before launch)
    char *hbm_state;           // HBM tier: base of per-wave slots; nullptr = LDS tier
    uint64_t hbm_stride;
    int32_t lds_state_bytes;   // LDS tier: bytes of state per wave
    int32_t waves_per_block;
};

// ------------------------------------------------------------------ views
struct Traj {
    const TrajArgs &a;
    uint16_t *deg;
    uint32_t *tree;
    float *r, *c;
    int32_t *stamp, *lst_a, *lst_b, *loc_r, *loc_c;
    float *new_r, *new_c;
    uint32_t *rem;
    int32_t n;

    __device__ Traj(const TrajArgs &args, char *state, uint32_t *tree_lds)
        : a(args), tree(tree_lds), n(args.A.n) {
        const StateLayout &s = args.st;
        deg = reinterpret_cast<uint16_t *>(state + s.deg);
        r = args.own_rc ? reinterpret_cast<float *>(state + s.r) : nullptr;
        c = args.own_rc ? reinterpret_cast<float *>(state + s.c) : nullptr;
        stamp = reinterpret_cast<int32_t *>(state + s.stamp);
        lst_a = reinterpret_cast<int32_t *>(state + s.lst_a);
        lst_b = reinterpret_cast<int32_t *>(state + s.lst_b);
        loc_r = reinterpret_cast<int32_t *>(state + s.loc_r);
        loc_c = reinterpret_cast<int32_t *>(state + s.loc_c);
        new_r = reinterpret_cast<float *>(state + s.new_r);
        new_c = reinterpret_cast<float *>(state + s.new_c);
        rem = args.dm_policy != kDmNone ? reinterpret_cast<uint32_t *>(state + s.rem) : nullptr;
    }

    __device__ __forceinline__ bool active(int32_t x) const { return deg[x] != kRetired; }
    __device__ __forceinline__ bool removed(int32_t e) const {
        return rem != nullptr && ((rem[e >> 5] >> (e & 31)) & 1u);
    }
    __device__ __forceinline__ float rv(int32_t i) const {
        return r ? r[i] : (a.r0 ? a.r0[i] : 1.0f);
    }
    __device__ __forceinline__ float cv(int32_t j) const {
        return c ? c[j] : (a.c0 ? a.c0[j] : 1.0f);
    }
    // neighbour list of vertex x: [beg, end) in CSR (row) or CSC (column)
    __device__ __forceinline__ void list(int32_t x, int32_t &beg, int32_t &end) const {
        if (x < n) { beg = a.A.row_ptr[x]; end = a.A.row_ptr[x + 1]; }
        else { beg = a.A.col_ptr[x - n]; end = a.A.col_ptr[x - n + 1]; }
    }
    // entry p of vertex x's list: neighbour id, CSR edge id, value
    __device__ __forceinline__ void entry(bool row, int32_t p, int32_t &y, int32_t &e, float &bv) const {
        if (row) {
            y = n + a.A.col_idx[p];
            e = p;
            bv = a.A.val ? a.A.val[p] : 1.0f;
        } else {
            y = a.A.row_idx[p];
            e = rem ? a.A.csc2csr[p] : 0;
            bv = a.A.val_csc ? a.A.val_csc[p] : 1.0f;
        }
    }

    // ------------------------------------------------------ min-tree
    __device__ __forceinline__ uint32_t *level(int k) const { return tree + a.tree.off[k]; }

    // lower a node chain after deg[x] dropped to d
    __device__ __forceinline__ void tree_lower(int32_t x, uint32_t d) const {
        atomicMin(level(0) + (x >> 8), d);
        if (a.tree.levels > 1) atomicMin(level(1) + (x >> 14), d);
        if (a.tree.levels > 2) atomicMin(level(2) + (x >> 20), d);
    }

    // min of the 256 leaves of group g, computed by the whole wave
    __device__ __forceinline__ uint32_t leaf_group_min(int32_t g) const {
        const int l = lane_id();
        const uint2 q = reinterpret_cast<const uint2 *>(deg + 256 * g)[l];
        uint32_t m = min(min(q.x & 0xFFFFu, q.x >> 16), min(q.y & 0xFFFFu, q.y >> 16));
        return wave_min_u32(m);
    }

    // recompute the chain above vertex x (after x was retired)
    __device__ void tree_refresh(int32_t x) const {
        const int l = lane_id();
        int32_t g = x >> 8;
        uint32_t m = leaf_group_min(g);
        if (l == 0) level(0)[g] = m;
        wave_fence();
        for (int k = 1; k < a.tree.levels; ++k) {
            const int32_t h = g >> 6;
            const int32_t idx = 64 * h + l;
            uint32_t v = idx < a.tree.size[k - 1] ? level(k - 1)[idx] : 0xFFFFFFFFu;
            v = wave_min_u32(v);
            if (l == 0) level(k)[h] = v;
            wave_fence();
            g = h;
        }
    }

    // active vertex of minimum degree, smallest id; returns the degree
    __device__ uint32_t select_min(int32_t &vsel) const {
        const int l = lane_id();
        const int top = a.tree.levels - 1;
        uint32_t v = l < a.tree.size[top] ? level(top)[l] : 0xFFFFFFFFu;
        const uint32_t m = wave_min_u32(v);
        uint64_t hit = ballot(v == m);
        int32_t g = __ffsll((unsigned long long)hit) - 1;
        for (int k = top - 1; k >= 0 && hit; --k) {
            const int32_t idx = 64 * g + l;
            uint32_t w = idx < a.tree.size[k] ? level(k)[idx] : 0xFFFFFFFFu;
            hit = ballot(w == m);
            g = 64 * g + __ffsll((unsigned long long)hit) - 1;
        }
        if (!hit) { vsel = -1; return m; }  // inconsistent tree: caller aborts
        const uint2 q = reinterpret_cast<const uint2 *>(deg + 256 * g)[l];
        const uint32_t d0 = q.x & 0xFFFFu, d1 = q.x >> 16, d2 = q.y & 0xFFFFu, d3 = q.y >> 16;
        const int j = d0 == m ? 0 : d1 == m ? 1 : d2 == m ? 2 : d3 == m ? 3 : 4;
        hit = ballot(j < 4);
        if (!hit) { vsel = -1; return m; }
        const int src = __ffsll((unsigned long long)hit) - 1;
        const int jj = read_lane(j, src);
        vsel = 256 * g + 4 * src + jj;
        return m;
    }

    __device__ __forceinline__ uint32_t global_min() const {
        const int top = a.tree.levels - 1;
        const int l = lane_id();
        uint32_t v = l < a.tree.size[top] ? level(top)[l] : 0xFFFFFFFFu;
        return wave_min_u32(v);
    }

    // ------------------------------------------------------------ SK
    // one full iteration over the residual: columns with the old r, then
    // rows with the new c; sequential binary32 sums in list order
    __device__ void sk_sweep() const {
        const int l = lane_id();
        for (int32_t j = l; j < n; j += kWave) {
            if (!active(n + j)) continue;
            float acc = 0.0f;
            for (int32_t p = a.A.col_ptr[j]; p < a.A.col_ptr[j + 1]; ++p) {
                const int32_t i = a.A.row_idx[p];
                if (!active(i)) continue;
                if (rem && removed(a.A.csc2csr[p])) continue;
                const float bv = a.A.val_csc ? a.A.val_csc[p] : 1.0f;
                const float prod = bv * r[i];
                acc = acc + prod;
            }
            if (acc != 0.0f) c[j] = 1.0f / acc;
        }
        wave_fence();
        for (int32_t i = l; i < n; i += kWave) {
            if (!active(i)) continue;
            float acc = 0.0f;
            for (int32_t e = a.A.row_ptr[i]; e < a.A.row_ptr[i + 1]; ++e) {
                const int32_t j = a.A.col_idx[e];
                if (!active(n + j) || removed(e)) continue;
                const float bv = a.A.val ? a.A.val[e] : 1.0f;
                const float prod = bv * c[j];
                acc = acc + prod;
            }
            if (acc != 0.0f) r[i] = 1.0f / acc;
        }
        wave_fence();
    }

    // append the active, non-removed neighbours of vertex x that are not
    // yet stamped with `mark` to out[*cnt...]; x's own list entries are
    // distinct, so one pass of the wave needs no intra-wave deduplication
    __device__ void gather_unmarked(int32_t x, int32_t mark, int32_t *out, int32_t &cnt) const {
        int32_t beg, end;
        list(x, beg, end);
        const bool row = x < n;
        for (int32_t base = beg; base < end; base += kWave) {
            const int32_t p = base + lane_id();
            bool take = false;
            int32_t y = 0;
            if (p < end) {
                int32_t e; float bv;
                entry(row, p, y, e, bv);
                take = active(y) && !removed(e) && stamp[y] != mark;
            }
            const uint64_t msk = ballot(take);
            if (take) {
                stamp[y] = mark;
                out[cnt + rank_below(msk)] = y;
            }
            cnt += __popcll(msk);
            wave_fence();
        }
    }

    __device__ float repair_row(int32_t i) const {
        float acc = 0.0f;
        for (int32_t e = a.A.row_ptr[i]; e < a.A.row_ptr[i + 1]; ++e) {
            const int32_t j = a.A.col_idx[e];
            if (!active(n + j) || removed(e)) continue;
            const float bv = a.A.val ? a.A.val[e] : 1.0f;
            const float prod = bv * c[j];
            acc = acc + prod;
        }
        return acc != 0.0f ? 1.0f / acc : r[i];
    }

    __device__ float repair_col(int32_t j) const {
        float acc = 0.0f;
        for (int32_t p = a.A.col_ptr[j]; p < a.A.col_ptr[j + 1]; ++p) {
            const int32_t i = a.A.row_idx[p];
            if (!active(i)) continue;
            if (rem && removed(a.A.csc2csr[p])) continue;
            const float bv = a.A.val_csc ? a.A.val_csc[p] : 1.0f;
            const float prod = bv * r[i];
            acc = acc + prod;
        }
        return acc != 0.0f ? 1.0f / acc : c[j];
    }

    // Eq. (local): rho_list = N_t(rho)\{gam} (column ids n+j), gam_list =
    // N_t(gam)\{rho} (row ids); `skip` is excluded from the list it lies in
    __device__ void local_repair(const int32_t *rho_list, int32_t k_rho, int32_t skip_rho,
                                 const int32_t *gam_list, int32_t k_gam, int32_t skip_gam,
                                 int32_t mark) const {
        const int l = lane_id();
        int32_t nc = 0, nr = 0;
        // C_loc: rho's other columns, then the child columns of gam's other rows
        for (int32_t base = 0; base < k_rho; base += kWave) {
            const int32_t idx = base + l;
            const int32_t y = idx < k_rho ? rho_list[idx] : -1;
            const bool take = idx < k_rho && y != skip_rho;
            const uint64_t msk = ballot(take);
            if (take) { stamp[y] = mark; loc_c[nc + rank_below(msk)] = y - n; }
            nc += __popcll(msk);
        }
        // R_loc: gam's other rows first
        for (int32_t base = 0; base < k_gam; base += kWave) {
            const int32_t idx = base + l;
            const int32_t y = idx < k_gam ? gam_list[idx] : -1;
            const bool take = idx < k_gam && y != skip_gam;
            const uint64_t msk = ballot(take);
            if (take) { stamp[y] = mark; loc_r[nr + rank_below(msk)] = y; }
            nr += __popcll(msk);
        }
        wave_fence();
        for (int32_t q = 0; q < k_gam; ++q) {
            const int32_t i = gam_list[q];
            if (i == skip_gam) continue;
            const int32_t before = nc;
            gather_unmarked(i, mark, loc_c, nc);
            // stored as column vertex ids; convert the new ones to column indices
            for (int32_t idx = before + l; idx < nc; idx += kWave) loc_c[idx] -= n;
            wave_fence();
        }
        for (int32_t q = 0; q < k_rho; ++q) {
            const int32_t y = rho_list[q];
            if (y == skip_rho) continue;
            gather_unmarked(y, mark, loc_r, nr);
        }
        wave_fence();
        for (int32_t idx = l; idx < nr; idx += kWave) new_r[idx] = repair_row(loc_r[idx]);
        for (int32_t idx = l; idx < nc; idx += kWave) new_c[idx] = repair_col(loc_c[idx]);
        wave_fence();
        for (int32_t idx = l; idx < nr; idx += kWave) r[loc_r[idx]] = new_r[idx];
        for (int32_t idx = l; idx < nc; idx += kWave) c[loc_c[idx]] = new_c[idx];
        wave_fence();
    }
};

// ------------------------------------------------------------------ kernel
__device__ void run_trajectory(const TrajArgs &a, Traj &T, int64_t q) {
    const int l = lane_id();
    const int32_t n = a.A.n;
    const uint32_t k = (uint32_t)(a.first + q);
    int32_t *path = a.path ? a.path + (size_t)q * 2 * n : nullptr;

    // ---- initial state: template degrees, tree, scaling copies, marks
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(a.deg0);
        uint4 *dst = reinterpret_cast<uint4 *>(T.deg);
        for (int32_t i = l; i < a.n_leaf / 8; i += kWave) dst[i] = src[i];
        for (int32_t i = l; i < a.tree.total; i += kWave) T.tree[i] = a.tree0[i];
        if (a.own_rc) {
            for (int32_t i = l; i < n; i += kWave) {
                T.r[i] = a.r0 ? a.r0[i] : 1.0f;
                T.c[i] = a.c0 ? a.c0[i] : 1.0f;
            }
        }
        if (a.sk_policy == kSkLocal)
            for (int32_t i = l; i < 2 * n; i += kWave) T.stamp[i] = 0;
        if (T.rem)
            for (int32_t i = l; i < (a.A.m + 31) / 32; i += kWave) T.rem[i] = 0;
        if (path)
            for (int32_t i = l; i < 2 * n; i += kWave) path[i] = -1;
        wave_fence();
    }

    double mant = 1.0;
    int64_t ex = 0;
    double track = 1.0;
    uint64_t h = 0;
    int32_t steps = 0, n_dm = 0, n_sweeps = 0, n_local = 0;
    bool alive = a.ok0 != 0;

    for (int32_t t = 0; alive && t < n; ++t) {
        // ---- choose the vertex
        int32_t v;
        if (a.vertex_rule == 1) v = t;
        else T.select_min(v);
        if (v < 0 || v >= 2 * n) {  // internal inconsistency: report, never index
            if (l == 0) atomicOr(a.err, 1u);
            alive = false;
            break;
        }
        const bool v_row = v < n;

        // ---- pass A: candidates N_t(v) (into lst_a), their count, max score
        int32_t beg, end;
        T.list(v, beg, end);
        int32_t kc = 0;
        float lmax = 0.0f;
        for (int32_t base = beg; base < end; base += kWave) {
            const int32_t p = base + l;
            bool cand = false;
            int32_t y = 0, e = 0;
            float bv = 0.0f;
            if (p < end) {
                T.entry(v_row, p, y, e, bv);
                cand = T.active(y) && !T.removed(e);
            }
            const uint64_t msk = ballot(cand);
            if (cand) {
                T.lst_a[kc + rank_below(msk)] = y;
                if (a.scaled) {
                    const float sc = v_row ? T.cv(y - n) : T.rv(y);
                    const float s = bv * sc;
                    lmax = (s > lmax) ? s : lmax;
                } else {
                    lmax = (bv > lmax) ? bv : lmax;
                }
            }
            kc += __popcll(msk);
        }
        if (kc == 0) { alive = false; break; }
        const float smax = wave_max_f32(lmax);
        const bool uniform = !(smax > 0.0f) || __builtin_isinf(smax);

        // ---- pass B: integer weights w_i and W
        auto weight = [&](float s) -> uint64_t {
            if (uniform) return 1ull;
            const float ratio = s / smax;
            const float rr = rintf(ratio * 16777216.0f);
            return rr >= 1.0f ? (uint64_t)rr : 1ull;
        };
        auto score = [&](int32_t y, float bv) -> float {
            if (!a.scaled) return bv;
            const float sc = v_row ? T.cv(y - n) : T.rv(y);
            return bv * sc;
        };
        uint64_t W = 0;
        if (kc > 1) {
            for (int32_t base = beg; base < end; base += kWave) {
                const int32_t p = base + l;
                uint64_t w = 0;
                if (p < end) {
                    int32_t y, e; float bv;
                    T.entry(v_row, p, y, e, bv);
                    if (T.active(y) && !T.removed(e)) w = weight(score(y, bv));
                }
                W += wave_sum_u64(w);
            }
        }
        // ---- draw u ~ q_t(.|v) and locate it (pass C)
        const uint64_t j = kc > 1 ? uniform_below(a.seed, k, a.b, (uint32_t)t, 0u, W) : 0ull;
        int32_t u = -1;
        float b_vu = 1.0f;
        uint64_t w_u = 1, pre = 0;
        for (int32_t base = beg; base < end; base += kWave) {
            const int32_t p = base + l;
            uint64_t w = 0;
            int32_t y = 0, e = 0;
            float bv = 0.0f;
            if (p < end) {
                T.entry(v_row, p, y, e, bv);
                if (T.active(y) && !T.removed(e)) w = kc > 1 ? weight(score(y, bv)) : 1ull;
            }
            const uint64_t incl = wave_incl_scan_u64(w) + pre;
            const bool hit = w != 0 && incl > j && incl - w <= j;
            const uint64_t msk = ballot(hit);
            if (msk) {
                const int src = __ffsll((unsigned long long)msk) - 1;
                u = read_lane(y, src);
                b_vu = read_lane(bv, src);
                w_u = read_lane(w, src);
                break;
            }
            pre = read_lane(incl, kWave - 1);
        }
        if (u < 0) {  // no candidate matched the draw: internal inconsistency
            if (l == 0) atomicOr(a.err, 2u);
            alive = false;
            break;
        }
        if (kc == 1) W = w_u;

        // ---- importance correction X <- X * B_vu / q(u|v), extended exponent
        {
            const double factor = (double)b_vu * ((double)W / (double)w_u);
            int e2;
            mant = frexp(mant * factor, &e2);
            ex += e2;
        }
        const int32_t rho = v_row ? v : u;
        const int32_t gam = v_row ? u : v;   // column vertex id
        const double z = (double)T.rv(rho) * (double)T.cv(gam - n);
        if (path && l == 0) { path[2 * t] = v; path[2 * t + 1] = u; }
        h = splitmix_fold(h, ((uint64_t)(uint32_t)v << 32) | (uint32_t)u);

        // ---- N_t(u) \ {v} into lst_b
        int32_t kb = 0;
        {
            int32_t ub, ue;
            T.list(u, ub, ue);
            const bool u_row = u < n;
            for (int32_t base = ub; base < ue; base += kWave) {
                const int32_t p = base + l;
                bool take = false;
                int32_t y = 0;
                if (p < ue) {
                    int32_t e; float bv;
                    T.entry(u_row, p, y, e, bv);
                    take = y != v && T.active(y) && !T.removed(e);
                }
                const uint64_t msk = ballot(take);
                if (take) T.lst_b[kb + rank_below(msk)] = y;
                kb += __popcll(msk);
            }
        }
        wave_fence();

        // ---- B^(t+1) = B^(t) \ {v,u}: retire both, lower their neighbours
        if (l == 0) { T.deg[v] = kRetired; T.deg[u] = kRetired; }
        for (int32_t idx = l; idx < kc; idx += kWave) {
            const int32_t y = T.lst_a[idx];
            if (y == u) continue;
            const uint32_t d = (uint32_t)T.deg[y] - 1u;
            T.deg[y] = (uint16_t)d;
            T.tree_lower(y, d);
        }
        for (int32_t idx = l; idx < kb; idx += kWave) {
            const int32_t y = T.lst_b[idx];
            const uint32_t d = (uint32_t)T.deg[y] - 1u;
            T.deg[y] = (uint16_t)d;
            T.tree_lower(y, d);
        }
        wave_fence();
        T.tree_refresh(v);
        T.tree_refresh(u);
        steps = t + 1;
        track = track * z;
        if (t + 1 >= n) break;

        if (T.global_min() == 0) { alive = false; break; }   // child dead end

        // ---- P_DM (inner support filtering is rejected by the host for now)
        bool run_dm = false;
        if (a.dm_policy == kDmAll) run_dm = true;
        else if (a.dm_policy == kDmThrs && z < a.theta_th) run_dm = true;
        else if (a.dm_policy == kDmTrck && track < a.theta_tr) run_dm = true;
        if (run_dm) { n_dm += 1; track = 1.0; }

        // ---- P_SK on the child
        if (a.sk_policy == kSkFixed || a.sk_policy == kSkAdaptive) {
            int nit = a.K;
            if (a.sk_policy == kSkAdaptive) {
                double want = ceil((1.0 - z) * (double)a.K);
                if (!(want > 0.0)) want = 0.0;
                if (want > (double)a.K) want = (double)a.K;
                nit = (int)want;
            }
            for (int it = 0; it < nit; ++it) T.sk_sweep();
            n_sweeps += nit;
        } else if (a.sk_policy == kSkLocal) {
            // rho_list = N_t(rho)\{gam}, gam_list = N_t(gam)\{rho}
            if (v_row) T.local_repair(T.lst_a, kc, u, T.lst_b, kb, -1, t + 1);
            else T.local_repair(T.lst_b, kb, -1, T.lst_a, kc, u, t + 1);
            n_local += 1;
        }
    }

    if (l == 0) {
        const bool done = alive && steps == n;
        if (a.logw) a.logw[q] = done ? log(mant) + (double)ex * kLn2 : -__builtin_huge_val();
        if (a.alive) a.alive[q] = done ? 1 : 0;
        if (a.path_hash) a.path_hash[q] = done ? h : 0ull;
        if (a.counters) {
            int32_t *cn = a.counters + 4 * q;
            cn[0] = steps; cn[1] = n_dm; cn[2] = n_sweeps; cn[3] = n_local;
        }
    }
    wave_fence();
}

__global__ void __launch_bounds__(256) traj_kernel(TrajArgs a) {
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x / kWave;
    const size_t per_wave = (size_t)a.tree.total * 4 + (size_t)a.lds_state_bytes;
    char *mine = smem + (size_t)wave * per_wave;
    uint32_t *tree = reinterpret_cast<uint32_t *>(mine);
    char *state;
    if (a.hbm_state) {
        const uint64_t slot = (uint64_t)blockIdx.x * a.waves_per_block + wave;
        state = a.hbm_state + slot * a.hbm_stride;
    } else {
        state = mine + (size_t)a.tree.total * 4;
    }
    Traj T(a, state, tree);
    for (;;) {
        uint32_t q = 0;
        if (lane_id() == 0) q = atomicAdd(a.work_next, 1u);
        q = read_lane(q, 0);
        if ((int64_t)q >= a.count) break;
        run_trajectory(a, T, (int64_t)q);
    }
}

}  // namespace pe
