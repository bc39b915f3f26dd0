// traj.hpp -- the trajectory kernel: one wave64 runs one trajectory of the
// generic estimator (Alg. 2) at a time and pulls trajectory ids from a
// global counter until the range is exhausted.
//
// Per-trajectory state (one block per wave, in LDS for small n or in an HBM
// scratch slot for large n):
//   deg    u16[n_leaf]  residual degree of every vertex (rows 0..n-1,
//                       columns n..2n-1), 0xFFFF once matched; padded with
//                       0xFFFF to a multiple of 256
//   rec    {f32,i32}[2n] per vertex: its scaling value (r_i for a row, c_j
//                       for a column; negative once matched) and the stamp
//                       of the local repair's set membership
//   lst_a  i32[dmax]    N_t(v) for lists longer than a wave
//   lst_b  i32[dmax]    N_t(u) \ {v} for lists longer than a wave
//   loc_r, loc_c i32[n] R_loc, C_loc of Eq. (local)
//   new_v  f32[2n]      staged values of a repair larger than one wave
//   rem    u32[m/32]    edges removed by inner DM (CSR edge ids)
//   mate_r, mate_c i32[n] perfect matching kept for inner DM
//   ws     i32[6n]      inner-DM work space (BFS, Tarjan)
// Minimum-degree selection uses a min-tree whose internal nodes are u32 in
// LDS: level-1 node g is the minimum of leaves [256g, 256g+256), higher
// levels have fan-out 64, the top level has at most 64 nodes.  The leftmost
// minimum is followed down, so the selected vertex is the active vertex of
// minimum degree with the smallest id.
#pragma once
#include "device.hpp"
#include "reduce.hpp"
#include "mlp.hpp"

namespace pe {

struct DevMat {
    int32_t n, m;
    const int32_t *row_ptr, *col_idx, *col_ptr, *row_idx, *csc2csr;
    const int32_t *edge_row;  // row of every CSR edge
    const float *val;         // CSR order, nullptr = 0/1
    const float *val_csc;     // CSC order, nullptr = 0/1
};

// the matrix arrays as global-memory pointers (device code)
struct GMat {
    const PE_G int32_t *row_ptr, *col_idx, *col_ptr, *row_idx, *csc2csr, *edge_row;
    const PE_G float *val, *val_csc;
    template <class DM>
    __device__ explicit GMat(const DM &A)
        : row_ptr(gptr(A.row_ptr)), col_idx(gptr(A.col_idx)), col_ptr(gptr(A.col_ptr)), row_idx(gptr(A.row_idx)),
          csc2csr(gptr(A.csc2csr)), edge_row(gptr(A.edge_row)), val(gptr(A.val)), val_csc(gptr(A.val_csc)) {}
};

struct TreeLayout {
    int32_t levels;   // internal levels, 1..3
    int32_t size[3];  // nodes per level (level 1 first)
    int32_t off[3];   // u32 offset of each level within the tree block
    int32_t total;    // u32 count of the tree block
};

struct StateLayout {  // byte offsets in one trajectory's state block
    uint32_t deg, rec, lst_a, lst_b, loc_r, loc_c, new_v, rem, mate_r, mate_c, ws;
    uint32_t lvl0;   // the min-tree's lowest internal level, when TrajArgs::l0_state
    uint32_t bytes;
};

struct Rec {
    float s;        // scaling value; < 0 once the vertex is matched
    int32_t stamp;  // (step + 1) << 6 | lane of the last local-repair visit
};

// kSkLearnedGated: the learned proposal with the gated local-repair fallback
// (own scaling values, Eq. (local) after a low-probability step or an inner
// DM call, the scaled proposal of Eq. (q) on the step after such a repair)
enum : int32_t { kSkNone = 0, kSkFixed = 1, kSkAdaptive = 2, kSkLocal = 3, kSkLearned = 4, kSkLearnedGated = 5 };
__host__ __device__ constexpr bool learned_kind(int sk) { return sk == kSkLearned || sk == kSkLearnedGated; }
enum : int32_t { kDmNone = 0, kDmAll = 1, kDmThrs = 2, kDmTrck = 3 };

struct TrajArgs {
    DevMat A;
    const float *r0, *c0;      // shared outer scaling, nullptr = all ones
    const uint16_t *deg0;      // leaf template [n_leaf]
    const uint32_t *tree0;     // internal-node template [tree.total]
    const uint32_t *tree0a;    // the same with level 1 as (degree << 8 | position)
    const int32_t *mate0_r;    // perfect matching of the filtered input, or nullptr
    const int32_t *mate0_c;
    int32_t n_leaf;
    TreeLayout tree;           // the internal levels the wave keeps in LDS (offsets there)
    int32_t l0_state;          // 1: level 0 lives in the state slot (st.lvl0), LDS holds levels 1..
    int32_t tree_l1_src;       // with l0_state: u32 offset of level 1 in the tree templates
    StateLayout st;
    int32_t ok0;               // 0: the input has no perfect matching
    int32_t lds_tier;          // 1: this matrix's state lives in the wave's LDS slot
    int32_t vertex_rule, sk_policy, dm_policy, K;
    int32_t local_cap;         // bounded-work local repair: 0 = Eq. (local) exactly
    int32_t scaled;            // proposal uses r/c
    double theta_th, theta_tr;
    uint64_t seed;
    uint32_t b;
    int64_t first, count;
    double *logw;
    uint8_t *alive;
    uint64_t *path_hash;
    int32_t *path;             // [count][2n] or nullptr
    int32_t *counters;         // [count][4] or nullptr
    uint32_t *err;             // internal-consistency error bits (zeroed before launch)
    // learned proposal: network parameters on the inference grid, softmax table
    const float *mlp;
    const int64_t *etab;
    double mix_alpha;
    // training-pair recording (nullptr = off): every rec_stride-th step with at
    // least two candidates and a list of at most one wave writes the
    // candidates' features and the current proposal as one group
    float *rec_x;              // [rec_cap][8]
    float *rec_y;              // [rec_cap]
    int64_t *rec_gstart;       // [rec_gcap] first record of the group
    int32_t *rec_ginfo;        // [rec_gcap][4] = {length, matrix b, trajectory k, step t}
    unsigned long long *rec_counter;  // claimed (records << 32) | groups
    unsigned long long *rec_written;  // written (records << 32) | groups
    int64_t rec_cap, rec_gcap;
    int32_t rec_stride;
};

// Bounded-work local repair: a list of L > cap entries is examined at the
// cap positions (o + floor(i L / cap)) mod L, i = 0..cap-1 (a systematic
// sample; distinct since L / cap > 1), with the offset o = floor(R L / 2^32)
// from the low 32 bits R of the trajectory's draw 2^31 + x at step t.
// L <= 65534 and cap <= 65535 keep i * L below 2^32.
__device__ __forceinline__ uint32_t sample_offset(uint64_t seed, uint32_t k, uint32_t b, uint32_t t, int32_t x,
                                                  int32_t L) {
    const uint32_t R = (uint32_t)rand64(seed, k, b, t, 0x80000000u | (uint32_t)x);
    return (uint32_t)(((uint64_t)R * (uint64_t)(uint32_t)L) >> 32);
}
__device__ __forceinline__ int32_t sample_pos(uint32_t o, int32_t i, int32_t L, int32_t cap) {
    const uint32_t p = o + ((uint32_t)i * (uint32_t)L) / (uint32_t)cap;
    return (int32_t)(p >= (uint32_t)L ? p - (uint32_t)L : p);
}

// ------------------------------------------------------------------ views
// AS: address space of the trajectory's state (kAsLds: the wave's LDS
// slot, kAsGlobal: its HBM slot)
template <bool OWN, bool DM, bool WT, int AS>
struct Traj {
    const PE_G TrajArgs &a;
    GMat M;
    const PE_G float *r0, *c0;  // shared outer scaling, nullptr = all ones
    as_ptr<AS, uint16_t> deg;
    uint32_t *tree;
    as_ptr<AS, Rec> rec;
    as_ptr<AS, int32_t> lst_a, lst_b, loc_r, loc_c;
    as_ptr<AS, float> new_v;
    as_ptr<AS, uint32_t> rem;
    as_ptr<AS, int32_t> mate_r, mate_c, ws;
    uint32_t *lvl0;  // the tree's lowest internal level (LDS, or the state slot)
    int32_t n;

    __device__ Traj(const PE_G TrajArgs &args, char *state_any, uint32_t *tree_lds)
        : a(args), M(args.A), r0(gptr(args.r0)), c0(gptr(args.c0)), tree(tree_lds), n(args.A.n) {
        const auto &s = args.st;
        lvl0 = args.l0_state ? reinterpret_cast<uint32_t *>(state_any + s.lvl0) : tree_lds + args.tree.off[0];
        const auto state = to_as<AS>(state_any);
        deg = recast<uint16_t>(state + s.deg);
        rec = OWN ? recast<Rec>(state + s.rec) : nullptr;
        lst_a = recast<int32_t>(state + s.lst_a);
        lst_b = recast<int32_t>(state + s.lst_b);
        loc_r = recast<int32_t>(state + s.loc_r);
        loc_c = recast<int32_t>(state + s.loc_c);
        new_v = recast<float>(state + s.new_v);
        rem = DM ? recast<uint32_t>(state + s.rem) : nullptr;
        mate_r = recast<int32_t>(state + s.mate_r);
        mate_c = recast<int32_t>(state + s.mate_c);
        ws = recast<int32_t>(state + s.ws);
    }

    __device__ __forceinline__ bool active(int32_t x) const { return deg[x] != kRetired; }
    __device__ __forceinline__ bool removed(int32_t e) const {
        if (!DM) return false;
        return (rem[e >> 5] >> (e & 31)) & 1u;
    }
    // scaling value of vertex y (r_y for a row, c_{y-n} for a column)
    __device__ __forceinline__ float scale(int32_t y) const {
        if (OWN) return rec[y].s;
        if (y < n) return r0 ? r0[y] : 1.0f;
        return c0 ? c0[y - n] : 1.0f;
    }
    __device__ __forceinline__ void list(int32_t x, int32_t &beg, int32_t &end) const {
        if (x < n) { beg = M.row_ptr[x]; end = M.row_ptr[x + 1]; }
        else { beg = M.col_ptr[x - n]; end = M.col_ptr[x - n + 1]; }
    }
    // entry p of a list: neighbour vertex id, CSR edge id, value
    __device__ __forceinline__ void entry(bool row, int32_t p, int32_t &y, int32_t &e, float &bv) const {
        if (row) {
            y = n + M.col_idx[p];
            e = p;
            bv = WT ? M.val[p] : 1.0f;
        } else {
            y = M.row_idx[p];
            e = DM ? M.csc2csr[p] : 0;
            bv = WT ? M.val_csc[p] : 1.0f;
        }
    }

    // ------------------------------------------------------ min-tree
    __device__ __forceinline__ uint32_t *level(int k) const { return k == 0 ? lvl0 : tree + a.tree.off[k]; }

    __device__ __forceinline__ void tree_lower(int32_t x, uint32_t d) const {
        atomicMin(level(0) + (x >> 8), d);
        if (a.tree.levels > 1) atomicMin(level(1) + (x >> 14), d);
        if (a.tree.levels > 2) atomicMin(level(2) + (x >> 20), d);
    }

    __device__ __forceinline__ uint32_t leaf_group_min(int32_t g) const {
        const int l = lane_id();
        const uint2 q = recast<const uint2>(deg + 256 * g)[l];
        uint32_t m = min(min(q.x & 0xFFFFu, q.x >> 16), min(q.y & 0xFFFFu, q.y >> 16));
        return wave_min_u32(m);
    }

    __device__ void refresh_upper(int32_t g) const {
        const int l = lane_id();
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

    // recompute the chain above vertex x from memory
    __device__ void tree_refresh(int32_t x) const {
        const int32_t g = x >> 8;
        const uint32_t m = leaf_group_min(g);
        if (lane_id() == 0) level(0)[g] = m;
        wave_fence();
        refresh_upper(g);
    }

    // rebuild every internal node from the leaves
    __device__ void tree_rebuild() const {
        const int l = lane_id();
        for (int32_t g = 0; g < a.tree.size[0]; ++g) {
            const uint32_t m = leaf_group_min(g);
            if (l == 0) level(0)[g] = m;
        }
        wave_fence();
        for (int k = 1; k < a.tree.levels; ++k) {
            for (int32_t h = 0; h < a.tree.size[k]; ++h) {
                const int32_t idx = 64 * h + l;
                uint32_t v = idx < a.tree.size[k - 1] ? level(k - 1)[idx] : 0xFFFFFFFFu;
                v = wave_min_u32(v);
                if (l == 0) level(k)[h] = v;
            }
            wave_fence();
        }
    }

    __device__ __forceinline__ uint32_t global_min() const {
        const int top = a.tree.levels - 1;
        const int l = lane_id();
        uint32_t v = l < a.tree.size[top] ? level(top)[l] : 0xFFFFFFFFu;
        return wave_min_u32(v);
    }

    // Minimum-degree selection; also hands back the leaf group of the
    // selected vertex and this lane's four leaves of it, so the group
    // minimum can be refreshed from registers after the step, and the
    // selected vertex's list bounds, loaded for the whole group together
    // with its leaves (one memory round trip instead of two).
    __device__ bool select_min(int32_t &vsel, int32_t &gsel, uint2 &leaves, int32_t &vb, int32_t &ve,
                               uint32_t &m) const {
        const int l = lane_id();
        const int top = a.tree.levels - 1;
        uint32_t v = l < a.tree.size[top] ? level(top)[l] : 0xFFFFFFFFu;
        m = wave_min_u32(v);
        uint64_t hit = ballot(v == m);
        int32_t g = __ffsll((unsigned long long)hit) - 1;
        for (int k = top - 1; k >= 0 && hit; --k) {
            const int32_t idx = 64 * g + l;
            const uint32_t w = idx < a.tree.size[k] ? level(k)[idx] : 0xFFFFFFFFu;
            hit = ballot(w == m);
            g = 64 * g + __ffsll((unsigned long long)hit) - 1;
        }
        if (!hit) return false;
        leaves = recast<const uint2>(deg + 256 * g)[l];
        // list bounds of this lane's four vertices from five consecutive
        // pointers (a list ends where the next begins, except at the last row)
        int32_t pp[5], lb[4], le[4];
        const int32_t x0 = 256 * g + 4 * l;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const int32_t x = x0 + i;
            const int32_t xc = x - n < n ? x - n : n;  // past the columns: their end
            pp[i] = *(x < n ? M.row_ptr + x : M.col_ptr + xc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            lb[i] = pp[i];
            le[i] = x0 + i == n - 1 ? M.row_ptr[n] : pp[i + 1];
        }
        const uint32_t d0 = leaves.x & 0xFFFFu, d1 = leaves.x >> 16, d2 = leaves.y & 0xFFFFu,
                       d3 = leaves.y >> 16;
        const int j = d0 == m ? 0 : d1 == m ? 1 : d2 == m ? 2 : d3 == m ? 3 : 4;
        hit = ballot(j < 4);
        if (!hit) return false;
        const int src = __ffsll((unsigned long long)hit) - 1;
        const int js = read_lane(j, src);
        vsel = 256 * g + 4 * src + js;
        gsel = g;
        const int32_t mb = js == 0 ? lb[0] : js == 1 ? lb[1] : js == 2 ? lb[2] : lb[3];
        const int32_t me = js == 0 ? le[0] : js == 1 ? le[1] : js == 2 ? le[2] : le[3];
        vb = read_lane(mb, src);
        ve = read_lane(me, src);
        return true;
    }

    // ------------------------------------------------------------ SK
    // one full iteration over the residual: columns with the old r, then
    // rows with the new c; sequential binary32 sums in list order
    // One SK iteration on the residual: every active column from the old
    // rows, then every active row from the new columns (sums in list order,
    // eight entries' loads in flight at a time; a matched vertex has a
    // negative scale).
    __device__ void sk_sweep() const {
        const int l = lane_id();
        for (int32_t j = l; j < n; j += kWave) {
            const int32_t x = n + j;
            if (!(rec[x].s >= 0.0f)) continue;
            const float acc = residual_sum(x);
            if (acc != 0.0f) rec[x].s = 1.0f / acc;
        }
        wave_fence();
        for (int32_t i = l; i < n; i += kWave) {
            if (!(rec[i].s >= 0.0f)) continue;
            const float acc = residual_sum(i);
            if (acc != 0.0f) rec[i].s = 1.0f / acc;
        }
        wave_fence();
    }

    // Sum of B_xy * s_y over the residual neighbours y of vertex x in list
    // order (binary32, no FMA); loads are issued eight entries at a time.
    __device__ float residual_sum(int32_t x) const {
        const bool row = x < n;
        int32_t beg, end;
        list(x, beg, end);
        float acc = 0.0f;
        for (int32_t p0 = beg; p0 < end; p0 += 8) {
            int32_t y[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int32_t p = p0 + i < end ? p0 + i : end - 1;
                y[i] = row ? n + M.col_idx[p] : M.row_idx[p];
            }
            float sv[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) sv[i] = rec[y[i]].s;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int32_t p = p0 + i;
                if (p < end && sv[i] >= 0.0f) {
                    if (DM) {
                        const int32_t e = row ? p : M.csc2csr[p];
                        if (removed(e)) continue;
                    }
                    const float bv = WT ? (row ? M.val[p] : M.val_csc[p]) : 1.0f;
                    const float prod = bv * sv[i];
                    acc = acc + prod;
                }
            }
        }
        return acc;
    }

    // Bounded-work form of residual_sum for a list longer than cap: the sum
    // of B_xy * s_y over the active entries at the cap sample positions of
    // x's list (offset o, sample order, binary32, no FMA) and their count.
    __device__ float sampled_sum(int32_t x, uint32_t o, int32_t cap, int32_t &cnt) const {
        const bool row = x < n;
        int32_t beg, end;
        list(x, beg, end);
        const int32_t L = end - beg;
        float acc = 0.0f;
        int32_t c = 0;
        for (int32_t i = 0; i < cap; ++i) {
            const int32_t p = beg + sample_pos(o, i, L, cap);
            const int32_t y = row ? n + M.col_idx[p] : M.row_idx[p];
            const float sv = rec[y].s;
            if (!(sv >= 0.0f)) continue;
            if (DM) {
                const int32_t e = row ? p : M.csc2csr[p];
                if (removed(e)) continue;
            }
            const float bv = WT ? (row ? M.val[p] : M.val_csc[p]) : 1.0f;
            const float prod = bv * sv;
            acc = acc + prod;
            ++c;
        }
        cnt = c;
        return acc;
    }

    // ------------------------------------------------- inner support filter
    // Alg. 2 InnerDM on the child residual: repair the kept perfect matching
    // (one BFS augmentation per row that lost its partner), strongly
    // connected components of the contracted alternating digraph (matched
    // pair (i, mate_r[i]) = node i; entry (i, j) off the matching gives the
    // arc mate_c[j] -> i) by an iterative Tarjan, then remove every entry
    // off the matching whose endpoints lie in different components.
    // Sequential parts run on lane 0; returns false if the child has no
    // perfect matching.
    __device__ bool augment_from(int32_t s, as_ptr<AS, int32_t> queue, as_ptr<AS, int32_t> parent,
                                 as_ptr<AS, int32_t> vis,
                                 int32_t stamp, uint64_t &examined) const {
        int32_t head = 0, tail = 0, found = -1;
        queue[tail++] = s;
        while (head < tail && found < 0) {
            const int32_t i = queue[head++];
            for (int32_t e = M.row_ptr[i]; e < M.row_ptr[i + 1]; ++e) {
                ++examined;
                const int32_t j = M.col_idx[e];
                if (!active(n + j) || removed(e) || vis[j] == stamp) continue;
                vis[j] = stamp;
                parent[j] = i;
                if (mate_c[j] < 0) { found = j; break; }
                queue[tail++] = mate_c[j];
            }
        }
        if (found < 0) return false;
        int32_t j = found;
        for (;;) {
            const int32_t i = parent[j];
            const int32_t nj = mate_r[i];
            mate_r[i] = j;
            mate_c[j] = i;
            if (i == s) break;
            j = nj;
        }
        return true;
    }

    // Matching repair of the inner filter: every active row whose partner
    // column left the residual gets a new one by one BFS augmentation (on
    // lane 0, rows in index order; the rows that need one are found across
    // the wave); false (in every lane) if the child has no perfect matching.
    // `examined` counts on lane 0.
    __device__ bool dm_match(uint64_t &examined) const {
        const int l = lane_id();
        const auto queue = ws, parent = ws + n, vis = ws + 2 * n;
        for (int32_t j = l; j < n; j += kWave) {
            vis[j] = 0;
            if (active(n + j) && mate_c[j] >= 0 && !active(mate_c[j])) mate_c[j] = -1;
        }
        wave_fence();
        int32_t stamp = 0;
        for (int32_t base = 0; base < n; base += kWave) {
            const int32_t i = base + l;
            bool need = false;
            if (i < n && active(i)) {
                const int32_t j = mate_r[i];
                need = !(j >= 0 && active(n + j));
            }
            // an augmentation re-pairs only rows that already had a partner,
            // so the rows found here still need one when their turn comes
            uint64_t msk = ballot(need);
            while (msk) {
                const int32_t i0 = base + __ffsll((unsigned long long)msk) - 1;
                msk &= msk - 1;
                int ok = 1;
                if (l == 0) {
                    mate_r[i0] = -1;
                    ok = augment_from(i0, queue, parent, vis, ++stamp, examined) ? 1 : 0;
                }
                ok = read_lane(ok, 0);
                wave_fence();
                if (!ok) return false;
            }
        }
        return true;
    }

    // The contracted alternating digraph: node x = active row x with its
    // partner column mate_r[x]; arcs x -> y for every other active row y of
    // that column whose entry is not removed.  scan_arcs visits the arcs of x
    // eight entries at a time, with the loads of each batch in flight
    // together (rows, then their colours, visit marks and edge ids, then the
    // removed bits): f(y, colour[y], vis[y]) for every arc whose head is
    // live (colour >= 0: inactive rows and rows already in a component have
    // colour -1).  Returns the entries examined.
    template <bool NEED_VIS, class F>
    __device__ __forceinline__ uint32_t scan_arcs(int32_t x, as_ptr<AS, int32_t> colour, as_ptr<AS, int32_t> vis,
                                                  F &&f) const {
        const int32_t jm = mate_r[x];
        const int32_t beg = M.col_ptr[jm], end = M.col_ptr[jm + 1];
        for (int32_t p0 = beg; p0 < end; p0 += 8) {
            int32_t y[8], cy[8], vy[8], e[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) y[i] = M.row_idx[p0 + i < end ? p0 + i : end - 1];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                cy[i] = colour[y[i]];
                vy[i] = NEED_VIS ? vis[y[i]] : 0;
                e[i] = M.csc2csr[p0 + i < end ? p0 + i : end - 1];
            }
            bool rm[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) rm[i] = removed(e[i]);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (p0 + i < end && y[i] != x && cy[i] >= 0 && !rm[i]) f(y[i], cy[i], vy[i]);
        }
        return (uint32_t)(end - beg);
    }

    // Strongly connected components of that digraph across the wave, by
    // rounds of max-label colouring: colour[y] becomes the largest live node
    // id that reaches y (forward propagation to a fixed point); a node whose
    // colour is its own id is a root, and the live nodes of its colour that
    // reach it (a backward closure inside the colour class) form its
    // component -- a path from such a node to the root stays in the class,
    // since anything reaching a node on it reaches the root too.  Components
    // found are removed and the next round colours what is left.
    // comp[x] = the root of x's component.  false when kSccRounds rounds do
    // not finish (long chains of components), leaving the work to Tarjan.
    static constexpr int kSccRounds = 8;
    __device__ bool scc_colouring(uint64_t &examined) const {
        const int l = lane_id();
        const auto colour = ws, vis = ws + n, comp = ws + 2 * n;
        uint64_t ex = 0;
        for (int32_t x = l; x < n; x += kWave) comp[x] = -1;
        wave_fence();
        bool done = false;
        for (int round = 0; round < kSccRounds && !done; ++round) {
            bool live_any = false;
            for (int32_t x = l; x < n; x += kWave) {
                const bool live = active(x) && comp[x] < 0;
                colour[x] = live ? x : -1;
                vis[x] = 0;
                live_any = live_any || live;
            }
            wave_fence();
            if (!ballot(live_any)) { done = true; break; }
            for (;;) {  // forward: the largest id reaching each live node
                bool ch = false;
                for (int32_t x = l; x < n; x += kWave) {
                    const int32_t cx = colour[x];
                    if (cx < 0) continue;
                    ex += scan_arcs<false>(x, colour, vis, [&](int32_t y, int32_t cy, int32_t) {
                        if (cy < cx && atomicMax(&colour[y], cx) < cx) ch = true;
                    });
                }
                wave_fence();
                if (!ballot(ch)) break;
            }
            for (int32_t x = l; x < n; x += kWave)
                if (colour[x] == x) vis[x] = 1;
            wave_fence();
            for (;;) {  // backward inside each colour class: the nodes reaching its root
                bool ch = false;
                for (int32_t x = l; x < n; x += kWave) {
                    const int32_t cx = colour[x];
                    if (cx < 0 || vis[x]) continue;
                    bool reach = false;
                    ex += scan_arcs<true>(x, colour, vis, [&](int32_t, int32_t cy, int32_t vy) {
                        if (vy && cy == cx) reach = true;
                    });
                    if (reach) { vis[x] = 1; ch = true; }
                }
                wave_fence();
                if (!ballot(ch)) break;
            }
            for (int32_t x = l; x < n; x += kWave)
                if (colour[x] >= 0 && vis[x]) comp[x] = colour[x];
            wave_fence();
        }
        if (!done) {  // components may remain only if the last round left live nodes
            bool left = false;
            for (int32_t x = l; x < n; x += kWave) left = left || (active(x) && comp[x] < 0);
            done = !ballot(left);
        }
        examined += wave_sum_u64(ex);
        return done;
    }

    // The same components by an iterative Tarjan on lane 0 (comp[x] = the
    // root of x's component); the fallback of scc_colouring.
    __device__ void scc_tarjan(uint64_t &examined) const {
        const auto idx = ws, low = ws + n, comp = ws + 2 * n, stk = ws + 3 * n, fnode = ws + 4 * n,
                fpos = ws + 5 * n;
        for (int32_t i = 0; i < n; ++i) { idx[i] = -1; comp[i] = -1; }
        int32_t counter = 0, sp = 0;
        for (int32_t root = 0; root < n; ++root) {
            if (!active(root) || idx[root] >= 0) continue;
            int32_t top = 0;
            fnode[0] = root;
            fpos[0] = M.col_ptr[mate_r[root]];
            idx[root] = low[root] = counter++;
            stk[sp++] = root;
            while (top >= 0) {
                const int32_t x = fnode[top];
                const int32_t jm = mate_r[x];
                const int32_t end = M.col_ptr[jm + 1];
                bool descended = false;
                while (fpos[top] < end) {
                    const int32_t p = fpos[top]++;
                    ++examined;
                    const int32_t y = M.row_idx[p];
                    if (y == x || !active(y) || removed(M.csc2csr[p])) continue;
                    if (idx[y] < 0) {
                        ++top;
                        fnode[top] = y;
                        fpos[top] = M.col_ptr[mate_r[y]];
                        idx[y] = low[y] = counter++;
                        stk[sp++] = y;
                        descended = true;
                        break;
                    }
                    if (comp[y] < 0 && idx[y] < low[x]) low[x] = idx[y];
                }
                if (descended) continue;
                if (low[x] == idx[x]) {
                    int32_t z;
                    do { z = stk[--sp]; comp[z] = x; } while (z != x);
                }
                --top;
                if (top >= 0 && low[x] < low[fnode[top]]) low[fnode[top]] = low[x];
            }
        }
    }

    // remove entries off the matching whose endpoints lie in different
    // components (bitmap words in parallel), recount degrees, rebuild tree
    __device__ void dm_apply() const {
        const int l = lane_id();
        const auto comp = ws + 2 * n;
        // one edge per lane: 64 edges = two bitmap words per pass, the cut
        // bits gathered by a ballot and or-ed in by lanes 0 and 32
        for (int32_t base = 0; base < a.A.m; base += kWave) {
            const int32_t e = base + l;
            bool cut = false;
            if (e < a.A.m && !removed(e)) {
                const int32_t i = M.edge_row[e];
                const int32_t j = M.col_idx[e];
                if (active(i) && active(n + j) && mate_r[i] != j) cut = comp[i] != comp[mate_c[j]];
            }
            const uint64_t b = ballot(cut);
            if (l == 0 && (uint32_t)b) rem[base >> 5] |= (uint32_t)b;
            if (l == 32 && (b >> 32)) rem[(base >> 5) + 1] |= (uint32_t)(b >> 32);
        }
        wave_fence();
        for (int32_t x = l; x < 2 * n; x += kWave)
            if (active(x)) deg[x] = (uint16_t)residual_count(x);
        wave_fence();
        tree_rebuild();
    }

    // number of residual neighbours of x (active, entry not removed), with
    // eight entries' loads in flight at a time
    __device__ int32_t residual_count(int32_t x) const {
        const bool row = x < n;
        int32_t beg, end;
        list(x, beg, end);
        int32_t c = 0;
        for (int32_t p0 = beg; p0 < end; p0 += 8) {
            int32_t y[8], e[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int32_t p = p0 + i < end ? p0 + i : end - 1;
                y[i] = row ? n + M.col_idx[p] : M.row_idx[p];
                e[i] = row ? p : (DM ? M.csc2csr[p] : 0);
            }
            uint32_t d[8];
            bool rm[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) { d[i] = deg[y[i]]; rm[i] = removed(e[i]); }
#pragma unroll
            for (int i = 0; i < 8; ++i) c += (p0 + i < end && d[i] != kRetired && !rm[i]) ? 1 : 0;
        }
        return c;
    }
};

// ------------------------------------------------------------ helpers
// per-wave work units (kept in registers, added once to the launch totals:
// adjacency entries scanned at the two endpoints, degree decrements,
// local-repair entries, local values, full SK sweeps)
struct Work {
    uint64_t scan = 0;        // adjacency entries read at the two endpoints
    uint64_t dec = 0;         // residual-degree decrements
    uint64_t loc_entries = 0; // entries gathered or summed by local repairs
    uint64_t loc_values = 0;  // scaling values recomputed by local repairs
    uint64_t sweeps = 0;      // full SK iterations
    uint64_t mlp_tiles = 0;   // 16-candidate tiles through the proposal network
    uint64_t scan_v = 0;      // adjacency entries read at the selected vertex
    // device time by phase (wall-clock ticks of the wave, summed over its
    // trajectories) and the entries the inner filter examined
    uint64_t t_all = 0, t_sk = 0, t_dm = 0, t_loc = 0;
    uint64_t dm_entries = 0;
};

// the device's constant-rate wall clock (ticks; the rate is a device attribute)
__device__ __forceinline__ uint64_t wall_ticks() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ uint64_t lemire_from(uint64_t x, uint64_t W, uint64_t seed, uint32_t k,
                                                uint32_t b, uint32_t t) {
    const uint64_t lo = x * W;
    if (lo < W) {
        const uint64_t thr = (0ull - W) % W;
        if (lo < thr) return uniform_below(seed, k, b, t, 1u, W);
    }
    return __umul64hi(x, W);
}

// last lane whose exclusive offset is <= f (offsets non-decreasing)
__device__ __forceinline__ int owner_lane(int32_t f, int32_t off) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int cand = lo + step;
        const int32_t oc = __shfl(off, cand < kWave ? cand : kWave - 1);
        if (cand < kWave && oc <= f) lo = cand;
    }
    return lo;
}

// The same owner for every flattened position base + lane at once, when an
// LDS array of kWave ints is free: each list that starts inside the pass
// writes its lane at its start, and an inclusive max-scan carries it to the
// positions that follow (carry: the owner at the end of the previous pass).
// Lanes with empty lists never own a position, so the largest lane with a
// start at or before a position is its owner, as in owner_lane.
__device__ __forceinline__ int owners_in_pass(int32_t off, int32_t len, int32_t base, int32_t &carry,
                                              int32_t *scratch) {
    const int l = lane_id();
    scratch[l] = -1;
    wave_fence();
    const int32_t s = off - base;
    if (len > 0 && s >= 0 && s < kWave) scratch[s] = l;
    wave_fence();
    uint32_t v = (uint32_t)scratch[l];
    v = wave_scan_u32(v, 0x80000000u, [](uint32_t x, uint32_t y) { return (int32_t)y > (int32_t)x ? y : x; });
    int32_t o = (int32_t)v > carry ? (int32_t)v : carry;
    carry = read_lane(o, kWave - 1);
    wave_fence();
    return o;
}

__device__ __forceinline__ int32_t wave_excl_scan_i32(int32_t x, int32_t &total) {
    const uint32_t incl = wave_scan_u32((uint32_t)x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
    total = (int32_t)read_lane(incl, kWave - 1);
    return (int32_t)incl - x;
}

// New scaling value of x for Eq. (local) from the pre-repair values: the
// reciprocal of its child sum, or under a cap for a longer list the sampled
// sum scaled by residual degree / sampled active count; unchanged when the
// sum is zero (or nothing active was sampled).  `examined` counts entries.
template <class TT>
__device__ __forceinline__ float local_new_value(const TT &T, int32_t x, uint32_t k, int32_t t,
                                                 uint64_t &examined) {
    const float old = T.rec[x].s;
    int32_t b0, e0;
    T.list(x, b0, e0);
    const int32_t L = e0 - b0, cap = T.a.local_cap;
    if (cap > 0 && L > cap) {
        int32_t cnt;
        const float acc = T.sampled_sum(x, sample_offset(T.a.seed, k, T.a.b, (uint32_t)t, x, L), cap, cnt);
        examined += (uint64_t)cap;
        if (cnt > 0 && acc != 0.0f) {
            const float est = acc * ((float)T.deg[x] / (float)cnt);
            return 1.0f / est;
        }
        return old;
    }
    const float acc = T.residual_sum(x);
    examined += (uint64_t)L;
    return acc != 0.0f ? 1.0f / acc : old;
}

// Eq. (local).  rho_y: a column vertex of N_t(rho)\{gam} held by this lane
// (or -1); gam_y: a row of N_t(gam)\{rho} (or -1).  R_loc / C_loc membership
// is marked with stamps (step+1) << 6 | lane; when several lanes reach the
// same vertex in one instruction the lane whose stamp survives keeps it.
template <class TT>
__device__ __forceinline__ void local_repair_lanes(const TT &T, int32_t rho_y, int32_t gam_y, uint32_t k,
                                                   int32_t t, Work &work) {
    const int l = lane_id();
    const int32_t n = T.n;
    const int32_t mark = t + 1;
    const int32_t mine = (mark << 6) | l;
    int32_t nc = 0, nr = 0;
    {
        const uint64_t mc = ballot(rho_y >= 0);
        if (rho_y >= 0) { T.rec[rho_y].stamp = mine; T.loc_c[rank_below(mc)] = rho_y - n; }
        nc = __popcll(mc);
        const uint64_t mr = ballot(gam_y >= 0);
        if (gam_y >= 0) { T.rec[gam_y].stamp = mine; T.loc_r[rank_below(mr)] = gam_y; }
        nr = __popcll(mr);
    }
    // examined entries per first-hop list: all of it, or cap sample positions
    const int32_t cap = T.a.local_cap;
    int32_t gb = 0, gl = 0, rb = 0, rl = 0, gL = 0, rL = 0;
    uint32_t go = 0, ro = 0;
    if (gam_y >= 0) {
        gb = T.M.row_ptr[gam_y];
        gL = gl = T.M.row_ptr[gam_y + 1] - gb;
        if (cap > 0 && gL > cap) { gl = cap; go = sample_offset(T.a.seed, k, T.a.b, (uint32_t)t, gam_y, gL); }
    }
    if (rho_y >= 0) {
        rb = T.M.col_ptr[rho_y - n];
        rL = rl = T.M.col_ptr[rho_y - n + 1] - rb;
        if (cap > 0 && rL > cap) { rl = cap; ro = sample_offset(T.a.seed, k, T.a.b, (uint32_t)t, rho_y, rL); }
    }
    int32_t TG, TR;
    const int32_t og = wave_excl_scan_i32(gl, TG);
    const int32_t orr = wave_excl_scan_i32(rl, TR);
    wave_fence();
    for (int32_t base = 0; base < TG + TR; base += kWave) {
        const int32_t f = base + l;
        const bool in_g = f < TG;
        const bool in_r = !in_g && f < TG + TR;
        // every lane takes part in every shuffle (no divergent cross-lane reads)
        const int32_t fg = in_g ? f : 0;
        const int og_o = owner_lane(fg, og);
        const int32_t gb_o = __shfl(gb, og_o), og_v = __shfl(og, og_o);
        const int32_t fr = in_r ? f - TG : 0;
        const int or_o = owner_lane(fr, orr);
        const int32_t rb_o = __shfl(rb, or_o), or_v = __shfl(orr, or_o);
        int32_t gL_o = 0, rL_o = 0;
        uint32_t go_o = 0, ro_o = 0;
        if (cap > 0) {
            gL_o = __shfl(gL, og_o);
            go_o = (uint32_t)__shfl((int32_t)go, og_o);
            rL_o = __shfl(rL, or_o);
            ro_o = (uint32_t)__shfl((int32_t)ro, or_o);
        }
        int32_t tgt = -1, e = 0;
        if (in_g) {
            const int32_t i = fg - og_v;
            const int32_t p = gb_o + (cap > 0 && gL_o > cap ? sample_pos(go_o, i, gL_o, cap) : i);
            tgt = n + T.M.col_idx[p];
            e = p;
        } else if (in_r) {
            const int32_t i = fr - or_v;
            const int32_t p = rb_o + (cap > 0 && rL_o > cap ? sample_pos(ro_o, i, rL_o, cap) : i);
            tgt = T.M.row_idx[p];
            e = T.rem ? T.M.csc2csr[p] : 0;
        }
        bool cand = false;
        if (tgt >= 0) {
            const Rec rc = T.rec[tgt];
            cand = rc.s >= 0.0f && (rc.stamp >> 6) != mark && !T.removed(e);
        }
        if (cand) T.rec[tgt].stamp = mine;
        wave_fence();
        const bool win = cand && T.rec[tgt].stamp == mine;
        const uint64_t wc = ballot(win && in_g);
        const uint64_t wr = ballot(win && in_r);
        if (win && in_g) T.loc_c[nc + rank_below(wc)] = tgt - n;
        if (win && in_r) T.loc_r[nr + rank_below(wr)] = tgt;
        nc += __popcll(wc);
        nr += __popcll(wr);
    }
    wave_fence();
    const int32_t ne = nr + nc;
    uint64_t summed = 0;
    if (ne <= kWave) {
        int32_t x = -1;
        float val = 0.0f;
        if (l < ne) x = l < nr ? T.loc_r[l] : n + T.loc_c[l - nr];
        if (x >= 0) val = local_new_value(T, x, k, t, summed);
        wave_fence();
        if (x >= 0) T.rec[x].s = val;
    } else {
        for (int32_t idx = l; idx < ne; idx += kWave) {
            const int32_t x = idx < nr ? T.loc_r[idx] : n + T.loc_c[idx - nr];
            T.new_v[idx] = local_new_value(T, x, k, t, summed);
        }
        wave_fence();
        for (int32_t idx = l; idx < ne; idx += kWave) {
            const int32_t x = idx < nr ? T.loc_r[idx] : n + T.loc_c[idx - nr];
            T.rec[x].s = T.new_v[idx];
        }
    }
    wave_fence();
    work.loc_entries += (uint64_t)(TG + TR) + wave_sum_u64(summed);
    work.loc_values += (uint64_t)ne;
}

// Eq. (local) with lists kept in memory (either list longer than a wave):
// the same sets and values, built one list at a time.
template <class TT, class LP>
__device__ void local_repair_lists(const TT &T, LP rho_list, int32_t k_rho, int32_t skip_rho,
                                   LP gam_list, int32_t k_gam, int32_t skip_gam, uint32_t k, int32_t t,
                                   Work &work) {
    const int32_t cap = T.a.local_cap;
    const int l = lane_id();
    const int32_t n = T.n;
    const int32_t mark = t + 1;
    int32_t nc = 0, nr = 0;
    uint64_t gathered = 0;
    for (int32_t base = 0; base < k_rho; base += kWave) {
        const int32_t idx = base + l;
        const int32_t y = idx < k_rho ? rho_list[idx] : -1;
        const bool take = idx < k_rho && y != skip_rho;
        const uint64_t msk = ballot(take);
        if (take) { T.rec[y].stamp = mark << 6; T.loc_c[nc + rank_below(msk)] = y - n; }
        nc += __popcll(msk);
    }
    for (int32_t base = 0; base < k_gam; base += kWave) {
        const int32_t idx = base + l;
        const int32_t y = idx < k_gam ? gam_list[idx] : -1;
        const bool take = idx < k_gam && y != skip_gam;
        const uint64_t msk = ballot(take);
        if (take) { T.rec[y].stamp = mark << 6; T.loc_r[nr + rank_below(msk)] = y; }
        nr += __popcll(msk);
    }
    wave_fence();
    // child neighbours, one source vertex at a time (its entries are distinct)
    auto gather = [&](int32_t x, auto out, int32_t &cnt, bool to_col) {
        int32_t beg, end;
        T.list(x, beg, end);
        const bool row = x < n;
        const int32_t L = end - beg;
        const bool smp = cap > 0 && L > cap;
        const int32_t ne_x = smp ? cap : L;
        const uint32_t o = smp ? sample_offset(T.a.seed, k, T.a.b, (uint32_t)t, x, L) : 0u;
        gathered += ne_x;
        for (int32_t base = 0; base < ne_x; base += kWave) {
            const int32_t i = base + l;
            const int32_t p = beg + (smp ? (i < ne_x ? sample_pos(o, i, L, cap) : 0) : i);
            bool take = false;
            int32_t y = 0;
            if (i < ne_x) {
                int32_t e; float bv;
                T.entry(row, p, y, e, bv);
                const Rec rc = T.rec[y];
                take = rc.s >= 0.0f && !T.removed(e) && (rc.stamp >> 6) != mark;
            }
            const uint64_t msk = ballot(take);
            if (take) {
                T.rec[y].stamp = mark << 6;
                out[cnt + rank_below(msk)] = to_col ? y - n : y;
            }
            cnt += __popcll(msk);
            wave_fence();
        }
    };
    for (int32_t q = 0; q < k_gam; ++q) {
        const int32_t i = gam_list[q];
        if (i != skip_gam) gather(i, T.loc_c, nc, true);
    }
    for (int32_t q = 0; q < k_rho; ++q) {
        const int32_t y = rho_list[q];
        if (y != skip_rho) gather(y, T.loc_r, nr, false);
    }
    wave_fence();
    const int32_t ne = nr + nc;
    uint64_t summed = 0;
    for (int32_t idx = l; idx < ne; idx += kWave) {
        const int32_t x = idx < nr ? T.loc_r[idx] : n + T.loc_c[idx - nr];
        T.new_v[idx] = local_new_value(T, x, k, t, summed);
    }
    wave_fence();
    for (int32_t idx = l; idx < ne; idx += kWave) {
        const int32_t x = idx < nr ? T.loc_r[idx] : n + T.loc_c[idx - nr];
        T.rec[x].s = T.new_v[idx];
    }
    wave_fence();
    work.loc_entries += gathered + wave_sum_u64(summed);
    work.loc_values += (uint64_t)ne;
}

// ------------------------------------------------------------------ kernel
template <int SK>
struct OwnRC {
    static constexpr bool value = SK == kSkFixed || SK == kSkAdaptive || SK == kSkLocal || SK == kSkLearnedGated;
};

// Features of the candidate edge of Eq. (q) for the learned proposal. The
// definition (the oracle's) is FP64: Q(y) = clamp(rint(64 y), -256, 255) / 64
// and plog2(s) = e - 2 + 2m with (m, e) = frexp(s). The grid integers are
// formed here with integer operations that give the same values:
// * for a positive normal binary32 s = 2^(E-127) (1 + M/2^23),
//   plog2(s) = E - 127 + M/2^23, so 64 plog2(s)/4 = (bits >> 19) - 2032
//   plus the low 19 bits over 2^19, rounded half to even. (In FP64 the sum
//   e - 2 + 2m is exact to 2^-42 in these units, far finer than the 2^-19
//   steps of a binary32 input, so no rounding of the definition differs.)
//   Zero, subnormal and other inputs take the FP64 definition;
// * for an integer S >= 1 with 2^p <= S < 2^(p+1), 16 plog2(S) = 16 p +
//   16 S / 2^p - 16, exact in integers; S / 2^20 shifts it by -320;
// * t/n's grid integer rint(64 t / n) is kept incrementally by the caller
//   (k4); the rational 64 t / n is a tie exactly when the FP64 quotient is.
__device__ __forceinline__ int32_t q_clamp(int32_t k) { return k < -256 ? -256 : (k > 255 ? 255 : k); }

__device__ __forceinline__ float q64_plog2_quarter(float s) {
    const uint32_t b = __float_as_uint(s);
    int32_t k;
    if (b >= 0x00800000u && b < 0x7F800000u) {
        const uint32_t q = b >> 19, r = b & 0x7FFFFu;
        const uint32_t up = (r > 0x40000u || (r == 0x40000u && (q & 1u))) ? 1u : 0u;
        k = (int32_t)(q + up) - 2032;
    } else {
        int e;
        const double m = frexp((double)s, &e);
        const double y = rint(((double)e - 2.0 + 2.0 * m) / 4.0 * 64.0);
        k = y < -256.0 ? -256 : (y > 255.0 ? 255 : (int32_t)y);
    }
    return (float)q_clamp(k) * (1.0f / 64.0f);
}

// Q(plog2(S / 2^20) / 4) for the integer S (at most 2^53)
__device__ __forceinline__ float q64_plog2_quarter_fixed20(uint64_t S) {
    int32_t k = -32;  // plog2(0) = -2
    if (S != 0) {
        const int p = 63 - __builtin_clzll(S);
        const uint64_t t16 = S << 4;
        const uint32_t q = (uint32_t)(t16 >> p);  // 16 .. 31
        uint32_t up = 0;
        if (p > 0) {
            const uint64_t r = t16 & ((1ull << p) - 1ull), half = 1ull << (p - 1);
            up = (r > half || (r == half && (q & 1u))) ? 1u : 0u;
        }
        k = 16 * p + (int32_t)(q + up) - 16 - 320;
    }
    return (float)q_clamp(k) * (1.0f / 64.0f);
}

// k4 = rint(64 t / n) (ties to even), advanced from step t - 1 to step t
__device__ __forceinline__ int32_t advance_t_grid(int32_t k4, int32_t t, int32_t n) {
    for (;;) {
        const int64_t lhs = 128 * (int64_t)t, rhs = (2 * (int64_t)k4 + 1) * n;
        if (lhs > rhs || (lhs == rhs && (k4 & 1))) ++k4;
        else return k4;
    }
}

__device__ __forceinline__ void learned_features(float *x, uint32_t deg_rho, uint32_t deg_gam, float r0_rho,
                                                 float c0_gam, int32_t k4, bool v_row, uint64_t s_u,
                                                 int32_t c2_u) {
    x[0] = (float)(deg_rho < 255u ? deg_rho : 255u) / 64.0f;
    x[1] = (float)(deg_gam < 255u ? deg_gam : 255u) / 64.0f;
    x[2] = q64_plog2_quarter(r0_rho);
    x[3] = q64_plog2_quarter(c0_gam);
    x[4] = (float)q_clamp(k4) * (1.0f / 64.0f);
    x[5] = v_row ? 1.0f : 0.0f;
    x[6] = q64_plog2_quarter_fixed20(s_u);
    x[7] = (float)(c2_u < 255 ? c2_u : 255) / 64.0f;
}

// per-wave LDS scratch of the learned proposal (the owner search of the
// flattened candidate lists; the network itself runs in registers)
struct WaveScratch {
    int32_t i[kWave];
};

// The candidates' flattened lists as read by candidate_stats when they fit
// one pass of the wave: the step reuses them for N_t(u) once u is drawn.
struct NbrCache {
    bool valid = false;   // wave-uniform: all candidate lists fit one pass
    int32_t off = 0;      // per candidate lane: first flattened lane of its list
    int32_t ub = 0;       // per candidate lane: its list start
    int32_t len = 0;      // per candidate lane: its list length
    int32_t w = -1;       // per flattened lane: the neighbour
    uint32_t dw = 0;      // its residual degree (kRetired if matched)
    bool live = false;    // active and the edge not removed
};

// Neighbourhood statistics of the candidate u held by each lane (cand), whose
// list [ub, ue) the caller has read: s_u = sum over the residual neighbours w
// of u of floor(2^20 / deg w) and c2_u = #{w != v : deg w <= 2}.  The
// candidates' lists are flattened over the wave (64 entries per pass) and
// summed per owner with a segmented scan; integer sums, so the result does
// not depend on the order.
// scratch: kWave ints of the wave's LDS for the owner search, or nullptr
template <class TT>
__device__ void candidate_stats(const TT &T, bool cand, int32_t u, int32_t ub, int32_t ue, int32_t v,
                                uint64_t &s_u, int32_t &c2_u, NbrCache &nc, int32_t *scratch) {
    const int l = lane_id();
    const bool u_row = u < T.n;
    const int32_t len = cand ? ue - ub : 0;
    int32_t total;
    const int32_t off = wave_excl_scan_i32(len, total);
    s_u = 0;
    c2_u = 0;
    nc.valid = total <= kWave;
    nc.off = off;
    nc.ub = ub;
    nc.len = len;
    int32_t carry = -1;
    for (int32_t base = 0; base < total; base += kWave) {
        const int32_t f = base + l;
        const bool valid = f < total;
        int own;
        if (scratch) {
            // past the end (f >= total) this is the last list's lane, as below
            own = owners_in_pass(off, len, base, carry, scratch);
            own = own < 0 ? 0 : own;
        } else {
            own = owner_lane(valid ? f : total - 1, off);
        }
        const int32_t o_off = __shfl(off, own);
        const int32_t o_ub = __shfl(ub, own);
        const bool o_row = __shfl((int)u_row, own) != 0;
        uint32_t sv = 0;
        int32_t cv = 0;
        int32_t w = -1;
        uint32_t dw = 0;
        bool live = false;
        if (valid) {
            int32_t e;
            float bv;
            T.entry(o_row, o_ub + (f - o_off), w, e, bv);
            dw = T.deg[w];
            live = dw != kRetired && !T.removed(e);
            if (live && dw != 0) {
                sv = (1u << 20) / dw;
                cv = (w != v && dw <= 2u) ? 1 : 0;
            }
        }
        nc.w = w;
        nc.dw = dw;
        nc.live = live;
        // inclusive scan within runs of equal owner (runs are contiguous, so
        // a lane adds a shifted partial exactly when it carries its own key)
        auto seg = [&](uint32_t ys, uint32_t yc, uint32_t yo) {
            if ((int)yo == own) { sv += ys; cv += (int32_t)yc; }
        };
        seg(dpp<kRowShr1>(0u, sv), dpp<kRowShr1>(0u, (uint32_t)cv), dpp<kRowShr1>(~0u, (uint32_t)own));
        seg(dpp<kRowShr2>(0u, sv), dpp<kRowShr2>(0u, (uint32_t)cv), dpp<kRowShr2>(~0u, (uint32_t)own));
        seg(dpp<kRowShr4>(0u, sv), dpp<kRowShr4>(0u, (uint32_t)cv), dpp<kRowShr4>(~0u, (uint32_t)own));
        seg(dpp<kRowShr8>(0u, sv), dpp<kRowShr8>(0u, (uint32_t)cv), dpp<kRowShr8>(~0u, (uint32_t)own));
        seg(dpp<kRowBcast15, 0xA>(0u, sv), dpp<kRowBcast15, 0xA>(0u, (uint32_t)cv),
            dpp<kRowBcast15, 0xA>(~0u, (uint32_t)own));
        seg(dpp<kRowBcast31, 0xC>(0u, sv), dpp<kRowBcast31, 0xC>(0u, (uint32_t)cv),
            dpp<kRowBcast31, 0xC>(~0u, (uint32_t)own));
        // each candidate lane takes the scan value at the last lane of its run
        const int32_t lo_f = off > base ? off : base;
        int32_t hi_f = off + len;
        const int32_t cap = base + kWave < total ? base + kWave : total;
        hi_f = hi_f < cap ? hi_f : cap;
        const int src = hi_f > lo_f ? hi_f - 1 - base : 0;
        const uint32_t seg_s = __shfl(sv, src);
        const int32_t seg_c = __shfl(cv, src);
        if (hi_f > lo_f) { s_u += seg_s; c2_u += seg_c; }
    }
}

// Logits (units of 1/16) of the candidates held by the lanes of one list
// chunk: the quantised network on matrix cores in 16-candidate tiles, the
// feature tile assembled and the logits returned by cross-lane moves (only
// the layer-1 activations pass through LDS).  Lanes without a candidate
// return 0.
__device__ int32_t learned_logits(const MlpLds *W, bool cand, uint32_t deg_rho,
                                  uint32_t deg_gam, float r0_rho, float c0_gam, int32_t k4,
                                  bool v_row, uint64_t s_u, int32_t c2_u, int32_t chunk_len) {
    const int l = lane_id();
    float x[8];
    learned_features(x, deg_rho, deg_gam, r0_rho, c0_gam, k4, v_row, s_u, c2_u);
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = cand ? x[k] : 0.0f;
    const int grp = l >> 4;  // A-operand features 4 grp .. 4 grp + 3 (grp < 2)
    int32_t mine = 0;
    const int ntiles = (chunk_len + 15) / 16;
    for (int ti = 0; ti < ntiles; ++ti) {
        const int src = 16 * ti + (l & 15);
        bf16x4 xa;
        if (ti == 0) {
            // candidates 0..15 sit in lanes 0..15: row 0 keeps its own
            // features 0..3, and a row swap gives row 1 their features 4..7
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t xu = __float_as_uint(x[4 + j]);
                const float hi = __uint_as_float(__builtin_amdgcn_permlane16_swap(xu, xu, false, false)[0]);
                xa[j] = grp == 0 ? to_bf16(x[j]) : (grp == 1 ? to_bf16(hi) : (short)0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float lo = __shfl(x[j], src), hi = __shfl(x[4 + j], src);
                xa[j] = grp == 0 ? to_bf16(lo) : (grp == 1 ? to_bf16(hi) : (short)0);
            }
        }
        // every lane: the logit of record l % 16 of this tile
        const float y = mlp_tile_logit_grid(W, xa);
        if (grp == ti) {
            float L = rintf(y * 16.0f);
            L = L < -1024.0f ? -1024.0f : (L > 1023.0f ? 1023.0f : L);
            mine = (int32_t)L;
        }
    }
    return cand ? mine : 0;
}

template <int SK, bool DM, bool WT, int AS>
__device__ __forceinline__ void run_trajectory(const PE_G TrajArgs &a, const Traj<OwnRC<SK>::value, DM, WT, AS> &T,
                                               int64_t q, Work &work, const LearnedLds *lrn, WaveScratch *scr) {
    const MlpLds *mlpw = &lrn->net;
    const uint32_t *etab = lrn->etab;
    constexpr bool OWN = OwnRC<SK>::value;
    const int l = lane_id();
    const int32_t n = a.A.n;
    const uint32_t k = (uint32_t)(a.first + q);
    const uint64_t t_begin = wall_ticks();
    PE_G int32_t *path = a.path ? gptr(a.path) + (size_t)q * 2 * n : nullptr;

    // ---- initial state: template degrees, tree, scaling values, matching
    {
        const auto src = gptr(reinterpret_cast<const uint4 *>(a.deg0));
        const auto dst = recast<uint4>(T.deg);
        for (int32_t i = l; i < a.n_leaf / 8; i += kWave) dst[i] = src[i];
        if (a.l0_state) {
            for (int32_t i = l; i < a.tree.size[0]; i += kWave) T.lvl0[i] = gptr(a.tree0)[i];
            for (int32_t i = l; i < a.tree.total; i += kWave) T.tree[i] = gptr(a.tree0)[a.tree_l1_src + i];
        } else {
            for (int32_t i = l; i < a.tree.total; i += kWave) T.tree[i] = gptr(a.tree0)[i];
        }
        if (OWN) {
            for (int32_t x = l; x < 2 * n; x += kWave) {
                float s = 1.0f;
                if (x < n) { if (T.r0) s = T.r0[x]; }
                else if (T.c0) s = T.c0[x - n];
                T.rec[x] = Rec{s, 0};
            }
        }
        if (DM) {
            for (int32_t i = l; i < (a.A.m + 31) / 32; i += kWave) T.rem[i] = 0;
            for (int32_t i = l; i < n; i += kWave) {
                T.mate_r[i] = a.mate0_r ? gptr(a.mate0_r)[i] : -1;
                T.mate_c[i] = a.mate0_c ? gptr(a.mate0_c)[i] : -1;
            }
        }
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

    int32_t k4 = 0;  // learned feature x4: rint(64 t / n)
    bool fb = false;  // gated fallback: this step draws from the scaled proposal
    for (int32_t t = 0; alive && t < n; ++t) {
        k4 = advance_t_grid(k4, t, n);
        const bool net = learned_kind(SK) && !fb;  // the network proposes this step
        // ---- choose the vertex
        int32_t v = -1, gsel = -1;
        int32_t vb = 0, ve = 0;
        uint32_t m_sel = 0;  // the minimum degree at selection (v's group minimum)
        uint2 gleaves = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
        if (a.vertex_rule == 1) {
            v = t;
            T.list(v, vb, ve);
        } else if (!T.select_min(v, gsel, gleaves, vb, ve, m_sel)) {
            v = -1;
        }
        if (v < 0 || v >= 2 * n) {  // internal inconsistency: report, never index
            if (l == 0) atomicOr(a.err, 1u);
            alive = false;
            break;
        }
        const bool v_row = v < n;
        const bool fast_v = ve - vb <= kWave;

        // ---- candidates N_t(v), proposal of Eq. (q), draw, pick
        int32_t kc = 0, u = -1;
        float b_vu = 1.0f;
        uint64_t W = 0, w_u = 1;
        uint32_t d_u = 0;
        int32_t cy = -1;   // this lane's candidate (lists up to a wave)
        uint32_t cd = 0;
        bool cand = false;
        NbrCache nc;       // learned: the candidates' lists, reused for N_t(u)
        int u_lane = -1;   // fast path: the lane that held u
        int32_t u_ub = 0, u_ue = 0;  // fast path: u's list bounds
        if (fast_v) {
            const int32_t p = vb + l;
            int32_t e = 0;
            float bv = 0.0f, sc = 1.0f;
            int32_t cub = 0, cue = 0;
            if (p < ve) {
                T.entry(v_row, p, cy, e, bv);
                cd = T.deg[cy];
                if (a.scaled && !net) sc = T.scale(cy);
                T.list(cy, cub, cue);  // issued with the degree load; u's list comes from here
                cand = cd != kRetired && !T.removed(e);
            }
            kc = __popcll(ballot(cand));
            if (kc == 0) { alive = false; break; }
            const float s = a.scaled ? bv * sc : bv;
            uint64_t w = 0;
            if (net) {
                // quantised network logits -> integer softmax table -> uniform mix
                const uint32_t deg_v = (uint32_t)kc;
                const int32_t rho_c = v_row ? v : cy, gam_c = v_row ? cy : v;
                int32_t L = 0;
                if (kc > 1) {
                    const float r0r = T.r0 ? T.r0[cand ? rho_c : 0] : 1.0f;
                    const float c0g = T.c0 ? T.c0[cand ? gam_c - n : 0] : 1.0f;
                    uint64_t su;
                    int32_t c2;
                    candidate_stats(T, cand, cy, cub, cue, v, su, c2, nc, scr->i);
                    L = learned_logits(mlpw, cand, v_row ? deg_v : cd, v_row ? cd : deg_v, r0r, c0g,
                                       k4, v_row, su, c2, ve - vb);
                    work.mlp_tiles += (uint64_t)((ve - vb + 15) / 16);
                }
                const int32_t lmx = wave_max_i32(cand ? L : -2147483647);
                int64_t E = 0;
                if (cand) {
                    const int32_t d = lmx - L;
                    E = d < kEtabLds ? (int64_t)etab[d] : 0;
                }
                // at most 2^24 per lane: the 64-lane total fits 32 bits
                const int64_t S = (int64_t)read_lane(wave_incl_scan_add_u32((uint32_t)E), kWave - 1);
                if (cand) {
                    if (kc == 1) w = 1;
                    else {
                        const double qq = (1.0 - a.mix_alpha) * (double)E / (double)S + a.mix_alpha / (double)kc;
                        const double rr = rint(16777216.0 * qq);
                        w = rr >= 1.0 ? (uint64_t)rr : 1ull;
                    }
                }
            } else {
                const float lmax = (cand && s > 0.0f) ? s : 0.0f;
                const float smax = wave_max_f32(lmax);
                const bool uniform = !(smax > 0.0f) || __builtin_isinf(smax);
                if (cand) {
                    if (kc == 1 || uniform) w = 1;
                    else {
                        const float rr = rintf((s / smax) * 16777216.0f);
                        w = rr >= 1.0f ? (uint64_t)rr : 1ull;
                    }
                }
                // training pairs: features and the current scaled proposal.
                // Records and groups are claimed by one packed atomic, so the
                // groups that fit are a prefix of the claim order and their
                // records are contiguous.
                if (a.rec_x && kc >= 2 && (t % a.rec_stride) == 0) {
                    const float ssum = wave_sum_f32(cand ? s : 0.0f);
                    uint64_t su;
                    int32_t c2;
                    int32_t rub = 0, rue = 0;
                    if (cand) T.list(cy, rub, rue);
                    NbrCache rnc;
                    candidate_stats(T, cand, cy, rub, rue, v, su, c2, rnc, nullptr);
                    unsigned long long old = 0;
                    if (l == 0) {
                        const unsigned long long cur = __hip_atomic_load(a.rec_counter, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT);
                        if ((int64_t)(cur >> 32) + kc <= a.rec_cap && (int64_t)(cur & 0xFFFFFFFFull) < a.rec_gcap)
                            old = atomicAdd(a.rec_counter, ((unsigned long long)kc << 32) | 1ull);
                        else
                            old = ~0ull;
                    }
                    old = read_lane(old, 0);
                    const int64_t base = (int64_t)(old >> 32);
                    const int64_t gid = (int64_t)(old & 0xFFFFFFFFull);
                    if (old != ~0ull && base + kc <= a.rec_cap && gid < a.rec_gcap) {
                        const uint64_t cm = ballot(cand);
                        if (cand) {
                            const int64_t r = base + rank_below(cm);
                            const uint32_t deg_v = (uint32_t)kc;
                            const int32_t rho_c = v_row ? v : cy, gam_c = v_row ? cy : v;
                            float x[8];
                            learned_features(x, v_row ? deg_v : cd, v_row ? cd : deg_v,
                                             T.r0 ? T.r0[rho_c] : 1.0f, T.c0 ? T.c0[gam_c - n] : 1.0f, k4, v_row,
                                             su, c2);
                            float4 *xo = reinterpret_cast<float4 *>(a.rec_x + r * 8);
                            xo[0] = make_float4(x[0], x[1], x[2], x[3]);
                            xo[1] = make_float4(x[4], x[5], x[6], x[7]);
                            a.rec_y[r] = ssum > 0.0f ? s / ssum : 1.0f / (float)kc;
                        }
                        if (l == 0) {
                            a.rec_gstart[gid] = base;
                            a.rec_ginfo[4 * gid + 0] = kc;
                            a.rec_ginfo[4 * gid + 1] = (int32_t)a.b;
                            a.rec_ginfo[4 * gid + 2] = (int32_t)k;
                            a.rec_ginfo[4 * gid + 3] = t;
                            atomicAdd(a.rec_written, ((unsigned long long)kc << 32) | 1ull);
                        }
                    }
                }
            }
            const uint64_t incl = wave_incl_scan_add_u32((uint32_t)w);
            W = read_lane(incl, kWave - 1);
            const uint64_t j = kc > 1 ? lemire_from(rand64(a.seed, k, a.b, (uint32_t)t, 0u), W, a.seed, k, a.b, (uint32_t)t) : 0ull;
            const uint64_t hm = ballot(w != 0 && incl > j && incl - w <= j);
            if (hm) {
                const int src = __ffsll((unsigned long long)hm) - 1;
                u = read_lane(cy, src);
                b_vu = read_lane(bv, src);
                w_u = read_lane(w, src);
                d_u = read_lane(cd, src);
                u_ub = read_lane(cub, src);
                u_ue = read_lane(cue, src);
                u_lane = src;
            }
            if (kc == 1) W = w_u;
        } else {
            // long list: three passes over memory, candidates into lst_a
            float lmax = 0.0f;
            for (int32_t base = vb; base < ve; base += kWave) {
                const int32_t p = base + l;
                bool c0 = false;
                int32_t y = 0, e = 0;
                float bv = 0.0f;
                if (p < ve) {
                    T.entry(v_row, p, y, e, bv);
                    c0 = T.active(y) && !T.removed(e);
                }
                const uint64_t msk = ballot(c0);
                if (c0) {
                    T.lst_a[kc + rank_below(msk)] = y;
                    const float s = a.scaled ? bv * T.scale(y) : bv;
                    lmax = (s > lmax) ? s : lmax;
                }
                kc += __popcll(msk);
            }
            if (kc == 0) { alive = false; break; }
            const float smax = wave_max_f32(lmax);
            const bool uniform = !(smax > 0.0f) || __builtin_isinf(smax);
            // learned: logits of every candidate chunk into lst_b (free here)
            int32_t lmx = -2147483647;
            int64_t Ssum = 0;
            if (net && kc > 1) {
                int32_t idx0 = 0;
                for (int32_t base = vb; base < ve; base += kWave) {
                    const int32_t p = base + l;
                    bool c0 = false;
                    int32_t y = 0, e = 0;
                    float bv = 0.0f;
                    uint32_t dy = 0;
                    if (p < ve) {
                        T.entry(v_row, p, y, e, bv);
                        dy = T.deg[y];
                        c0 = dy != kRetired && !T.removed(e);
                    }
                    const int32_t rho_c = v_row ? v : y, gam_c = v_row ? y : v;
                    const float r0r = T.r0 ? T.r0[c0 ? rho_c : 0] : 1.0f;
                    const float c0g = T.c0 ? T.c0[c0 ? gam_c - n : 0] : 1.0f;
                    uint64_t su;
                    int32_t c2;
                    int32_t yub = 0, yue = 0;
                    if (c0) T.list(y, yub, yue);
                    NbrCache lnc;
                    candidate_stats(T, c0, y, yub, yue, v, su, c2, lnc, scr->i);
                    const int32_t L = learned_logits(mlpw, c0, v_row ? (uint32_t)kc : dy,
                                                     v_row ? dy : (uint32_t)kc, r0r, c0g, k4, v_row, su, c2,
                                                     min(kWave, ve - base));
                    work.mlp_tiles += (uint64_t)((min(kWave, ve - base) + 15) / 16);
                    const uint64_t msk = ballot(c0);
                    if (c0) { T.lst_b[idx0 + rank_below(msk)] = L; lmx = L > lmx ? L : lmx; }
                    idx0 += __popcll(msk);
                }
                lmx = wave_max_i32(lmx);
                wave_fence();
                uint64_t part = 0;
                for (int32_t idx = l; idx < kc; idx += kWave) {
                    const int32_t d = lmx - T.lst_b[idx];
                    part += d < kEtabLds ? (uint64_t)etab[d] : 0ull;
                }
                Ssum = (int64_t)wave_sum_u64(part);
            }
            // ci: the candidate's rank among all candidates (learned logits in lst_b)
            auto weight_of = [&](int32_t y, float bv, int32_t ci) -> uint64_t {
                if (net) {
                    if (kc == 1) return 1ull;
                    const int32_t d = lmx - T.lst_b[ci];
                    const int64_t E = d < kEtabLds ? (int64_t)etab[d] : 0;
                    const double qq = (1.0 - a.mix_alpha) * (double)E / (double)Ssum + a.mix_alpha / (double)kc;
                    const double rr = rint(16777216.0 * qq);
                    return rr >= 1.0 ? (uint64_t)rr : 1ull;
                }
                if (kc == 1 || uniform) return 1ull;
                const float s = a.scaled ? bv * T.scale(y) : bv;
                const float rr = rintf((s / smax) * 16777216.0f);
                return rr >= 1.0f ? (uint64_t)rr : 1ull;
            };
            int32_t cbase = 0;
            for (int32_t base = vb; base < ve; base += kWave) {
                const int32_t p = base + l;
                uint64_t w = 0;
                bool c0 = false;
                int32_t y = 0, e = 0;
                float bv = 0.0f;
                if (p < ve) {
                    T.entry(v_row, p, y, e, bv);
                    c0 = T.active(y) && !T.removed(e);
                }
                const uint64_t msk = ballot(c0);
                if (c0) w = weight_of(y, bv, cbase + rank_below(msk));
                cbase += __popcll(msk);
                W += read_lane(wave_incl_scan_add_u32((uint32_t)w), kWave - 1);
            }
            const uint64_t j = kc > 1 ? lemire_from(rand64(a.seed, k, a.b, (uint32_t)t, 0u), W, a.seed, k, a.b, (uint32_t)t) : 0ull;
            uint64_t pre = 0;
            cbase = 0;
            for (int32_t base = vb; base < ve; base += kWave) {
                const int32_t p = base + l;
                uint64_t w = 0;
                int32_t y = 0, e = 0;
                float bv = 0.0f;
                bool c0 = false;
                if (p < ve) {
                    T.entry(v_row, p, y, e, bv);
                    c0 = T.active(y) && !T.removed(e);
                }
                const uint64_t msk = ballot(c0);
                if (c0) w = weight_of(y, bv, cbase + rank_below(msk));
                cbase += __popcll(msk);
                const uint64_t incl = wave_incl_scan_add_u32((uint32_t)w) + pre;
                const uint64_t hm = ballot(w != 0 && incl > j && incl - w <= j);
                if (hm) {
                    const int src = __ffsll((unsigned long long)hm) - 1;
                    u = read_lane(y, src);
                    b_vu = read_lane(bv, src);
                    w_u = read_lane(w, src);
                    break;
                }
                pre = read_lane(incl, kWave - 1);
            }
            if (kc == 1) W = w_u;
            if (u >= 0) d_u = T.deg[u];
        }
        if (u < 0) {  // no candidate matched the draw: internal inconsistency
            if (l == 0) atomicOr(a.err, 2u);
            alive = false;
            break;
        }
        // u's leaf group needs a new minimum after the step when u is that
        // minimum (and the group is not v's, refreshed from the selection's
        // leaves): read its leaves now, before this step's stores, so the
        // refresh needs no memory round trip. Stale values are harmless:
        // the step only lowers degrees (the new ones are known) and retires
        // v and u (masked).
        const int32_t gu = u >> 8;
        const uint32_t l1u_before = T.level(0)[gu];
        const bool refresh_u = gu != gsel && d_u <= l1u_before;
        uint2 uleaves = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
        if (refresh_u && gsel >= 0) uleaves = recast<const uint2>(T.deg + 256 * gu)[l];

        // ---- importance correction X <- X * B_vu / q(u|v), extended exponent
        {
            const double factor = (double)b_vu * ((double)W / (double)w_u);
            int e2;
            mant = frexp(mant * factor, &e2);
            ex += e2;
        }
        const int32_t rho = v_row ? v : u;
        const int32_t gam = v_row ? u : v;  // column vertex id
        const double z = net ? (double)w_u / (double)W : (double)T.scale(rho) * (double)T.scale(gam);
        if (path && l == 0) { path[2 * t] = v; path[2 * t + 1] = u; }
        h = splitmix_fold(h, ((uint64_t)(uint32_t)v << 32) | (uint32_t)u);

        // ---- N_t(u) \ {v}
        int32_t ub, ue;
        // learned: u's list, its neighbours and their degrees were read for
        // the features (nothing has changed since); move them into place
        const bool from_cache = net && nc.valid && u_lane >= 0;
        int32_t u_off = 0;
        if (from_cache) u_off = read_lane(nc.off, u_lane);
        if (u_lane >= 0) {
            ub = u_ub;
            ue = u_ue;
        } else {
            T.list(u, ub, ue);
        }
        const bool fast_u = ue - ub <= kWave;
        const bool u_row = u < n;
        int32_t by = -1;
        uint32_t bd = 0;
        bool take = false;
        int32_t kb = 0;
        if (from_cache) {
            const int srcl = (u_off + l) & (kWave - 1);
            const int32_t w2 = __shfl(nc.w, srcl);
            const uint32_t d2 = __shfl(nc.dw, srcl);
            const bool live2 = __shfl((int)nc.live, srcl) != 0;
            if (ub + l < ue) {
                by = w2;
                bd = d2;
                take = by != v && live2;
            }
            kb = __popcll(ballot(take));
        } else if (fast_u) {
            const int32_t p = ub + l;
            if (p < ue) {
                int32_t e; float bv;
                T.entry(u_row, p, by, e, bv);
                bd = T.deg[by];
                take = by != v && bd != kRetired && !T.removed(e);
            }
            kb = __popcll(ballot(take));
        } else {
            for (int32_t base = ub; base < ue; base += kWave) {
                const int32_t p = base + l;
                bool tk = false;
                int32_t y = 0;
                if (p < ue) {
                    int32_t e; float bv;
                    T.entry(u_row, p, y, e, bv);
                    tk = y != v && T.active(y) && !T.removed(e);
                }
                const uint64_t msk = ballot(tk);
                if (tk) T.lst_b[kb + rank_below(msk)] = y;
                kb += __popcll(msk);
            }
        }
        wave_fence();

        // ---- B^(t+1) = B^(t) \ {v,u}: retire both, lower their neighbours
        if (l == 0) {
            T.deg[v] = kRetired;
            T.deg[u] = kRetired;
            if (OWN) { T.rec[v].s = -1.0f; T.rec[u].s = -1.0f; }
        }
        uint32_t dec_min_g = 0xFFFFFFFFu;  // lowest new degree inside v's leaf group
        uint32_t dec_min_u = 0xFFFFFFFFu;  // ... and inside u's
        auto lower = [&](int32_t y, uint32_t nd) {
            T.deg[y] = (uint16_t)nd;
            T.tree_lower(y, nd);
            if ((y >> 8) == gsel && nd < dec_min_g) dec_min_g = nd;
            if ((y >> 8) == gu && nd < dec_min_u) dec_min_u = nd;
        };
        if (fast_v) {
            if (cand && cy != u) lower(cy, cd - 1u);
        } else {
            for (int32_t idx = l; idx < kc; idx += kWave) {
                const int32_t y = T.lst_a[idx];
                if (y == u) continue;
                lower(y, (uint32_t)T.deg[y] - 1u);
            }
        }
        if (fast_u) {
            if (take) lower(by, bd - 1u);
        } else {
            for (int32_t idx = l; idx < kb; idx += kWave) {
                const int32_t y = T.lst_b[idx];
                lower(y, (uint32_t)T.deg[y] - 1u);
            }
        }
        work.scan += (uint64_t)(ve - vb) + (uint64_t)(ue - ub);
        work.scan_v += (uint64_t)(ve - vb);
        work.dec += (uint64_t)(kc - 1 + kb);
        wave_fence();
        // refresh the group of v from the leaves read at selection time
        if (gsel >= 0) {
            const int32_t base_id = 256 * gsel + 4 * l;
            uint32_t d0 = gleaves.x & 0xFFFFu, d1 = gleaves.x >> 16, d2 = gleaves.y & 0xFFFFu,
                     d3 = gleaves.y >> 16;
            if (base_id == v || base_id == u) d0 = 0xFFFFu;
            if (base_id + 1 == v || base_id + 1 == u) d1 = 0xFFFFu;
            if (base_id + 2 == v || base_id + 2 == u) d2 = 0xFFFFu;
            if (base_id + 3 == v || base_id + 3 == u) d3 = 0xFFFFu;
            uint32_t mm = min(min(d0, d1), min(d2, d3));
            mm = wave_min_u32(min(mm, dec_min_g));
            if (l == 0) T.level(0)[gsel] = mm;
            wave_fence();
            // the upper levels hold every lower value already (atomic
            // minima of the decrements); they change only if the group's
            // minimum rose above the selected degree
            if (mm > m_sel) T.refresh_upper(gsel);
            if (refresh_u) {
                const int32_t ub_id = 256 * gu + 4 * l;
                uint32_t e0 = uleaves.x & 0xFFFFu, e1 = uleaves.x >> 16, e2 = uleaves.y & 0xFFFFu,
                         e3 = uleaves.y >> 16;
                if (ub_id == u) e0 = 0xFFFFu;
                if (ub_id + 1 == u) e1 = 0xFFFFu;
                if (ub_id + 2 == u) e2 = 0xFFFFu;
                if (ub_id + 3 == u) e3 = 0xFFFFu;
                uint32_t mu = min(min(e0, e1), min(e2, e3));
                mu = wave_min_u32(min(mu, dec_min_u));
                if (l == 0) T.level(0)[gu] = mu;
                wave_fence();
                if (mu > d_u) T.refresh_upper(gu);
            }
        } else {
            T.tree_refresh(v);
            if (refresh_u) T.tree_refresh(u);
        }
        steps = t + 1;
        track = track * z;
        if (t + 1 >= n) break;

        // child dead end. Under minimum-degree selection without inner SK or
        // DM nothing runs before the next selection, which then picks a
        // vertex of degree 0 and stops the trajectory at the same point with
        // the same counters, so the check is left to it.
        const bool next_select_checks = (SK == kSkNone || SK == kSkLearned) && !DM && a.vertex_rule != 1;
        if (!next_select_checks && T.global_min() == 0) { alive = false; break; }

        // ---- P_DM: support filtering of the child
        bool ran_dm = false;
        if (DM) {
            bool run_dm = false;
            if (a.dm_policy == kDmAll) run_dm = true;
            else if (a.dm_policy == kDmThrs && z < a.theta_th) run_dm = true;
            else if (a.dm_policy == kDmTrck && track < a.theta_tr) run_dm = true;
            if (run_dm) {
                n_dm += 1;
                const uint64_t c0 = wall_ticks();
                uint64_t dm_ex = 0;
                const bool ok = T.dm_match(dm_ex);
                if (!ok) {
                    work.dm_entries += read_lane(dm_ex, 0);
                    work.t_dm += wall_ticks() - c0;
                    alive = false;
                    break;
                }
                uint64_t scc_ex = 0;
                if (!T.scc_colouring(scc_ex)) {
                    if (l == 0) T.scc_tarjan(dm_ex);
                    wave_fence();
                }
                work.dm_entries += read_lane(dm_ex, 0) + scc_ex;
                T.dm_apply();
                work.t_dm += wall_ticks() - c0;
                track = 1.0;
                ran_dm = true;
            }
        }

        // ---- P_SK on the child
        if (SK == kSkFixed || SK == kSkAdaptive) {
            int nit = a.K;
            if (SK == kSkAdaptive) {
                double want = ceil((1.0 - z) * (double)a.K);
                if (!(want > 0.0)) want = 0.0;
                if (want > (double)a.K) want = (double)a.K;
                nit = (int)want;
            }
            const uint64_t c0 = wall_ticks();
            for (int it = 0; it < nit; ++it) T.sk_sweep();
            work.t_sk += wall_ticks() - c0;
            n_sweeps += nit;
            work.sweeps += (uint64_t)nit;
        } else if (SK == kSkLocal || SK == kSkLearnedGated) {
            // Local: every step.  Gated learned: after a step whose sampled
            // probability fell below theta_th or after inner DM, and then the
            // next step draws from the scaled proposal.
            bool repair = true;
            if (SK == kSkLearnedGated) {
                repair = z < a.theta_th || ran_dm;
                fb = repair;
            }
            if (repair) {
                const uint64_t c0 = wall_ticks();
                // rho_list = N_t(rho)\{gam} (columns), gam_list = N_t(gam)\{rho} (rows)
                if (fast_v && fast_u) {
                    const int32_t other_v = (cand && cy != u) ? cy : -1;
                    const int32_t other_u = take ? by : -1;
                    if (v_row) local_repair_lanes(T, other_v, other_u, k, t, work);
                    else local_repair_lanes(T, other_u, other_v, k, t, work);
                } else {
                    if (fast_v) {
                        const uint64_t msk = ballot(cand);
                        if (cand) T.lst_a[rank_below(msk)] = cy;
                    }
                    if (fast_u) {
                        const uint64_t msk = ballot(take);
                        if (take) T.lst_b[rank_below(msk)] = by;
                    }
                    wave_fence();
                    if (v_row) local_repair_lists(T, T.lst_a, kc, u, T.lst_b, kb, -1, k, t, work);
                    else local_repair_lists(T, T.lst_b, kb, -1, T.lst_a, kc, u, k, t, work);
                }
                work.t_loc += wall_ticks() - c0;
                n_local += 1;
            }
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
    work.t_all += wall_ticks() - t_begin;
    wave_fence();
}

// A launch runs the trajectories of one or more matrices (same schedule).
// Work items are numbered over the matrices taken in `order` (most
// expensive first, for a short tail); item q maps to matrix order[i] with
// item_off[i] <= q < item_off[i+1] and trajectory q - item_off[i].
struct BatchArgs {
    const TrajArgs *mats;     // [count] per-matrix argument blocks (device)
    const int32_t *order;     // [count] processing order
    const int64_t *item_off;  // [count+1] prefix sums of trajectory counts, in order
    int32_t count;
    int64_t total;
    uint32_t *work_next;      // item counter (zeroed before launch)
    unsigned long long *work_totals;  // [12]: scanned, decrements, local entries, local values, sweeps,
                                      // tiles, scanned at the selected vertex, wave ticks in trajectories,
                                      // in full SK, in inner DM, in local repairs, DM entries examined
    char *hbm_state;          // base of the per-wave HBM slots, or nullptr if every matrix is LDS tier
    uint64_t hbm_stride;
    int32_t lds_tree_bytes;   // LDS bytes reserved per wave for min-tree nodes
    int32_t lds_mlp_bytes;    // LDS bytes per wave for the network's tiles (learned)
    int32_t lds_state_bytes;  // bytes of LDS state per wave (largest LDS-tier matrix), or 0
    int32_t waves_per_block;
    const float *mlp;         // learned proposal parameters (staged per block), or nullptr
    const int64_t *etab;      // learned proposal's softmax table (staged per block)
    // statistics reduced by the kernel's last block (the learned row
    // kernel), or nullptr: a separate reduction kernel follows
    const ReduceSeg *seg;
    DevStats *stats;
    uint32_t *blocks_done;    // finished-block counter (zeroed before launch)
};

constexpr int kMlpWaveBytes = (int)sizeof(WaveScratch);
constexpr int kMlpBlockBytes = ((int)sizeof(LearnedLds) + 15) / 16 * 16;

// The argument blocks live in device memory (uniform fields become scalar
// loads; no private copy of a by-value parameter is needed).
template <int SK, bool DM, bool WT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((SK == kSkNone || !DM) ? 4 : 1, 8)))
traj_kernel(const BatchArgs *__restrict__ bp) {
    const PE_G BatchArgs &B = *gptr(bp);
    extern __shared__ __align__(16) char smem[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));  // wave-uniform
    // block: [network weights (learned)] then per wave [tree | network tiles | state]
    LearnedLds *lrn = reinterpret_cast<LearnedLds *>(smem);
    MlpLds *mlpw = &lrn->net;
    char *waves = smem + (learned_kind(SK) ? kMlpBlockBytes : 0);
    if (learned_kind(SK)) {
        stage_weights<true>(mlpw, B.mlp);
        for (int i = threadIdx.x; i < kEtabLds; i += blockDim.x) lrn->etab[i] = (uint32_t)B.etab[i];
        __syncthreads();
    }
    const size_t per_wave = (size_t)B.lds_tree_bytes + (size_t)B.lds_mlp_bytes + (size_t)B.lds_state_bytes;
    char *mine = waves + (size_t)wave * per_wave;
    uint32_t *tree = reinterpret_cast<uint32_t *>(mine);
    WaveScratch *scr = reinterpret_cast<WaveScratch *>(mine + B.lds_tree_bytes);
    // per-matrix tier: the wave's LDS slot (sized for the largest LDS-tier
    // matrix of the launch) or its HBM slot
    char *lds_state = mine + B.lds_tree_bytes + B.lds_mlp_bytes;
    char *hbm_state = B.hbm_state ? B.hbm_state + ((uint64_t)blockIdx.x * B.waves_per_block + wave) * B.hbm_stride
                                  : nullptr;
    Work work;
    for (;;) {
        uint32_t q = 0;
        if (lane_id() == 0) q = atomicAdd(gptr(B.work_next), 1u);
        q = read_lane(q, 0);
        if ((int64_t)q >= B.total) break;
        // matrix of item q: last i with item_off[i] <= q
        int32_t lo = 0, hi = B.count - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (gptr(B.item_off)[mid] <= (int64_t)q) lo = mid; else hi = mid - 1;
        }
        const PE_G TrajArgs &a = gptr(B.mats)[gptr(B.order)[lo]];
        const int64_t k = (int64_t)q - gptr(B.item_off)[lo];
        if (a.lds_tier) {
            const Traj<OwnRC<SK>::value, DM, WT, kAsLds> T(a, lds_state, tree);
            run_trajectory<SK, DM, WT, kAsLds>(a, T, k, work, lrn, scr);
        } else {
            const Traj<OwnRC<SK>::value, DM, WT, kAsGlobal> T(a, hbm_state, tree);
            run_trajectory<SK, DM, WT, kAsGlobal>(a, T, k, work, lrn, scr);
        }
    }
    if (lane_id() == 0 && B.work_totals) {
        atomicAdd(B.work_totals + 0, (unsigned long long)work.scan);
        atomicAdd(B.work_totals + 1, (unsigned long long)work.dec);
        atomicAdd(B.work_totals + 2, (unsigned long long)work.loc_entries);
        atomicAdd(B.work_totals + 3, (unsigned long long)work.loc_values);
        atomicAdd(B.work_totals + 4, (unsigned long long)work.sweeps);
        atomicAdd(B.work_totals + 5, (unsigned long long)work.mlp_tiles);
        atomicAdd(B.work_totals + 6, (unsigned long long)work.scan_v);
        atomicAdd(B.work_totals + 7, (unsigned long long)work.t_all);
        atomicAdd(B.work_totals + 8, (unsigned long long)work.t_sk);
        atomicAdd(B.work_totals + 9, (unsigned long long)work.t_dm);
        atomicAdd(B.work_totals + 10, (unsigned long long)work.t_loc);
        atomicAdd(B.work_totals + 11, (unsigned long long)work.dm_entries);
    }
}

}  // namespace pe
