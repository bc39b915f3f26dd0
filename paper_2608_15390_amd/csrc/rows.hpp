// rows.hpp -- four trajectories per wave: each 16-lane row of a wave64 runs
// its own trajectory of the plain estimator (Alg. 2 with minimum-degree
// selection, the outer scaling only: no inner SK, no inner support filter).
//
// Large sparse matrices give short candidate lists (the minimum-degree
// vertex has a handful of neighbours; average lists hold ~8 entries), so a
// full wave per trajectory leaves most lanes idle while every step waits
// on a chain of dependent memory accesses.  Rows let one instruction serve
// four trajectories: four times the memory-level parallelism per wave and a
// quarter of the instructions per trajectory step.  Row-wide reductions and
// scans are DPP row shifts and row broadcasts.
//
// Results are identical to traj_kernel's for the same (seed, trajectory,
// matrix index): the step is the same sequence of integer decisions and
// FP64 operations; only the lane layout differs.
#pragma once
#include "traj.hpp"

namespace pe {

constexpr int kRowLanes = 16;

__device__ __forceinline__ int row_id() { return lane_id() >> 4; }
__device__ __forceinline__ int row_lane() { return lane_id() & 15; }

// this row's 16 bits of a wave mask
__device__ __forceinline__ uint32_t row_bits(uint64_t m) { return (uint32_t)(m >> (16 * row_id())) & 0xFFFFu; }

// lane L of each row, broadcast within the row
template <int L>
__device__ __forceinline__ uint32_t row_bcast(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + L, 0xF, 0xF, false);
}
template <int L>
__device__ __forceinline__ uint64_t row_bcast64(uint64_t v) {
    return ((uint64_t)row_bcast<L>((uint32_t)(v >> 32)) << 32) | row_bcast<L>((uint32_t)v);
}
template <int L>
__device__ __forceinline__ int32_t row_bcast_i(int32_t v) { return (int32_t)row_bcast<L>((uint32_t)v); }
template <int L>
__device__ __forceinline__ float row_bcast_f(float v) { return __uint_as_float(row_bcast<L>(__float_as_uint(v))); }

// lane src (per row, 0..15) of each row; src may differ between rows
template <typename T>
__device__ __forceinline__ T row_read(T v, int src) { return __shfl(v, 16 * row_id() + src); }

// inclusive scan within each row, op with identity id
template <typename Op>
__device__ __forceinline__ uint32_t row_scan_u32(uint32_t x, uint32_t id, Op op) {
    x = op(x, dpp<kRowShr1>(id, x));
    x = op(x, dpp<kRowShr2>(id, x));
    x = op(x, dpp<kRowShr4>(id, x));
    x = op(x, dpp<kRowShr8>(id, x));
    return x;
}
__device__ __forceinline__ uint32_t row_min_u32(uint32_t x) {
    return row_bcast<15>(row_scan_u32(x, 0xFFFFFFFFu, [](uint32_t a, uint32_t b) { return b < a ? b : a; }));
}
__device__ __forceinline__ int32_t row_max_i32(int32_t x) {
    return (int32_t)row_bcast<15>(row_scan_u32((uint32_t)x, 0x80000000u, [](uint32_t a, uint32_t b) {
        return (int32_t)b > (int32_t)a ? b : a;
    }));
}
__device__ __forceinline__ float row_max_f32(float x) {
    const uint32_t r = row_scan_u32(__float_as_uint(x), __float_as_uint(-__builtin_huge_valf()),
                                    [](uint32_t a, uint32_t b) {
                                        return __uint_as_float(b) > __uint_as_float(a) ? b : a;
                                    });
    return __uint_as_float(row_bcast<15>(r));
}
// exact 64-bit inclusive scan within each row
__device__ __forceinline__ uint64_t row_incl_scan_u64(uint64_t x) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    auto step = [&](uint32_t ylo, uint32_t yhi) {
        const uint32_t s = lo + ylo;
        hi = hi + yhi + (s < lo ? 1u : 0u);
        lo = s;
    };
    step(dpp<kRowShr1>(0u, lo), dpp<kRowShr1>(0u, hi));
    step(dpp<kRowShr2>(0u, lo), dpp<kRowShr2>(0u, hi));
    step(dpp<kRowShr4>(0u, lo), dpp<kRowShr4>(0u, hi));
    step(dpp<kRowShr8>(0u, lo), dpp<kRowShr8>(0u, hi));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t row_sum_u64(uint64_t x) { return row_bcast64<15>(row_incl_scan_u64(x)); }
// 32-bit inclusive prefix sum within each row (16 proposal weights of at
// most 2^24 + 1 fit)
__device__ __forceinline__ uint32_t row_incl_scan_add_u32(uint32_t x) {
    return row_scan_u32(x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}
__device__ __forceinline__ int32_t row_excl_scan_i32(int32_t x, int32_t &total) {
    const uint32_t incl = row_scan_u32((uint32_t)x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
    total = (int32_t)row_bcast<15>(incl);
    return (int32_t)incl - x;
}
// last lane of the row whose exclusive offset is <= f (offsets non-decreasing)
__device__ __forceinline__ int row_owner(int32_t f, int32_t off) {
    int lo = 0;
#pragma unroll
    for (int step = 8; step > 0; step >>= 1) {
        const int c = lo + step;
        const int32_t oc = row_read(off, c < kRowLanes ? c : kRowLanes - 1);
        if (c < kRowLanes && oc <= f) lo = c;
    }
    return lo;
}

// the scaling value of an unscaled matrix, at a fixed global address
__device__ const float kUnitScale = 1.0f;

// One row's trajectory state and views (all values uniform within the row).
// L0AS: address space of the min-tree's lowest internal level (LDS, or the
// row's state slot in global memory); the levels above it are in LDS.  Each
// level is reached through a pointer of its own address space, so no tree
// access becomes a flat instruction (a flat access also holds up every later
// wait for LDS results until its memory round trip ends).
template <int L0AS>
struct RowTraj {
    const PE_C TrajArgs &a;
    GMat M;
    PE_G uint16_t *deg;
    PE_G int32_t *lst_a, *lst_b;
    PE_L uint32_t *tree;          // the internal levels kept in LDS
    int32_t n;
    as_ptr<L0AS, uint32_t> lvl0;  // the lowest internal level

    // node i of internal level k: read, write, atomic minimum
    __device__ uint32_t node(int k, int32_t i) const { return k == 0 ? lvl0[i] : tree[a.tree.off[k] + i]; }
    __device__ void set_node(int k, int32_t i, uint32_t v) const {
        if (k == 0) lvl0[i] = v;
        else tree[a.tree.off[k] + i] = v;
    }
    __device__ void min_node(int k, int32_t i, uint32_t v) const {
        if (k == 0) atomicMin(lvl0 + i, v);
        else atomicMin(tree + a.tree.off[k] + i, v);
    }
    // nodes base .. base + 3 of level k (base a multiple of 4), read by every
    // lane with one choice of address space for all four, so the reads issue
    // together; values past the level's end are unspecified (callers mask
    // them).  Level 0 in the state slot is padded to whole 64-node blocks and
    // 256-byte aligned: one 16-byte load.
    __device__ void nodes4(int k, int32_t base, uint32_t (&w)[4]) const {
        if constexpr (L0AS == kAsGlobal) {
            if (k == 0) {
                const uint4 q = *reinterpret_cast<const PE_G uint4 *>(lvl0 + base);
                w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
                return;
            }
        }
        const int32_t last = a.tree.size[k] - 1;
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = node(k, base + i < last ? base + i : last);
    }
    // The accessors below pick their array by a select rather than a branch:
    // lanes of one row may read rows and columns alike, and a load in each
    // arm of a divergent branch would be waited for at the join before the
    // next load could issue.
    __device__ void list(int32_t x, int32_t &b, int32_t &e) const {
        const bool row = x < n;
        const PE_G int32_t *ptr = row ? M.row_ptr : M.col_ptr;
        const int32_t i = row ? x : x - n;
        b = ptr[i];
        e = ptr[i + 1];
    }
    template <bool WT>
    __device__ void entry(bool row, int32_t p, int32_t &y, float &bv) const {
        y = (row ? M.col_idx : M.row_idx)[p] + (row ? n : 0);
        bv = WT ? (row ? M.val : M.val_csc)[p] : 1.0f;
    }
    __device__ float scale0(int32_t y) const {
        if (y < n) return a.r0 ? gptr(a.r0)[y] : 1.0f;
        return a.c0 ? gptr(a.c0)[y - n] : 1.0f;
    }
    // the outer scaling of a vertex known to be a row / a column, read
    // without a branch (an unscaled matrix reads a constant 1)
    __device__ float scale_row(int32_t x) const { return *(a.r0 ? gptr(a.r0) + x : gptr(&kUnitScale)); }
    __device__ float scale_col(int32_t x) const { return *(a.c0 ? gptr(a.c0) + (x - n) : gptr(&kUnitScale)); }
    __device__ void tree_lower(int32_t x, uint32_t d) const {
        min_node(0, x >> 8, d);
        if (a.tree.levels > 1) min_node(1, x >> 14, d);
        if (a.tree.levels > 2) min_node(2, x >> 20, d);
    }
    // min over nodes [64 h, 64 h + 64) of level k (4 per lane)
    __device__ uint32_t block_min(int k, int32_t h) const {
        const int32_t base = 64 * h + 4 * row_lane();
        uint32_t w[4];
        nodes4(k, base, w);
        uint32_t m = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (base + i < a.tree.size[k]) m = w[i] < m ? w[i] : m;
        return row_min_u32(m);
    }
    __device__ void refresh_upper(int32_t g) const {
        for (int k = 1; k < a.tree.levels; ++k) {
            const int32_t h = g >> 6;
            const uint32_t m = block_min(k - 1, h);
            if (row_lane() == 0) set_node(k, h, m);
            wave_fence();
            g = h;
        }
    }
    // this lane's 16 leaves of group g (vertices 256 g + 16 rl .. + 15)
    __device__ void load_leaves(int32_t g, uint4 &q0, uint4 &q1) const {
        const auto p = recast<const uint4>(deg + 256 * g + 16 * row_lane());
        q0 = p[0];
        q1 = p[1];
    }
    __device__ uint32_t global_min() const {
        const int top = a.tree.levels - 1;
        return block_min(top, 0);
    }
};

__device__ __forceinline__ uint32_t min16(const uint4 &q0, const uint4 &q1) {
    uint32_t m = 0xFFFFFFFFu;
    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t lo = w[i] & 0xFFFFu, hi = w[i] >> 16;
        m = lo < m ? lo : m;
        m = hi < m ? hi : m;
    }
    return m;
}

// first leaf index (0..15) of this lane equal to d, or 16
__device__ __forceinline__ int first16(const uint4 &q0, const uint4 &q1, uint32_t d) {
    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    int j = 16;
#pragma unroll
    for (int i = 7; i >= 0; --i) {
        if ((w[i] >> 16) == d) j = 2 * i + 1;
        if ((w[i] & 0xFFFFu) == d) j = 2 * i;
    }
    return j;
}

// min over this lane's 16 leaves, vertices in `skip_a`, `skip_b` left out
__device__ __forceinline__ uint32_t min16_skip(const uint4 &q0, const uint4 &q1, int32_t base, int32_t skip_a,
                                               int32_t skip_b) {
    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    uint32_t m = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int32_t x0 = base + 2 * i, x1 = x0 + 1;
        const uint32_t lo = (x0 == skip_a || x0 == skip_b) ? 0xFFFFu : (w[i] & 0xFFFFu);
        const uint32_t hi = (x1 == skip_a || x1 == skip_b) ? 0xFFFFu : (w[i] >> 16);
        m = lo < m ? lo : m;
        m = hi < m ? hi : m;
    }
    return m;
}

}  // namespace pe

namespace pe {

// scaled proposal weight of one candidate (Eq. q, integerised)
__device__ __forceinline__ uint64_t scaled_weight(float s, float smax, bool uniform, int32_t kc) {
    if (kc == 1 || uniform) return 1ull;
    const float rr = rintf((s / smax) * 16777216.0f);
    return rr >= 1.0f ? (uint64_t)rr : 1ull;
}

// the plain estimator (Alg. 2 with minimum degree, outer scaling only),
// four trajectories per wave; WT: weighted entries
template <bool WT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
traj_rows_kernel(const BatchArgs *__restrict__ bp) {
    const PE_C BatchArgs &B = *cptr(bp);
    const PE_C TrajArgs &a = cptr(B.mats)[0];
    extern __shared__ __align__(16) char smem[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int r = row_id(), rl = row_lane();
    const int32_t n = a.A.n;
    char *mine = smem + (size_t)wave * 4 * (size_t)B.lds_tree_bytes;
    PE_G char *state = gptr(B.hbm_state) + (((uint64_t)blockIdx.x * B.waves_per_block + wave) * 4 + r) * B.hbm_stride;
    const auto &L = a.st;
    PE_L uint32_t *tree_row = (PE_L uint32_t *)reinterpret_cast<uint32_t *>(mine + (size_t)r * B.lds_tree_bytes);
    const RowTraj<kAsLds> T{a, GMat(a.A), recast<uint16_t>(state + L.deg), recast<int32_t>(state + L.lst_a),
                            recast<int32_t>(state + L.lst_b), tree_row, n, tree_row + a.tree.off[0]};
    Work work;
    // per-row trajectory registers (uniform within the row)
    int phase = 0;  // 0 claim, 1 running, 2 no more work
    int64_t q = 0;
    uint32_t k = 0;
    int32_t t = 0, steps = 0;
    double mant = 1.0;
    int64_t ex = 0;
    uint64_t h = 0;
    bool alive = false;

    for (;;) {
        // ---- claim and initialise (rows that finished their trajectory)
        if (phase == 0) {
            uint32_t qq = 0;
            if (rl == 0) qq = atomicAdd(gptr(B.work_next), 1u);
            qq = row_bcast<0>(qq);
            if ((int64_t)qq >= B.total) {
                phase = 2;
            } else {
                phase = 1;
                q = (int64_t)qq;
                k = (uint32_t)(a.first + q);
                t = 0;
                steps = 0;
                mant = 1.0;
                ex = 0;
                h = 0;
                alive = a.ok0 != 0;
                const auto src = gptr(reinterpret_cast<const uint4 *>(a.deg0));
                const auto dst = recast<uint4>(T.deg);
                for (int32_t i = rl; i < a.n_leaf / 8; i += kRowLanes) dst[i] = src[i];
                for (int32_t i = rl; i < a.tree.total; i += kRowLanes) T.tree[i] = gptr(a.tree0)[i];
                wave_fence();
            }
        }
        if (!ballot(phase != 2)) break;
        const bool run = phase == 1 && alive && t < n;
        bool finished = phase == 1 && !run;  // completed or dead at the previous step
        if (run) {
            // ---- minimum-degree selection down the row's min-tree, then the leaf group
            int32_t v = -1, gsel = -1;
            uint4 lq0 = make_uint4(0, 0, 0, 0), lq1 = lq0;  // this lane's 16 leaves of v's group
            uint32_t m_sel = 0;  // the minimum degree at selection
            {
                const int top = a.tree.levels - 1;
                const uint32_t m = T.global_min();
                m_sel = m;
                int32_t g = 0;
                for (int kk = top; kk >= 0 && g >= 0; --kk) {
                    // first node of the block [64 g, 64 g + 64) of level kk holding m
                    const int32_t base = 64 * g + 4 * rl;
                    int j = 4;
                    uint32_t w[4];
                    T.nodes4(kk, base, w);
#pragma unroll
                    for (int i = 3; i >= 0; --i)
                        if (w[i] == m && base + i < a.tree.size[kk]) j = i;
                    const uint32_t bits = row_bits(ballot(j < 4));
                    const int src = __ffs(bits) - 1;
                    const int js = row_read(j, src < 0 ? 0 : src);
                    g = bits ? 64 * g + 4 * src + js : -1;
                }
                if (g >= 0) {
                    T.load_leaves(g, lq0, lq1);
                    const int j = first16(lq0, lq1, m);
                    const uint32_t bits = row_bits(ballot(j < 16));
                    const int src = __ffs(bits) - 1;
                    const int js = row_read(j, src < 0 ? 0 : src);
                    if (bits) {
                        v = 256 * g + 16 * src + js;
                        gsel = g;
                    }
                }
            }
            bool dead = false;
            if (v < 0 || v >= 2 * n) {  // internal inconsistency: report, never index
                if (rl == 0) atomicOr(a.err, 1u);
                dead = true;
            }
            int32_t u = -1, kc = 0, vb = 0, ve = 0, cy = -1;
            uint32_t cd = 0, d_u = 0;
            bool cand = false, fast_v = false;
            float b_vu = 1.0f;
            uint64_t Wt = 0, w_u = 1;
            const bool v_row = v < n;
            if (!dead) {
                T.list(v, vb, ve);
                fast_v = ve - vb <= kRowLanes;
            }
            // ---- candidates, proposal of Eq. (q) (outer scaling), draw
            if (!dead && fast_v) {
                const int32_t p = vb + rl;
                float bv = 0.0f;
                if (p < ve) {
                    T.entry<WT>(v_row, p, cy, bv);
                    cd = T.deg[cy];
                    cand = cd != kRetired;
                }
                kc = __popc(row_bits(ballot(cand)));
                if (kc == 0) {
                    dead = true;
                } else {
                    const float s = a.scaled ? bv * T.scale0(cy) : bv;
                    const float smax = row_max_f32((cand && s > 0.0f) ? s : 0.0f);
                    const bool uniform = !(smax > 0.0f) || __builtin_isinf(smax);
                    const uint64_t w = cand ? scaled_weight(s, smax, uniform, kc) : 0ull;
                    const uint64_t incl = row_incl_scan_add_u32((uint32_t)w);
                    Wt = row_bcast<15>((uint32_t)incl);
                    const uint64_t j = kc > 1 ? lemire_from(rand64(a.seed, k, a.b, (uint32_t)t, 0u), Wt, a.seed, k,
                                                            a.b, (uint32_t)t)
                                              : 0ull;
                    const uint32_t hm = row_bits(ballot(w != 0 && incl > j && incl - w <= j));
                    const int src = hm ? __ffs(hm) - 1 : 0;
                    u = hm ? row_read(cy, src) : -1;
                    b_vu = row_read(bv, src);
                    w_u = row_read(w, src);
                    d_u = row_read(cd, src);
                    if (kc == 1) Wt = w_u;
                }
            } else if (!dead) {
                // long list: candidates into lst_a, weights in passes of 16
                float lmaxf = 0.0f;
                for (int32_t base = vb; base < ve; base += kRowLanes) {
                    const int32_t p = base + rl;
                    bool c0 = false;
                    int32_t y = 0;
                    float bvv = 0.0f;
                    if (p < ve) {
                        T.entry<WT>(v_row, p, y, bvv);
                        c0 = T.deg[y] != kRetired;
                    }
                    const uint32_t msk = row_bits(ballot(c0));
                    if (c0) {
                        T.lst_a[kc + __popc(msk & ((1u << rl) - 1u))] = y;
                        const float s = a.scaled ? bvv * T.scale0(y) : bvv;
                        lmaxf = s > lmaxf ? s : lmaxf;
                    }
                    kc += __popc(msk);
                }
                wave_fence();
                if (kc == 0) {
                    dead = true;
                } else {
                    const float smax = row_max_f32(lmaxf);
                    const bool uniform = !(smax > 0.0f) || __builtin_isinf(smax);
                    auto weight_of = [&](int32_t y, float bvv) -> uint64_t {
                        const float s = a.scaled ? bvv * T.scale0(y) : bvv;
                        return scaled_weight(s, smax, uniform, kc);
                    };
                    for (int32_t base = vb; base < ve; base += kRowLanes) {
                        const int32_t p = base + rl;
                        uint64_t w = 0;
                        int32_t y = 0;
                        float bvv = 0.0f;
                        if (p < ve) {
                            T.entry<WT>(v_row, p, y, bvv);
                            if (T.deg[y] != kRetired) w = weight_of(y, bvv);
                        }
                        Wt += row_bcast<15>(row_incl_scan_add_u32((uint32_t)w));
                    }
                    const uint64_t j = kc > 1 ? lemire_from(rand64(a.seed, k, a.b, (uint32_t)t, 0u), Wt, a.seed, k,
                                                            a.b, (uint32_t)t)
                                              : 0ull;
                    uint64_t pre = 0;
                    bool found = false;
                    for (int32_t base = vb; base < ve && !found; base += kRowLanes) {
                        const int32_t p = base + rl;
                        uint64_t w = 0;
                        int32_t y = 0;
                        float bvv = 0.0f;
                        if (p < ve) {
                            T.entry<WT>(v_row, p, y, bvv);
                            if (T.deg[y] != kRetired) w = weight_of(y, bvv);
                        }
                        const uint64_t incl = row_incl_scan_add_u32((uint32_t)w) + pre;
                        const uint32_t hm = row_bits(ballot(w != 0 && incl > j && incl - w <= j));
                        if (hm) {
                            const int src = __ffs(hm) - 1;
                            u = row_read(y, src);
                            b_vu = row_read(bvv, src);
                            w_u = row_read(w, src);
                            found = true;
                        }
                        pre = row_bcast64<15>(incl);
                    }
                    if (kc == 1) Wt = w_u;
                    if (u >= 0) d_u = T.deg[u];
                }
            }
            if (!dead && u < 0) {  // no candidate matched the draw: internal inconsistency
                if (rl == 0) atomicOr(a.err, 2u);
                dead = true;
            }
            if (dead) {
                alive = false;
            } else {
                // importance correction X <- X * B_vu / q(u|v), extended exponent
                {
                    const double factor = (double)b_vu * ((double)Wt / (double)w_u);
                    int e2;
                    mant = frexp(mant * factor, &e2);
                    ex += e2;
                }
                h = splitmix_fold(h, ((uint64_t)(uint32_t)v << 32) | (uint32_t)u);

                // N_t(u) \ {v}
                int32_t ub, ue;
                T.list(u, ub, ue);
                const bool fast_u = ue - ub <= kRowLanes;
                const bool u_row = u < n;
                int32_t by = -1;
                uint32_t bd = 0;
                bool take = false;
                int32_t kb = 0;
                if (fast_u) {
                    const int32_t p = ub + rl;
                    if (p < ue) {
                        float bvv;
                        T.entry<false>(u_row, p, by, bvv);
                        bd = T.deg[by];
                        take = by != v && bd != kRetired;
                    }
                    kb = __popc(row_bits(ballot(take)));
                } else {
                    for (int32_t base = ub; base < ue; base += kRowLanes) {
                        const int32_t p = base + rl;
                        bool tk = false;
                        int32_t y = 0;
                        if (p < ue) {
                            float bvv;
                            T.entry<false>(u_row, p, y, bvv);
                            tk = y != v && T.deg[y] != kRetired;
                        }
                        const uint32_t msk = row_bits(ballot(tk));
                        if (tk) T.lst_b[kb + __popc(msk & ((1u << rl) - 1u))] = y;
                        kb += __popc(msk);
                    }
                }
                const int32_t gu = u >> 8;
                const uint32_t l1u_before = T.lvl0[gu];
                // u's group needs a new minimum when u is it: read its leaves
                // before this step's stores (stale values are only higher;
                // the new degrees and u are patched in below)
                const bool refresh_u = gu != gsel && d_u <= l1u_before;
                uint4 uq0 = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu), uq1 = uq0;
                if (refresh_u) T.load_leaves(gu, uq0, uq1);
                wave_fence();
                // retire v and u, lower their other neighbours
                if (rl == 0) {
                    T.deg[v] = kRetired;
                    T.deg[u] = kRetired;
                }
                uint32_t dec_min_g = 0xFFFFFFFFu, dec_min_u = 0xFFFFFFFFu;
                if (fast_v) {
                    if (cand && cy != u) {
                        const uint32_t nd = cd - 1u;
                        T.deg[cy] = (uint16_t)nd;
                        T.tree_lower(cy, nd);
                        if ((cy >> 8) == gsel) dec_min_g = nd;
                        if ((cy >> 8) == gu) dec_min_u = nd;
                    }
                } else {
                    for (int32_t idx = rl; idx < kc; idx += kRowLanes) {
                        const int32_t y = T.lst_a[idx];
                        if (y == u) continue;
                        const uint32_t nd = (uint32_t)T.deg[y] - 1u;
                        T.deg[y] = (uint16_t)nd;
                        T.tree_lower(y, nd);
                        if ((y >> 8) == gsel && nd < dec_min_g) dec_min_g = nd;
                        if ((y >> 8) == gu && nd < dec_min_u) dec_min_u = nd;
                    }
                }
                if (fast_u) {
                    if (take) {
                        const uint32_t nd = bd - 1u;
                        T.deg[by] = (uint16_t)nd;
                        T.tree_lower(by, nd);
                        if ((by >> 8) == gsel && nd < dec_min_g) dec_min_g = nd;
                        if ((by >> 8) == gu && nd < dec_min_u) dec_min_u = nd;
                    }
                } else {
                    for (int32_t idx = rl; idx < kb; idx += kRowLanes) {
                        const int32_t y = T.lst_b[idx];
                        const uint32_t nd = (uint32_t)T.deg[y] - 1u;
                        T.deg[y] = (uint16_t)nd;
                        T.tree_lower(y, nd);
                        if ((y >> 8) == gsel && nd < dec_min_g) dec_min_g = nd;
                        if ((y >> 8) == gu && nd < dec_min_u) dec_min_u = nd;
                    }
                }
                if (rl == 0) {
                    work.scan += (uint64_t)(ve - vb) + (uint64_t)(ue - ub);
                    work.scan_v += (uint64_t)(ve - vb);
                    work.dec += (uint64_t)(kc - 1 + kb);
                }
                wave_fence();
                // refresh v's group from the leaves read at selection time
                {
                    uint32_t mm = min16_skip(lq0, lq1, 256 * gsel + 16 * rl, v, u);
                    mm = row_min_u32(mm < dec_min_g ? mm : dec_min_g);
                    if (rl == 0) T.lvl0[gsel] = mm;
                    wave_fence();
                    // the upper levels hold every lowered value already
                    if (mm > m_sel) T.refresh_upper(gsel);
                }
                if (refresh_u) {
                    uint32_t mu = min16_skip(uq0, uq1, 256 * gu + 16 * rl, v, u);
                    mu = row_min_u32(mu < dec_min_u ? mu : dec_min_u);
                    if (rl == 0) T.lvl0[gu] = mu;
                    wave_fence();
                    if (mu > d_u) T.refresh_upper(gu);
                }
                steps = t + 1;
                t += 1;
                // a dead child is found by the next selection (a degree-0
                // vertex without candidates), at the same step count
            }
            finished = !alive || t >= n;
        }
        if (phase == 1 && finished) {
            if (rl == 0) {
                const bool done = alive && steps == n;
                if (a.logw) a.logw[q] = done ? log(mant) + (double)ex * kLn2 : -__builtin_huge_val();
                if (a.alive) a.alive[q] = done ? 1 : 0;
                if (a.path_hash) a.path_hash[q] = done ? h : 0ull;
                if (a.counters) {
                    int32_t *cn = a.counters + 4 * q;
                    cn[0] = steps; cn[1] = 0; cn[2] = 0; cn[3] = 0;
                }
            }
            wave_fence();
            phase = 0;
        }
    }
    // launch totals: one atomic per row leader
    if (rl == 0 && B.work_totals) {
        atomicAdd(B.work_totals + 0, (unsigned long long)work.scan);
        atomicAdd(B.work_totals + 1, (unsigned long long)work.dec);
        atomicAdd(B.work_totals + 6, (unsigned long long)work.scan_v);
    }
}

}  // namespace pe
