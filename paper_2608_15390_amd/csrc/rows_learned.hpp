// rows_learned.hpp -- four trajectories per wave for the learned proposal.
//
// Each 16-lane row of a wave64 runs its own trajectory of Alg. 2 with
// minimum-degree selection and the learned per-edge proposal (no inner SK,
// no inner support filter), as the whole-wave learned kernel does, with the
// same sequence of integer decisions and FP64 operations.  What differs is
// the layout: the candidate features of all four rows are packed into
// 16-record matrix-core tiles, so one pass of the network serves four
// trajectory steps, and a wave keeps four trajectories' dependent memory
// chains in flight instead of one.
//
// Per step of a row: selection down the row's min-tree (upper levels in LDS,
// the lowest in LDS or in the row's state slot), whose lowest level names
// the vertex; the candidates of v (one per lane for lists of up to 16 entries, a
// buffer in the state slot beyond that); the neighbourhood statistics of
// every candidate from its flattened residual list (two 16-entry passes per
// memory round trip, the first 32 entries kept in registers so that the
// drawn candidate's list costs no second read); features written to the
// wave's LDS record area; the tiles; logits read back; integer softmax,
// uniform mix and the draw; removal and min-tree maintenance as in the
// plain row kernel (v's leaf group, read at selection, for its refresh).
// When every row is done, the last block to finish reduces the launch's
// statistics.
#pragma once
#include "rows.hpp"

namespace pe {

// per-wave LDS: one round's records (at most 16 per row) as bf16 features,
// and their logits
struct RowNetScratch {
    uint4 x[4 * kRowLanes];          // 8 bf16 features per record
    int32_t logit[4 * kRowLanes];
};
constexpr int kRowNetScratchBytes = ((int)sizeof(RowNetScratch) + 15) / 16 * 16;

// exclusive prefix over the wave's rows of a row-uniform count, and the total
__device__ __forceinline__ int32_t rows_excl_prefix(int32_t c, int32_t &total) {
    const int32_t c0 = read_lane(c, 0), c1 = read_lane(c, 16), c2 = read_lane(c, 32), c3 = read_lane(c, 48);
    total = c0 + c1 + c2 + c3;
    const int r = row_id();
    return r == 0 ? 0 : (r == 1 ? c0 : (r == 2 ? c0 + c1 : c0 + c1 + c2));
}

// The first 32 flattened entries of the row's candidate lists (neighbour
// and its residual degree at the step's start), and each candidate lane's
// offset and length in that flattening.
struct RowNbrCache {
    int32_t w0 = -1, w1 = -1;
    uint32_t d0 = kRetired, d1 = kRetired;
    int32_t off = 0, len = 0, total = 0;
};

// s_u = sum over the residual neighbours w of the lane's candidate y of
// floor(2^20 / deg w) and c2_u = #{w != v : deg w <= 2}: the row's
// candidates' lists flattened over its 16 lanes and summed per owner with a
// segmented scan (integer sums: the result does not depend on the order).
template <bool WT, int L0AS>
__device__ __forceinline__ void row_candidate_stats(const RowTraj<L0AS> &T, bool ok, int32_t y, int32_t yb, int32_t ye,
                                                    int32_t v, uint64_t &s_u, int32_t &c2_u, RowNbrCache &nc) {
    const int rl = row_lane();
    const int32_t len = ok ? ye - yb : 0;
    int32_t total;
    const int32_t off = row_excl_scan_i32(len, total);
    nc.off = off;
    nc.len = len;
    nc.total = total;
    s_u = 0;
    c2_u = 0;
    const int y_row = (ok && y < T.n) ? 1 : 0;
    for (int32_t base = 0; ballot(base < total); base += 2 * kRowLanes) {
        int32_t w[2];
        uint32_t dw[2];
        int own[2];
        bool valid[2];
        // both passes' entries, then both passes' degrees: one round trip each
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int32_t f = base + kRowLanes * i + rl;
            valid[i] = f < total;
            own[i] = row_owner(valid[i] ? f : (total > 0 ? total - 1 : 0), off);
            const int32_t o_off = row_read(off, own[i]);
            const int32_t o_yb = row_read(yb, own[i]);
            const bool o_row = row_read(y_row, own[i]) != 0;
            // every lane loads (an invalid one reads entry 0), then masks:
            // no branch, so both passes' reads issue before either is waited for
            float bv;
            T.template entry<false>(o_row, valid[i] ? o_yb + (f - o_off) : 0, w[i], bv);
            if (!valid[i]) w[i] = -1;
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            // every lane loads (an invalid one reads vertex 0), then masks
            const uint32_t d = (uint32_t)T.deg[valid[i] ? w[i] : 0];
            dw[i] = valid[i] ? d : (uint32_t)kRetired;
        }
        if (base == 0) {
            nc.w0 = w[0]; nc.d0 = dw[0];
            nc.w1 = w[1]; nc.d1 = dw[1];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            uint32_t sv = 0, cv = 0;
            if (valid[i] && dw[i] != kRetired && dw[i] != 0) {
                sv = (1u << 20) / dw[i];
                cv = (w[i] != v && dw[i] <= 2u) ? 1u : 0u;
            }
            const int me = own[i];
            auto seg = [&](uint32_t ys, uint32_t yc, uint32_t yo) {
                if ((int)yo == me) { sv += ys; cv += yc; }
            };
            seg(dpp<kRowShr1>(0u, sv), dpp<kRowShr1>(0u, cv), dpp<kRowShr1>(~0u, (uint32_t)me));
            seg(dpp<kRowShr2>(0u, sv), dpp<kRowShr2>(0u, cv), dpp<kRowShr2>(~0u, (uint32_t)me));
            seg(dpp<kRowShr4>(0u, sv), dpp<kRowShr4>(0u, cv), dpp<kRowShr4>(~0u, (uint32_t)me));
            seg(dpp<kRowShr8>(0u, sv), dpp<kRowShr8>(0u, cv), dpp<kRowShr8>(~0u, (uint32_t)me));
            // each candidate lane takes the value at the last lane of its run
            const int32_t pbase = base + kRowLanes * i;
            const int32_t lo_f = off > pbase ? off : pbase;
            int32_t hi_f = off + len;
            const int32_t cap = pbase + kRowLanes < total ? pbase + kRowLanes : total;
            hi_f = hi_f < cap ? hi_f : cap;
            const int src = hi_f > lo_f ? hi_f - 1 - pbase : 0;
            const uint32_t seg_s = row_read(sv, src);
            const uint32_t seg_c = row_read(cv, src);
            if (hi_f > lo_f) { s_u += seg_s; c2_u += (int32_t)seg_c; }
        }
    }
}

// The row's min-tree with level 1 packed as (degree << 8 | position): each
// level-1 node holds the minimum of its 256 leaves together with the
// position of the first leaf of that degree, so selection names the vertex
// from LDS alone; higher levels hold degrees.
template <int L0AS>
struct ArgTree {
    const RowTraj<L0AS> &T;
    __device__ uint32_t deg_at(int k, uint32_t val) const { return k == 0 ? val >> 8 : val; }
    // a decrement of vertex y to degree nd
    __device__ void lower(int32_t y, uint32_t nd) const {
        T.min_node(0, y >> 8, (nd << 8) | (uint32_t)(y & 255));
        if (T.a.tree.levels > 1) T.min_node(1, y >> 14, nd);
        if (T.a.tree.levels > 2) T.min_node(2, y >> 20, nd);
    }
    // recompute the degree chain above level-1 node g
    __device__ void refresh_upper(int32_t g) const {
        const int rl = row_lane();
        for (int k = 1; k < T.a.tree.levels; ++k) {
            const int32_t h = g >> 6;
            const int32_t base = 64 * h + 4 * rl;
            uint32_t raw[4];
            T.nodes4(k - 1, base, raw);
            uint32_t m = 0xFFFFFFFFu;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t w = deg_at(k - 1, raw[i]);
                if (base + i < T.a.tree.size[k - 1]) m = w < m ? w : m;
            }
            m = row_min_u32(m);
            if (rl == 0) T.set_node(k, h, m);
            wave_fence();
            g = h;
        }
    }
};

// (degree << 8 | position in the group) minimum over this lane's 16 leaves
// (positions 16 rl .. 16 rl + 15 of group g), vertices skip_a, skip_b left out
__device__ __forceinline__ uint32_t argmin16_skip(const uint4 &q0, const uint4 &q1, int32_t g, int32_t skip_a,
                                                  int32_t skip_b) {
    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    const int32_t p0 = 16 * row_lane();
    uint32_t m = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int32_t pa = p0 + 2 * i, pb = pa + 1;
        const int32_t xa = 256 * g + pa, xb = xa + 1;
        const uint32_t lo = (xa == skip_a || xa == skip_b) ? 0xFFFFu : (w[i] & 0xFFFFu);
        const uint32_t hi = (xb == skip_a || xb == skip_b) ? 0xFFFFu : (w[i] >> 16);
        const uint32_t ca = (lo << 8) | (uint32_t)pa, cb = (hi << 8) | (uint32_t)pb;
        m = ca < m ? ca : m;
        m = cb < m ? cb : m;
    }
    return m;
}

// The learned proposal, four trajectories per wave; WT: weighted entries;
// L0AS: where the min-tree's lowest level lives (kAsGlobal: the row's state
// slot, as the launch chose for this matrix; kAsLds: with the levels above).
template <bool WT, int L0AS>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3, 8)))
traj_rows_learned_kernel(const BatchArgs *__restrict__ bp) {
    const PE_C BatchArgs &B = *cptr(bp);
    const PE_C TrajArgs &a = cptr(B.mats)[0];
    extern __shared__ __align__(16) char smem[];
    LearnedLds *lrn = reinterpret_cast<LearnedLds *>(smem);
    stage_weights<true>(&lrn->net, gptr(B.mlp));
    for (int i = threadIdx.x; i < kEtabLds; i += blockDim.x) lrn->etab[i] = (uint32_t)gptr(B.etab)[i];
    __syncthreads();
    const MlpLds *mlpw = &lrn->net;
    const uint32_t *etab = lrn->etab;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int l = lane_id();
    const int r = row_id(), rl = row_lane();
    const int32_t n = a.A.n;
    char *mine = smem + kMlpBlockBytes + (size_t)wave * (4 * (size_t)B.lds_tree_bytes + kRowNetScratchBytes);
    RowNetScratch *scr = reinterpret_cast<RowNetScratch *>(mine + 4 * (size_t)B.lds_tree_bytes);
    PE_G char *state = gptr(B.hbm_state) + (((uint64_t)blockIdx.x * B.waves_per_block + wave) * 4 + r) * B.hbm_stride;
    const auto &L = a.st;
    // the tree's lowest level lives in the row's state slot when the launch
    // moved it there (LDS then holds the levels above, offsets from 0)
    PE_L uint32_t *tree_row = (PE_L uint32_t *)reinterpret_cast<uint32_t *>(mine + (size_t)r * B.lds_tree_bytes);
    as_ptr<L0AS, uint32_t> lvl0;
    if constexpr (L0AS == kAsGlobal) lvl0 = recast<uint32_t>(state + L.lvl0);
    else lvl0 = tree_row + a.tree.off[0];
    const RowTraj<L0AS> T{a, GMat(a.A), recast<uint16_t>(state + L.deg), recast<int32_t>(state + L.lst_a),
                          recast<int32_t>(state + L.lst_b), tree_row, n, lvl0};
    const double alpha = a.mix_alpha;
    const ArgTree<L0AS> AT{T};
    Work work;
    // per-row trajectory registers (uniform within the row)
    int phase = 0;  // 0 claim, 1 running, 2 no more work
    int64_t q = 0;
    uint32_t k = 0;
    int32_t t = 0, steps = 0, k4 = 0;
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
                k4 = 0;
                mant = 1.0;
                ex = 0;
                h = 0;
                alive = a.ok0 != 0;
                const auto src = gptr(reinterpret_cast<const uint4 *>(a.deg0));
                const auto dst = recast<uint4>(T.deg);
                for (int32_t i = rl; i < a.n_leaf / 8; i += kRowLanes) dst[i] = src[i];
                if constexpr (L0AS == kAsGlobal) {
                    for (int32_t i = rl; i < a.tree.size[0]; i += kRowLanes) T.lvl0[i] = gptr(a.tree0a)[i];
                    for (int32_t i = rl; i < a.tree.total; i += kRowLanes)
                        T.tree[i] = gptr(a.tree0a)[a.tree_l1_src + i];
                } else {
                    for (int32_t i = rl; i < a.tree.total; i += kRowLanes) T.tree[i] = gptr(a.tree0a)[i];
                }
                wave_fence();
            }
        }
        if (!ballot(phase != 2)) break;
        const bool run = phase == 1 && alive && t < n;
        bool finished = phase == 1 && !run;  // completed or dead at the previous step
        // every row takes part in the wave-wide parts (the network tiles), so
        // the step runs with predicates; `run` rows do the work
        if (ballot(run)) {
            if (run) k4 = advance_t_grid(k4, t, n);
            // ---- minimum-degree selection down the row's min-tree, then the leaf group
            int32_t v = -1, gsel = -1;
            uint4 lq0 = make_uint4(0, 0, 0, 0), lq1 = lq0;  // this lane's 16 leaves of v's group
            uint32_t m_sel = 0;
            if (run) {
                // the leftmost node of the minimum degree at each level is the
                // row minimum of the code (lane, position) over the matches; at
                // level 1 the code also carries the position of the vertex
                const int top = a.tree.levels - 1;
                const int32_t tb = 4 * rl;
                uint32_t raw4[4], w4[4];
                T.nodes4(top, tb, raw4);
#pragma unroll
                for (int i = 0; i < 4; ++i) w4[i] = tb + i < a.tree.size[top] ? AT.deg_at(top, raw4[i]) : 0xFFFFFFFFu;
                const uint32_t m = row_min_u32(min(min(w4[0], w4[1]), min(w4[2], w4[3])));
                m_sel = m;
                int32_t g = 0;
                uint32_t pos = 0;
                if (top == 0) {
                    uint32_t code = 0xFFFFFFFFu;
#pragma unroll
                    for (int i = 3; i >= 0; --i)
                        if (w4[i] == m) code = ((uint32_t)(tb + i) << 8) | (raw4[i] & 255u);
                    const uint32_t cm = row_min_u32(code);
                    g = (int32_t)(cm >> 8);
                    pos = cm & 255u;
                } else {
                    uint32_t code = 0xFFFFFFFFu;
#pragma unroll
                    for (int i = 3; i >= 0; --i)
                        if (w4[i] == m) code = (uint32_t)(tb + i);
                    g = (int32_t)row_min_u32(code);
                    for (int kk = top - 1; kk >= 0 && g >= 0; --kk) {
                        const int32_t base = 64 * g + tb;
                        code = 0xFFFFFFFFu;
                        uint32_t val[4];
                        T.nodes4(kk, base, val);
#pragma unroll
                        for (int i = 3; i >= 0; --i)
                            if (base + i < a.tree.size[kk] && AT.deg_at(kk, val[i]) == m)
                                code = kk == 0 ? (((uint32_t)(tb + i) << 8) | (val[i] & 255u)) : (uint32_t)(tb + i);
                        const uint32_t cm = row_min_u32(code);
                        if (cm == 0xFFFFFFFFu) {
                            g = -1;
                        } else if (kk == 0) {
                            g = 64 * g + (int32_t)(cm >> 8);
                            pos = cm & 255u;
                        } else {
                            g = 64 * g + (int32_t)cm;
                        }
                    }
                }
                if (g >= 0 && g < a.tree.size[0]) {
                    v = 256 * g + (int32_t)pos;
                    gsel = g;
                    // the group's leaves for its refresh after the step
                    T.load_leaves(g, lq0, lq1);
                }
            }
            bool dead = !run;
            if (run && (v < 0 || v >= 2 * n)) {  // internal inconsistency: report, never index
                if (rl == 0) atomicOr(a.err, 1u);
                dead = true;
            }
            const bool v_row = v < n;
            int32_t vb = 0, ve = 0;
            if (!dead) T.list(v, vb, ve);
            const bool fast_v = ve - vb <= kRowLanes;
            // ---- candidates: one per lane (short lists) or into lst_a
            int32_t kc = 0, cy = -1, cub = 0, cue = 0;
            uint32_t cd = 0;
            bool cand = false;
            float cbv = 0.0f;
            if (!dead && fast_v) {
                const int32_t p = vb + rl;
                if (p < ve) {
                    T.template entry<WT>(v_row, p, cy, cbv);
                    cd = T.deg[cy];
                    T.list(cy, cub, cue);  // issued with the degree load
                    cand = cd != kRetired;
                }
                kc = __popc(row_bits(ballot(cand)));
            } else if (!dead) {
                for (int32_t base = vb; base < ve; base += kRowLanes) {
                    const int32_t p = base + rl;
                    bool c0 = false;
                    int32_t y = 0;
                    float bvv = 0.0f;
                    if (p < ve) {
                        T.template entry<WT>(v_row, p, y, bvv);
                        c0 = T.deg[y] != kRetired;
                    }
                    const uint32_t msk = row_bits(ballot(c0));
                    if (c0) T.lst_a[kc + __popc(msk & ((1u << rl) - 1u))] = y;
                    kc += __popc(msk);
                }
                wave_fence();
            }
            if (!dead && kc == 0) dead = true;
            // ---- network logits of every candidate, in rounds of up to 16
            // candidates per row; a long row's logits go to lst_b
            const bool net = !dead && kc >= 2;
            const int32_t my_rounds = net ? (fast_v ? 1 : (kc + kRowLanes - 1) / kRowLanes) : 0;
            int32_t rounds = my_rounds;
            {
                const int32_t r0 = read_lane(rounds, 0), r1 = read_lane(rounds, 16), r2 = read_lane(rounds, 32),
                              r3 = read_lane(rounds, 48);
                rounds = max(max(r0, r1), max(r2, r3));
            }
            int32_t Lmine = 0;  // fast rows: this lane's candidate's logit
            RowNbrCache nc;
            for (int32_t c = 0; c < rounds; ++c) {
                // this lane's candidate in round c
                bool ok = false;
                int32_t y = -1, yb = 0, ye = 0;
                uint32_t dy = 0;
                int32_t idx = 0;
                if (c < my_rounds) {
                    if (fast_v) {
                        ok = cand;
                        y = cy; yb = cub; ye = cue; dy = cd;
                    } else {
                        idx = kRowLanes * c + rl;
                        if (idx < kc) {
                            ok = true;
                            y = T.lst_a[idx];
                            dy = T.deg[y];
                            T.list(y, yb, ye);
                        }
                    }
                }
                uint64_t su;
                int32_t c2;
                RowNbrCache ncc;
                // the candidate edge's outer scaling, read before the
                // statistics so that its latency overlaps theirs
                const int32_t rho = v_row ? v : y, gam = v_row ? y : v;
                const float s_rho = T.scale_row(ok ? rho : 0), s_gam = T.scale_col(ok ? gam : n);
                row_candidate_stats<WT>(T, ok, y, yb, ye, v, su, c2, ncc);
                if (c == 0) nc = ncc;
                // features into the wave's record area
                const uint32_t okm = row_bits(ballot(ok));
                int32_t all_recs;
                const int32_t rbase = rows_excl_prefix(__popc(okm), all_recs);
                const int32_t rec = rbase + __popc(okm & ((1u << rl) - 1u));
                if (ok) {
                    float x[8];
                    learned_features(x, v_row ? (uint32_t)kc : dy, v_row ? dy : (uint32_t)kc, s_rho, s_gam, k4, v_row,
                                     su, c2);
                    uint4 pk;
                    pk.x = (uint32_t)(uint16_t)to_bf16(x[0]) | ((uint32_t)(uint16_t)to_bf16(x[1]) << 16);
                    pk.y = (uint32_t)(uint16_t)to_bf16(x[2]) | ((uint32_t)(uint16_t)to_bf16(x[3]) << 16);
                    pk.z = (uint32_t)(uint16_t)to_bf16(x[4]) | ((uint32_t)(uint16_t)to_bf16(x[5]) << 16);
                    pk.w = (uint32_t)(uint16_t)to_bf16(x[6]) | ((uint32_t)(uint16_t)to_bf16(x[7]) << 16);
                    scr->x[rec] = pk;
                }
                wave_fence();
                const int ntiles = (all_recs + 15) / 16;
                for (int ti = 0; ti < ntiles; ++ti) {
                    const int ridx = 16 * ti + (l & 15);
                    const int grp = l >> 4;
                    bf16x4 xb = {0, 0, 0, 0};
                    if (grp < 2 && ridx < all_recs) {
                        const uint4 pk = scr->x[ridx];
                        const uint32_t lo = grp == 0 ? pk.x : pk.z, hi = grp == 0 ? pk.y : pk.w;
                        xb[0] = (short)(lo & 0xFFFFu);
                        xb[1] = (short)(lo >> 16);
                        xb[2] = (short)(hi & 0xFFFFu);
                        xb[3] = (short)(hi >> 16);
                    }
                    const float yv = mlp_tile_logit_grid(mlpw, xb);
                    if (l < 16 && ridx < all_recs) {
                        float Lf = rintf(yv * 16.0f);
                        Lf = Lf < -1024.0f ? -1024.0f : (Lf > 1023.0f ? 1023.0f : Lf);
                        scr->logit[ridx] = (int32_t)Lf;
                    }
                }
                if (l == 0) work.mlp_tiles += (uint64_t)ntiles;
                wave_fence();
                if (ok) {
                    const int32_t Lv = scr->logit[rec];
                    if (fast_v) Lmine = Lv;
                    else T.lst_b[idx] = Lv;
                }
                wave_fence();
            }
            // ---- proposal weights (integer softmax, uniform mix) and the draw
            int32_t u = -1, u_src = -1;
            float b_vu = 1.0f;
            uint64_t Wt = 0, w_u = 1;
            uint32_t d_u = 0;
            if (!dead && fast_v) {
                uint64_t w = 0;
                if (kc == 1) {
                    w = cand ? 1ull : 0ull;
                } else {
                    const int32_t lmx = row_max_i32(cand ? Lmine : -2147483647);
                    int64_t E = 0;
                    if (cand) {
                        const int32_t d = lmx - Lmine;
                        E = d < kEtabLds ? (int64_t)etab[d] : 0;
                    }
                    // at most 2^24 per lane: the row's total fits 32 bits
                    const int64_t S = (int64_t)row_bcast<15>(row_incl_scan_add_u32((uint32_t)E));
                    if (cand) {
                        const double qq = (1.0 - alpha) * (double)E / (double)S + alpha / (double)kc;
                        const double rr = rint(16777216.0 * qq);
                        w = rr >= 1.0 ? (uint64_t)rr : 1ull;
                    }
                }
                const uint64_t incl = row_incl_scan_add_u32((uint32_t)w);
                Wt = row_bcast<15>((uint32_t)incl);
                const uint64_t j = kc > 1 ? lemire_from(rand64(a.seed, k, a.b, (uint32_t)t, 0u), Wt, a.seed, k, a.b,
                                                        (uint32_t)t)
                                          : 0ull;
                const uint32_t hm = row_bits(ballot(w != 0 && incl > j && incl - w <= j));
                const int src = hm ? __ffs(hm) - 1 : 0;
                u = hm ? row_read(cy, src) : -1;
                u_src = hm ? src : -1;
                b_vu = row_read(cbv, src);
                w_u = row_read(w, src);
                d_u = row_read(cd, src);
                if (kc == 1) Wt = w_u;
            } else if (!dead) {
                // long list: max and sum over lst_b, then weights in passes of 16
                int32_t lmx = -2147483647;
                uint64_t Ssum = 0;
                if (kc >= 2) {
                    for (int32_t idx = rl; idx < kc + kRowLanes - 1; idx += kRowLanes) {
                        const int32_t Lv = idx < kc ? T.lst_b[idx] : -2147483647;
                        lmx = Lv > lmx ? Lv : lmx;
                    }
                    lmx = row_max_i32(lmx);
                    uint64_t part = 0;
                    for (int32_t idx = rl; idx < kc; idx += kRowLanes) {
                        const int32_t d = lmx - T.lst_b[idx];
                        part += d < kEtabLds ? (uint64_t)etab[d] : 0ull;
                    }
                    Ssum = row_sum_u64(part);
                }
                auto weight_of = [&](int32_t ci) -> uint64_t {
                    if (kc == 1) return 1ull;
                    const int32_t d = lmx - T.lst_b[ci];
                    const int64_t E = d < kEtabLds ? (int64_t)etab[d] : 0;
                    const double qq = (1.0 - alpha) * (double)E / (double)Ssum + alpha / (double)kc;
                    const double rr = rint(16777216.0 * qq);
                    return rr >= 1.0 ? (uint64_t)rr : 1ull;
                };
                for (int32_t ci0 = 0; ci0 < kc; ci0 += kRowLanes) {
                    const int32_t ci = ci0 + rl;
                    const uint64_t w = ci < kc ? weight_of(ci) : 0ull;
                    Wt += row_bcast<15>(row_incl_scan_add_u32((uint32_t)w));
                }
                const uint64_t j = kc > 1 ? lemire_from(rand64(a.seed, k, a.b, (uint32_t)t, 0u), Wt, a.seed, k, a.b,
                                                        (uint32_t)t)
                                          : 0ull;
                uint64_t pre = 0;
                int32_t pick = -1;
                for (int32_t ci0 = 0; ci0 < kc && pick < 0; ci0 += kRowLanes) {
                    const int32_t ci = ci0 + rl;
                    const uint64_t w = ci < kc ? weight_of(ci) : 0ull;
                    const uint64_t incl = row_incl_scan_add_u32((uint32_t)w) + pre;
                    const uint32_t hm = row_bits(ballot(w != 0 && incl > j && incl - w <= j));
                    if (hm) {
                        const int src = __ffs(hm) - 1;
                        pick = ci0 + src;
                        w_u = row_read(w, src);
                    }
                    pre = row_bcast64<15>(incl);
                }
                if (kc == 1) { pick = 0; w_u = 1; Wt = 1; }
                if (pick >= 0) {
                    u = T.lst_a[pick];
                    d_u = T.deg[u];
                    // B_vu: u's entry in v's list
                    for (int32_t base = vb; base < ve; base += kRowLanes) {
                        const int32_t p = base + rl;
                        int32_t y = -1;
                        float bvv = 0.0f;
                        if (p < ve) T.template entry<WT>(v_row, p, y, bvv);
                        const uint32_t hit = row_bits(ballot(p < ve && y == u));
                        if (hit) b_vu = row_read(bvv, __ffs(hit) - 1);
                    }
                }
            }
            if (!dead && u < 0) {  // no candidate matched the draw: internal inconsistency
                if (rl == 0) atomicOr(a.err, 2u);
                dead = true;
            }
            if (run && dead) alive = false;
            if (!dead) {
                // importance correction X <- X * B_vu / q(u|v), extended exponent
                {
                    const double factor = (double)b_vu * ((double)Wt / (double)w_u);
                    int e2;
                    mant = frexp(mant * factor, &e2);
                    ex += e2;
                }
                h = splitmix_fold(h, ((uint64_t)(uint32_t)v << 32) | (uint32_t)u);

                const int32_t gu = u >> 8;
                // u's group needs a new minimum when u is its recorded argmin:
                // read its leaves before this step's stores (stale values are
                // only higher; the new degrees and u are patched in below)
                const bool refresh_u = gu != gsel && T.lvl0[gu] == ((d_u << 8) | (uint32_t)(u & 255));
                uint4 uq0 = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu), uq1 = uq0;
                if (refresh_u) T.load_leaves(gu, uq0, uq1);
                // N_t(u) \ {v}: from the statistics' cache when u's list lies
                // in its first 32 flattened entries, else read
                int32_t ub, ue;
                if (fast_v && u_src >= 0) {
                    ub = row_read(cub, u_src);
                    ue = row_read(cue, u_src);
                } else {
                    T.list(u, ub, ue);
                }
                const bool fast_u = ue - ub <= kRowLanes;
                const bool u_row = u < n;
                int32_t u_off = 0;
                if (fast_v && u_src >= 0) u_off = row_read(nc.off, u_src);
                const bool from_cache = fast_v && kc >= 2 && u_src >= 0 && fast_u && u_off + (ue - ub) <= 2 * kRowLanes;
                int32_t by = -1;
                uint32_t bd = 0;
                bool take = false;
                int32_t kb = 0;
                if (from_cache) {
                    const int32_t pos = u_off + rl;
                    const int sl = pos & (kRowLanes - 1);
                    const int32_t wa = row_read(nc.w0, sl), wb = row_read(nc.w1, sl);
                    const uint32_t da = row_read(nc.d0, sl), db = row_read(nc.d1, sl);
                    if (ub + rl < ue) {
                        by = pos < kRowLanes ? wa : wb;
                        bd = pos < kRowLanes ? da : db;
                        take = by != v && bd != kRetired;
                    }
                    kb = __popc(row_bits(ballot(take)));
                } else if (fast_u) {
                    const int32_t p = ub + rl;
                    if (p < ue) {
                        float bvv;
                        T.template entry<false>(u_row, p, by, bvv);
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
                            T.template entry<false>(u_row, p, y, bvv);
                            tk = y != v && T.deg[y] != kRetired;
                        }
                        const uint32_t msk = row_bits(ballot(tk));
                        if (tk) T.lst_b[kb + __popc(msk & ((1u << rl) - 1u))] = y;
                        kb += __popc(msk);
                    }
                }
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
                        AT.lower(cy, nd);
                        const uint32_t pk = (nd << 8) | (uint32_t)(cy & 255);
                        if ((cy >> 8) == gsel) dec_min_g = pk;
                        if ((cy >> 8) == gu) dec_min_u = pk;
                    }
                } else {
                    for (int32_t idx = rl; idx < kc; idx += kRowLanes) {
                        const int32_t y = T.lst_a[idx];
                        if (y == u) continue;
                        const uint32_t nd = (uint32_t)T.deg[y] - 1u;
                        T.deg[y] = (uint16_t)nd;
                        AT.lower(y, nd);
                        const uint32_t pk = (nd << 8) | (uint32_t)(y & 255);
                        if ((y >> 8) == gsel && pk < dec_min_g) dec_min_g = pk;
                        if ((y >> 8) == gu && pk < dec_min_u) dec_min_u = pk;
                    }
                }
                if (fast_u) {
                    if (take) {
                        const uint32_t nd = bd - 1u;
                        T.deg[by] = (uint16_t)nd;
                        AT.lower(by, nd);
                        const uint32_t pk = (nd << 8) | (uint32_t)(by & 255);
                        if ((by >> 8) == gsel && pk < dec_min_g) dec_min_g = pk;
                        if ((by >> 8) == gu && pk < dec_min_u) dec_min_u = pk;
                    }
                } else {
                    for (int32_t idx = rl; idx < kb; idx += kRowLanes) {
                        const int32_t y = T.lst_b[idx];
                        const uint32_t nd = (uint32_t)T.deg[y] - 1u;
                        T.deg[y] = (uint16_t)nd;
                        AT.lower(y, nd);
                        const uint32_t pk = (nd << 8) | (uint32_t)(y & 255);
                        if ((y >> 8) == gsel && pk < dec_min_g) dec_min_g = pk;
                        if ((y >> 8) == gu && pk < dec_min_u) dec_min_u = pk;
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
                    uint32_t mm = argmin16_skip(lq0, lq1, gsel, v, u);
                    mm = row_min_u32(mm < dec_min_g ? mm : dec_min_g);
                    if (rl == 0) T.lvl0[gsel] = mm;
                    wave_fence();
                    // the upper levels hold every lowered value already
                    if ((mm >> 8) > m_sel) AT.refresh_upper(gsel);
                }
                if (refresh_u) {
                    uint32_t mu = argmin16_skip(uq0, uq1, gu, v, u);
                    mu = row_min_u32(mu < dec_min_u ? mu : dec_min_u);
                    if (rl == 0) T.lvl0[gu] = mu;
                    wave_fence();
                    if ((mu >> 8) > d_u) AT.refresh_upper(gu);
                }
                steps = t + 1;
                t += 1;
                // a dead child is found by the next selection (a degree-0
                // vertex without candidates), at the same step count
            }
            if (run) finished = !alive || t >= n;
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
        atomicAdd(B.work_totals + 5, (unsigned long long)work.mlp_tiles);
        atomicAdd(B.work_totals + 6, (unsigned long long)work.scan_v);
    }
    // the launch's statistics, reduced by the last block to finish (its flag
    // in the softmax table's first word, unused once every wave is done)
    if (B.stats) reduce_in_last_block(B.seg, B.stats, B.blocks_done, lrn->etab);
}

}  // namespace pe
