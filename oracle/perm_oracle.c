/*
 * perm_oracle.c -- plain, slow CPU oracle for the adaptive sparse-permanent
 * estimator ("The Quick and the Dead", Elbek, Manafi, Gurdal, Yildirim, Kaya).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or helper with
 * the HIP library; the two meet only through the seeded input generators.
 *
 * What it computes, and where the paper defines it:
 *   - per(A), Eq. (per1); Ryser inclusion-exclusion (Sec. 2) in exact
 *     128-bit integers for 0/1 matrices and in long double for weights.
 *   - one trajectory of the generic estimator, Alg. 2 (Alg. 1 when the vertex
 *     rule is the fixed row order and nothing is scaled): vertex selection,
 *     the scaled proposal Eq. (q) with its importance correction, removal,
 *     degree bookkeeping, the DM policies All/Thrs/Trck (Sec. 3.3), the SK
 *     policies Fixed/Adaptive/Local with the local repair Eq. (local).
 *   - support filtering (Sec. 2, "Support filtering with DM"): a maximum
 *     matching (Hopcroft-Karp), the alternating digraph, its strongly
 *     connected components (Tarjan), keep an edge iff it is matched or its
 *     endpoints share a component.
 *   - outer Sinkhorn-Knopp (Sec. 3.1 and the column-then-row update of
 *     Sec. 3.3).
 *   - the reported statistics (Sec. 2 and Sec. 4 "Metrics"): mean,
 *     p_match, relative spread with the M-1 denominator, RSE, effective
 *     sample size -- in log space.
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - MD tie-break: the active vertex of minimum current degree with the
 *     smallest id; rows are ids 0..n-1, columns n..2n-1 (found with a
 *     binary heap of (degree, id) keys, lazily discarding stale keys).
 *   - a trajectory is dead as soon as some active vertex of the child has
 *     degree 0 (for the MD rule this is exactly the next step's dead end;
 *     in every case X = 0 as Alg. 2 would return).
 *   - CONTRACT precision: scaling vectors and every SK sum in IEEE binary32,
 *     summed sequentially in list order, no fused multiply-add; the
 *     proposal is integerised, w_i = max(1, rint(2^24 * s_i / s_max)), and
 *     sampled exactly with Lemire's unbiased bounded integer method
 *     (ACM TOMACS 2019), so the correction B*W/w_u uses the probability
 *     actually sampled.  PAPER precision keeps binary64 scaling and the
 *     exact ratio q = s / sum(s) (used for replay along a given path).
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     key = seed, counter = (trajectory, matrix, step, draw).
 *   - path hash: SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014)
 *     folded over (v_t, u_t).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -lm -lpthread
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ types */
typedef struct {
    int32_t n;
    int64_t m;
    const int32_t *row_ptr, *col_idx; /* CSR, ascending lists            */
    const int32_t *col_ptr, *row_idx; /* CSC, ascending lists            */
    const float *val;                 /* CSR-order values, NULL = 0/1   */
    int32_t *csc2csr;                 /* filled by or_mat_init           */
} or_mat;

typedef struct {
    int32_t vertex_rule; /* 0 = two-sided minimum degree, 1 = row order    */
    int32_t sk_policy;   /* 0 none, 1 fixed, 2 adaptive, 3 local            */
    int32_t dm_policy;   /* 0 none, 1 all, 2 thrs, 3 trck                   */
    int32_t initial_dm;  /* 1 = filter the input once before trajectories  */
    int32_t K0;          /* outer SK iterations                            */
    int32_t K;           /* inner SK cap                                    */
    double theta_th, theta_tr;
    int32_t precision;   /* 0 = CONTRACT (binary32 scaling), 1 = PAPER      */
    int32_t local_gate;  /* learned proposal: 1 = gated local-repair fallback */
    const double *model; /* learned proposal: quantised MLP parameters       */
    double mix_alpha;    /* uniform share mixed into the learned proposal    */
    int32_t local_cap;   /* local repair: 0 = exact Eq. (local); B > 0 = a
                            list longer than B entries is examined at B
                            sampled positions only (bounded-work repair)  */
} or_sched;

enum { VR_MD = 0, VR_ROW = 1 };
enum { SK_NONE = 0, SK_FIXED = 1, SK_ADAPTIVE = 2, SK_LOCAL = 3, SK_LEARNED = 4 };
enum { DM_NONE = 0, DM_ALL = 1, DM_THRS = 2, DM_TRCK = 3 };
enum { PREC_CONTRACT = 0, PREC_PAPER = 1 };

#define LN2_D 0.69314718055994530941723212145818

/* ---------------------------------------------------------------- Philox */
/* Philox4x32 with 10 rounds, from the SC'11 definition: each round takes
 * two 32x32->64 products of counter words with the round multipliers, and
 * the key is bumped by the Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 64 random bits for (seed; trajectory k, matrix b, step t, draw d). */
uint64_t or_rng64(uint64_t seed, uint32_t k, uint32_t b, uint32_t t, uint32_t d)
{
    uint32_t ctr[4] = {k, b, t, d};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    return ((uint64_t)o[1] << 32) | o[0];
}

/* Uniform integer in [0, W) by Lemire's multiply-and-reject method; every
 * rejection consumes the next draw index. */
uint64_t or_uniform_below(uint64_t seed, uint32_t k, uint32_t b, uint32_t t, uint32_t d0, uint64_t W)
{
    uint32_t d = d0;
    for (;;) {
        uint64_t x = or_rng64(seed, k, b, t, d);
        unsigned __int128 prod = (unsigned __int128)x * W;
        uint64_t lo = (uint64_t)prod;
        if (lo < W) {
            uint64_t thr = (0 - W) % W;
            if (lo < thr) { ++d; continue; }
        }
        return (uint64_t)(prod >> 64);
    }
}

uint64_t or_splitmix_fold(uint64_t h, uint64_t x)
{
    uint64_t z = h + 0x9E3779B97F4A7C15ull + x;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* --------------------------------------------------------------- Ryser */
/* per(A) = (-1)^n sum_{S subset of columns} (-1)^{|S|} prod_i sum_{j in S} a_ij
 * visited in Gray-code order; exact in 128-bit integers for every 0/1
 * matrix with n <= 20 (row sums <= n, so each product is below 20^20). */
void or_ryser_u01(int32_t n, const uint8_t *dense, uint64_t out[2])
{
    __int128 total = 0;
    int64_t rowsum[64];
    memset(rowsum, 0, sizeof(rowsum));
    uint64_t gray_prev = 0;
    uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t s = 1; s < nsub; ++s) {
        uint64_t gray = s ^ (s >> 1);
        uint64_t diff = gray ^ gray_prev;
        int j = __builtin_ctzll(diff);
        int add = (gray & diff) ? 1 : -1;
        for (int i = 0; i < n; ++i) rowsum[i] += add * (int64_t)dense[i * n + j];
        __int128 prod = 1;
        for (int i = 0; i < n && prod != 0; ++i) prod *= rowsum[i];
        int card = __builtin_popcountll(gray);
        if ((n - card) & 1) total -= prod; else total += prod;
        gray_prev = gray;
    }
    unsigned __int128 u = (unsigned __int128)total;
    out[0] = (uint64_t)u;
    out[1] = (uint64_t)(u >> 64);
}

double or_ryser_f64(int32_t n, const double *dense)
{
    long double total = 0.0L;
    long double rowsum[64];
    for (int i = 0; i < 64; ++i) rowsum[i] = 0.0L;
    uint64_t gray_prev = 0;
    uint64_t nsub = (uint64_t)1 << n;
    for (uint64_t s = 1; s < nsub; ++s) {
        uint64_t gray = s ^ (s >> 1);
        uint64_t diff = gray ^ gray_prev;
        int j = __builtin_ctzll(diff);
        int add = (gray & diff) ? 1 : -1;
        for (int i = 0; i < n; ++i) rowsum[i] += add * (long double)dense[i * n + j];
        long double prod = 1.0L;
        for (int i = 0; i < n; ++i) prod *= rowsum[i];
        int card = __builtin_popcountll(gray);
        if ((n - card) & 1) total -= prod; else total += prod;
        gray_prev = gray;
    }
    return (double)total;
}

/* Permanent of a dense nonnegative matrix (n <= 26) by the row-by-row
 * expansion over column subsets: f(S) is the permanent of the first |S|
 * rows restricted to the columns in S, f(empty) = 1 and
 *     f(S) = sum over j in S of a[|S| - 1][j] * f(S without j),
 * so per(A) = f(all columns).  Every term is nonnegative, so the binary64
 * result carries no cancellation (relative error about 2n ulps), unlike
 * Ryser's alternating sum.  Needs 2^n doubles of workspace; returns -1.0
 * when that cannot be allocated. */
double or_perm_subset_dp(int32_t n, const double *dense)
{
    if (n == 0) return 1.0;
    if (n > 26) return -1.0;
    size_t N = (size_t)1 << n;
    double *f = malloc(sizeof(double) * N);
    if (!f) return -1.0;
    f[0] = 1.0;
    for (size_t S = 1; S < N; ++S) {
        int i = __builtin_popcountll((unsigned long long)S) - 1;   /* the row added last */
        const double *row = dense + (size_t)i * (size_t)n;
        double acc = 0.0;
        for (size_t R = S; R; R &= R - 1) {
            int j = __builtin_ctzll((unsigned long long)R);
            if (row[j] != 0.0) acc += row[j] * f[S & ~((size_t)1 << j)];
        }
        f[S] = acc;
    }
    double out = f[N - 1];
    free(f);
    return out;
}

/* ---------------------------------------------------------- matrix setup */
/* csc2csr[p] = CSR position of the entry at CSC position p. */
int or_mat_init(or_mat *A, int32_t *csc2csr_out)
{
    int32_t n = A->n;
    for (int32_t j = 0; j < n; ++j) {
        for (int32_t p = A->col_ptr[j]; p < A->col_ptr[j + 1]; ++p) {
            int32_t i = A->row_idx[p];
            int32_t lo = A->row_ptr[i], hi = A->row_ptr[i + 1] - 1, found = -1;
            while (lo <= hi) {
                int32_t mid = lo + (hi - lo) / 2;
                if (A->col_idx[mid] == j) { found = mid; break; }
                if (A->col_idx[mid] < j) lo = mid + 1; else hi = mid - 1;
            }
            if (found < 0) return -1;
            csc2csr_out[p] = found;
        }
    }
    A->csc2csr = csc2csr_out;
    return 0;
}

static inline double entry_d(const or_mat *A, int64_t e) { return A->val ? (double)A->val[e] : 1.0; }
static inline float entry_f(const or_mat *A, int64_t e) { return A->val ? A->val[e] : 1.0f; }

/* --------------------------------------------------- support filtering */
/* The residual is given by vertex activity flags (act[0..n) rows,
 * act[n..2n) columns) and a removed flag per CSR edge.  On success the
 * edges lying in no perfect matching get removed[e] = 1 and the function
 * returns 1; if the residual has no perfect matching it returns 0 and
 * leaves removed[] untouched. */
typedef struct {
    int32_t *mate_r, *mate_c, *dist, *queue, *stk_v, *stk_e;
    int32_t *idx, *low, *comp, *tstack;
    uint8_t *onstack;
} dm_work;

static int dm_alloc(dm_work *w, int32_t n)
{
    size_t N = (size_t)2 * n + 2;
    w->mate_r = malloc(sizeof(int32_t) * N);
    w->mate_c = malloc(sizeof(int32_t) * N);
    w->dist = malloc(sizeof(int32_t) * N);
    w->queue = malloc(sizeof(int32_t) * N);
    w->stk_v = malloc(sizeof(int32_t) * N);
    w->stk_e = malloc(sizeof(int32_t) * N);
    w->idx = malloc(sizeof(int32_t) * N);
    w->low = malloc(sizeof(int32_t) * N);
    w->comp = malloc(sizeof(int32_t) * N);
    w->tstack = malloc(sizeof(int32_t) * N);
    w->onstack = malloc(N);
    return (w->mate_r && w->mate_c && w->dist && w->queue && w->stk_v && w->stk_e &&
            w->idx && w->low && w->comp && w->tstack && w->onstack) ? 0 : -1;
}

static void dm_free(dm_work *w)
{
    free(w->mate_r); free(w->mate_c); free(w->dist); free(w->queue);
    free(w->stk_v); free(w->stk_e); free(w->idx); free(w->low);
    free(w->comp); free(w->tstack); free(w->onstack);
}

#define INF_DIST 0x3fffffff

/* Hopcroft-Karp: BFS layers from free rows, then vertex-disjoint shortest
 * augmenting paths by (iterative) depth-first search. */
static int32_t hk_matching(const or_mat *A, const uint8_t *act, const uint8_t *removed, dm_work *w)
{
    int32_t n = A->n, size = 0;
    for (int32_t i = 0; i < n; ++i) { w->mate_r[i] = -1; w->mate_c[i] = -1; }
    for (;;) {
        /* BFS over rows; dist[i] = layer of row i */
        int32_t qh = 0, qt = 0, found = 0;
        for (int32_t i = 0; i < n; ++i) {
            if (act[i] && w->mate_r[i] < 0) { w->dist[i] = 0; w->queue[qt++] = i; }
            else w->dist[i] = INF_DIST;
        }
        int32_t limit = INF_DIST;
        while (qh < qt) {
            int32_t i = w->queue[qh++];
            if (w->dist[i] >= limit) continue;
            for (int32_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
                int32_t j = A->col_idx[e];
                if (removed[e] || !act[n + j]) continue;
                int32_t i2 = w->mate_c[j];
                if (i2 < 0) { found = 1; if (limit == INF_DIST) limit = w->dist[i] + 1; }
                else if (w->dist[i2] == INF_DIST) { w->dist[i2] = w->dist[i] + 1; w->queue[qt++] = i2; }
            }
        }
        if (!found) break;
        /* DFS from every free row along dist+1 layers */
        for (int32_t s = 0; s < n; ++s) {
            if (!act[s] || w->mate_r[s] >= 0 || w->dist[s] != 0) continue;
            int32_t top = 0;
            w->stk_v[0] = s; w->stk_e[0] = A->row_ptr[s];
            int augmented = 0;
            while (top >= 0 && !augmented) {
                int32_t i = w->stk_v[top];
                int32_t e = w->stk_e[top];
                if (e >= A->row_ptr[i + 1]) { w->dist[i] = INF_DIST; --top; continue; }
                w->stk_e[top] = e + 1;
                int32_t j = A->col_idx[e];
                if (removed[e] || !act[n + j]) continue;
                int32_t i2 = w->mate_c[j];
                if (i2 < 0) {
                    if (w->dist[i] + 1 != limit) continue;
                    /* augment along the stack */
                    for (int32_t l = top; l >= 0; --l) {
                        int32_t ri = w->stk_v[l];
                        int32_t cj = A->col_idx[w->stk_e[l] - 1];
                        w->mate_r[ri] = cj; w->mate_c[cj] = ri;
                    }
                    augmented = 1; ++size;
                } else if (w->dist[i2] == w->dist[i] + 1) {
                    ++top; w->stk_v[top] = i2; w->stk_e[top] = A->row_ptr[i2];
                }
            }
        }
    }
    return size;
}

/* Tarjan's strongly connected components on the alternating digraph:
 * matched edges go row -> column, all other residual edges column -> row.
 * Node ids: row i = i, column j = n + j.  Iterative. */
static void tarjan_scc(const or_mat *A, const uint8_t *act, const uint8_t *removed, dm_work *w)
{
    int32_t n = A->n, N = 2 * n, counter = 0, ncomp = 0, tsp = 0;
    for (int32_t x = 0; x < N; ++x) { w->idx[x] = -1; w->onstack[x] = 0; w->comp[x] = -1; }
    for (int32_t root = 0; root < N; ++root) {
        if (!act[root] || w->idx[root] >= 0) continue;
        int32_t top = 0;
        w->stk_v[0] = root; w->stk_e[0] = -1; /* -1 = not yet entered */
        while (top >= 0) {
            int32_t x = w->stk_v[top];
            if (w->stk_e[top] == -1) {
                w->idx[x] = w->low[x] = counter++;
                w->tstack[tsp++] = x; w->onstack[x] = 1;
                w->stk_e[top] = (x < n) ? 0 : A->col_ptr[x - n];
            }
            int32_t y = -1;
            if (x < n) {
                /* row: single out-edge to its mate column */
                if (w->stk_e[top] == 0) { w->stk_e[top] = 1; y = n + w->mate_r[x]; }
            } else {
                int32_t j = x - n;
                while (w->stk_e[top] < A->col_ptr[j + 1]) {
                    int32_t p = w->stk_e[top]++;
                    int32_t i = A->row_idx[p];
                    int32_t e = A->csc2csr[p];
                    if (!act[i] || removed[e] || w->mate_c[j] == i) continue;
                    y = i; break;
                }
            }
            if (y >= 0) {
                if (w->idx[y] < 0) { ++top; w->stk_v[top] = y; w->stk_e[top] = -1; }
                else if (w->onstack[y] && w->idx[y] < w->low[x]) w->low[x] = w->idx[y];
                continue;
            }
            /* x finished */
            if (w->low[x] == w->idx[x]) {
                int32_t z;
                do { z = w->tstack[--tsp]; w->onstack[z] = 0; w->comp[z] = ncomp; } while (z != x);
                ++ncomp;
            }
            --top;
            if (top >= 0) {
                int32_t par = w->stk_v[top];
                if (w->low[x] < w->low[par]) w->low[par] = w->low[x];
            }
        }
    }
}

static int support_filter(const or_mat *A, const uint8_t *act, uint8_t *removed, dm_work *w)
{
    int32_t n = A->n, need = 0;
    for (int32_t i = 0; i < n; ++i) need += act[i];
    int32_t got = hk_matching(A, act, removed, w);
    if (got != need) return 0;
    tarjan_scc(A, act, removed, w);
    for (int32_t i = 0; i < n; ++i) {
        if (!act[i]) continue;
        for (int32_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
            int32_t j = A->col_idx[e];
            if (removed[e] || !act[n + j]) continue;
            if (w->mate_r[i] == j) continue;
            if (w->comp[i] != w->comp[n + j]) removed[e] = 1;
        }
    }
    return 1;
}

/* Exported: filter the whole (or a masked) matrix.  act may be NULL (all
 * active).  Returns 1 if a perfect matching exists (removed[] updated),
 * 0 otherwise, -1 on allocation failure. */
int or_support_filter(const or_mat *A, const uint8_t *act_in, uint8_t *removed)
{
    int32_t n = A->n;
    uint8_t *act = malloc((size_t)2 * n);
    dm_work w;
    if (!act || dm_alloc(&w, n)) { free(act); return -1; }
    for (int32_t x = 0; x < 2 * n; ++x) act[x] = act_in ? act_in[x] : 1;
    int ok = support_filter(A, act, removed, &w);
    dm_free(&w);
    free(act);
    return ok;
}

/* ------------------------------------------------------- scaling (SK) */
/* One SK iteration on the residual: every active column first (with the
 * old r), then every active row (with the new c).  A zero sum leaves the
 * value unchanged.  CONTRACT: binary32 products and sequential binary32
 * sums; PAPER: binary64. */
static void sk_sweep(const or_mat *A, const uint8_t *act, const uint8_t *removed,
                     double *r, double *c, int prec)
{
    int32_t n = A->n;
    for (int32_t j = 0; j < n; ++j) {
        if (!act[n + j]) continue;
        if (prec == PREC_CONTRACT) {
            float acc = 0.0f;
            for (int32_t p = A->col_ptr[j]; p < A->col_ptr[j + 1]; ++p) {
                int32_t i = A->row_idx[p], e = A->csc2csr[p];
                if (!act[i] || removed[e]) continue;
                float prod = entry_f(A, e) * (float)r[i];
                acc = acc + prod;
            }
            if (acc != 0.0f) c[j] = (double)(1.0f / acc);
        } else {
            double acc = 0.0;
            for (int32_t p = A->col_ptr[j]; p < A->col_ptr[j + 1]; ++p) {
                int32_t i = A->row_idx[p], e = A->csc2csr[p];
                if (!act[i] || removed[e]) continue;
                acc = acc + entry_d(A, e) * r[i];
            }
            if (acc != 0.0) c[j] = 1.0 / acc;
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        if (!act[i]) continue;
        if (prec == PREC_CONTRACT) {
            float acc = 0.0f;
            for (int32_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
                int32_t j = A->col_idx[e];
                if (!act[n + j] || removed[e]) continue;
                float prod = entry_f(A, e) * (float)c[j];
                acc = acc + prod;
            }
            if (acc != 0.0f) r[i] = (double)(1.0f / acc);
        } else {
            double acc = 0.0;
            for (int32_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
                int32_t j = A->col_idx[e];
                if (!act[n + j] || removed[e]) continue;
                acc = acc + entry_d(A, e) * c[j];
            }
            if (acc != 0.0) r[i] = 1.0 / acc;
        }
    }
}

/* Preprocessing of Alg. 2: optional initial DM, r = c = 1, K0 outer SK
 * iterations.  removed[] (CSR order) must be zeroed by the caller.
 * Returns 1 (ok), 0 (no perfect matching: per(A) = 0), -1 (error). */
int or_prep(const or_mat *A, int32_t initial_dm, int32_t K0, int32_t prec,
            uint8_t *removed, double *r, double *c)
{
    int32_t n = A->n;
    int ok = 1;
    if (initial_dm) {
        ok = or_support_filter(A, NULL, removed);
        if (ok < 0) return -1;
    }
    for (int32_t i = 0; i < n; ++i) { r[i] = 1.0; c[i] = 1.0; }
    if (!ok) return 0;
    uint8_t *act = malloc((size_t)2 * n);
    if (!act) return -1;
    memset(act, 1, (size_t)2 * n);
    for (int32_t it = 0; it < K0; ++it) sk_sweep(A, act, removed, r, c, prec);
    free(act);
    return 1;
}

/* ------------------------------------------------- learned proposal */
/* A small per-edge network replaces the scaling-based scores (no inner SK).
 * Its inference is defined on fixed grids so that every sum is exact:
 *   features x[0..7] of the candidate edge (rho = row end, gam = column
 *   end) at step t:
 *     x0 = min(deg rho, 255)/64, x1 = min(deg gam, 255)/64,
 *     x2 = Q(plog2(r0[rho])/4), x3 = Q(plog2(c0[gam])/4), x4 = Q(t/n),
 *     x5 = 1 if the selected vertex is a row,
 *     x6 = Q(plog2(S_u / 2^20)/4) with S_u = sum over the residual
 *          neighbours w of the candidate u (v included) of
 *          floor(2^20 / deg w): one half-step of SK from unit scaling,
 *          in exact integer arithmetic,
 *     x7 = min(#{w in N(u), w != v, deg w <= 2}, 255)/64 (neighbours of u
 *          the step leaves with at most one option);
 *   Q(y) = clamp(rint(64 y), -256, 255)/64; plog2(s) = e - 2 + 2m for
 *   s = m 2^e, m in [0.5, 1) (piecewise-linear log2, exact);
 *   h1 = A(x W1 + b1), h2 = A(h1 W2 + b2), L = Lq(h2 . w3 + b3) with
 *   A(y) = clamp(rint(64 max(y, 0)), 0, 255)/64 and Lq(y) = clamp(rint(16 y),
 *   -1024, 1023) (logit in units of 1/16); weights are multiples of 1/64.
 * Softmax by the integer table E[d] = rint(2^24 exp(-d/16)), d = L_max - L_i,
 * then w_i = max(1, rint(2^24 ((1 - a) E_i / sum E + a / k))).
 * Parameter layout (doubles): W1[8][64], b1[64], W2[64][64], b2[64],
 * w3[64], b3. */
#define MLP_H 64
#define MLP_IN 8
#define MLP_NPARAM (MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)
#define ETAB_N 2048

static double q64(double y, double lo, double hi)
{
    double k = rint(y * 64.0);
    if (k < lo) k = lo;
    if (k > hi) k = hi;
    return k / 64.0;
}

double or_plog2(double s)
{
    int e;
    double m = frexp(s, &e);
    return (double)e - 2.0 + 2.0 * m;
}

void or_learned_features(int32_t deg_rho, int32_t deg_gam, double r0_rho, double c0_gam,
                         int32_t t, int32_t n, int32_t v_is_row, int64_t s_u, int32_t c2_u, double *x)
{
    x[0] = (double)(deg_rho < 255 ? deg_rho : 255) / 64.0;
    x[1] = (double)(deg_gam < 255 ? deg_gam : 255) / 64.0;
    x[2] = q64(or_plog2(r0_rho) / 4.0, -256.0, 255.0);
    x[3] = q64(or_plog2(c0_gam) / 4.0, -256.0, 255.0);
    x[4] = q64((double)t / (double)n, -256.0, 255.0);
    x[5] = v_is_row ? 1.0 : 0.0;
    x[6] = q64(or_plog2((double)s_u / 1048576.0) / 4.0, -256.0, 255.0);
    x[7] = (double)(c2_u < 255 ? c2_u : 255) / 64.0;
}

/* logit in units of 1/16 (exact grid arithmetic) */
int32_t or_learned_logit(const double *P, const double *x)
{
    const double *W1 = P, *b1 = W1 + MLP_IN * MLP_H, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
    const double *w3 = b2 + MLP_H, *b3 = w3 + MLP_H;
    double h1[MLP_H], h2[MLP_H];
    for (int j = 0; j < MLP_H; ++j) {
        double acc = b1[j];
        for (int k = 0; k < MLP_IN; ++k) acc += x[k] * W1[k * MLP_H + j];
        h1[j] = q64(acc > 0.0 ? acc : 0.0, 0.0, 255.0);
    }
    for (int j = 0; j < MLP_H; ++j) {
        double acc = b2[j];
        for (int k = 0; k < MLP_H; ++k) acc += h1[k] * W2[k * MLP_H + j];
        h2[j] = q64(acc > 0.0 ? acc : 0.0, 0.0, 255.0);
    }
    double acc = b3[0];
    for (int k = 0; k < MLP_H; ++k) acc += h2[k] * w3[k];
    double L = rint(acc * 16.0);
    if (L < -1024.0) L = -1024.0;
    if (L > 1023.0) L = 1023.0;
    return (int32_t)L;
}

static int64_t etab(int32_t d)
{
    if (d >= ETAB_N) return 0;
    return (int64_t)rint(16777216.0 * exp(-(double)d / 16.0));
}

/* integer weights of the learned proposal for k candidates with logits L */
void or_learned_weights(const int32_t *L, int32_t k, double alpha, uint64_t *w)
{
    int32_t lmax = L[0];
    for (int32_t a = 1; a < k; ++a) if (L[a] > lmax) lmax = L[a];
    int64_t S = 0;
    for (int32_t a = 0; a < k; ++a) S += etab(lmax - L[a]);
    for (int32_t a = 0; a < k; ++a) {
        double q = (1.0 - alpha) * (double)etab(lmax - L[a]) / (double)S + alpha / (double)k;
        double r = rint(16777216.0 * q);
        w[a] = r >= 1.0 ? (uint64_t)r : 1;
    }
}

/* ---------------------------------------------------------- trajectory */
typedef struct {
    uint8_t *act;      /* 2n */
    int32_t *deg;      /* 2n */
    uint8_t *removed;  /* m  */
    double *r, *c;     /* n each */
    int32_t *cand_v, *cand_e; /* candidate vertex / CSR edge */
    uint64_t *cand_w;
    double *cand_s;
    int32_t *cand_L;   /* learned-proposal logits of the candidates */
    int32_t *nb_v;     /* N_t(v)\{u} (other candidates of v)  */
    int32_t *nb_u;     /* N_t(u)\{v} */
    uint8_t *mark_r, *mark_c;
    int32_t *list_r, *list_c;
    double *new_r, *new_c;
    int32_t *pos_buf;  /* list positions examined by the local repair (n)  */
    int32_t *kept_buf; /* a list as the trajectories start it (n)          */
    uint64_t *heap;    /* binary min-heap of (degree << 32 | vertex) keys  */
    int64_t heap_n, heap_cap;
    dm_work dm;
} traj_work;

/* ---- binary min-heap with lazy deletion: the minimum-degree rule is
 * "smallest (degree, id) among active vertices"; every degree change
 * pushes the new key and stale keys are discarded when they surface. */
static int heap_push(traj_work *w, uint64_t key)
{
    if (w->heap_n == w->heap_cap) {
        int64_t cap = w->heap_cap ? 2 * w->heap_cap : 1024;
        uint64_t *h = realloc(w->heap, sizeof(uint64_t) * (size_t)cap);
        if (!h) return -1;
        w->heap = h; w->heap_cap = cap;
    }
    int64_t i = w->heap_n++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (w->heap[p] <= key) break;
        w->heap[i] = w->heap[p];
        i = p;
    }
    w->heap[i] = key;
    return 0;
}

static void heap_pop(traj_work *w)
{
    uint64_t last = w->heap[--w->heap_n];
    int64_t i = 0, N = w->heap_n;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        uint64_t best = last;
        if (l < N && w->heap[l] < best) { m = l; best = w->heap[l]; }
        if (r < N && w->heap[r] < best) { m = r; }
        if (m == i) break;
        w->heap[i] = w->heap[m];
        i = m;
    }
    if (N > 0) w->heap[i] = last;
}

static inline uint64_t heap_key(int32_t deg, int32_t x) { return ((uint64_t)(uint32_t)deg << 32) | (uint32_t)x; }

/* smallest (degree, id) over the active vertices; -1 if none */
static int32_t heap_min(traj_work *w, int32_t *deg_out)
{
    while (w->heap_n > 0) {
        uint64_t k = w->heap[0];
        int32_t x = (int32_t)(uint32_t)k, d = (int32_t)(k >> 32);
        if (w->act[x] && w->deg[x] == d) { *deg_out = d; return x; }
        heap_pop(w);
    }
    return -1;
}

static int heap_reset(const or_mat *A, traj_work *w)
{
    w->heap_n = 0;
    for (int32_t x = 0; x < 2 * A->n; ++x)
        if (w->act[x] && heap_push(w, heap_key(w->deg[x], x))) return -1;
    return 0;
}

static int tw_alloc(traj_work *w, const or_mat *A)
{
    int32_t n = A->n;
    size_t N = (size_t)n;
    memset(w, 0, sizeof(*w));
    w->act = malloc(2 * N);
    w->deg = malloc(sizeof(int32_t) * 2 * N);
    w->removed = malloc((size_t)A->m + 1);
    w->r = malloc(sizeof(double) * N);
    w->c = malloc(sizeof(double) * N);
    w->cand_v = malloc(sizeof(int32_t) * N);
    w->cand_e = malloc(sizeof(int32_t) * N);
    w->cand_w = malloc(sizeof(uint64_t) * N);
    w->cand_s = malloc(sizeof(double) * N);
    w->cand_L = malloc(sizeof(int32_t) * N);
    w->nb_v = malloc(sizeof(int32_t) * N);
    w->nb_u = malloc(sizeof(int32_t) * N);
    w->mark_r = calloc(N, 1);
    w->mark_c = calloc(N, 1);
    w->list_r = malloc(sizeof(int32_t) * N);
    w->list_c = malloc(sizeof(int32_t) * N);
    w->new_r = malloc(sizeof(double) * N);
    w->new_c = malloc(sizeof(double) * N);
    w->pos_buf = malloc(sizeof(int32_t) * N);
    w->kept_buf = malloc(sizeof(int32_t) * N);
    if (!w->pos_buf || !w->kept_buf || !w->act || !w->deg || !w->removed || !w->r || !w->c || !w->cand_v || !w->cand_e || !w->cand_L ||
        !w->cand_w || !w->cand_s || !w->nb_v || !w->nb_u || !w->mark_r || !w->mark_c ||
        !w->list_r || !w->list_c || !w->new_r || !w->new_c)
        return -1;
    return dm_alloc(&w->dm, n);
}

static void tw_free(traj_work *w)
{
    free(w->act); free(w->deg); free(w->removed); free(w->r); free(w->c);
    free(w->cand_v); free(w->cand_e); free(w->cand_w); free(w->cand_s); free(w->cand_L);
    free(w->nb_v); free(w->nb_u); free(w->mark_r); free(w->mark_c);
    free(w->list_r); free(w->list_c); free(w->new_r); free(w->new_c); free(w->pos_buf); free(w->kept_buf);
    free(w->heap);
    dm_free(&w->dm);
}

/* active, non-removed neighbours of vertex x; returns the count and writes
 * vertex ids / CSR edge ids in list order when the arrays are given. */
static int32_t residual_neighbours(const or_mat *A, const traj_work *w, int32_t x,
                                   int32_t *nv, int32_t *ne)
{
    int32_t n = A->n, k = 0;
    if (x < n) {
        for (int32_t e = A->row_ptr[x]; e < A->row_ptr[x + 1]; ++e) {
            int32_t y = n + A->col_idx[e];
            if (!w->act[y] || w->removed[e]) continue;
            if (nv) nv[k] = y;
            if (ne) ne[k] = e;
            ++k;
        }
    } else {
        int32_t j = x - n;
        for (int32_t p = A->col_ptr[j]; p < A->col_ptr[j + 1]; ++p) {
            int32_t y = A->row_idx[p], e = A->csc2csr[p];
            if (!w->act[y] || w->removed[e]) continue;
            if (nv) nv[k] = y;
            if (ne) ne[k] = e;
            ++k;
        }
    }
    return k;
}

/* S_u and the degree-<=2 count of features x6 / x7 of the learned proposal */
static void candidate_stats(const or_mat *A, const traj_work *w, int32_t u, int32_t v, int64_t *s_u,
                            int32_t *c2_u)
{
    int32_t n = A->n;
    int64_t S = 0;
    int32_t c2 = 0;
    int32_t beg, end;
    if (u < n) { beg = A->row_ptr[u]; end = A->row_ptr[u + 1]; }
    else { beg = A->col_ptr[u - n]; end = A->col_ptr[u - n + 1]; }
    for (int32_t p = beg; p < end; ++p) {
        int32_t y = u < n ? n + A->col_idx[p] : A->row_idx[p];
        int32_t e = u < n ? p : A->csc2csr[p];
        if (!w->act[y] || w->removed[e] || w->deg[y] <= 0) continue;
        S += 1048576 / w->deg[y];
        if (y != v && w->deg[y] <= 2) ++c2;
    }
    *s_u = S;
    *c2_u = c2;
}

static void recount_degrees(const or_mat *A, traj_work *w)
{
    for (int32_t x = 0; x < 2 * A->n; ++x)
        w->deg[x] = w->act[x] ? residual_neighbours(A, w, x, NULL, NULL) : 0;
}

/* Bounded-work local repair (the sampled variant that Sec. 3.3 suggests
 * for hub vertices and leaves open).  The list of a vertex x here is the
 * list trajectories start from: x's entries that the shared initial
 * filter kept, in list order.  With a cap B > 0, a vertex whose list holds
 * L_x > B entries is examined at B of them only, the ones at list indices
 *     p_k = (o_x + floor(k L_x / B)) mod L_x,  k = 0 .. B-1  (in k order),
 * a systematic sample whose offset o_x = floor(R L_x / 2^32) takes R, the
 * low 32 bits of the Philox draw (seed; trajectory, matrix, step t,
 * draw 2^31 + x).  The active, non-removed entries among them are x's
 * sampled child neighbourhood: it stands for N_{t+1}(x) when x's
 * neighbours join R_loc or C_loc, and x's normalisation sum is estimated
 * from it by the ratio d_x / a (d_x = x's residual degree in the child,
 * a = the number of those entries):
 *     new value of x = 1 / ((sum over them, in k order) * (d_x / a)),
 * unchanged when a = 0 or the sum is 0.  Lists of at most B entries (and
 * every list when B = 0) are used whole, as in Eq. (local).  Only the
 * proposal changes, so the estimator stays unbiased (Sec. 3.1). */
#define LOCAL_DRAW_BASE 0x80000000u

typedef struct {
    uint64_t seed;
    uint32_t k, b, t;
    int32_t cap;
    const uint8_t *removed0;  /* entries the shared initial filter removed */
} local_draw;

/* x's list as the trajectories start it: absolute CSR (row x) or CSC
 * (column x) positions of the entries the initial filter kept. */
static int32_t start_list(const or_mat *A, const uint8_t *removed0, int32_t x, int32_t *out)
{
    int32_t n = A->n, L = 0;
    if (x < n) {
        for (int32_t e = A->row_ptr[x]; e < A->row_ptr[x + 1]; ++e)
            if (!removed0[e]) out[L++] = e;
    } else {
        for (int32_t p = A->col_ptr[x - n]; p < A->col_ptr[x - n + 1]; ++p)
            if (!removed0[A->csc2csr[p]]) out[L++] = p;
    }
    return L;
}

/* The positions of x's list that the repair examines, in examination
 * order; *sampled tells whether the list was longer than the cap. */
static int32_t examined_positions(const or_mat *A, const local_draw *ld, int32_t x, int32_t *kept,
                                  int32_t *pos, int *sampled)
{
    int32_t L = start_list(A, ld->removed0, x, kept);
    if (ld->cap <= 0 || L <= ld->cap) {
        for (int32_t i = 0; i < L; ++i) pos[i] = kept[i];
        *sampled = 0;
        return L;
    }
    uint32_t R = (uint32_t)or_rng64(ld->seed, ld->k, ld->b, ld->t, LOCAL_DRAW_BASE | (uint32_t)x);
    uint64_t o = ((uint64_t)R * (uint64_t)L) >> 32;
    for (int32_t i = 0; i < ld->cap; ++i)
        pos[i] = kept[(o + ((uint64_t)i * (uint64_t)L) / (uint64_t)ld->cap) % (uint64_t)L];
    *sampled = 1;
    return ld->cap;
}

/* Eq. (local): Jacobi repair of r on R_loc and c on C_loc, computed from
 * the pre-repair vectors and committed together. rho/gam are the removed
 * row/column, nb_rho = N_t(rho)\{gam} (columns), nb_gam = N_t(gam)\{rho}
 * (rows), given as vertex ids.  ld->cap > 0 selects the bounded-work
 * variant above. */
static void local_repair(const or_mat *A, traj_work *w, int prec,
                         const int32_t *nb_rho, int32_t k_rho,
                         const int32_t *nb_gam, int32_t k_gam, const local_draw *ld)
{
    int32_t *pos = w->pos_buf, *kept = w->kept_buf;
    int32_t n = A->n, nr = 0, nc = 0;
    int smp;
    /* C_loc = N_t(rho)\{gam}  U  N_{t+1}(N_t(gam)\{rho}) */
    for (int32_t a = 0; a < k_rho; ++a) {
        int32_t j = nb_rho[a] - n;
        if (!w->mark_c[j]) { w->mark_c[j] = 1; w->list_c[nc++] = j; }
    }
    for (int32_t a = 0; a < k_gam; ++a) {
        int32_t i = nb_gam[a];
        int32_t np = examined_positions(A, ld, i, kept, pos, &smp);
        for (int32_t q = 0; q < np; ++q) {
            int32_t e = pos[q];
            int32_t j = A->col_idx[e];
            if (!w->act[n + j] || w->removed[e]) continue;
            if (!w->mark_c[j]) { w->mark_c[j] = 1; w->list_c[nc++] = j; }
        }
    }
    /* R_loc = N_t(gam)\{rho}  U  N_{t+1}(N_t(rho)\{gam}) */
    for (int32_t a = 0; a < k_gam; ++a) {
        int32_t i = nb_gam[a];
        if (!w->mark_r[i]) { w->mark_r[i] = 1; w->list_r[nr++] = i; }
    }
    for (int32_t a = 0; a < k_rho; ++a) {
        int32_t j = nb_rho[a] - n;
        int32_t np = examined_positions(A, ld, n + j, kept, pos, &smp);
        for (int32_t q = 0; q < np; ++q) {
            int32_t p = pos[q];
            int32_t i = A->row_idx[p], e = A->csc2csr[p];
            if (!w->act[i] || w->removed[e]) continue;
            if (!w->mark_r[i]) { w->mark_r[i] = 1; w->list_r[nr++] = i; }
        }
    }
    /* new values from the old vectors */
    for (int32_t a = 0; a < nr; ++a) {
        int32_t i = w->list_r[a];
        double val = w->r[i];
        int32_t np = examined_positions(A, ld, i, kept, pos, &smp);
        if (smp) {
            /* sampled sum, ratio-scaled to the residual degree (binary32) */
            int32_t cnt = 0;
            float acc = 0.0f;
            for (int32_t q = 0; q < np; ++q) {
                int32_t e = pos[q];
                int32_t j = A->col_idx[e];
                if (!w->act[n + j] || w->removed[e]) continue;
                float prod = entry_f(A, e) * (float)w->c[j];
                acc = acc + prod;
                ++cnt;
            }
            if (cnt > 0 && acc != 0.0f) {
                float est = acc * ((float)w->deg[i] / (float)cnt);
                val = (double)(1.0f / est);
            }
        } else if (prec == PREC_CONTRACT) {
            float acc = 0.0f;
            for (int32_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
                int32_t j = A->col_idx[e];
                if (!w->act[n + j] || w->removed[e]) continue;
                float prod = entry_f(A, e) * (float)w->c[j];
                acc = acc + prod;
            }
            if (acc != 0.0f) val = (double)(1.0f / acc);
        } else {
            double acc = 0.0;
            for (int32_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
                int32_t j = A->col_idx[e];
                if (!w->act[n + j] || w->removed[e]) continue;
                acc = acc + entry_d(A, e) * w->c[j];
            }
            if (acc != 0.0) val = 1.0 / acc;
        }
        w->new_r[a] = val;
    }
    for (int32_t a = 0; a < nc; ++a) {
        int32_t j = w->list_c[a];
        double val = w->c[j];
        int32_t np = examined_positions(A, ld, n + j, kept, pos, &smp);
        if (smp) {
            int32_t cnt = 0;
            float acc = 0.0f;
            for (int32_t q = 0; q < np; ++q) {
                int32_t p = pos[q];
                int32_t i = A->row_idx[p], e = A->csc2csr[p];
                if (!w->act[i] || w->removed[e]) continue;
                float prod = entry_f(A, e) * (float)w->r[i];
                acc = acc + prod;
                ++cnt;
            }
            if (cnt > 0 && acc != 0.0f) {
                float est = acc * ((float)w->deg[n + j] / (float)cnt);
                val = (double)(1.0f / est);
            }
        } else if (prec == PREC_CONTRACT) {
            float acc = 0.0f;
            for (int32_t p = A->col_ptr[j]; p < A->col_ptr[j + 1]; ++p) {
                int32_t i = A->row_idx[p], e = A->csc2csr[p];
                if (!w->act[i] || w->removed[e]) continue;
                float prod = entry_f(A, e) * (float)w->r[i];
                acc = acc + prod;
            }
            if (acc != 0.0f) val = (double)(1.0f / acc);
        } else {
            double acc = 0.0;
            for (int32_t p = A->col_ptr[j]; p < A->col_ptr[j + 1]; ++p) {
                int32_t i = A->row_idx[p], e = A->csc2csr[p];
                if (!w->act[i] || w->removed[e]) continue;
                acc = acc + entry_d(A, e) * w->r[i];
            }
            if (acc != 0.0) val = 1.0 / acc;
        }
        w->new_c[a] = val;
    }
    for (int32_t a = 0; a < nr; ++a) { w->r[w->list_r[a]] = w->new_r[a]; w->mark_r[w->list_r[a]] = 0; }
    for (int32_t a = 0; a < nc; ++a) { w->c[w->list_c[a]] = w->new_c[a]; w->mark_c[w->list_c[a]] = 0; }
}

/* Per-trajectory result. */
typedef struct {
    double logw;        /* ln X, -inf when X = 0 */
    int32_t alive;
    int32_t steps;      /* completed matching steps */
    int32_t n_dm, n_sk_sweeps, n_local;
    uint64_t path_hash;
} traj_out;

/* Probe interface used for exact enumeration and replay: the first
 * n_forced steps take the candidate whose vertex id is forced_choice[t]
 * (stopped = -1 if it is not a candidate) instead of a random draw (and, if forced_events is given, DM on/off and the number of SK
 * sweeps from forced_events[2t], forced_events[2t+1]); at step n_forced the
 * trajectory stops and reports its candidates with their probabilities. */
typedef struct {
    const int32_t *forced_choice;
    const int32_t *forced_events;
    int32_t n_forced;
    int32_t stop_at;        /* stop before drawing at this step (-1 = never) */
    int32_t *cand_out;      /* [n] vertex ids at stop step */
    double *prob_out;       /* [n] sampling probabilities at stop step */
    int32_t *ncand_out;
    int32_t *stopped;
    /* state snapshot when the probe stops or the trajectory ends (nullable) */
    uint8_t *act_out, *removed_out;
    double *r_out, *c_out;
    int32_t *deg_out;
} probe_ctl;

static void snapshot(const or_mat *A, const traj_work *w, const probe_ctl *pc)
{
    if (!pc) return;
    int32_t n = A->n;
    if (pc->act_out) memcpy(pc->act_out, w->act, (size_t)2 * n);
    if (pc->removed_out) memcpy(pc->removed_out, w->removed, (size_t)A->m);
    if (pc->r_out) memcpy(pc->r_out, w->r, sizeof(double) * n);
    if (pc->c_out) memcpy(pc->c_out, w->c, sizeof(double) * n);
    if (pc->deg_out) memcpy(pc->deg_out, w->deg, sizeof(int32_t) * 2 * n);
}

static void run_traj(const or_mat *A, const or_sched *S, const uint8_t *removed0,
                     const double *r0, const double *c0, int ok0,
                     uint64_t seed, uint32_t b, uint32_t k, traj_work *w,
                     traj_out *out, int32_t *path, int32_t *events, const probe_ctl *pc)
{
    int32_t n = A->n;
    int prec = S->precision;
    out->logw = -INFINITY; out->alive = 0; out->steps = 0;
    out->n_dm = out->n_sk_sweeps = out->n_local = 0;
    out->path_hash = 0;
    if (path) for (int32_t t = 0; t < 2 * n; ++t) path[t] = -1;
    if (events) for (int32_t t = 0; t < 2 * n; ++t) events[t] = 0;
    if (pc && pc->stopped) *pc->stopped = 0;
    if (!ok0) return;

    memset(w->act, 1, (size_t)2 * n);
    memcpy(w->removed, removed0, (size_t)A->m);
    for (int32_t i = 0; i < n; ++i) { w->r[i] = r0[i]; w->c[i] = c0[i]; }
    recount_degrees(A, w);
    if (heap_reset(A, w)) return;

    double mant = 1.0;
    int64_t ex = 0;
    double track = 1.0;
    /* Learned proposal with the gated fallback: the trajectory keeps its own
     * r, c (from the outer scaling), repairs them by Eq. (local) after a
     * step whose sampled probability fell below theta_th or after an inner
     * DM call, and the step after such a repair draws from the scaled
     * proposal of Eq. (q) instead of the network. */
    const int gate = S->sk_policy == SK_LEARNED && S->local_gate;
    int fb = 0;
    uint64_t h = 0;

    for (int32_t t = 0; t < n; ++t) {
        /* ---- choose an active vertex */
        int32_t v = -1;
        if (S->vertex_rule == VR_ROW) {
            for (int32_t i = 0; i < n; ++i) if (w->act[i]) { v = i; break; }
        } else {
            int32_t dmin;
            v = heap_min(w, &dmin);
        }
        /* ---- candidates N_t(v) */
        int32_t kc = residual_neighbours(A, w, v, w->cand_v, w->cand_e);
        if (kc == 0) return; /* dead end: X = 0 */

        /* ---- proposal scores s = B_{v,u} * (c_u for a row v, r_u for a column v) */
        int v_is_row = v < n;
        uint64_t W = 0;
        double S_paper = 0.0;
        if (S->sk_policy == SK_LEARNED && !fb) {
            int32_t *Lg = w->cand_L;
            for (int32_t a = 0; a < kc; ++a) {
                int32_t y = w->cand_v[a];
                int32_t rho = v_is_row ? v : y, gam = v_is_row ? y : v;
                double x[MLP_IN];
                int64_t s_u;
                int32_t c2_u;
                candidate_stats(A, w, y, v, &s_u, &c2_u);
                or_learned_features(w->deg[rho], w->deg[gam], r0[rho], c0[gam - n], t, n, v_is_row, s_u, c2_u,
                                    x);
                Lg[a] = or_learned_logit(S->model, x);
            }
            or_learned_weights(Lg, kc, S->mix_alpha, w->cand_w);
            for (int32_t a = 0; a < kc; ++a) W += w->cand_w[a];
        } else if (prec == PREC_CONTRACT || S->sk_policy == SK_LEARNED) {
            float smax = 0.0f;
            float sv[1];
            (void)sv;
            for (int32_t a = 0; a < kc; ++a) {
                int32_t y = w->cand_v[a];
                float sc = v_is_row ? (float)w->c[y - n] : (float)w->r[y];
                float s = entry_f(A, w->cand_e[a]) * sc;
                w->cand_s[a] = (double)s;
                if (s > smax) smax = s;
            }
            int uniform = !(smax > 0.0f) || isinf(smax);
            for (int32_t a = 0; a < kc; ++a) {
                uint64_t wi = 1;
                if (!uniform) {
                    float ratio = (float)w->cand_s[a] / smax;
                    float scaled = ratio * 16777216.0f;
                    float rr = rintf(scaled);
                    wi = (rr >= 1.0f) ? (uint64_t)rr : 1;
                }
                w->cand_w[a] = wi;
                W += wi;
            }
        } else {
            for (int32_t a = 0; a < kc; ++a) {
                int32_t y = w->cand_v[a];
                double sc = v_is_row ? w->c[y - n] : w->r[y];
                double s = entry_d(A, w->cand_e[a]) * sc;
                w->cand_s[a] = s;
                S_paper = S_paper + s;
            }
        }

        if (pc && pc->stop_at == t) {
            for (int32_t a = 0; a < kc; ++a) {
                pc->cand_out[a] = w->cand_v[a];
                pc->prob_out[a] = (prec == PREC_CONTRACT || S->sk_policy == SK_LEARNED)
                                      ? (double)w->cand_w[a] / (double)W : w->cand_s[a] / S_paper;
            }
            *pc->ncand_out = kc;
            *pc->stopped = 1;
            out->steps = t;
            snapshot(A, w, pc);
            return;
        }

        /* ---- draw u ~ q_t(.|v) */
        int32_t pick;
        if (pc && t < pc->n_forced) {
            pick = -1;
            for (int32_t a = 0; a < kc; ++a) if (w->cand_v[a] == pc->forced_choice[t]) pick = a;
            if (pick < 0) { if (pc->stopped) *pc->stopped = -1; out->steps = t; return; }
        } else if (kc == 1) {
            pick = 0;
        } else if (prec == PREC_CONTRACT || S->sk_policy == SK_LEARNED) {
            uint64_t j = or_uniform_below(seed, k, b, (uint32_t)t, 0, W);
            uint64_t pre = 0;
            pick = kc - 1;
            for (int32_t a = 0; a < kc; ++a) { pre += w->cand_w[a]; if (pre > j) { pick = a; break; } }
        } else {
            uint64_t x = or_rng64(seed, k, b, (uint32_t)t, 0);
            double U = (double)(x >> 11) * 0x1.0p-53;
            double target = U * S_paper, pre = 0.0;
            pick = kc - 1;
            for (int32_t a = 0; a < kc; ++a) { pre = pre + w->cand_s[a]; if (pre > target) { pick = a; break; } }
        }
        int32_t u = w->cand_v[pick];
        int32_t e_vu = w->cand_e[pick];

        /* ---- importance correction X <- X * B_{v,u} / q_t(u|v) */
        double factor;
        if (prec == PREC_CONTRACT || S->sk_policy == SK_LEARNED)
            factor = entry_d(A, e_vu) * ((double)W / (double)w->cand_w[pick]);
        else factor = entry_d(A, e_vu) * (S_paper / w->cand_s[pick]);
        {
            int e2;
            mant = frexp(mant * factor, &e2);
            ex += e2;
        }

        /* ---- z = r_rho * c_gam with the pre-step vectors */
        int32_t rho = v_is_row ? v : u;
        int32_t gam = v_is_row ? u : v; /* vertex id n + j */
        double z = w->r[rho] * w->c[gam - n];
        if (S->sk_policy == SK_LEARNED && !fb) z = (double)w->cand_w[pick] / (double)W;

        if (path) { path[2 * t] = v; path[2 * t + 1] = u; }
        h = or_splitmix_fold(h, ((uint64_t)(uint32_t)v << 32) | (uint32_t)u);

        /* N_t(rho)\{gam}, N_t(gam)\{rho} for the local repair */
        int32_t k_rho = 0, k_gam = 0;
        {
            int32_t kk = residual_neighbours(A, w, rho, w->nb_v, NULL);
            for (int32_t a = 0; a < kk; ++a) if (w->nb_v[a] != gam) w->nb_v[k_rho++] = w->nb_v[a];
            kk = residual_neighbours(A, w, gam, w->nb_u, NULL);
            for (int32_t a = 0; a < kk; ++a) if (w->nb_u[a] != rho) w->nb_u[k_gam++] = w->nb_u[a];
        }

        /* ---- B^{(t+1)} = B^{(t)} \ {v,u}; degree bookkeeping */
        w->act[v] = 0; w->act[u] = 0;
        for (int32_t a = 0; a < k_rho; ++a) {
            int32_t y = w->nb_v[a];
            w->deg[y] -= 1;
            if (heap_push(w, heap_key(w->deg[y], y))) return;
        }
        for (int32_t a = 0; a < k_gam; ++a) {
            int32_t y = w->nb_u[a];
            w->deg[y] -= 1;
            if (heap_push(w, heap_key(w->deg[y], y))) return;
        }
        out->steps = t + 1;
        track = track * z;

        if (t + 1 >= n) break;

        /* child dead end: some active vertex has no residual neighbour */
        {
            int32_t dmin = -1;
            if (heap_min(w, &dmin) < 0 || dmin == 0) return;
        }

        /* ---- DM policy */
        int run_dm = 0;
        if (S->dm_policy == DM_ALL) run_dm = 1;
        else if (S->dm_policy == DM_THRS && z < S->theta_th) run_dm = 1;
        else if (S->dm_policy == DM_TRCK && track < S->theta_tr) run_dm = 1;
        if (pc && pc->forced_events && t < pc->n_forced) run_dm = pc->forced_events[2 * t] != 0;
        if (run_dm) {
            out->n_dm += 1;
            int ok = support_filter(A, w->act, w->removed, &w->dm);
            if (events) events[2 * t] = 1;
            if (!ok) return;
            recount_degrees(A, w);
            if (heap_reset(A, w)) return;
            track = 1.0;
        }

        /* ---- SK policy on the child */
        const local_draw ld = {seed, k, b, (uint32_t)t, S->local_cap, removed0};
        int nit = 0;
        if (S->sk_policy == SK_FIXED) nit = S->K;
        else if (S->sk_policy == SK_ADAPTIVE) {
            double want = ceil((1.0 - z) * (double)S->K);
            if (!(want > 0.0)) want = 0.0; /* also maps NaN to 0 */
            if (want > (double)S->K) want = (double)S->K;
            nit = (int)want;
        }
        if (pc && pc->forced_events && t < pc->n_forced && S->sk_policy != SK_LOCAL)
            nit = pc->forced_events[2 * t + 1];
        if (S->sk_policy == SK_FIXED || S->sk_policy == SK_ADAPTIVE) {
            for (int it = 0; it < nit; ++it) sk_sweep(A, w->act, w->removed, w->r, w->c, prec);
            out->n_sk_sweeps += nit;
            if (events) events[2 * t + 1] = nit;
        } else if (S->sk_policy == SK_LOCAL) {
            local_repair(A, w, prec, w->nb_v, k_rho, w->nb_u, k_gam, &ld);
            out->n_local += 1;
            if (events) events[2 * t + 1] = 1;
        } else if (gate) {
            fb = z < S->theta_th || run_dm;
            if (fb) {
                local_repair(A, w, prec, w->nb_v, k_rho, w->nb_u, k_gam, &ld);
                out->n_local += 1;
                if (events) events[2 * t + 1] = 1;
            }
        }
    }
    out->alive = 1;
    out->logw = log(mant) + (double)ex * LN2_D;
    out->path_hash = h;
    snapshot(A, w, pc);
}

/* ------------------------------------------------------------- drivers */
typedef struct {
    const or_mat *A;
    const or_sched *S;
    const uint8_t *removed0;
    const double *r0, *c0;
    int ok0;
    uint64_t seed;
    uint32_t b;
    int64_t first, count;
    double *logw;
    uint8_t *alive;
    int32_t *path;
    uint64_t *path_hash;
    int32_t *counters;
    int64_t lo, hi;
    int status;
} run_job;

static void *run_worker(void *arg)
{
    run_job *J = arg;
    traj_work w;
    if (tw_alloc(&w, J->A)) { J->status = -1; tw_free(&w); return NULL; }
    int32_t n = J->A->n;
    for (int64_t q = J->lo; q < J->hi; ++q) {
        traj_out o;
        uint32_t k = (uint32_t)(J->first + q);
        run_traj(J->A, J->S, J->removed0, J->r0, J->c0, J->ok0, J->seed, J->b, k, &w, &o,
                 J->path ? J->path + (size_t)q * 2 * n : NULL, NULL, NULL);
        if (J->logw) J->logw[q] = o.logw;
        if (J->alive) J->alive[q] = (uint8_t)o.alive;
        if (J->path_hash) J->path_hash[q] = o.path_hash;
        if (J->counters) {
            J->counters[4 * q + 0] = o.steps;
            J->counters[4 * q + 1] = o.n_dm;
            J->counters[4 * q + 2] = o.n_sk_sweeps;
            J->counters[4 * q + 3] = o.n_local;
        }
    }
    tw_free(&w);
    J->status = 0;
    return NULL;
}

/* Run trajectories first..first+count-1 of matrix b.  Output arrays are
 * indexed 0..count-1 and may be NULL; path holds 2n int32 per trajectory
 * (v_t, u_t, -1 after the last completed step); counters holds (steps,
 * DM calls, full SK sweeps, local repairs).  Results do not depend on
 * nthreads. */
int or_run(const or_mat *A, const or_sched *S, const uint8_t *removed0,
           const double *r0, const double *c0, int32_t ok0, uint64_t seed,
           uint32_t b, int64_t first, int64_t count, int32_t nthreads,
           double *logw, uint8_t *alive, int32_t *path, uint64_t *path_hash,
           int32_t *counters)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (count < nthreads) nthreads = count > 0 ? (int32_t)count : 1;
    run_job jobs[256];
    pthread_t th[256];
    for (int32_t i = 0; i < nthreads; ++i) {
        run_job *J = &jobs[i];
        J->A = A; J->S = S; J->removed0 = removed0; J->r0 = r0; J->c0 = c0; J->ok0 = ok0;
        J->seed = seed; J->b = b; J->first = first; J->count = count;
        J->logw = logw; J->alive = alive; J->path = path; J->path_hash = path_hash;
        J->counters = counters;
        J->lo = count * i / nthreads; J->hi = count * (i + 1) / nthreads;
        J->status = 0;
    }
    if (nthreads == 1) {
        run_worker(&jobs[0]);
    } else {
        for (int32_t i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, run_worker, &jobs[i]);
        for (int32_t i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    }
    for (int32_t i = 0; i < nthreads; ++i) if (jobs[i].status) return -1;
    return 0;
}

/* One trajectory under probe control (enumeration and replay).  Returns
 * 0 ok, -1 error.  result[0] = logw, result[1] = alive, result[2] =
 * stopped (1 if the trajectory stopped at stop_at and reported
 * candidates), result[3] = completed steps.  The *_out arrays (nullable)
 * receive the residual state (activity, removed edges, r, c, degrees) at
 * the stop, or at the end of a completed trajectory. */
int or_probe(const or_mat *A, const or_sched *S, const uint8_t *removed0,
             const double *r0, const double *c0, int32_t ok0, uint64_t seed,
             uint32_t b, uint32_t k, const int32_t *forced_choice,
             const int32_t *forced_events, int32_t n_forced, int32_t stop_at,
             int32_t *ncand, int32_t *cand, double *prob, int32_t *path,
             int32_t *events, int32_t *counters, double *result,
             uint8_t *act_out, uint8_t *removed_out, double *r_out, double *c_out,
             int32_t *deg_out)
{
    traj_work w;
    if (tw_alloc(&w, A)) { tw_free(&w); return -1; }
    int32_t stopped = 0;
    probe_ctl pc = {forced_choice, forced_events, n_forced, stop_at, cand, prob, ncand, &stopped,
                    act_out, removed_out, r_out, c_out, deg_out};
    traj_out o;
    run_traj(A, S, removed0, r0, c0, ok0, seed, b, k, &w, &o, path, events, &pc);
    result[0] = o.logw;
    result[1] = o.alive;
    result[2] = stopped;
    result[3] = o.steps;
    if (counters) {
        counters[0] = o.steps; counters[1] = o.n_dm;
        counters[2] = o.n_sk_sweeps; counters[3] = o.n_local;
    }
    tw_free(&w);
    return 0;
}

/* --------------------------------------------------------- statistics */
/* Sec. 2 and Sec. 4 "Metrics", zeros included, in log space:
 * L = max ln X over surviving trajectories, S1 = sum e^{lnX-L},
 * S2 = sum e^{2(lnX-L)}.  out = {ln mean, p_match, relative spread
 * (sd with M-1 over |mean|), RSE, ESS = S1^2/S2, var of ln X over the
 * survivors, L, n_alive}.  Sums are compensated (Neumaier). */
void or_stats(const double *logw, const uint8_t *alive, int64_t M, double *out)
{
    double L = -INFINITY;
    int64_t na = 0;
    for (int64_t q = 0; q < M; ++q)
        if (alive[q]) { ++na; if (logw[q] > L) L = logw[q]; }
    double s1 = 0, c1 = 0, s2 = 0, c2 = 0, m1 = 0, m1c = 0;
    for (int64_t q = 0; q < M; ++q) {
        if (!alive[q]) continue;
        double a = exp(logw[q] - L), bq = a * a;
        double t = s1 + a; if (fabs(s1) >= fabs(a)) c1 += (s1 - t) + a; else c1 += (a - t) + s1; s1 = t;
        t = s2 + bq; if (fabs(s2) >= fabs(bq)) c2 += (s2 - t) + bq; else c2 += (bq - t) + s2; s2 = t;
        t = m1 + logw[q]; if (fabs(m1) >= fabs(logw[q])) m1c += (m1 - t) + logw[q]; else m1c += (logw[q] - t) + m1; m1 = t;
    }
    s1 += c1; s2 += c2; m1 += m1c;
    double Md = (double)M;
    out[6] = L;
    out[7] = (double)na;
    out[1] = Md > 0 ? (double)na / Md : NAN;
    if (na == 0) {
        out[0] = -INFINITY; out[2] = NAN; out[3] = NAN; out[4] = 0.0; out[5] = NAN;
        return;
    }
    out[0] = L + log(s1) - log(Md);
    double cv2 = M > 1 ? Md * (Md * s2 / (s1 * s1) - 1.0) / (Md - 1.0) : NAN;
    if (cv2 < 0) cv2 = 0;
    out[2] = sqrt(cv2);
    out[3] = out[2] / sqrt(Md);
    out[4] = s1 * s1 / s2;
    double mean = m1 / (double)na, v = 0, vc = 0;
    for (int64_t q = 0; q < M; ++q) {
        if (!alive[q]) continue;
        double d = (logw[q] - mean) * (logw[q] - mean);
        double t = v + d; if (fabs(v) >= fabs(d)) vc += (v - t) + d; else vc += (d - t) + v; v = t;
    }
    out[5] = na > 1 ? (v + vc) / (double)(na - 1) : 0.0;
}
