// reduce.hpp -- FP64 reduction of the trajectory log-weights into the
// statistics of Sec. 2 and Sec. 4 "Metrics" (zeros included), in log space
// so that per(A) beyond the FP64 range is representable.
//   L  = max ln X over survivors, S1 = sum e^{lnX - L}, S2 = sum e^{2(lnX-L)}
//   ln mean = L + ln S1 - ln M; CV^2 = M (M S2 / S1^2 - 1) / (M - 1);
//   RSE = CV / sqrt(M); ESS = S1^2 / S2; p_match = n_alive / M.
// One wave per segment (matrix), all segments in one launch; each lane owns
// a strided subset and the wave combines partials in a fixed butterfly
// order, so results do not depend on scheduling.
#pragma once
#include "device.hpp"

namespace pe {

// one matrix's per-trajectory outputs
struct ReduceSeg {
    const double *logw;
    const uint8_t *alive;
    const int32_t *counters;  // [count][4] or nullptr
    int64_t count;
};

struct DevStats {
    double log_estimate, p_match, rel_spread, rse, ess, var_logw, max_logw;
    int64_t n_traj, n_alive, n_dm, n_full_sk, n_local_sk, n_steps;
};

// compensated accumulation (Neumaier)
struct KSum {
    double s = 0.0, c = 0.0;
    __device__ void add(double x) {
        const double t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x; else c += (x - t) + s;
        s = t;
    }
    __device__ double value() const { return s + c; }
};

// Butterfly combination of one value per lane across the wave: every lane
// ends with op over all 64, combined in the same fixed order (xor distances
// 32, 16, .., 1), so the result does not depend on scheduling.
template <typename T, typename Op>
__device__ T wave_allreduce(T v, Op op) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o));
    return v;
}

// One wave reduces one segment (matrix) into *out.
__device__ void reduce_segment(const ReduceSeg &sg, DevStats *out) {
    const double *logw = sg.logw;
    const uint8_t *alive = sg.alive;
    const int32_t *counters = sg.counters;
    const int64_t lo = 0, hi = sg.count;
    const int t = lane_id(), B = kWave;
    auto dmax = [](double a, double b) { return a > b ? a : b; };
    auto dadd = [](double a, double b) { return a + b; };
    auto iadd = [](long long a, long long b) { return a + b; };

    double L = -__builtin_huge_val();
    long long na = 0, c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    for (int64_t q = lo + t; q < hi; q += B) {
        if (alive[q]) { ++na; L = logw[q] > L ? logw[q] : L; }
        if (counters) {
            c0 += counters[4 * q + 0]; c1 += counters[4 * q + 1];
            c2 += counters[4 * q + 2]; c3 += counters[4 * q + 3];
        }
    }
    L = wave_allreduce(L, dmax);
    na = wave_allreduce(na, iadd);
    c0 = wave_allreduce(c0, iadd);
    c1 = wave_allreduce(c1, iadd);
    c2 = wave_allreduce(c2, iadd);
    c3 = wave_allreduce(c3, iadd);

    KSum s1, s2, m1;
    for (int64_t q = lo + t; q < hi; q += B) {
        if (!alive[q]) continue;
        const double a = exp(logw[q] - L);
        s1.add(a);
        s2.add(a * a);
        m1.add(logw[q]);
    }
    const double S1 = wave_allreduce(s1.value(), dadd);
    const double S2 = wave_allreduce(s2.value(), dadd);
    const double M1 = wave_allreduce(m1.value(), dadd);
    const double mean = na > 0 ? M1 / (double)na : 0.0;
    KSum vv;
    for (int64_t q = lo + t; q < hi; q += B) {
        if (!alive[q]) continue;
        const double d = logw[q] - mean;
        vv.add(d * d);
    }
    const double V = wave_allreduce(vv.value(), dadd);

    if (t == 0) {
        DevStats r;
        const double M = (double)(hi - lo);
        r.n_traj = hi - lo;
        r.n_alive = na;
        r.n_steps = c0; r.n_dm = c1; r.n_full_sk = c2; r.n_local_sk = c3;
        r.max_logw = L;
        r.p_match = M > 0 ? (double)na / M : __builtin_nan("");
        if (na == 0) {
            r.log_estimate = -__builtin_huge_val();
            r.rel_spread = r.rse = r.var_logw = __builtin_nan("");
            r.ess = 0.0;
        } else {
            r.log_estimate = L + log(S1) - log(M);
            double cv2 = M > 1 ? M * (M * S2 / (S1 * S1) - 1.0) / (M - 1.0) : __builtin_nan("");
            if (cv2 < 0) cv2 = 0;
            r.rel_spread = sqrt(cv2);
            r.rse = r.rel_spread / sqrt(M);
            r.ess = S1 * S1 / S2;
            r.var_logw = na > 1 ? V / (double)(na - 1) : 0.0;
        }
        *out = r;
    }
}

// One wave per segment: a single-wave block with no LDS, so the reduction
// can start on any CU with a free wave slot even while persistent trajectory
// kernels of other streams hold the chip's LDS.
__global__ void __launch_bounds__(64) k_reduce_stats(const ReduceSeg *segs, DevStats *out) {
    reduce_segment(segs[blockIdx.x], out + blockIdx.x);
}

// The launch's statistics from inside a persistent trajectory kernel of one
// matrix: the last block to finish reduces every block's outputs with its
// first wave.  A register-heavy trajectory kernel (its own launch or those
// of other streams) can leave no SIMD room for a separate reduction wave,
// which then waits for one of its waves to end; here the reduction runs on
// waves already resident.  Every thread of the block must reach this call;
// `flag` is a word of the block's LDS that no wave reads any more.
__device__ void reduce_in_last_block(const ReduceSeg *seg, DevStats *stats, uint32_t *blocks_done, uint32_t *flag) {
    __threadfence();  // this thread's outputs, device-wide, before the count
    __syncthreads();
    if (threadIdx.x == 0) *flag = atomicAdd(blocks_done, 1u) == gridDim.x - 1 ? 1u : 0u;
    __syncthreads();
    if (*flag && threadIdx.x < kWave) {
        __threadfence();  // every block's outputs before reading them
        reduce_segment(*seg, stats);
    }
}

}  // namespace pe
