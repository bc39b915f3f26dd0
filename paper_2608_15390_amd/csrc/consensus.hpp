// Multi-seed consensus diagnostics for a permanent with no known value
// (Sec. 4.4): host code over the final statistics of V variants x R seeds.
//
// Every estimate Y is handled as exp(ln Y - L), L the largest ln Y, so the
// large permanents of big matrices do not overflow; degree-one quantities
// are returned as logarithms, ratios as they are.
//
// Quantiles come from their definitions, without tables:
// * Phi^{-1}(p): bisection on Phi(x) = erfc(-x / sqrt 2) / 2;
// * Student t with an integer number of degrees of freedom nu: the finite
//   trigonometric series for A(t | nu) = P(|T| <= t) (Abramowitz & Stegun,
//   26.7.3 for odd and 26.7.4 for even nu, theta = atan(t / sqrt nu)),
//   inverted by bisection.
#pragma once

#include <cmath>
#include <cstdint>
#include <vector>

#include "perm_est.h"

namespace pe {
namespace consensus {

inline double phi_inv(double p) {
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 400 && hi - lo > 0.0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// P(|T| <= t) for Student's t with nu >= 1 degrees of freedom, t >= 0
inline double t_abs_cdf(double t, int nu) {
    const double th = std::atan(t / std::sqrt((double)nu));
    const double s = std::sin(th), c = std::cos(th), c2 = c * c;
    if (nu % 2 == 0) {
        double term = 1.0, sum = 1.0;
        for (int k = 1; k <= (nu - 2) / 2; ++k) {
            term *= (2.0 * k - 1.0) / (2.0 * k) * c2;
            sum += term;
        }
        return s * sum;
    }
    const double pi = 3.14159265358979323846;
    if (nu == 1) return 2.0 * th / pi;
    double term = c, sum = c;
    for (int k = 1; k <= (nu - 3) / 2; ++k) {
        term *= (2.0 * k) / (2.0 * k + 1.0) * c2;
        sum += term;
    }
    return 2.0 / pi * (th + s * sum);
}

// two-sided critical value: P(|T| <= t) = level
inline double t_crit(int nu, double level) {
    double lo = 0.0, hi = 1e7;
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (t_abs_cdf(mid, nu) < level) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

inline int run(int32_t V, int32_t R, const perm_est_result *runs, double alpha, perm_est_consensus_result *out,
               double *log_ybar, double *rel_e) {
    const size_t N = (size_t)V * (size_t)R;
    bool present = true;
    double L = -INFINITY;
    for (size_t i = 0; i < N; ++i) {
        if (runs[i].n_traj <= 0 || std::isnan(runs[i].log_estimate)) present = false;
        if (std::isfinite(runs[i].log_estimate)) L = std::max(L, runs[i].log_estimate);
    }
    if (!std::isfinite(L)) L = 0.0;
    std::vector<double> ybar(V), eP(V);
    double min_ess = INFINITY;
    bool alive_ok = true, ess_ok = true;
    for (int32_t p = 0; p < V; ++p) {
        double sy = 0.0, se2 = 0.0;
        std::vector<double> y(R);
        for (int32_t r = 0; r < R; ++r) {
            const perm_est_result &q = runs[(size_t)p * R + r];
            const double yr = std::isfinite(q.log_estimate) ? std::exp(q.log_estimate - L) : 0.0;
            // within-run standard error s / sqrt(M) = RSE * |Y| (0 without survivors)
            const double er = yr > 0.0 && std::isfinite(q.rse) ? q.rse * yr : 0.0;
            y[r] = yr;
            sy += yr;
            se2 += er * er;
            min_ess = std::min(min_ess, q.ess);
            if (q.n_alive < 1000) alive_ok = false;
            if (!(q.ess >= 1000.0)) ess_ok = false;
        }
        const double m = sy / R;
        double ss = 0.0;
        for (int32_t r = 0; r < R; ++r) ss += (y[r] - m) * (y[r] - m);
        const double e_in = std::sqrt(se2) / R;
        const double e_seed = std::sqrt(ss / (R - 1)) / std::sqrt((double)R);
        ybar[p] = m;
        eP[p] = std::max(e_in, e_seed);
    }
    double pcon = 0.0, e2 = 0.0, ymax = ybar[0], ymin = ybar[0];
    for (int32_t p = 0; p < V; ++p) {
        pcon += ybar[p];
        e2 += eP[p] * eP[p];
        ymax = std::max(ymax, ybar[p]);
        ymin = std::min(ymin, ybar[p]);
    }
    pcon /= V;
    const double econ = std::sqrt(e2) / V;
    double dmax = 0.0;
    for (int32_t a = 0; a < V; ++a)
        for (int32_t b = a + 1; b < V; ++b) {
            const double den = std::sqrt(eP[a] * eP[a] + eP[b] * eP[b]);
            const double diff = std::fabs(ybar[a] - ybar[b]);
            const double d = den > 0.0 ? diff / den : (diff == 0.0 ? 0.0 : INFINITY);
            dmax = std::max(dmax, d);
        }
    const double pairs = 0.5 * V * (V - 1);
    const double cb = phi_inv(1.0 - alpha / (2.0 * pairs));
    const double tc = t_crit(R - 1, 0.95);
    double lo_max = -INFINITY, hi_min = INFINITY;
    for (int32_t p = 0; p < V; ++p) {
        lo_max = std::max(lo_max, ybar[p] - tc * eP[p]);
        hi_min = std::min(hi_min, ybar[p] + tc * eP[p]);
    }
    const double rel_hw = pcon != 0.0 ? 1.96 * econ / std::fabs(pcon) : INFINITY;
    uint32_t checks = 0;
    if (present) checks |= PE_CON_ALL_RUNS;
    if (lo_max <= hi_min) checks |= PE_CON_T_INTERVALS;
    if (dmax <= cb) checks |= PE_CON_BONFERRONI;
    if (alive_ok) checks |= PE_CON_ALIVE;
    if (ess_ok) checks |= PE_CON_ESS;
    if (rel_hw <= 0.10) checks |= PE_CON_HALF_WIDTH;
    out->log_p_con = pcon > 0.0 ? L + std::log(pcon) : -INFINITY;
    out->log_e_con = econ > 0.0 ? L + std::log(econ) : -INFINITY;
    out->rel_half_width = rel_hw;
    out->variant_ratio = ymin > 0.0 ? ymax / ymin : INFINITY;
    out->min_ess = min_ess;
    out->d_max = dmax;
    out->c_bonf = cb;
    out->t_crit = tc;
    out->checks = checks;
    out->provisional = checks == PE_CON_ALL ? 1 : 0;
    for (int32_t p = 0; p < V; ++p) {
        if (log_ybar) log_ybar[p] = ybar[p] > 0.0 ? L + std::log(ybar[p]) : -INFINITY;
        if (rel_e) rel_e[p] = ybar[p] > 0.0 ? eP[p] / ybar[p] : INFINITY;
    }
    return PE_OK;
}

}  // namespace consensus
}  // namespace pe
