// Host-side constants of the Robust-l0 decoder: the posteriors p_breve_z and p_breve_e
// for Gaussian signal and noise, their float32 tables, the t-sweep and the outer-test
// thresholds.  Plain C++ in fp64; no device code.
//
// Paper references (arXiv 1704.09012):
//   eq:pz_gaussian / eq:pe_gaussian  full-series posteriors (Sec. 3, centred Gaussian case)
//   eq:pz_approx / eq:pe_approx      ell explicit terms plus one moment-matched Gaussian for
//                                    the remainder, variance from Lemma "Sums of centred
//                                    density functions"
//   eq:breve                         normalisation by the maximum, attained at w = 0
//   eq:finetune_c_cont / _quant      default decrement c of the t-sweep (continuous and
//                                    quantised scores)
//   Table "scores"                   quantised scores: indicators of the same posteriors
//   Sec. 4 "Stopping conditions"     tolerance m sigma sqrt(2/pi)
#include "constants.h"

#include "general.h"

#include <cmath>
#include <cstdint>
#include <cstring>

namespace rl0 {

namespace {

// lam^q / q!
double poisson_weight(double lam, int q) {
    if (lam <= 0.0) return q == 0 ? 1.0 : 0.0;
    return std::exp(q * std::log(lam) - std::lgamma(q + 1.0));
}

// sum_{q > ell} lam^q / q!  (the e^lam minus partial-sum remainder, summed directly)
double remainder_after(double lam, int ell) {
    double total = 0.0;
    int q = ell + 1;
    double term = poisson_weight(lam, q);
    for (;;) {
        total += term;
        ++q;
        term = term * lam / q;
        if (term <= total * 1e-18 || q > ell + 400) break;
    }
    return total;
}

// Odds form of one posterior: p(w) = 1 / (1 + sum_t C_t exp(a_t w^2)).  The q = 0 term
// (variance v0, weight 1) is the numerator density itself.
struct Odds {
    int count = 0;
    double C[40];
    double a[40];
    double eval(double w) const {
        const double w2 = w * w;
        double s = 0.0;
        for (int t = 0; t < count; ++t) s += C[t] * std::exp(a[t] * w2);
        return s;
    }
};

// kind 'z': rate d rho, base variance sn^2; kind 'e': rate 2 d rho, base variance 2 sn^2
Odds build_odds(char kind, int d, double rho, double sn, double ss, int ell, double* v0_out) {
    const double lam = (kind == 'z') ? d * rho : 2.0 * d * rho;
    const double v0 = (kind == 'z') ? sn * sn : 2.0 * sn * sn;
    Odds o;
    for (int q = 1; q <= ell; ++q) {
        const double wq = poisson_weight(lam, q);
        const double var = q * ss * ss + v0;
        o.C[o.count] = wq * std::sqrt(v0 / var);
        o.a[o.count] = 0.5 * (1.0 / v0 - 1.0 / var);
        ++o.count;
    }
    const double R = remainder_after(lam, ell);
    const double R_prev = remainder_after(lam, ell - 1);
    if (R > 0.0) {
        const double var_tail = (ss * ss * lam * R_prev + v0 * R) / R;
        o.C[o.count] = R * std::sqrt(v0 / var_tail);
        o.a[o.count] = 0.5 * (1.0 / v0 - 1.0 / var_tail);
        ++o.count;
    }
    *v0_out = v0;
    return o;
}

constexpr double kCutoff = 1.0 / 134217728.0;  // 2^-27

void build_table(char kind, int d, double rho, double sn, double ss, int ell, float* T,
                 float* inv_h, double* range) {
    double v0 = 0.0;
    const Odds o = build_odds(kind, d, rho, sn, ss, ell, &v0);
    const double one_plus_S0 = 1.0 + o.eval(0.0);
    auto breve = [&](double w) { return one_plus_S0 / (1.0 + o.eval(w)); };
    const double h0 = std::sqrt(v0) / 8.0;
    int q = 8;
    while (breve(q * h0) >= kCutoff) ++q;
    const double R = q * h0;
    for (int i = 0; i <= kTableN; ++i) T[i] = static_cast<float>(breve((double)i * R / kTableN));
    T[0] = 1.0f;
    *inv_h = static_cast<float>(kTableN / R);
    *range = R;
}

}  // namespace

float table_score(const float* T, float inv_h, float a) {
    // float32, each operation rounded, no contraction (this file is built with
    // -ffp-contract=off and x86-64 evaluates float in SSE single precision)
    const float u = a * inv_h;
    if (!(u < static_cast<float>(kTableN))) return 0.0f;
    const int i = static_cast<int>(u);
    const float f = u - static_cast<float>(i);
    const float t0 = T[i];
    const float t1 = T[i + 1];
    return t0 + f * (t1 - t0);
}

static uint32_t f2u(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }

// Smallest non-negative float a with fl32(1 - Tz(a)) >= t, as its bit pattern.  The
// tabulated score is non-increasing in a, so the outer test of Alg. 1 is a threshold.
static uint32_t outer_threshold_bits(const HostConstants& hc, float t) {
    if (hc.exact) return 1u;  // Parallel-l0: r != 0  <=>  |r| >= smallest subnormal
    auto passes = [&](uint32_t bits) {
        const float z = table_score(hc.table_z, hc.inv_h_z, u2f(bits));
        return (1.0f - z) >= t;
    };
    uint32_t lo = 0, hi = 0x7F800000u;  // +inf always passes for t <= 1
    if (passes(lo)) return 0u;
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (passes(mid)) hi = mid; else lo = mid;
    }
    return hi;
}

// Largest non-negative float a with T(a) >= level, as its bit pattern: the tabulated score
// is non-increasing in a, so the indicator 1{T(|a|) >= level} of the quantised scores is
// the threshold bits(|a|) <= this.  T(0) = 1 >= level for every level <= 1.
static uint32_t indicator_threshold_bits(const float* T, float inv_h, float level) {
    uint32_t lo = 0, hi = 0x7F800000u;   // T(lo) >= level; T(+inf) = 0
    if (table_score(T, inv_h, u2f(hi)) >= level) return hi;
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (table_score(T, inv_h, u2f(mid)) >= level) lo = mid; else hi = mid;
    }
    return lo;
}

double c_rule(double delta, double rho, bool quantised) {
    if (delta <= 0.05) return 0.01;
    if (!quantised) return 0.025;
    if (rho <= 0.1) return 0.05;
    if (rho <= 0.2) return 0.075;
    return 0.1;
}

int iterations_for(double c) { return static_cast<int>(std::ceil(1.0 / c - 1e-9)); }

bool compute_constants(const Problem& pr, HostConstants* hc) {
    hc->exact = (pr.sigma == 0.0);
    hc->quant = pr.variant == 1 && !hc->exact;   // sigma = 0: Parallel-l0's indicators either way
    hc->c = pr.c > 0.0 ? pr.c
                       : c_rule(static_cast<double>(pr.m) / pr.n, static_cast<double>(pr.k) / pr.m, pr.variant == 1);
    hc->n_iters = iterations_for(hc->c);
    if (pr.max_iters > 0 && pr.max_iters < hc->n_iters) hc->n_iters = pr.max_iters;
    const Law mu{pr.signal_law, pr.sigma_s}, nu{pr.noise_law, pr.sigma};
    // Sec. 4: ||r||_1 <= E||eta||_1 = m E|eta_i| (m sigma sqrt(2/pi) for Gaussian noise)
    hc->tol = pr.noise_law == kLawGaussian ? pr.m * pr.sigma * std::sqrt(2.0 / M_PI) : pr.m * pr.sigma / std::sqrt(2.0);
    const double rho = (pr.k_post > 0.0 ? pr.k_post : static_cast<double>(pr.k)) / pr.m;
    if (hc->exact) {
        std::memset(hc->table_z, 0, sizeof(hc->table_z));
        std::memset(hc->table_e, 0, sizeof(hc->table_e));
        hc->inv_h_z = hc->inv_h_e = 0.0f;
        hc->range_z = hc->range_e = 0.0;
    } else if (pr.tables) {
        std::memcpy(hc->table_z, pr.tables, sizeof(hc->table_z));
        std::memcpy(hc->table_e, pr.tables + kTableN + 1, sizeof(hc->table_e));
        hc->inv_h_z = pr.tables[2 * (kTableN + 1)];
        hc->inv_h_e = pr.tables[2 * (kTableN + 1) + 1];
        hc->range_z = kTableN / static_cast<double>(hc->inv_h_z);
        hc->range_e = kTableN / static_cast<double>(hc->inv_h_e);
    } else if (pr.signal_law != kLawGaussian || pr.noise_law != kLawGaussian) {
        if (!build_general_table('z', pr.d, rho, mu, nu, hc->table_z, &hc->inv_h_z, &hc->range_z) ||
            !build_general_table('e', pr.d, rho, mu, nu, hc->table_e, &hc->inv_h_e, &hc->range_e))
            return false;
    } else {
        build_table('z', pr.d, rho, pr.sigma, pr.sigma_s, pr.ell, hc->table_z, &hc->inv_h_z,
                    &hc->range_z);
        build_table('e', pr.d, rho, pr.sigma, pr.sigma_s, pr.ell, hc->table_e, &hc->inv_h_e,
                    &hc->range_e);
    }
    hc->t.resize(hc->n_iters);
    hc->tau_bits.resize(hc->n_iters);
    hc->qe_bits.assign(hc->n_iters, 0u);
    hc->qz_bits.assign(hc->n_iters, 0u);
    for (int it = 0; it < hc->n_iters; ++it) {
        hc->t[it] = static_cast<float>(1.0 - it * hc->c);
        hc->tau_bits[it] = outer_threshold_bits(*hc, hc->t[it]);
        if (hc->quant) {
            hc->qe_bits[it] = indicator_threshold_bits(hc->table_e, hc->inv_h_e, hc->t[it]);
            hc->qz_bits[it] = indicator_threshold_bits(hc->table_z, hc->inv_h_z, 1.0f - hc->t[it]);
        }
    }
    // smallest |difference| whose e-score is 0 (the table ends): bits of that float
    if (hc->exact) {
        hc->e_zero_bits = 1u;
    } else {
        uint32_t lo = 0, hi = 0x7F800000u;
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (!(u2f(mid) * hc->inv_h_e < static_cast<float>(kTableN))) hi = mid; else lo = mid;
        }
        hc->e_zero_bits = hi;
    }
    return true;
}

}  // namespace rl0
