// Posteriors for non-Gaussian laws (Thm "Probabilities for general signal and noise
// distributions") and their score tables.  Plain C++ in fp64; no device code.
//
// With lambda = d rho (p_z) or 2 d rho (p_e) and B the noise density nu (p_z) or the
// density nu~ of the difference of two noise values (p_e), both posteriors have the form
// B(w) / D(w) with
//     D(w) = sum_{q >= 0} lambda^q / q! (B * mu_q)(w)
//          = B(w) + lambda (B * mu)(w) + R(w),
// mu_q the q-fold convolution of the signal law (symmetric, so mu-bar = mu).  The q = 1
// term is one convolution of two known densities, taken here by Gauss-Legendre
// quadrature in direct space (B is narrow: 60 of its standard deviations either side,
// panel breaks at the kinks of the Laplace densities).  The rest, R, has the Fourier
// transform phi_B (exp(lambda phi_mu) - 1 - lambda phi_mu) (the characteristic
// functions of B and mu), which decays at least as fast as phi_B phi_mu^2, so
//     R(w) = (1/pi) int_0^inf phi_B(t) (exp(lambda phi_mu(t)) - 1 - lambda phi_mu(t)) cos(w t) dt
// is taken by Gauss-Legendre quadrature on panels no wider than a quarter period of the
// fastest cosine, up to where the integrand's tail is negligible.
#include "general.h"

#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "constants.h"

namespace rl0 {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kCutoff = 1.0 / 134217728.0;   // 2^-27
constexpr int kGL = 8;                           // Gauss-Legendre nodes per panel

// Nodes x and weights w of the kGL-point Gauss-Legendre rule on [-1, 1], by Newton's
// iteration on the Legendre polynomial (three-term recurrence).
struct GaussLegendre {
    double x[kGL], w[kGL];
    GaussLegendre() {
        for (int i = 0; i < kGL; ++i) {
            double z = std::cos(kPi * (i + 0.75) / (kGL + 0.5));
            double dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= kGL; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = kGL * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};
const GaussLegendre& gl() {
    static const GaussLegendre g;
    return g;
}

double density(const Law& L, double x) {
    if (L.family == kLawGaussian) return std::exp(-0.5 * (x / L.s) * (x / L.s)) / (L.s * std::sqrt(2.0 * kPi));
    const double b = L.s / kSqrt2;
    return std::exp(-std::fabs(x) / b) / (2.0 * b);
}

double charfun(const Law& L, double t) {
    if (L.family == kLawGaussian) return std::exp(-0.5 * L.s * L.s * t * t);
    const double b = L.s / kSqrt2;
    return 1.0 / (1.0 + b * b * t * t);
}

// The base density B and its characteristic function: nu (kind 'z') or nu~ (kind 'e').
struct Base {
    Law nu;
    bool diff;
    double s;   // its standard deviation
    double dens(double x) const {
        if (!diff) return density(nu, x);
        if (nu.family == kLawGaussian) return density(Law{kLawGaussian, nu.s * kSqrt2}, x);
        const double b = nu.s / kSqrt2, a = std::fabs(x) / b;
        return (1.0 + a) * std::exp(-a) / (4.0 * b);
    }
    double phi(double t) const {
        const double f = charfun(nu, t);
        return diff ? f * f : f;
    }
};

// exp(x) - 1 - x without cancellation for small x
double expm1_minus(double x) {
    if (std::fabs(x) < 1e-3) return x * x * 0.5 * (1.0 + x / 3.0 * (1.0 + x / 4.0 * (1.0 + x / 5.0)));
    return std::expm1(x) - x;
}

// (B * mu)(w) = int B(y) mu(w - y) dy by composite Gauss-Legendre over |y| <= 60 sd(B),
// with panel breaks at y = 0 and y = w
double conv_direct(const Base& B, const Law& mu, double w) {
    const GaussLegendre& g = gl();
    const double Y = 60.0 * B.s;
    double br[4] = {-Y, 0.0, w, Y};
    std::sort(br, br + 4);
    const double panel = B.s / 4.0;
    double total = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double a = br[k], b = br[k + 1];
        if (!(b > a)) continue;
        const int np = std::max(1, static_cast<int>(std::ceil((b - a) / panel)));
        const double h = (b - a) / np;
        for (int p = 0; p < np; ++p) {
            const double c = a + (p + 0.5) * h;
            double s = 0.0;
            for (int i = 0; i < kGL; ++i) {
                const double y = c + 0.5 * h * g.x[i];
                s += g.w[i] * B.dens(y) * density(mu, w - y);
            }
            total += 0.5 * h * s;
        }
    }
    return total;
}

// Nodes and weights (with 1/pi) of the remainder's Fourier integral, the weights already
// multiplied by the integrand without its cosine.
struct FourierRule {
    std::vector<double> t, gw;
};

// Empty if the integrand does not fall below the accuracy target within 2^24 nodes.
FourierRule fourier_rule(const Base& B, const Law& mu, double lam, double w_max) {
    const GaussLegendre& g = gl();
    auto integrand = [&](double t) { return B.phi(t) * expm1_minus(lam * charfun(mu, t)); };
    const double fine = 0.125 / std::max(mu.s, B.s);                   // the finest scale of phi_mu, phi_B
    const double dcos = 0.5 * kPi / std::max(w_max, 1e-300);            // a quarter period of cos(w_max t)
    // absolute accuracy: far below the denominator anywhere on the table range
    const double eps = 1e-17 * (B.dens(0.0) + lam * density(mu, 0.0));
    const double t_min = 64.0 / std::max(mu.s, B.s);
    FourierRule r;
    double t0 = 0.0;
    for (;;) {
        const double h = std::min(dcos, std::max(fine, 0.125 * t0));
        const double c = t0 + 0.5 * h;
        for (int i = 0; i < kGL; ++i) {
            const double t = c + 0.5 * h * g.x[i];
            r.t.push_back(t);
            r.gw.push_back(0.5 * h * g.w[i] * integrand(t) / kPi);
        }
        t0 += h;
        // the integrand decays at least as a power t^-p with p >= 4 past its features, so
        // its tail beyond t0 is below t0 |g(t0)|
        if (t0 >= t_min && t0 * std::fabs(integrand(t0)) < eps) break;
        if (r.t.size() > (1u << 24)) return FourierRule{};
    }
    return r;
}

struct Posterior {
    bool ok = false;
    Base B;
    Law mu;
    double lam;
    FourierRule rule;
    double value(double w) const {
        double R = 0.0;
        for (size_t i = 0; i < rule.t.size(); ++i) R += rule.gw[i] * std::cos(w * rule.t[i]);
        const double num = B.dens(w);
        return num / (num + lam * conv_direct(B, mu, w) + R);
    }
};

Posterior make_posterior(char kind, int d, double rho, Law mu, Law nu, double w_max) {
    Posterior P;
    P.B.nu = nu;
    P.B.diff = kind == 'e';
    P.B.s = P.B.diff ? nu.s * kSqrt2 : nu.s;
    P.mu = mu;
    P.lam = (kind == 'e' ? 2.0 : 1.0) * d * rho;
    P.rule = fourier_rule(P.B, mu, P.lam, w_max);
    P.ok = !P.rule.t.empty();
    return P;
}

}  // namespace

double general_posterior(char kind, int d, double rho, Law mu, Law nu, double w) {
    const Posterior P = make_posterior(kind, d, rho, mu, nu, std::max(std::fabs(w), 1e-300));
    return P.ok ? P.value(w) : NAN;
}

bool build_general_table(char kind, int d, double rho, Law mu, Law nu, float* T, float* inv_h, double* range) {
    const double v0 = nu.s * nu.s * (kind == 'e' ? 2.0 : 1.0);
    const double h0 = std::sqrt(v0) / 8.0;
    const Posterior P0 = make_posterior(kind, d, rho, mu, nu, 1e-300);
    if (!P0.ok) return false;
    const double p0 = P0.value(0.0);
    // the range search: each candidate with a rule fitted to its own frequency
    int q = 8;
    for (;;) {
        const double w = q * h0;
        const Posterior Pw = make_posterior(kind, d, rho, mu, nu, w);
        if (!Pw.ok) return false;
        if (Pw.value(w) / p0 < kCutoff) break;
        if (++q > (1 << 16)) return false;
    }
    const double R = q * h0;
    const Posterior P = make_posterior(kind, d, rho, mu, nu, R);
    if (!P.ok) return false;
    const int nt = static_cast<int>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    std::vector<double> vals(kTableN + 1);
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int i = t; i <= kTableN; i += nt) vals[i] = P.value(static_cast<double>(i) * R / kTableN);
        });
    for (auto& th : pool) th.join();
    T[0] = 1.0f;
    for (int i = 1; i <= kTableN; ++i) {
        T[i] = static_cast<float>(vals[i] / p0);
        if (T[i] > T[i - 1]) T[i] = T[i - 1];
    }
    *inv_h = static_cast<float>(kTableN / R);
    *range = R;
    return true;
}

double noise_abs_mean(Law nu) {
    if (nu.family == kLawGaussian) return nu.s * std::sqrt(2.0 / kPi);
    return nu.s / kSqrt2;
}

}  // namespace rl0
