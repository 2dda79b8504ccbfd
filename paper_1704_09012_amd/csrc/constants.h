// Host-side constants of the Robust-l0 decoder (see constants.cpp).
#pragma once

#include <cstdint>
#include <vector>

namespace rl0 {

constexpr int kTableN = 4096;

struct Problem {
    int n = 0, m = 0, d = 0, k = 0;
    double sigma = 0.0, sigma_s = 1.0;
    double c = 0.0;
    int ell = 4;
    int max_iters = 0;
    int variant = 0;   // 0 continuous scores, 1 quantised
    double k_post = 0.0;   // the sparsity the posteriors assume (adaptive_k); 0 = k
    int signal_law = 0, noise_law = 0;   // LawFamily of mu and nu (both Gaussian: eq:pz_approx)
    const float* tables = nullptr;       // given score tables: T_z, T_e ([kTableN + 1] each), inv_h_z, inv_h_e
    unsigned long long tables_hash = 0;  // of those floats (the constants cache's key)
};

struct HostConstants {
    bool exact = false;
    double c = 0.0, tol = 0.0;
    int n_iters = 0;
    double range_z = 0.0, range_e = 0.0;
    float inv_h_z = 0.0f, inv_h_e = 0.0f;
    float table_z[kTableN + 1];
    float table_e[kTableN + 1];
    std::vector<float> t;            // t_it = fl32(1 - it c)
    std::vector<uint32_t> tau_bits;  // outer test threshold per iteration (float bits)
    uint32_t e_zero_bits = 0;        // |v_p - v_l| >= this  =>  e-score 0
    bool quant = false;              // quantised scores (never with exact = true)
    std::vector<uint32_t> qe_bits;   // per iteration: Te(a) >= t      iff bits(a) <= qe_bits
    std::vector<uint32_t> qz_bits;   // per iteration: Tz(a) >= 1 - t  iff bits(a) <= qz_bits
};

double c_rule(double delta, double rho = 0.0, bool quantised = false);
int iterations_for(double c);
// False if the posteriors of the given laws cannot be tabulated.
bool compute_constants(const Problem& pr, HostConstants* hc);
float table_score(const float* T, float inv_h, float a);

}  // namespace rl0
