// Score tables for non-Gaussian signal and noise laws (Thm "Probabilities for general
// signal and noise distributions", eq:pz_general / eq:pe_general).  Host code, fp64.
#pragma once

namespace rl0 {

// Laws of the signal entries (mu) and of the noise (nu): symmetric about 0, each given by
// its standard deviation.
enum LawFamily { kLawGaussian = 0, kLawLaplace = 1 };

struct Law {
    int family = kLawGaussian;
    double s = 1.0;   // standard deviation
};

// T[0..kTableN] = fl32(p_breve(i R / kTableN)) of p_z (kind 'z') or p_e (kind 'e') for
// GM with rate d rho, the same construction as the Gaussian tables: R = q h0 for the
// smallest q >= 8 with p_breve(q h0) < 2^-27, h0 = sqrt(v0) / 8, v0 = Var(nu) (z) or
// 2 Var(nu) (e); T[0] = 1; p_breve = p / p(0); a later entry above an earlier one is
// lowered to it (the kernels take the tables to be non-increasing).  False if the
// posterior's numerics do not settle (no table is written then).
bool build_general_table(char kind, int d, double rho, Law mu, Law nu, float* T, float* inv_h, double* range);

// p_z(w) or p_e(w) of the theorem (unnormalised), for tests of the builder.
double general_posterior(char kind, int d, double rho, Law mu, Law nu, double w);

// E|eta| for eta ~ nu: s sqrt(2/pi) (Gaussian), s / sqrt(2) (Laplace).
double noise_abs_mean(Law nu);

}  // namespace rl0
