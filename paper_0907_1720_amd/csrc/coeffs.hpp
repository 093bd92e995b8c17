// Host-side model construction (once per problem): relaxation polynomials,
// beta_k, the corrections A_k0, the auxiliary moments Pi_k0, the scaled
// moments Pi_bar_k and their collapse through M_q^{-1} into one polynomial in
// phi per population.  All arithmetic is 113-bit (__float128) on the exact
// binary values of the inputs; every table entry is rounded to double once.
#pragma once

#include <cstdint>

#include "lbmhpde.h"

namespace lbm {

constexpr int kMaxQ = 7;
constexpr int kMaxDeg = 19;   // Pi_1 of degree 4: (Pi_1')^6 has degree 18, Pi_60 degree 19
constexpr int kGClasses = 4;  // non-polynomial Pi: distinct fractional parts of the exponents
constexpr int kGDeg = 11;     // non-polynomial Pi: integer degree within one class

struct Model {
  int q = 5;
  int m = 1;
  int D = 1;                   // degree of the equilibrium polynomials
  int scheme = 1;
  double tau = 1.0;
  double c = 1.0;              // dx / dt
  // f_eq_j(phi) = sum_d G[j][d] phi^d  (steps a2-a3 collapsed)
  double G[kMaxQ][kMaxDeg + 1] = {};
  // BGK with omega = 1/tau folded in: f*_j = w0 f_j + sum_d wG[j][d] phi^d
  double wG[kMaxQ][kMaxDeg + 1] = {};
  double w0 = 0.0;
  // FP32 deviation storage about the rest state phi_rest:
  // f_eq_j(phi_rest + delta) - f_rest_j = sum_{d >= 1} H[j][d] delta^d
  double phi_rest = 0.0;
  double f_rest[kMaxQ] = {};
  double wfrest[kMaxQ] = {};   // omega * f_rest_j
  double wG0rest[kMaxQ] = {};  // omega * (G[j][0] - f_rest_j), rounded once
  double H[kMaxQ][kMaxDeg + 1] = {};
  double wH[kMaxQ][kMaxDeg + 1] = {};
  // the 113-bit table, kept for the rest-state shift
  __float128 Gq[kMaxQ][kMaxDeg + 1] = {};
  // Non-polynomial Pi (real exponents, Sec. III.C families with real n, p, q):
  // f_eq_j(phi) = sum_c phi^gnu[c] sum_d gG[c][j][d] phi^d, gnu[0] = 0 and
  // gnu[c] in (0, 1) the distinct fractional parts; G above is unused then
  int gF = 0;                  // number of classes; 0 = polynomial model
  double gnu[kGClasses] = {};
  double gG[kGClasses][kMaxQ][kGDeg + 1] = {};
  double gwG[kGClasses][kMaxQ][kGDeg + 1] = {};   // omega * gG
  __float128 gGq[kGClasses][kMaxQ][kGDeg + 1] = {};
  __float128 gnuq[kGClasses] = {};
  // strided layout of each class (the kernels evaluate it by Horner in
  // phi^gstep): every nonzero degree of class c is gd0[c] + gstep[c] i, i < gK[c]
  int gd0[kGClasses] = {};
  int gstep[kGClasses] = {};
  int gK[kGClasses] = {};
};

// f_eq_j(phi) of a non-polynomial model in long double (host checks, rest state)
long double general_feq(const Model& m, int j, long double phi);
// d f_eq_j / d phi of a non-polynomial model (phi > 0)
long double general_dfeq(const Model& m, int j, long double phi);

// Validates the descriptor and builds the model; changes nothing on failure.
lbm_status build_model(const lbm_desc& d, Model* out);

// Fills phi_rest, f_rest, H and wH for the rest state phi_rest.
void set_rest_state(Model* mdl, double phi_rest);

// Resolved order m and lattice size q of a descriptor (0 on invalid input).
int resolved_order(const lbm_desc& d);
int resolved_lattice(const lbm_desc& d);

int lattice_velocity(int q, int j);   // e_j of D1Q<q>

// Largest |eigenvalue| over Fourier modes kappa in (0, pi] of the scheme
// linearised about uniform states phi_bar in [phi_min, phi_max] (5 states,
// 128 modes): the growth factor per step of the most amplified mode.
double stability_growth(const Model& m, double phi_min, double phi_max);

}  // namespace lbm
