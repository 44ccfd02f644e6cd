// The paper's reduced-rank basis model on the device (Sec. 2.1, Eqs. BMKL,
// Solin_representation and hpar_prior; features in the appendix on the
// reduced-rank representation): f = Phi a + b with sinusoidal features
// sin(pi m (x + L) / 2L) per Gaussian-kernel covariate and the covariate
// itself per linear one, a_j ~ N(0, var_j) with var_j = c_g V_m(sigma_g) or
// c_l, b ~ N(0, Sigma), and inverse-Gamma priors on c_g, sigma_g, c_l.
// q = (a_1..a_F, b, c_g, sigma_g, c_l), D = F + 4.
#pragma once
#include "common.h"

namespace rmhmc {

struct BasisDev {
  int N = 0;          // records
  int F = 0;          // basis features (coefficients a)
  int Fa = 0;         // F + 1: the features and the bias column
  double bias_var = 1.0;
  double ig_a[3] = {0, 0, 0}, ig_b[3] = {0, 0, 0};   // InvGamma of (c_g, sigma_g, c_l)
  double* Phi = nullptr;     // N x Fa, column-major (ld N); column F is all ones
  int* kind = nullptr;       // F: 0 Gaussian kernel (c_g, sigma_g), 1 linear (c_l)
  double* kappa = nullptr;   // F: pi^2 m^2 / (16 L^2) for Gaussian features, 0 for linear
};

// Phi from the covariates X (dx x N, X[c * N + i]) and, per feature, its
// covariate column and frequency m (0 for linear features).
void basis_features(const BasisDev& bd, const double* X, const int* col, const int* freq,
                    double L, hipStream_t st);

// U (scal[1]), sum of the per-record l (scal[3]), grad U (D) and the
// Hessian H (Dp x Dp, ld Dp, zero padding) at q; f (N) and lik
// (LIK_SLOTS x N, as lik_derivs) are written on the way.  work: N x Fa.
// A hyperparameter outside (0, inf) leaves non-finite values in U and H.
void basis_hessian(const BasisDev& bd, int lik, double noise_var, double beta, const double* y,
                   const double* q, double* f, double* likv, double* H, int Dp, double* gradU,
                   double* scal, double* work, hipStream_t st);

// v_i = tr(W dH/dq_i) (W symmetric, Dp x Dp, ld Dp; v of length D) at the
// point whose likelihood derivatives basis_hessian left in likv.
// work: N x Fa + N.
void basis_contract(const BasisDev& bd, double beta, const double* q, const double* likv,
                    const double* W, int Dp, double* v, double* work, hipStream_t st);

}  // namespace rmhmc
