// Softabs eigendecomposition: block Jacobi workspace and helpers.
#pragma once
#include "common.h"

namespace rmhmc {

struct EigWork {
  double* M = nullptr;     // Dp x Dp working matrix (ld Dp)
  double* M2 = nullptr;    // second buffer
  double* Psi = nullptr;   // Dp x Dp eigenvectors (columns), identity-padded
  double* V = nullptr;     // per-slot 32 x 32 rotations, two sets (eig_rotation_doubles)
  double* part = nullptr;  // reduction partials
  double* ctrl = nullptr;  // device control block (EIG_CTRL_DOUBLES): norm, stop flag, counts
  double* ctrl_host = nullptr;  // pinned host mirror of ctrl
};
constexpr int EIG_CTRL_DOUBLES = 32;
// Stopping rules of the Jacobi solve (see eig.hip); RMHMC_EIG_STOP=polish in
// the environment selects the older one.
enum { EIG_STOP_POLISH = 0, EIG_STOP_METRIC = 1 };
int eig_stop_rule();
double eig_stop_zeta_scaled();
bool eig_trace();
// Doubles of EigWork::part for a padded dimension Dp.
long eig_part_doubles(int Dp);

int eig_padded_dim(int D);
void eig_workspace_sizes(int D, long* doubles);
// Copy H (D x D, ldh) into w.M (symmetrised, zero-padded).
void eig_load_matrix(int D, const double* H, long ldh, EigWork& w, hipStream_t st);
// w.Psi = diag(Q, I) (Q == nullptr: identity).
void eig_load_basis(int D, const double* Q, long ldq, EigWork& w, hipStream_t st);
// Jacobi on w.M, rotations accumulated into w.Psi; converged matrix left in w.M.
// max_inner names the solve: JACOBI_INNER_DYNAMIC for a warm start,
// JACOBI_INNER_STATIC for a solve from the identity.  Both run one inner
// sweep per round on the cross schedule (up to four inner sweeps per round
// left a static solve at D = 1038 at the same 18 outer sweeps, 84 against
// 22 ms); they are timed as separate kernel families.
constexpr int JACOBI_INNER_STATIC = 4;
constexpr int JACOBI_INNER_DYNAMIC = 1;
// Doubles of EigWork::V for a padded dimension Dp: two sets of 32 x 32
// rotations, one per slot (double-buffered across rounds).
inline long eig_rotation_doubles(int Dp) { return 2L * (Dp / 32) * 32 * 32; }

// Result of a solve, known on the host only when it checked convergence.
struct JacobiResult {
  int sweeps = -1;          // sweeps applied (-1: not read back)
  bool converged = true;    // false: max_sweeps ran out (or non-finite entries)
  bool nonfinite = false;
};
// Sweeps are launched `blind` at a time without the host looking: every
// launch first reads a stop flag that the convergence check after each sweep
// sets on the device, so sweeps launched past convergence exit at once.  With
// host_check the host then reads the flag after each further sweep until it
// is set or max_sweeps have run; without it (graph capture) exactly
// max(blind, 1) sweeps are launched and nothing is read back.  On the device:
// *fail |= 4 if the solve did not converge, 8 if it met non-finite entries
// (fail may be null); dstats[0] += 1, dstats[1] += sweeps (may be null).
// gfloor: the smallest value of the softabs map (1 / alpha), the scale below
// which an eigenvalue's size no longer matters to G^-1.
// zeta_s: the tolerance of the scaled test of the metric stopping rule
// (<= 0: eig_stop_zeta_scaled()).
JacobiResult jacobi_eig(int D, EigWork& w, double zeta, double gfloor, int max_sweeps,
                        int max_inner, int blind, bool host_check, int* fail, double* dstats,
                        hipStream_t st, double zeta_s = -1.0);
// Rayleigh quotients lam_i = psi_i' H psi_i of the converged basis against the
// original H (D x D, ldh), written to diag(w.M); Z is Dp x Dp scratch.
// One Newton-Schulz step Psi <- Psi (3I - Psi'Psi) / 2 on the D x D block of
// a Dp-strided basis: removes the rounding drift from orthogonality to second
// order.  T1, T2: Dp x Dp scratch.
// (split: optional split-K partials, nsplit x D x D, for the D x D products)
void orthonormalise(int D, int Dp, double* Psi, double* T1, double* T2, hipStream_t st,
                    double* split = nullptr, int nsplit = 1);

void rayleigh_refine(int D, const double* H, long ldh, EigWork& w, double* Z, hipStream_t st,
                     double* split = nullptr, int nsplit = 1);
// lam = diag(M); g, g' and log|G| of the softabs map `kind` (rmhmc_softabs).
void softabs_finalize(int D, const double* M, long ldm, double alpha, int kind, double* lam,
                      double* g, double* gp, double* logdetG, hipStream_t st);
// M1(j,k) = T_jk b_j b_k with T the divided differences of g.
void t_bb(int D, const double* lam, const double* b, double alpha, int kind, double* M1, long ld,
          hipStream_t st);
// B(:, j) = A(:, j) * num[j] / den[j]  (either may be null)
void scale_cols(int m, int n, const double* A, long lda, const double* num, const double* den,
                double* B, long ldb, hipStream_t st);
// y = x * (sqrt)num / den elementwise (either may be null)
void vec_scale(int n, const double* x, const double* num, const double* den, bool sqrt_num,
               double* y, hipStream_t st);

}  // namespace rmhmc
