// Latent-GP model pieces on the device: kernel matrix and hyperparameter
// derivatives generated on the fly, likelihood derivatives, and the small
// reductions the Hessian and the third-derivative contraction need.
#pragma once
#include "common.h"

namespace rmhmc {

constexpr int MAX_TERMS = 8;
constexpr int MAX_P = 24;
constexpr int MAX_TUPLES = 64;

struct TermDev {
  int kind, ncols, p0, np;
  int cols[RMHMC_MAX_TERM_COLS];
  int fn;               // latent function the term belongs to (-1: all points)
};

// Everything a kernel needs to evaluate K(eta) and its derivatives at (i, j).
struct ModelDev {
  int N, dx, P, nterms;
  double jitter;
  const double* X;     // dx x N: X[c * N + i]
  int fn_col;          // column of X with each point's latent function, -1: one function
  TermDev terms[MAX_TERMS];
  int param_term[MAX_P];
};

// A derivative index tuple (order 1..3), all indices in one kernel term.
struct Tuple {
  int ord, l, m, n;
};

// K and K_l (materialised), jitter on the diagonal of K.
void kgen(const ModelDev& md, const double* eta, double* K, double* K1, hipStream_t st);

// out[w * nt + t] = sum_ij Wgt_w(i,j) * d^ord K / d eta_tuple(i,j).
// mode 0: one weight Phi = (K^-1 - alpha alpha')/2 built from Kinv and alpha;
// mode 1: nw weights from a stack (stride N*N).
// tuples: on the device; tuples_h: the same list on the host (its terms set
// the passes).
void kd_wsum(const ModelDev& md, const double* eta, const Tuple* tuples, const Tuple* tuples_h,
             int nt, int mode, const double* Kinv, const double* alpha, const double* Wstack,
             int nw, double* out, double* work, hipStream_t st);

// out[w * nt + t] = sum_ij W_w(i,j) * d^ord K / d eta_tuple(i,j) for nw weights
// from a stack (stride N*N): the tuple derivatives are generated once into
// KT (at most MAX_TUPLES x N*N values) and contracted with every weight by a
// deterministic tall-K GEMM (`tallwork`: tallk_splits(N*N) * MAX_TUPLES * nw).
void kd_wsum_stack(const ModelDev& md, const double* eta, const Tuple* tuples,
                   const Tuple* tuples_h, int nt, const double* Wstack, int nw, double* out,
                   double* KT, double* tallwork, hipStream_t st);

// y[(x * nt + t) * N + i] = sum_j d K_tuple(i,j) x_x(j), for nx vectors x (stride N).
// The j range is split over KD_MV_SPLIT workgroup columns; `work` holds
// KD_MV_SPLIT * min(nt, MAX_TUPLES) * nx * N partial sums.
constexpr int KD_MV_SPLIT = 32;
void kd_matvec(const ModelDev& md, const double* eta, const Tuple* tuples, const Tuple* tuples_h,
               int nt, const double* x, int nx, double* y, double* work, hipStream_t st);

// Likelihood derivatives in the latent coordinates, out[0..LIK_SLOTS * N):
//   [0, N)   l_i (per record; zero at the second function's points)
//   [N, 2N)  gradient;  [2N, 3N) diagonal of the Hessian;
//   [3N, 4N) diagonal third derivatives d^3 L / df_k^3;
// and, for the mean/variance model (R = N / 2 records, a = f1_i, b = f2_i):
//   [4N, 4N+R) l_ab, [4N+R, 5N) l_aab, [5N, 5N+R) l_abb, [5N+R, 6N) zero.
constexpr int LIK_SLOTS = 6;
void lik_derivs(int N, int lik, double noise_var, double delta, const double* f, const double* y,
                double* out, hipStream_t st);

// out[a * ny + b] = x_a . y_b  (length n, x stride sx, y stride sy)
void pair_dots(int n, const double* x, long sx, int nx, const double* y, long sy, int ny,
               double* out, hipStream_t st);

}  // namespace rmhmc
