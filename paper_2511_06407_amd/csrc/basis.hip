// Reduced-rank basis model (declarations and paper anchors in basis.h).
//
// Likelihood part, in the order of Sec. 2.3: with f = Phi (a, b),
//   grad = Phi' (beta l'),  H_ab = Phi' diag(beta l'') Phi,
//   v_ab(W) = Phi' [ beta l''' (.) rowsum((Phi W_ab) (.) Phi) ],
// two GEMMs on the matrix cores and a row reduction.  Prior part: each
// coefficient a_j enters u_j = a_j^2 e^{-s_j} / 2 + s_j / 2 (+ const) with
// s_j = ln var_j, a function of its hyperparameters only (ln c_g +
// ln sqrt(pi sigma_g) - kappa_j sigma_g, or ln c_l); every derivative of u_j
// follows from the chain rule through s_j, so the prior adds a diagonal, the
// couplings a_j - (c_g, sigma_g | c_l) and a 3 x 3 hyperparameter block, all
// O(F) work in one workgroup with fixed-order reductions.
#include "basis.h"
#include "gp.h"

namespace rmhmc {
namespace {

constexpr double kLn2Pi = 1.8378770664093454836;
constexpr double kPi = 3.14159265358979323846;
constexpr int BT = 256;   // threads of the prior workgroup

__global__ void basis_features_kernel(int N, int F, const double* __restrict__ X,
                                      const int* __restrict__ col, const int* __restrict__ freq,
                                      const int* __restrict__ kind, double L,
                                      double* __restrict__ Phi) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * (F + 1)) return;
  const int i = (int)(e % N), j = (int)(e / N);
  double v = 1.0;
  if (j < F) {
    const double x = X[(long)col[j] * N + i];
    v = kind[j] == 0 ? sin(kPi * freq[j] * (x + L) / (2.0 * L)) : x;
  }
  Phi[e] = v;
}

// out[i + j N] = s * l''_i Phi[i + j N]
__global__ void row_scale_kernel(int N, int Fa, double s, const double* __restrict__ l2,
                                 const double* __restrict__ Phi, double* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * Fa) return;
  out[e] = s * l2[e % N] * Phi[e];
}

// t_i = s * l'''_i * sum_j G[i + j N] Phi[i + j N]  (one thread per record)
// 64 rows per workgroup, their feature columns split over 16 phases (thread
// (row r, phase g) takes columns g, g + 16, ...), the phases' sums added in
// LDS in a fixed order: a few hundred rows still give every workgroup 16
// waves with short loops.
constexpr int RD_ROWS = 64, RD_PHASES = 16;
__global__ __launch_bounds__(RD_ROWS * RD_PHASES) void rowdot_kernel(
    int N, int Fa, double s, const double* __restrict__ l3, const double* __restrict__ G,
    const double* __restrict__ Phi, double* __restrict__ t) {
  __shared__ double sh[RD_PHASES][RD_ROWS];
  const int r = threadIdx.x % RD_ROWS, g = threadIdx.x / RD_ROWS;
  const int i = blockIdx.x * RD_ROWS + r;
  double acc = 0.0;
  if (i < N) {
#pragma unroll 4
    for (int j = g; j < Fa; j += RD_PHASES) acc += G[i + (long)j * N] * Phi[i + (long)j * N];
  }
  sh[g][r] = acc;
  __syncthreads();
  if (g == 0 && i < N) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < RD_PHASES; ++q) sum += sh[q][r];
    t[i] = s * l3[i] * sum;
  }
}

// Derivatives of s_j = ln var_j in its hyperparameters: index (into q),
// s_x, s_xx, s_xxx; the mixed second derivatives vanish.
struct SDerivs {
  int n;
  int idx[2];
  double s, sx[2], sxx[2], sxxx[2];
};

__device__ __forceinline__ SDerivs s_derivs(const BasisDev& bd, const double* q, int j) {
  const int F = bd.F;
  SDerivs d;
  if (bd.kind[j] == 0) {
    const double cg = q[F + 1], sg = q[F + 2];
    d.n = 2;
    d.idx[0] = F + 1;
    d.idx[1] = F + 2;
    d.s = log(cg) + 0.5 * log(kPi * sg) - bd.kappa[j] * sg;
    d.sx[0] = 1.0 / cg;
    d.sxx[0] = -1.0 / (cg * cg);
    d.sxxx[0] = 2.0 / (cg * cg * cg);
    d.sx[1] = 0.5 / sg - bd.kappa[j];
    d.sxx[1] = -0.5 / (sg * sg);
    d.sxxx[1] = 1.0 / (sg * sg * sg);
  } else {
    const double cl = q[F + 3];
    d.n = 1;
    d.idx[0] = F + 3;
    d.idx[1] = F + 3;
    d.s = log(cl);
    d.sx[0] = 1.0 / cl;
    d.sxx[0] = -1.0 / (cl * cl);
    d.sxxx[0] = 2.0 / (cl * cl * cl);
    d.sx[1] = d.sxx[1] = d.sxxx[1] = 0.0;
  }
  return d;
}

// hyperparameter slot (0 c_g, 1 sigma_g, 2 c_l) of an index into q
__device__ __forceinline__ int hslot(const BasisDev& bd, int idx) { return idx - bd.F - 1; }

// -ln InvGamma(theta; a, b) and its first three derivatives
__device__ __forceinline__ void inv_gamma(double th, double a, double b, double* g) {
  g[0] = -a * log(b) + lgamma(a) + (a + 1.0) * log(th) + b / th;
  g[1] = (a + 1.0) / th - b / (th * th);
  g[2] = -(a + 1.0) / (th * th) + 2.0 * b / (th * th * th);
  g[3] = 2.0 * (a + 1.0) / (th * th * th) - 6.0 * b / (th * th * th * th);
}

// Fixed-order block reduction of NV values per thread (in place in sh).
template <int NV>
__device__ __forceinline__ void block_reduce(double (*sh)[BT]) {
  __syncthreads();
  for (int s = BT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
    __syncthreads();
  }
}

// Prior part of U, grad U and H (one workgroup of BT threads).  Adds to the
// likelihood entries already in grad[0..F] and H[0..F, 0..F]; sets the
// hyperparameter entries of grad and H; U = beta * scal[3] + prior.
__global__ __launch_bounds__(BT) void basis_prior_kernel(BasisDev bd, double beta,
                                                         const double* __restrict__ q, double* H,
                                                         int Dp, double* grad, double* scal) {
  __shared__ double sh[8][BT];
  const int F = bd.F;
  // [0..2] grad of (c_g, sigma_g, c_l); [3] H_cc, [4] H_ss, [5] H_cs, [6] H_ll; [7] U
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = threadIdx.x; j < F; j += BT) {
    const SDerivs d = s_derivs(bd, q, j);
    const double a = q[j];
    const double e = exp(-d.s);
    const double us = 0.5 * (1.0 - a * a * e), uss = 0.5 * a * a * e;
    grad[j] += a * e;
    H[j + (long)j * Dp] += e;
    for (int x = 0; x < d.n; ++x) {
      const double c = -a * e * d.sx[x];
      H[j + (long)d.idx[x] * Dp] = c;
      H[d.idx[x] + (long)j * Dp] = c;
      acc[hslot(bd, d.idx[x])] += us * d.sx[x];
    }
    if (d.n == 2) {
      acc[3] += uss * d.sx[0] * d.sx[0] + us * d.sxx[0];
      acc[4] += uss * d.sx[1] * d.sx[1] + us * d.sxx[1];
      acc[5] += uss * d.sx[0] * d.sx[1];
    } else {
      acc[6] += uss * d.sx[0] * d.sx[0] + us * d.sxx[0];
    }
    acc[7] += 0.5 * a * a * e + 0.5 * d.s + 0.5 * kLn2Pi;
  }
  for (int k = 0; k < 8; ++k) sh[k][threadIdx.x] = acc[k];
  block_reduce<8>(sh);
  if (threadIdx.x != 0) return;
  const double b = q[F];
  grad[F] += b / bd.bias_var;
  H[F + (long)F * Dp] += 1.0 / bd.bias_var;
  double u = sh[7][0] + 0.5 * b * b / bd.bias_var + 0.5 * (kLn2Pi + log(bd.bias_var));
  double g[3][4];
  for (int h = 0; h < 3; ++h) {
    inv_gamma(q[F + 1 + h], bd.ig_a[h], bd.ig_b[h], g[h]);
    u += g[h][0];
    grad[F + 1 + h] = sh[h][0] + g[h][1];
  }
  const long iC = F + 1, iS = F + 2, iL = F + 3;
  H[iC + iC * Dp] = sh[3][0] + g[0][2];
  H[iS + iS * Dp] = sh[4][0] + g[1][2];
  H[iC + iS * Dp] = sh[5][0];
  H[iS + iC * Dp] = sh[5][0];
  H[iL + iL * Dp] = sh[6][0] + g[2][2];
  scal[1] = beta * scal[3] + u;
}

// Prior part of v(W): adds to v[0..F-1], sets the hyperparameter entries.
__global__ __launch_bounds__(BT) void basis_prior_contract_kernel(BasisDev bd,
                                                                  const double* __restrict__ q,
                                                                  const double* __restrict__ W,
                                                                  int Dp, double* v) {
  __shared__ double sh[3][BT];
  const int F = bd.F;
  double acc[3] = {0, 0, 0};
  auto w = [&](int r, int c) { return 0.5 * (W[r + (long)c * Dp] + W[c + (long)r * Dp]); };
  for (int j = threadIdx.x; j < F; j += BT) {
    const SDerivs d = s_derivs(bd, q, j);
    const double a = q[j];
    const double e = exp(-d.s);
    const double us = 0.5 * (1.0 - a * a * e), uss = 0.5 * a * a * e, usss = -uss;
    const double wjj = W[j + (long)j * Dp];
    double vj = 0.0;
    for (int xi = 0; xi < d.n; ++xi) {
      const int x = d.idx[xi];
      double vx = wjj * (-e * d.sx[xi]);             // d3 u / da da dx
      vj += 2.0 * w(j, x) * (-e * d.sx[xi]);
      for (int yi = 0; yi < d.n; ++yi) {
        const int y = d.idx[yi];
        const double sxy = xi == yi ? d.sxx[xi] : 0.0;
        const double daxy = a * e * (d.sx[xi] * d.sx[yi] - sxy);   // d3 u / da dx dy
        vj += w(x, y) * daxy;
        vx += 2.0 * w(j, y) * daxy;
        for (int zi = 0; zi < d.n; ++zi) {
          const int z = d.idx[zi];
          const double sxz = xi == zi ? d.sxx[xi] : 0.0;
          const double syz = yi == zi ? d.sxx[yi] : 0.0;
          double d3 = usss * d.sx[xi] * d.sx[yi] * d.sx[zi] +
                      uss * (sxy * d.sx[zi] + sxz * d.sx[yi] + syz * d.sx[xi]);
          if (xi == yi && yi == zi) d3 += us * d.sxxx[xi];
          vx += w(y, z) * d3;
        }
      }
      acc[hslot(bd, x)] += vx;
    }
    v[j] += vj;
  }
  for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = acc[k];
  block_reduce<3>(sh);
  if (threadIdx.x != 0) return;
  for (int h = 0; h < 3; ++h) {
    double g[4];
    inv_gamma(q[F + 1 + h], bd.ig_a[h], bd.ig_b[h], g);
    const long ih = F + 1 + h;
    v[ih] = sh[h][0] + W[ih + ih * Dp] * g[3];
  }
}

}  // namespace

void basis_features(const BasisDev& bd, const double* X, const int* col, const int* freq,
                    double L, hipStream_t st) {
  const long n = (long)bd.N * bd.Fa;
  hipLaunchKernelGGL(basis_features_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, bd.N, bd.F, X,
                     col, freq, (const int*)bd.kind, L, bd.Phi);
  RM_CHECK_LAUNCH();
}

void basis_hessian(const BasisDev& bd, int lik, double noise_var, double beta, const double* y,
                   const double* q, double* f, double* likv, double* H, int Dp, double* gradU,
                   double* scal, double* work, hipStream_t st) {
  const int N = bd.N, Fa = bd.Fa;
  gemv(N, Fa, 1.0, bd.Phi, N, false, 0, q, 0, 0.0, f, 0, 1, st);   // f = Phi (a, b)
  lik_derivs(N, lik, noise_var, 0.0, f, y, likv, st);
  hipLaunchKernelGGL(row_scale_kernel, dim3(cdiv((long)N * Fa, 256)), dim3(256), 0, st, N, Fa, beta,
                     (const double*)(likv + 2L * N), (const double*)bd.Phi, work);
  RM_CHECK_LAUNCH();
  fill(H, (long)Dp * Dp, 0.0, st);
  Gemm<double> g;   // H_ab = Phi' diag(beta l'') Phi
  g.m = Fa; g.n = Fa; g.k = N;
  g.A = bd.Phi; g.lda = N; g.tA = true;
  g.B = work; g.ldb = N;
  g.C = H; g.ldc = Dp;
  gemm(g, st);
  gemv(N, Fa, beta, bd.Phi, N, true, 0, likv + N, 0, 0.0, gradU, 0, 1, st);
  vsum(N, likv, scal + 3, st);
  hipLaunchKernelGGL(basis_prior_kernel, dim3(1), dim3(BT), 0, st, bd, beta, q, H, Dp, gradU, scal);
  RM_CHECK_LAUNCH();
  symmetrize(bd.F + 4, H, Dp, st);
}

void basis_contract(const BasisDev& bd, double beta, const double* q, const double* likv,
                    const double* W, int Dp, double* v, double* work, hipStream_t st) {
  const int N = bd.N, Fa = bd.Fa;
  double* G = work;
  double* t = work + (long)N * Fa;
  Gemm<double> g;   // G = Phi W_ab
  g.m = N; g.n = Fa; g.k = Fa;
  g.A = bd.Phi; g.lda = N;
  g.B = W; g.ldb = Dp;
  g.C = G; g.ldc = N;
  gemm(g, st);
  hipLaunchKernelGGL(rowdot_kernel, dim3(cdiv(N, RD_ROWS)), dim3(RD_ROWS * RD_PHASES), 0, st, N, Fa,
                     beta,
                     (const double*)(likv + 3L * N), (const double*)G, (const double*)bd.Phi, t);
  RM_CHECK_LAUNCH();
  gemv(N, Fa, 1.0, bd.Phi, N, true, 0, t, 0, 0.0, v, 0, 1, st);   // v_ab = Phi' t
  hipLaunchKernelGGL(basis_prior_contract_kernel, dim3(1), dim3(BT), 0, st, bd, q, W, Dp, v);
  RM_CHECK_LAUNCH();
}

}  // namespace rmhmc
