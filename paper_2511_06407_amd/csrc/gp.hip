// Kernel matrix K(eta) = sum of kernel terms + jitter I (Sec. 2.1,
// Eq. BMKL) and its hyperparameter derivatives, evaluated element by
// element from the covariates so that only K and the first derivatives are
// ever stored.  Squared-exponential terms differentiate exp(log K):
//   K_l = K c_l,  K_lm = K (c_l c_m + c_lm),
//   K_lmn = K (c_l c_m c_n + c_lm c_n + c_ln c_m + c_mn c_l + c_lmn),
// with log K = 2 eta_s - sum_g u_g / 2, u_g = r_g^2 exp(-2 eta_g), so
// c_s = 2, c_g = u_g, c_gg = -2 u_g, c_ggg = 4 u_g and all other entries 0.
#include <algorithm>

#include "gp.h"

namespace rmhmc {
namespace {

struct TermVals {
  double Kt;
  double u[RMHMC_MAX_TERM_COLS];
};

// Every loop below runs over compile-time bounds and every array is indexed
// by compile-time indices or through select(), so the per-element values
// stay in registers (a runtime index into a register array puts it in
// scratch memory, one memory round trip per access).
template <int NS>
__device__ __forceinline__ double select(const double (&v)[NS], int k) {
  double r = 0.0;
#pragma unroll
  for (int q = 0; q < NS; ++q) r = (q == k) ? v[q] : r;
  return r;
}

__device__ __forceinline__ void term_eval(const ModelDev& md, const double* __restrict__ eta,
                                          int t, int i, int j, TermVals& tv) {
  const TermDev& T = md.terms[t];
  const double* X = md.X;
  const int N = md.N;
  tv.Kt = 0.0;
#pragma unroll
  for (int c = 0; c < RMHMC_MAX_TERM_COLS; ++c) tv.u[c] = 0.0;
  if (T.fn >= 0) {
    // a term of one latent function's prior acts only between its points:
    // the term and every derivative of it vanish elsewhere
    const double* F = X + (long)md.fn_col * N;
    if (F[i] != (double)T.fn || F[j] != (double)T.fn) return;
  }
  if (T.kind == RMHMC_K_SE_ISO) {
    double r2 = 0.0;
#pragma unroll
    for (int c = 0; c < RMHMC_MAX_TERM_COLS; ++c) {
      if (c < T.ncols) {
        const double d = X[(long)T.cols[c] * N + i] - X[(long)T.cols[c] * N + j];
        r2 += d * d;
      }
    }
    const double u = r2 * exp(-2.0 * eta[T.p0 + 1]);
    tv.u[0] = u;
    tv.Kt = exp(2.0 * eta[T.p0] - 0.5 * u);
  } else if (T.kind == RMHMC_K_SE_ARD) {
    double su = 0.0;
#pragma unroll
    for (int c = 0; c < RMHMC_MAX_TERM_COLS; ++c) {
      if (c < T.ncols) {
        const double d = X[(long)T.cols[c] * N + i] - X[(long)T.cols[c] * N + j];
        const double u = d * d * exp(-2.0 * eta[T.p0 + 1 + c]);
        tv.u[c] = u;
        su += u;
      }
    }
    tv.Kt = exp(2.0 * eta[T.p0] - 0.5 * su);
  } else if (T.kind == RMHMC_K_LINEAR_ARD) {
    double s2 = 0.0;
#pragma unroll
    for (int c = 0; c < RMHMC_MAX_TERM_COLS; ++c) {
      if (c < T.ncols) {
        const double v =
            exp(eta[T.p0 + c]) * X[(long)T.cols[c] * N + i] * X[(long)T.cols[c] * N + j];
        tv.u[c] = v;
        s2 += v;
      }
    }
    tv.Kt = s2;
  } else {  // RMHMC_K_BINARY_SAME
    const long c = T.cols[0];
    tv.Kt = (X[c * N + i] == X[c * N + j]) ? exp(2.0 * eta[T.p0]) : 0.0;
  }
}

// Derivative of one term with respect to local parameter indices a, b, c
// (ord = 1, 2 or 3; unused indices ignored).
__device__ __forceinline__ double term_deriv(const TermDev& T, const TermVals& tv, int ord, int a,
                                             int b, int c) {
  if (T.kind == RMHMC_K_SE_ISO || T.kind == RMHMC_K_SE_ARD) {
    auto c1 = [&](int x) { return x == 0 ? 2.0 : select(tv.u, x - 1); };
    auto c2 = [&](int x, int y) { return (x == y && x > 0) ? -2.0 * select(tv.u, x - 1) : 0.0; };
    if (ord == 1) return tv.Kt * c1(a);
    if (ord == 2) return tv.Kt * (c1(a) * c1(b) + c2(a, b));
    const double c3 = (a == b && b == c && a > 0) ? 4.0 * select(tv.u, a - 1) : 0.0;
    return tv.Kt * (c1(a) * c1(b) * c1(c) + c2(a, b) * c1(c) + c2(a, c) * c1(b) +
                    c2(b, c) * c1(a) + c3);
  }
  if (T.kind == RMHMC_K_LINEAR_ARD) {
    if (ord >= 2 && a != b) return 0.0;
    if (ord == 3 && a != c) return 0.0;
    return select(tv.u, a);
  }
  return (ord == 1 ? 2.0 : (ord == 2 ? 4.0 : 8.0)) * tv.Kt;
}

__global__ __launch_bounds__(256) void kgen_kernel(ModelDev md, const double* __restrict__ eta,
                                                   double* __restrict__ K, double* __restrict__ K1) {
  const long NN = (long)md.N * md.N;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NN) return;
  const int i = (int)(e % md.N), j = (int)(e / md.N);
  double k = (i == j) ? md.jitter : 0.0;
#pragma unroll
  for (int t = 0; t < MAX_TERMS; ++t) {
    if (t < md.nterms) {
      TermVals tv;
      term_eval(md, eta, t, i, j, tv);
      k += tv.Kt;
      const TermDev& T = md.terms[t];
#pragma unroll
      for (int a = 0; a < RMHMC_MAX_TERM_COLS + 1; ++a)
        if (a < T.np) K1[(long)(T.p0 + a) * NN + e] = term_deriv(T, tv, 1, a, 0, 0);
    }
  }
  K[e] = k;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// The kernel-derivative sums by passes: a pass is up to KD_PASS tuples of
// one kernel term (the tuples of a term are consecutive), and workgroup
// layer blockIdx.z takes one pass, so every element evaluates that term
// only.  The term's derivative factors go to a per-thread LDS column (SE
// kinds: c_0 = 2, c_x = u_(x-1), so that dK = K (c_a c_b c_c + ...) with
// the second-order factors -2 c_x on the diagonal; linear-ARD: u_x), from
// which each tuple reads the factors of its indices, which are the same in
// every lane: the accumulators stay in registers and the code has one
// branch per term kind, outside the element loop.
constexpr int KD_PASS = 16;
constexpr int KD_MAX_PASSES = 16;
struct KdPasses {
  int n;
  int term[KD_MAX_PASSES], t0[KD_MAX_PASSES], cnt[KD_MAX_PASSES];
};

// The pass's tuples as local indices of its term (the same in every lane).
struct PassTuples {
  int t, nl, kind;
  int ord[KD_PASS], ia[KD_PASS], ib[KD_PASS], ic[KD_PASS];
};

__device__ __forceinline__ void load_pass(const ModelDev& md, const Tuple* __restrict__ tuples,
                                          const KdPasses& ps, int pz, PassTuples& P) {
  P.t = __builtin_amdgcn_readfirstlane(ps.term[pz]);
  const int t0 = __builtin_amdgcn_readfirstlane(ps.t0[pz]);
  P.nl = __builtin_amdgcn_readfirstlane(ps.cnt[pz]);
  P.kind = __builtin_amdgcn_readfirstlane(md.terms[P.t].kind);
  const int p0 = __builtin_amdgcn_readfirstlane(md.terms[P.t].p0);
#pragma unroll
  for (int k = 0; k < KD_PASS; ++k) {
    const Tuple tp = tuples[t0 + (k < P.nl ? k : 0)];
    P.ord[k] = __builtin_amdgcn_readfirstlane(tp.ord);
    P.ia[k] = __builtin_amdgcn_readfirstlane(tp.l - p0);
    P.ib[k] = __builtin_amdgcn_readfirstlane(tp.ord >= 2 ? tp.m - p0 : 0);
    P.ic[k] = __builtin_amdgcn_readfirstlane(tp.ord >= 3 ? tp.n - p0 : 0);
  }
}

// (i, j) of a grid-stride loop over the N x N elements e = i + j N, stepped
// without a division per element: e advances by stride = sj N + si.
struct ElemWalk {
  int i, j, si, sj;
  __device__ ElemWalk(long e, long stride, int N) {
    j = (int)(e / N);
    i = (int)(e - (long)j * N);
    sj = (int)(stride / N);
    si = (int)(stride - (long)sj * N);
  }
  __device__ __forceinline__ void step(int N) {
    i += si;
    j += sj;
    if (i >= N) { i -= N; ++j; }
  }
};

// acc[k] += wgt * (d^ord K / d eta_tuple k)(i, j) from the pass term's
// values tv at (i, j); cv is the LDS block of per-thread factor columns.
__device__ __forceinline__ void pass_accumulate(const PassTuples& P, const TermVals& tv, double wgt,
                                                double (*cv)[256], int tid,
                                                double (&acc)[KD_PASS]) {
  if (P.kind == RMHMC_K_SE_ISO || P.kind == RMHMC_K_SE_ARD) {
    cv[0][tid] = 2.0;
#pragma unroll
    for (int c = 0; c < RMHMC_MAX_TERM_COLS; ++c) cv[1 + c][tid] = tv.u[c];
    const double wk = wgt * tv.Kt;
#pragma unroll
    for (int k = 0; k < KD_PASS; ++k) {
      if (k < P.nl) {
        const int a = P.ia[k], b = P.ib[k], c = P.ic[k];
        const double ca = cv[a][tid];
        double d = ca;
        if (P.ord[k] >= 2) {
          const double cb = cv[b][tid];
          const double c2ab = (a == b && a > 0) ? -2.0 * ca : 0.0;
          if (P.ord[k] == 2) {
            d = ca * cb + c2ab;
          } else {
            const double cc = cv[c][tid];
            const double c2ac = (a == c && a > 0) ? -2.0 * ca : 0.0;
            const double c2bc = (b == c && b > 0) ? -2.0 * cb : 0.0;
            const double c3 = (a == b && b == c && a > 0) ? 4.0 * ca : 0.0;
            d = ca * cb * cc + c2ab * cc + c2ac * cb + c2bc * ca + c3;
          }
        }
        acc[k] += wk * d;
      }
    }
  } else if (P.kind == RMHMC_K_LINEAR_ARD) {
#pragma unroll
    for (int c = 0; c < RMHMC_MAX_TERM_COLS; ++c) cv[c][tid] = tv.u[c];
#pragma unroll
    for (int k = 0; k < KD_PASS; ++k) {
      const bool nz = P.ord[k] == 1 || (P.ia[k] == P.ib[k] && (P.ord[k] == 2 || P.ia[k] == P.ic[k]));
      if (k < P.nl && nz) acc[k] += wgt * cv[P.ia[k]][tid];
    }
  } else {  // same-value term: d^ord K = 2^ord K
    const double wk = wgt * tv.Kt;
#pragma unroll
    for (int k = 0; k < KD_PASS; ++k)
      if (k < P.nl) acc[k] += wk * (P.ord[k] == 1 ? 2.0 : (P.ord[k] == 2 ? 4.0 : 8.0));
  }
}

// Passes of a host tuple list: runs of consecutive tuples of one term, at
// most KD_PASS each.
KdPasses make_passes(const ModelDev& md, const Tuple* tuples_h, int nt) {
  KdPasses ps{};
  for (int k = 0; k < nt;) {
    const int t = md.param_term[tuples_h[k].l];
    int e = k + 1;
    while (e < nt && e - k < KD_PASS && md.param_term[tuples_h[e].l] == t) ++e;
    RM_REQUIRE(ps.n < KD_MAX_PASSES, "kernel-derivative passes: too many");
    ps.term[ps.n] = t;
    ps.t0[ps.n] = k;
    ps.cnt[ps.n] = e - k;
    ++ps.n;
    k = e;
  }
  return ps;
}

__global__ __launch_bounds__(256) void kd_wsum_pass_kernel(ModelDev md, const double* __restrict__ eta,
                                                           const Tuple* __restrict__ tuples, int nt,
                                                           KdPasses ps, int mode,
                                                           const double* __restrict__ Kinv,
                                                           const double* __restrict__ alpha,
                                                           const double* __restrict__ Wstack,
                                                           double* __restrict__ part) {
  constexpr int NC = RMHMC_MAX_TERM_COLS + 1;
  __shared__ double cv[NC][256];
  __shared__ double sh[4][KD_PASS];
  const long NN = (long)md.N * md.N;
  const int w = blockIdx.y;
  PassTuples P;
  load_pass(md, tuples, ps, blockIdx.z, P);
  double acc[KD_PASS];
#pragma unroll
  for (int k = 0; k < KD_PASS; ++k) acc[k] = 0.0;
  const int tid = threadIdx.x;
  const long stride = (long)gridDim.x * blockDim.x;
  const long e0 = (long)blockIdx.x * blockDim.x + tid;
  ElemWalk ij(e0, stride, md.N);
  for (long e = e0; e < NN; e += stride, ij.step(md.N)) {
    const int i = ij.i, j = ij.j;
    const double wgt = mode == 0 ? 0.5 * (Kinv[e] - alpha[i] * alpha[j]) : Wstack[(long)w * NN + e];
    TermVals tv;
    term_eval(md, eta, P.t, i, j, tv);
    pass_accumulate(P, tv, wgt, cv, tid, acc);
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int k = 0; k < KD_PASS; ++k) {
    if (k < P.nl) {
      const double sk = wave_sum(acc[k]);
      if (lane == 0) sh[wave][k] = sk;
    }
  }
  __syncthreads();
  const int t0 = ps.t0[blockIdx.z];
  for (int k = tid; k < P.nl; k += blockDim.x)
    part[((long)w * gridDim.x + blockIdx.x) * nt + t0 + k] = sh[0][k] + sh[1][k] + sh[2][k] + sh[3][k];
}

// out[w * nt + t] = sum over the per-block partials.  One wave per output:
// lanes take every 64th block and a shuffle tree adds the lane sums (a fixed
// order, so the result is deterministic).
__global__ __launch_bounds__(64) void kd_wsum_reduce(int nblk, int nt, const double* __restrict__ part,
                                                     double* __restrict__ out) {
  const int idx = blockIdx.x;
  const int w = idx / nt, t = idx % nt;
  double s = 0.0;
#pragma unroll 4
  for (int b = threadIdx.x; b < nblk; b += 64) s += part[((long)w * nblk + b) * nt + t];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x == 0) out[idx] = s;
}

// Partial sums of y = dK_tuple x over one j chunk, by passes:
// blockIdx.z = pass * nsplit + chunk.  Thread (row lane, wave g) takes every
// fourth j of the chunk; the four waves' sums are added in LDS in a fixed
// order.
__global__ __launch_bounds__(256) void kd_matvec_pass_kernel(ModelDev md, const double* __restrict__ eta,
                                                             const Tuple* __restrict__ tuples, int nt,
                                                             KdPasses ps, const double* __restrict__ x,
                                                             int nx, int jchunk, int nsplit,
                                                             double* __restrict__ part) {
  constexpr int NC = RMHMC_MAX_TERM_COLS + 1;
  __shared__ double cv[NC][256];
  __shared__ double sh[4][KD_PASS][64];
  const int N = md.N;
  const int xi = blockIdx.y, pz = blockIdx.z / nsplit, jz = blockIdx.z % nsplit;
  PassTuples P;
  load_pass(md, tuples, ps, pz, P);
  const double* xv = x + (long)xi * N;
  const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int i = blockIdx.x * 64 + r;
  const int j0 = jz * jchunk, j1 = min(N, j0 + jchunk);
  double acc[KD_PASS];
#pragma unroll
  for (int k = 0; k < KD_PASS; ++k) acc[k] = 0.0;
  if (i < N) {
    for (int j = j0 + g; j < j1; j += 4) {
      TermVals tv;
      term_eval(md, eta, P.t, i, j, tv);
      pass_accumulate(P, tv, xv[j], cv, tid, acc);
    }
  }
#pragma unroll
  for (int k = 0; k < KD_PASS; ++k) sh[g][k][r] = acc[k];
  __syncthreads();
  const int t0 = ps.t0[pz];
  for (int e = tid; e < P.nl * 64; e += 256) {
    const int k = e / 64, rr = e % 64, ii = blockIdx.x * 64 + rr;
    if (ii < N)
      part[(((long)jz * nx + xi) * nt + t0 + k) * N + ii] =
          sh[0][k][rr] + sh[1][k][rr] + sh[2][k][rr] + sh[3][k][rr];
  }
}

// y[(x * nt + t) * N + i] = sum over chunks in order.
__global__ void kd_matvec_reduce(long n, int nsplit, const double* __restrict__ part,
                                 double* __restrict__ y) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
#pragma unroll 8
  for (int z = 0; z < nsplit; ++z) s += part[(long)z * n + e];
  y[e] = s;
}

// KT[t * NN + e] = d^ord K / d eta_tuple at element e = i + j N.
// The tuple derivatives themselves, KT[t * NN + e], by passes (blockIdx.y).
__global__ __launch_bounds__(256) void kd_gen_pass_kernel(ModelDev md, const double* __restrict__ eta,
                                                          const Tuple* __restrict__ tuples,
                                                          KdPasses ps, double* __restrict__ KT) {
  constexpr int NC = RMHMC_MAX_TERM_COLS + 1;
  __shared__ double cv[NC][256];
  PassTuples P;
  load_pass(md, tuples, ps, blockIdx.y, P);
  const int t0 = ps.t0[blockIdx.y];
  const long NN = (long)md.N * md.N;
  const int tid = threadIdx.x;
  const long stride = (long)gridDim.x * blockDim.x;
  const long e0 = (long)blockIdx.x * blockDim.x + tid;
  ElemWalk ij(e0, stride, md.N);
  for (long e = e0; e < NN; e += stride, ij.step(md.N)) {
    const int i = ij.i, j = ij.j;
    TermVals tv;
    term_eval(md, eta, P.t, i, j, tv);
    double acc[KD_PASS];
#pragma unroll
    for (int k = 0; k < KD_PASS; ++k) acc[k] = 0.0;
    pass_accumulate(P, tv, 1.0, cv, tid, acc);
#pragma unroll
    for (int k = 0; k < KD_PASS; ++k)
      if (k < P.nl) KT[(long)(t0 + k) * NN + e] = acc[k];
  }
}

// Mean/variance model (Sec. 2.1, Eq. mvmodel), one thread per record:
// l = r^2 / (2v) + ln(2 pi v) / 2 with r = a - y, v = delta + e, e = exp(b),
// differentiated in a = f1_i and b = f2_i (dv/db = e).
__global__ void lik_mv_kernel(int R, double delta, const double* __restrict__ f,
                              const double* __restrict__ y, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R) return;
  const long N = 2L * R;
  const double a = f[i], b = f[R + i];
  const double e = exp(b), v = delta + e, r = a - y[i];
  const double iv = 1.0 / v, iv2 = iv * iv, iv3 = iv2 * iv, r2 = r * r;
  out[i] = 0.5 * r2 * iv + 0.5 * log(2.0 * M_PI * v);
  out[R + i] = 0.0;
  out[N + i] = r * iv;                                               // l_a
  out[N + R + i] = 0.5 * (e * iv - r2 * e * iv2);                    // l_b
  out[2 * N + i] = iv;                                               // l_aa
  out[2 * N + R + i] = 0.5 * (delta * e * iv2 - r2 * e * (v - 2.0 * e) * iv3);   // l_bb
  out[3 * N + i] = 0.0;                                              // l_aaa
  out[3 * N + R + i] = 0.5 * (delta * e * (v - 2.0 * e) * iv3 -
                              r2 * (e * iv2 - 6.0 * e * e * iv3 + 6.0 * e * e * e * iv3 * iv));  // l_bbb
  out[4 * N + i] = -r * e * iv2;                                     // l_ab
  out[4 * N + R + i] = -e * iv2;                                     // l_aab
  out[5 * N + i] = -r * e * (v - 2.0 * e) * iv3;                     // l_abb
  out[5 * N + R + i] = 0.0;
}

__global__ void lik_kernel(int N, int lik, double noise_var, const double* __restrict__ f,
                           const double* __restrict__ y, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double fi = f[i], yi = y[i];
  double l0, l1, l2, l3;
  if (lik == RMHMC_LIK_BERNOULLI_LOGIT) {
    // l = log(1 + e^f) - y f, written to avoid overflow for large |f|
    const double s = fi >= 0 ? 1.0 / (1.0 + exp(-fi)) : exp(fi) / (1.0 + exp(fi));
    l0 = (fi > 0 ? fi + log1p(exp(-fi)) : log1p(exp(fi))) - yi * fi;
    l1 = s - yi;
    l2 = s * (1.0 - s);
    l3 = l2 * (1.0 - 2.0 * s);
  } else {
    const double r = fi - yi;
    l0 = 0.5 * r * r / noise_var + 0.5 * log(2.0 * M_PI * noise_var);
    l1 = r / noise_var;
    l2 = 1.0 / noise_var;
    l3 = 0.0;
  }
  out[i] = l0;
  out[N + i] = l1;
  out[2 * N + i] = l2;
  out[3 * N + i] = l3;
}

__global__ __launch_bounds__(256) void pair_dots_kernel(int n, const double* __restrict__ x, long sx,
                                                        int nx, const double* __restrict__ y, long sy,
                                                        int ny, double* __restrict__ out) {
  __shared__ double sh[4];
  const int a = blockIdx.x / ny, b = blockIdx.x % ny;
  const double* xa = x + (long)a * sx;
  const double* yb = y + (long)b * sy;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += xa[i] * yb[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

}  // namespace

void kgen(const ModelDev& md, const double* eta, double* K, double* K1, hipStream_t st) {
  const long NN = (long)md.N * md.N;
  hipLaunchKernelGGL(kgen_kernel, dim3(cdiv(NN, 256)), dim3(256), 0, st, md, eta, K, K1);
  RM_CHECK_LAUNCH();
}

static void kd_wsum_chunk(const ModelDev& md, const double* eta, const Tuple* tuples,
                          const Tuple* tuples_h, int nt, int mode, const double* Kinv,
                          const double* alpha, const double* Wstack, int nw, double* out,
                          double* work, hipStream_t st);

void kd_wsum(const ModelDev& md, const double* eta, const Tuple* tuples, const Tuple* tuples_h,
             int nt, int mode, const double* Kinv, const double* alpha, const double* Wstack,
             int nw, double* out, double* work, hipStream_t st) {
  // out is nw x nt (row w); chunks of at most MAX_TUPLES tuples write their columns
  if (nt <= MAX_TUPLES) {
    kd_wsum_chunk(md, eta, tuples, tuples_h, nt, mode, Kinv, alpha, Wstack, nw, out, work, st);
    return;
  }
  double* tmp = work + 512L * MAX_P * MAX_TUPLES;
  for (int t0 = 0; t0 < nt; t0 += MAX_TUPLES) {
    const int c = std::min(MAX_TUPLES, nt - t0);
    kd_wsum_chunk(md, eta, tuples + t0, tuples_h + t0, c, mode, Kinv, alpha, Wstack, nw, tmp,
                  work, st);
    for (int w = 0; w < nw; ++w) copy(out + (long)w * nt + t0, tmp + (long)w * c, c, st);
  }
}

static void kd_wsum_chunk(const ModelDev& md, const double* eta, const Tuple* tuples,
                          const Tuple* tuples_h, int nt, int mode, const double* Kinv,
                          const double* alpha, const double* Wstack, int nw, double* out,
                          double* work, hipStream_t st) {
  if (nt <= 0 || nw <= 0) return;
  const long NN = (long)md.N * md.N;
  const KdPasses ps = make_passes(md, tuples_h, nt);
  // sixteen elements per thread at N = 1024 (256 workgroups per pass)
  int nblk = cdiv(NN, 256 * 16);
  if (nblk > 512) nblk = 512;
  if (nblk < 1) nblk = 1;
  const int slot = timing_begin(TK_KD_WSUM, st);
  hipLaunchKernelGGL(kd_wsum_pass_kernel, dim3(nblk, nw, ps.n), dim3(256), 0, st, md, eta, tuples,
                     nt, ps, mode, Kinv, alpha, Wstack, work);
  RM_CHECK_LAUNCH();
  timing_end(slot, st, 2.0 * (double)NN * nt * nw, (double)NN * nw * sizeof(double));
  hipLaunchKernelGGL(kd_wsum_reduce, dim3(nt * nw), dim3(64), 0, st, nblk, nt,
                     (const double*)work, out);
  RM_CHECK_LAUNCH();
}

void kd_matvec(const ModelDev& md, const double* eta, const Tuple* tuples, const Tuple* tuples_h,
               int nt, const double* x, int nx, double* y, double* work, hipStream_t st) {
  if (nt <= 0 || nx <= 0) return;
  RM_REQUIRE(nt <= MAX_TUPLES || nx == 1, "kd_matvec: chunked tuples need a single vector");
  if (nt > MAX_TUPLES) {
    for (int t0 = 0; t0 < nt; t0 += MAX_TUPLES)
      kd_matvec(md, eta, tuples + t0, tuples_h + t0, std::min(MAX_TUPLES, nt - t0), x, 1,
                y + (long)t0 * md.N, work, st);
    return;
  }
  const int N = md.N;
  const int jchunk = cdiv(N, KD_MV_SPLIT);
  const int nsplit = cdiv(N, jchunk);
  const long n = (long)nt * nx * N;
  const KdPasses ps = make_passes(md, tuples_h, nt);
  const int slot = timing_begin(TK_KD_MATVEC, st);
  hipLaunchKernelGGL(kd_matvec_pass_kernel, dim3(cdiv(N, 64), nx, nsplit * ps.n), dim3(256), 0, st,
                     md, eta, tuples, nt, ps, x, nx, jchunk, nsplit, work);
  RM_CHECK_LAUNCH();
  hipLaunchKernelGGL(kd_matvec_reduce, dim3(cdiv(n, 256)), dim3(256), 0, st, n, nsplit,
                     (const double*)work, y);
  RM_CHECK_LAUNCH();
  timing_end(slot, st, 2.0 * (double)N * N * nt * nx, (double)N * nx * (1.0 + nt) * sizeof(double));
}

void kd_wsum_stack(const ModelDev& md, const double* eta, const Tuple* tuples,
                   const Tuple* tuples_h, int nt, const double* Wstack, int nw, double* out,
                   double* KT, double* tallwork, hipStream_t st) {
  if (nt <= 0 || nw <= 0) return;
  const long NN = (long)md.N * md.N;
  const int nblk = std::max(1, std::min(2048, cdiv(NN, 256 * 4)));
  for (int t0 = 0; t0 < nt; t0 += MAX_TUPLES) {
    const int c = std::min(MAX_TUPLES, nt - t0);
    const KdPasses ps = make_passes(md, tuples_h + t0, c);
    const int slot = timing_begin(TK_KD_WSUM, st);
    hipLaunchKernelGGL(kd_gen_pass_kernel, dim3(nblk, ps.n), dim3(256), 0, st, md, eta,
                       tuples + t0, ps, KT);
    RM_CHECK_LAUNCH();
    timing_end(slot, st, 0.0, (double)NN * c * sizeof(double));
    // out(t, w) at out[w * nt + t]: C = KT' W with ldc = nt, columns offset by t0
    gemm_tallk(c, nw, NN, KT, NN, Wstack, NN, out + t0, nt, tallwork, tallk_splits(NN), st);
  }
}

void lik_derivs(int N, int lik, double noise_var, double delta, const double* f, const double* y,
                double* out, hipStream_t st) {
  if (lik == RMHMC_LIK_GAUSSIAN_MV) {
    const int R = N / 2;
    hipLaunchKernelGGL(lik_mv_kernel, dim3(cdiv(R, 256)), dim3(256), 0, st, R, delta, f, y, out);
  } else {
    hipLaunchKernelGGL(lik_kernel, dim3(cdiv(N, 256)), dim3(256), 0, st, N, lik, noise_var, f, y,
                       out);
  }
  RM_CHECK_LAUNCH();
}

void pair_dots(int n, const double* x, long sx, int nx, const double* y, long sy, int ny,
               double* out, hipStream_t st) {
  if (nx <= 0 || ny <= 0) return;
  hipLaunchKernelGGL(pair_dots_kernel, dim3(nx * ny), dim3(256), 0, st, n, x, sx, nx, y, sy, ny, out);
  RM_CHECK_LAUNCH();
}

}  // namespace rmhmc
