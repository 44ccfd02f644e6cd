// librmhmc: softabs RMHMC for latent-GP models on one MI355X.
//
// Host orchestration of the device kernels behind the C ABI in rmhmc.h:
//   hessian      U, grad U and H at q                      (Sec. 2.2 input)
//   softabs_eig  H = Psi diag(lam) Psi', g, g', log|G|     (Sec. 2.2, 2.4)
//   metric_grad  dH/dq, dH/dp and H(q,p)                   (Eq. d_Hamiltonian,
//                with W1, W2 of Eq. Betancourt_formula and the ordered
//                contraction of Sec. 2.3)
//   glf_step     generalized leapfrog                      (Eq. leapfrog)
//   chain        RMHMC moves with Metropolis-Hastings      (Algorithm 1)
//
// Notation: q = (f, eta), K = K(eta) + jitter I, alpha = K^-1 f, K_l = dK/deta_l,
// A_l = K^-1 K_l, B_l = A_l K^-1, Phi = (K^-1 - alpha alpha')/2.
// Everything a point q needs is cached in a Point; a leapfrog moves between
// three Points (move start, and two alternating trial points).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "basis.h"
#include "common.h"
#include "eig.h"
#include "gp.h"

namespace rmhmc {

static thread_local std::string g_last_error;
void timing_set(unsigned mask);
void timing_read(int kind, long long* launches, double* ms, double* flops, double* bytes);

namespace {

const double kLog2Pi = 1.8378770664093453;

struct Pool {
  std::vector<void*> ptrs;
  std::vector<void*> host;
  size_t bytes = 0;   // device bytes held
  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    bytes += n * sizeof(T);
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(RMHMC_E_NOMEM, "device allocation of " + std::to_string(n * sizeof(T)) +
                                     " bytes failed");
    }
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  template <class T>
  T* alloc_host(size_t n) {
    void* p = nullptr;
    RM_HIP(hipHostMalloc(&p, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault));
    host.push_back(p);
    return static_cast<T*>(p);
  }
  ~Pool() {
    for (void* p : ptrs) (void)hipFree(p);
    for (void* p : host) (void)hipHostFree(p);
  }
};

// ------------------------------------------------------------ small kernels

// H (Dp x Dp, padded with zeros): H_ff = K^-1 + beta L'', H_fl = -A_l alpha,
// H_lm = k_l.a_m + <Phi, K_lm> - tr(A_l A_m)/2 + delta_lm (symmetrised).
// L'' is diag(l'') for one latent function; with two (R > 0 records, the
// mean/variance model) each record also couples f1_i and f2_i = f_(R+i).
// Same-value terms with at most this many distinct values take the
// low-rank form of their derivative.
constexpr int LR_MAX_RANK = 4;

// UU[:, ncol + k] = UU[:, k] c_s(eta) for the columns k of slot s = k / rl:
// c = exp(eta_l) (linear-ARD), 2 exp(2 eta_l) (same-value).
__global__ void lr_scale_kernel(int N, int ncol, int rl, double* __restrict__ UU,
                                const int* __restrict__ lr_param, const int* __restrict__ lr_kind,
                                const double* __restrict__ eta) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)N * ncol) return;
  const int sl = (int)(e / N) / rl;
  const double h = eta[lr_param[sl]];
  const double c = lr_kind[sl] ? 2.0 * exp(2.0 * h) : exp(h);
  UU[(long)ncol * N + e] = UU[e] * c;
}

__global__ void assemble_H_kernel(int N, int P, int Dp, int R, double beta, const double* __restrict__ Kinv,
                                  const double* __restrict__ lik, const double* __restrict__ a,
                                  const double* __restrict__ kla, const double* __restrict__ phiK2,
                                  const double* __restrict__ trAA, const int* __restrict__ pidx,
                                  double* __restrict__ H) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)Dp * Dp) return;
  const int i = (int)(e % Dp), j = (int)(e / Dp);
  const int D = N + P;
  double v = 0.0;
  if (i < N && j < N) {
    v = Kinv[i + (long)j * N];
    if (i == j) v += beta * lik[2 * N + i];
    if (R > 0 && (i - j == R || j - i == R)) v += beta * lik[4 * N + min(i, j)];
  } else if (i < N && j < D) {
    v = -a[(long)(j - N) * N + i];
  } else if (j < N && i < D) {
    v = -a[(long)(i - N) * N + j];
  } else if (i < D && j < D) {
    const int l = i - N, m = j - N;
    v = 0.5 * (kla[l * P + m] + kla[m * P + l]) - 0.25 * (trAA[l + m * P] + trAA[m + l * P]);
    const int pi = pidx[l * P + m];
    if (pi >= 0) v += phiK2[pi];
    if (l == m) v += 1.0;
  }
  H[e] = v;
}

// grad U and U.  scal: [0] log|K|, [1] U (out), [3] sum l_i, [4] f.alpha.
__global__ void grad_U_kernel(int N, int P, double beta, const double* __restrict__ q,
                              const double* __restrict__ alpha, const double* __restrict__ lik,
                              const double* __restrict__ ak, const double* __restrict__ trK1,
                              double* __restrict__ gradU, double* __restrict__ scal) {
  const int D = N + P;
  for (int i = threadIdx.x; i < D; i += blockDim.x) {
    if (i < N) {
      gradU[i] = beta * lik[N + i] + alpha[i];
    } else {
      const int l = i - N;
      gradU[i] = -0.5 * ak[l] + 0.5 * trK1[l] + q[i];
    }
  }
  if (threadIdx.x == 0) {
    double ee = 0.0;
    for (int l = 0; l < P; ++l) ee += q[N + l] * q[N + l];
    scal[1] = beta * scal[3] + 0.5 * scal[4] + 0.5 * scal[0] + 0.5 * ee + 0.5 * D * kLog2Pi;
  }
}

// d H_lm / d eta_n for all n, l, m (W-independent part of the contraction).
__global__ void dHe_kernel(int P, const double* __restrict__ D1, const double* __restrict__ D2,
                           const double* __restrict__ D3, const double* __restrict__ t3,
                           const double* __restrict__ tB, const double* __restrict__ tau,
                           const int* __restrict__ pidx, const int* __restrict__ tidx,
                           const int* __restrict__ tauidx, int npairs,
                           double* __restrict__ dHe) {
  const int P2 = P * P, P3 = P2 * P;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < P3; e += gridDim.x * blockDim.x) {
    const int n = e / P2, l = (e / P) % P, m = e % P;
    double v = -D1[n * P2 + l * P + m] - D1[l * P2 + n * P + m] - D1[l * P2 + m * P + n];
    const int pln = pidx[l * P + n], pmn = pidx[m * P + n], plm = pidx[l * P + m];
    if (pln >= 0) v += D2[pln * P + m] - 0.5 * tB[m * npairs + pln];
    if (pmn >= 0) v += D3[l * npairs + pmn] - 0.5 * tB[l * npairs + pmn];
    if (plm >= 0) v += D3[n * npairs + plm] - 0.5 * tB[n * npairs + plm];
    const int t = tidx[(l * P + m) * P + n];
    if (t >= 0) v += t3[t];
    v += tau[tauidx[e]];
    dHe[e] = v;
  }
}

// z = sum_lm W_lm (2 K_l a_m - K_lm alpha)
// z_i = sum_lm W[eta_l, eta_m] (2 c1a_lm(i) - k2a_lm(i)).  A workgroup
// covers 64 rows i; its 16 waves split the P^2 (l, m) terms and the wave
// sums are added in a fixed order through LDS.
constexpr int ZV_WAVES = 16;
__global__ __launch_bounds__(64 * ZV_WAVES) void zvec_kernel(int N, int P, int Dp, const double* __restrict__ W,
                                                          const double* __restrict__ c1a, const double* __restrict__ k2a,
                                                          const int* __restrict__ pidx, double* __restrict__ z) {
  __shared__ double sh[ZV_WAVES][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + tx;
  double s = 0.0;
  if (i < N) {
    for (int k = ty; k < P * P; k += ZV_WAVES) {
      const int l = k / P, m = k % P;
      const double wlm = W[(N + l) + (long)(N + m) * Dp];
      double t = 2.0 * c1a[(long)k * N + i];
      const int pi = pidx[k];
      if (pi >= 0) t -= k2a[(long)pi * N + i];
      s += wlm * t;
    }
  }
  sh[ty][tx] = s;
  __syncthreads();
  if (ty == 0 && i < N) {
    double r = 0.0;
    for (int w = 0; w < ZV_WAVES; ++w) r += sh[w][tx];
    z[i] = r;
  }
}

// v = tr(W dH/dq) for the latent coordinates i < N, assembled from the pieces.
// The likelihood part is sum_mn W_mn d^3 L / df_i df_m df_n: W_ii l'''_i for
// one latent function; with two (R > 0), per record (a, b) = (f1_r, f2_r):
//   v_a = W_aa l_aaa + 2 W_ab l_aab + W_bb l_abb,
//   v_b = W_aa l_aab + 2 W_ab l_abb + W_bb l_bbb.
__global__ void contract_final_kernel(int N, int P, int Dp, int R, double beta,
                                      const double* __restrict__ W,
                                      const double* __restrict__ lik, const double* __restrict__ Au,
                                      const double* __restrict__ Kz, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double t3;
  if (R > 0) {
    const int r = i < R ? i : i - R;
    const double waa = W[r + (long)r * Dp], wbb = W[(r + R) + (long)(r + R) * Dp];
    const double wab = 0.5 * (W[r + (long)(r + R) * Dp] + W[(r + R) + (long)r * Dp]);
    const double laab = lik[4 * N + R + r], labb = lik[5 * N + r];
    t3 = i < R ? waa * lik[3 * N + r] + 2.0 * wab * laab + wbb * labb
               : waa * laab + 2.0 * wab * labb + wbb * lik[3 * N + R + r];
  } else {
    t3 = W[i + (long)i * Dp] * lik[3 * N + i];
  }
  double s = beta * t3 + Kz[i];
  for (int l = 0; l < P; ++l) s -= 2.0 * Au[(long)l * N + i];
  v[i] = s;
}

// v = tr(W dH/dq) for the hyperparameter coordinate N + n: one wave per n,
// lanes over the P^2 (l, m) terms, summed by a shuffle tree.
__global__ __launch_bounds__(64) void contract_eta_kernel(int N, int P, int Dp, const double* __restrict__ W,
                                                          const double* __restrict__ wB, const double* __restrict__ E1,
                                                          const double* __restrict__ E2, const double* __restrict__ dHe,
                                                          const int* __restrict__ pidx, int npairs,
                                                          double* __restrict__ v) {
  const int n = blockIdx.x, lane = threadIdx.x, P2 = P * P;
  double s = 0.0;
  for (int k = lane; k < P2; k += 64) {
    const int l = k / P, m = k % P;
    s += W[(N + l) + (long)(N + m) * Dp] * dHe[(long)n * P2 + k];
  }
  for (int l = lane; l < P; l += 64) {
    s += 2.0 * (E1[l * P2 + n * P + l] + E1[l * P2 + l * P + n]);
    const int pln = pidx[l * P + n];
    if (pln >= 0) s -= 2.0 * E2[l * npairs + pln];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) v[N + n] = s - wB[n];
}

// H(q,p) = U + log|G|/2 + sum c^2/g / 2 + D log(2 pi)/2, c = Psi' p.
__global__ void ham_kernel(int D, const double* __restrict__ c, const double* __restrict__ g,
                           const double* __restrict__ U, const double* __restrict__ logdetG,
                           double* __restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < D; i += 256) s += c[i] * c[i] / g[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0)
    out[0] = U[0] + 0.5 * logdetG[0] + 0.5 * (sh[0] + sh[1] + sh[2] + sh[3]) + 0.5 * D * kLog2Pi;
}

// ------------------------------------------------------------ chain randomness
// Philox4x64-10 (Salmon et al., SC 2011): ten rounds of two 64 x 64 -> 128-bit
// products of counter words 0 and 2 by fixed odd multipliers, the high halves
// mixed with the other counter words and the key, the key bumped by two Weyl
// constants between rounds.  key = (seed, stream_id); counter = (block j,
// move, purpose, 0), purpose 0 for the momentum normals and 1 for the
// Metropolis-Hastings uniform of the move.
struct Philox4 {
  unsigned long long w[4];
};
__device__ __forceinline__ Philox4 philox4x64(unsigned long long c0, unsigned long long c1,
                                              unsigned long long c2, unsigned long long c3,
                                              unsigned long long k0, unsigned long long k1) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const unsigned long long hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const unsigned long long hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const unsigned long long n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return Philox4{{c0, c1, c2, c3}};
}

// (0, 1) uniform from the top 53 bits of a word.
__device__ __forceinline__ double uniform53(unsigned long long w) {
  return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

// z[4j .. 4j+3] from block j: two Box-Muller pairs from words (0, 1), (2, 3).
// The move index comes from device memory when dmove is given (a chain's
// move counter, so that a captured move replays with the right counter).
__global__ void normals_kernel(int D, unsigned long long seed, unsigned long long stream,
                               unsigned long long move_imm, const long long* __restrict__ dmove,
                               double* __restrict__ z) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * j >= D) return;
  const unsigned long long move = dmove ? (unsigned long long)*dmove : move_imm;
  const Philox4 r = philox4x64((unsigned long long)j, move, 0ull, 0ull, seed, stream);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double u0 = uniform53(r.w[2 * h]), u1 = uniform53(r.w[2 * h + 1]);
    const double rad = sqrt(-2.0 * log(u0));
    const double t = (2.0 * M_PI) * u1;
    const int i = 4 * j + 2 * h;
    if (i < D) z[i] = rad * cos(t);
    if (i + 1 < D) z[i + 1] = rad * sin(t);
  }
}

// The Metropolis-Hastings uniform of a move (word 0 of block 0, purpose 1).
__global__ void uniform_kernel(unsigned long long seed, unsigned long long stream,
                               unsigned long long move, double* __restrict__ u) {
  if (threadIdx.x == 0) u[0] = uniform53(philox4x64(0ull, move, 1ull, 0ull, seed, stream).w[0]);
}

// Device statistics of a state (doubles).
enum {
  ST_EIG = 0, ST_SWEEPS = 1, ST_ACC = 2, ST_FAIL = 3, ST_NOTPD = 4, ST_NONFINITE = 5, ST_NOCONV = 6,
  ST_RESP = 8, ST_RESQ = 9, ST_ACC_KEPT = 11, ST_N = 16
};
// Failure bits of a move (device int): 1 K not positive definite, 4 an
// eigensolve did not converge, 8 non-finite values met.
enum { FAIL_NOT_PD = 1, FAIL_NOCONV = 4, FAIL_NONFINITE = 8 };

// Metropolis-Hastings test of Algorithm 1 (accept iff log r < H_old - H_new;
// the printed algorithm restores q on this event instead): a failed or
// non-finite move is a rejection.  acc[0] = decision; kept_acc (nullable) =
// the decision in the output of a kept move; the failure word is cleared for
// the next move.
__global__ void mh_kernel(unsigned long long seed, unsigned long long stream,
                          const long long* __restrict__ dmove, int n_burnin,
                          const double* __restrict__ ham, int* __restrict__ fail,
                          int* __restrict__ acc, double* __restrict__ stats,
                          int* __restrict__ accepted_out) {
  if (threadIdx.x != 0) return;
  const long long move = *dmove;
  const double u = uniform53(philox4x64(0ull, (unsigned long long)move, 1ull, 0ull, seed, stream).w[0]);
  const int f = *fail;
  const double h0 = ham[0], h1 = ham[1];
  const bool finite = isfinite(h0) && isfinite(h1);
  const bool ok = f == 0 && finite;
  const bool a = ok && log(u) < h0 - h1;
  acc[0] = a ? 1 : 0;
  stats[ST_ACC] += a ? 1.0 : 0.0;
  if (!ok) {
    stats[ST_FAIL] += 1.0;
    if (f & FAIL_NOT_PD) stats[ST_NOTPD] += 1.0;
    if ((f & FAIL_NONFINITE) || (!finite && !(f & FAIL_NOT_PD))) stats[ST_NONFINITE] += 1.0;
    if (f & FAIL_NOCONV) stats[ST_NOCONV] += 1.0;
  }
  if (move >= n_burnin) {
    accepted_out[move - n_burnin] = a ? 1 : 0;
    stats[ST_ACC_KEPT] += a ? 1.0 : 0.0;
  }
  *fail = 0;
}

// dst <- src over n 16-byte words when *flag is set (an accepted move's end
// point becomes the start point of the next move).
__global__ __launch_bounds__(256) void copy_if_kernel(long n, double2* __restrict__ dst,
                                                      const double2* __restrict__ src,
                                                      const int* __restrict__ flag) {
  if (*flag == 0) return;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    dst[i] = src[i];
}

// After a move: the position and log posterior of the chain's point go to
// the output row of a kept move; the move counter advances.  One workgroup.
__global__ __launch_bounds__(1024) void store_sample_kernel(int D, const double* __restrict__ q,
                                                            const double* __restrict__ U,
                                                            long long* __restrict__ dmove,
                                                            int n_burnin,
                                                            double* __restrict__ samples,
                                                            double* __restrict__ logpost) {
  const long long move = *dmove;
  if (move >= n_burnin) {
    const long long row = move - n_burnin;
    for (int i = threadIdx.x; i < D; i += 1024) samples[row * D + i] = q[i];
    if (threadIdx.x == 0) logpost[row] = -U[0];
  }
  __syncthreads();   // every thread has read the counter before it advances
  if (threadIdx.x == 0) *dmove = move + 1;
}

__global__ void set_counter_kernel(long long* __restrict__ c, long long v) {
  if (threadIdx.x == 0) *c = v;
}

// One fixed-point update dst <- base + c1 x + c2 y of the implicit leapfrog
// equations; when `res` is given, res = max(res, ||new - old|| / ||new||)
// (the relative residual of the iteration).  One workgroup.
__global__ __launch_bounds__(1024) void fp_update_kernel(int n, const double* __restrict__ base,
                                                         double c1, const double* __restrict__ x,
                                                         double c2, const double* __restrict__ y,
                                                         double* __restrict__ dst,
                                                         double* __restrict__ res) {
  __shared__ double sh[2][16];
  double d2 = 0.0, n2 = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const double v = base[i] + c1 * x[i] + c2 * y[i];
    const double d = v - dst[i];
    d2 += d * d;
    n2 += v * v;
    dst[i] = v;
  }
  if (!res) return;
  for (int o = 32; o > 0; o >>= 1) {
    d2 += __shfl_xor(d2, o, 64);
    n2 += __shfl_xor(n2, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = d2;
    sh[1][w] = n2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < 16; ++k) {
      a += sh[0][k];
      b += sh[1][k];
    }
    const double r = b > 0.0 ? sqrt(a / b) : sqrt(a);
    if (!(r <= res[0])) res[0] = r;   // a NaN residual is kept
  }
}

// fail |= bit when the Cholesky flag is set.
__global__ void fold_flag_kernel(const int* __restrict__ info, int* __restrict__ fail, int bit) {
  if (threadIdx.x == 0 && *info != 0) *fail |= bit;
}
__global__ void or_flag_kernel(int* __restrict__ fail, int bit) {
  if (threadIdx.x == 0) *fail |= bit;
}

__global__ void any_nonfinite_kernel(long n, const double* __restrict__ x, int* __restrict__ flag) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) flag[0] = 1;
}


}  // namespace

// ------------------------------------------------------------ model

// k-range layers for the single Dp x Dp warm-start products and K^-1 =
// L^-T L^-1: 17 x 17 tiles at Dp = 1088 become 1156 workgroups with 4
// layers, about four per CU.  The tuner may pick another count up to
// GSPLIT_MAX per model.
constexpr int GSPLIT_DEFAULT = 4;
constexpr int GSPLIT_MAX = 8;

// How an eigendecomposition is driven: host_check reads the stop flag after
// each sweep past the first `blind` (single calls and the chain); without it
// exactly `blind` sweeps are launched with nothing read back (graph capture).
// fail / dstats: the state's failure word and statistics (nullable).
struct EigCfg {
  double zeta = 1e-13;
  double zeta_s = -1.0;   // scaled test of the metric stopping rule (<= 0: its default)
  int max_sweeps = 60;
  int blind = 0;
  bool host_check = true;
  int* fail = nullptr;
  double* dstats = nullptr;
  int* max_seen = nullptr;   // [host] largest sweep count of a warm start (host-checked mode)
  int softabs = RMHMC_SOFTABS_COTH;   // the map g of the metric (rmhmc_softabs)
};
// Largest number of fixed-point iterations whose eigen-solves get their own
// sweep budget in a captured move.
constexpr int MAX_FP_BUDGETS = 16;
// The position equation's iterates before the last two are solved to these
// tolerances instead of zeta (norm-wise and scaled tests of the metric
// stopping rule): their metrics only steer the iteration.  A relative error
// e in G^-1 at iterate k moves q_(k+1) by about eps |G^-1 p| e / 2, and that
// reaches the result only through the later iterates' metrics, scaled by
// the iteration's contraction; the last two iterates, whose metrics enter
// the result directly (and the new point's, which the next step and the
// Hamiltonian use), keep zeta.
constexpr double LOOSE_ZETA = 1e-8, LOOSE_ZETA_S = 1e-7;

struct Model {
  int N = 0, dx = 0, P = 0, D = 0, Dp = 0;
  int lik = 0;
  int R = 0;            // records of the mean/variance model (two latent functions), else 0
  // the reduced-rank basis model (q = (a, b, c_g, sigma_g, c_l); N = records)
  bool basis = false;
  BasisDev bd;
  double* bwork = nullptr;   // N x (F + 1) + N
  double noise_var = 1.0, jitter = 1e-6, beta = 1.0, delta = 0.0;
  rmhmc_precision prec = RMHMC_FP64;
  ModelDev md{};
  Pool pool;
  double* y = nullptr;
  std::vector<Tuple> pairs_h, triples_h;
  Tuple* pairs = nullptr;
  Tuple* triples = nullptr;
  int npairs = 0, ntriples = 0, nyy = 0;
  std::vector<int> pidx_h, tidx_h, yidx_h, tauidx_h;
  int *pidx = nullptr, *tidx = nullptr, *tauidx = nullptr;
  // scratch
  CholWork chol;
  EigWork eig;
  double *tallwork = nullptr, *kdwork = nullptr, *mdwork = nullptr;
  long tallwork_n = 0;  // doubles of tallwork available to split partials
  double* gsplit = nullptr;   // split-K partials of the warm-start products (GSPLIT_MAX x Dp x Dp)
  int gsplit_layers = GSPLIT_DEFAULT;
  double *mvwork = nullptr;   // column-split partials of kd_matvec
  double *ktbuf = nullptr;    // generated second derivatives of K (<= MAX_TUPLES x N*N)
  double *W = nullptr, *Wt1 = nullptr, *Wt2 = nullptr;
  double *vc = nullptr, *vb = nullptr, *vtmp = nullptr, *vtmp2 = nullptr, *v1 = nullptr;
  double *u = nullptr, *Au = nullptr, *Ku = nullptr, *z = nullptr, *Kz = nullptr, *wB = nullptr;
  double* gvwork = nullptr;    // column-split GEMV partials
  double *E1 = nullptr, *E2 = nullptr, *D1 = nullptr, *D2 = nullptr, *D3 = nullptr;
  double *t3 = nullptr, *tB = nullptr, *tau = nullptr;
  // Low-rank hyperparameter derivatives.  A linear-ARD parameter's K_l is
  // exp(eta_l) x x' (rank one) and a same-value term's is 2 exp(2 eta_l)
  // times the indicator of equal values (one column per distinct value), so
  // K_l = U_l c_l(eta) U_l' with U_l of rl columns (zero-padded).  Such
  // parameters (slots, in parameter order) take their A_l = K^-1 K_l,
  // B_l = A_l K^-1 and Y products from thin factors instead of N^3 products.
  int nlr = 0, rl = 0;
  std::vector<int> lr_slot_h;                  // per parameter: slot, -1: full rank
  std::vector<std::pair<int, int>> runs_h;     // consecutive parameters of one class: (first, count)
  int *lr_param = nullptr, *lr_kind = nullptr; // per slot: parameter; 0: c = e^eta, 1: c = 2 e^(2 eta)
  double* UU = nullptr;                        // N x 2 nlr rl: [U | U C] (C set per point)
  double* Gy = nullptr;                        // (nyl + nyr) x N x rl: thin Y factors
  // formed Y pairs l <= m: both full rank; l low rank; only m low rank
  int nyf = 0, nyl = 0, nyr = 0;
  int* dflag = nullptr;
  int* hflag = nullptr;
  struct Point* api_pt = nullptr;
  std::unique_ptr<struct Point> api_pt_own;
  std::unique_ptr<struct State> chain_state;
  size_t device_bytes = 0;   // device memory held by the model (points, chain state, scratch)
  // Serialises every call that uses the model's scratch or its chain state
  // (calls on a model from several threads run one at a time).
  std::mutex busy;
  bool in_batch = false;   // admitted to a batch: its chain state belongs to the batch slot
  ~Model();
};

// Everything that depends on one point q.  The data arrays live in one
// contiguous device block (`data`, `data_bytes`), so an accepted move's end
// point can replace the start point with one predicated copy on the device;
// the device pointer arrays of the batched Y products point into the Point's
// own block and sit outside it.
struct Point {
  Pool meta;
  char* data = nullptr;
  size_t data_bytes = 0;
  int N, P, D, Dp;
  double *q, *K, *Kinv, *K1, *A, *At, *alpha, *lik, *scal, *k1a, *a, *gradU, *H;
  double *Psi, *lam, *g, *gp;
  double *B, *Yt, *k2a, *ik2a, *c1a, *Aam, *dHe, *vW2;
  double *trK1, *kla, *phiK2, *trAA, *ak;
  const double **Yap = nullptr, **Ybp = nullptr;
  double** Ycp = nullptr;
  // low-rank parameters: ZZ = [K^-1 U | K^-1 U C] (N x 2 nlr rl), and the
  // pointer arrays of the thin Y products (first factors with l low rank,
  // with only m low rank, then the outer products)
  double* ZZ = nullptr;
  const double **YLa = nullptr, **YLb = nullptr, **YRa = nullptr, **YRb = nullptr;
  double **YLc = nullptr, **YRc = nullptr;
  const double **Y2a = nullptr, **Y2b = nullptr;
  double** Y2c = nullptr;
  float** Y2cf = nullptr;
  // mixed precision: FP32 copies feeding the FP32 MFMA products
  float *Af = nullptr, *Atf = nullptr, *Ytf = nullptr;
  const float **Yapf = nullptr, **Ybpf = nullptr;
  float** Ycpf = nullptr;
  bool have_pre = false, have_vW2 = false, have_eig = false;
  // scal: [0] log|K|, [1] U, [2] log|G|, [3] sum l, [4] f.alpha, [5] ham
};

namespace {

// Sub-allocation of a Point's data block: the same layout is run once to
// size the block and once to hand out its pieces (256-byte aligned).
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

void layout_point(const Model& m, Point& p, Carve& c) {
  const long N = m.N, P = m.P, NN = N * N, Dp = m.Dp;
  const bool mixed = m.prec == RMHMC_MIXED;
  if (m.basis) {
    // f in alpha; the latent model's K-derived caches are not used
    p.q = c.take<double>(m.D);
    p.alpha = c.take<double>(N);
    p.lik = c.take<double>((long)LIK_SLOTS * N);
    p.scal = c.take<double>(8);
    p.gradU = c.take<double>(m.D);
    p.H = c.take<double>(Dp * Dp);
    p.Psi = c.take<double>(Dp * Dp);
    p.lam = c.take<double>(Dp);
    p.g = c.take<double>(Dp);
    p.gp = c.take<double>(Dp);
    p.vW2 = c.take<double>(m.D);
    return;
  }
  p.q = c.take<double>(m.D);
  p.K = c.take<double>(NN);
  p.Kinv = c.take<double>(NN);
  p.K1 = c.take<double>(P * NN);
  p.A = c.take<double>(P * NN);
  p.At = c.take<double>(mixed ? 1 : P * NN);
  p.alpha = c.take<double>(N);
  p.lik = c.take<double>((long)LIK_SLOTS * N);
  p.scal = c.take<double>(8);
  p.k1a = c.take<double>(P * N);
  p.a = c.take<double>(P * N);
  p.gradU = c.take<double>(m.D);
  p.H = c.take<double>(Dp * Dp);
  p.Psi = c.take<double>(Dp * Dp);
  p.lam = c.take<double>(Dp);
  p.g = c.take<double>(Dp);
  p.gp = c.take<double>(Dp);
  p.B = c.take<double>(P * NN);
  p.Yt = c.take<double>(mixed ? 1 : (long)m.nyy * NN);
  p.k2a = c.take<double>((long)std::max(m.npairs, 1) * N);
  p.ik2a = c.take<double>((long)std::max(m.npairs, 1) * N);
  p.c1a = c.take<double>(P * P * N);
  p.Aam = c.take<double>(P * P * N);
  p.dHe = c.take<double>(P * P * P);
  p.vW2 = c.take<double>(m.D);
  p.trK1 = c.take<double>(P);
  p.kla = c.take<double>(P * P);
  p.phiK2 = c.take<double>(std::max(m.npairs, 1));
  p.trAA = c.take<double>(P * P);
  p.ak = c.take<double>(P);
  p.ZZ = c.take<double>(N * 2L * m.nlr * m.rl);
  if (mixed) {
    p.Af = c.take<float>(P * NN);
    p.Atf = c.take<float>(P * NN);
    p.Ytf = c.take<float>((long)m.nyy * NN);
  }
}

// Device bytes of one Point of model m.
size_t point_bytes(const Model& m) {
  Point p;
  Carve c;
  layout_point(m, p, c);
  return (c.off + 255) & ~size_t(255);
}

// The split partials of a rows x cols tall-K product over the N^2 elements
// (tallk_splits(N^2) x rows x cols doubles), checked against the space held.
double* tall_space(const Model& m, int rows, int cols) {
  RM_REQUIRE((long)tallk_splits((long)m.N * m.N) * rows * cols <= m.tallwork_n,
             "internal: tall-K workspace too small");
  return m.tallwork;
}

// A product with a thin output (a few 64 x 64 tiles) over a long k range
// leaves most of the chip idle: its k range is split over up to 16 layers of
// workgroups (partials in the model's split-K space, added in order).
void thin_gemm(Model& m, const Gemm<double>& g, hipStream_t st) {
  const long tiles = (long)cdiv(g.m, 64) * cdiv(g.n, 64);
  const long room = (long)GSPLIT_MAX * std::max<long>((long)m.Dp * m.Dp, (long)m.N * m.N) /
                    std::max<long>(1, (long)g.m * g.n);
  const int sp = (int)std::max<long>(1, std::min<long>({16L, 256 / std::max(tiles, 1L), room}));
  gemm_splitk(g, m.gsplit, sp, st);
}

std::unique_ptr<Point> new_point(Model& m) {
  auto pt = std::make_unique<Point>();
  Point& p = *pt;
  p.N = m.N; p.P = m.P; p.D = m.D; p.Dp = m.Dp;
  p.data_bytes = point_bytes(m);
  p.data = p.meta.alloc<char>(p.data_bytes);
  Carve c;
  c.base = p.data;
  layout_point(m, p, c);
  if (m.basis) {
    RM_HIP(hipMemset(p.data, 0, p.data_bytes));
    return pt;
  }
  const long NN = (long)m.N * m.N;
  // pointer arrays for the Y_lm = A_l A_m products (the formed pairs l <= m):
  // both factors full rank in one batch; with a low-rank factor, thin
  // products through G (N x rl):
  //   l low rank:       G = A_m' U_l,    Y' = G Zc_l'
  //   only m low rank:  G = A_l Zc_m,    Y' = U_m G'
  // with Zc = K^-1 U C, so that A_l = Zc_l U_l' for a low-rank l
  std::vector<const double*> ya, yb;
  std::vector<double*> yc;
  std::vector<const float*> fa, fb;
  std::vector<float*> fc;
  std::vector<const double*> la, lb, ra, rb, a2l, b2l, a2r, b2r;
  std::vector<double*> lc, rc, c2l, c2r;
  std::vector<float*> c2lf, c2rf;
  const long ncol = (long)m.nlr * m.rl;
  for (int l = 0; l < m.P; ++l)
    for (int mm = l; mm < m.P; ++mm) {
      const int y = m.yidx_h[l * m.P + mm];
      if (y < 0) continue;
      const int sl = m.lr_slot_h[l], sm = m.lr_slot_h[mm];
      if (sl >= 0 || sm >= 0) {
        const bool caseL = sl >= 0;
        double* G = m.Gy + (long)(caseL ? la.size() : m.nyl + ra.size()) * m.N * m.rl;
        if (caseL) {
          la.push_back(p.A + mm * NN);
          lb.push_back(m.UU + (long)sl * m.rl * m.N);
          lc.push_back(G);
          a2l.push_back(G);
          b2l.push_back(p.ZZ + (ncol + (long)sl * m.rl) * m.N);
          c2l.push_back(p.Yt + (long)y * NN);
          c2lf.push_back(p.Ytf ? p.Ytf + (long)y * NN : nullptr);
        } else {
          ra.push_back(p.A + l * NN);
          rb.push_back(p.ZZ + (ncol + (long)sm * m.rl) * m.N);
          rc.push_back(G);
          a2r.push_back(m.UU + (long)sm * m.rl * m.N);
          b2r.push_back(G);
          c2r.push_back(p.Yt + (long)y * NN);
          c2rf.push_back(p.Ytf ? p.Ytf + (long)y * NN : nullptr);
        }
        continue;
      }
      if (m.prec == RMHMC_MIXED) {
        fa.push_back(p.Af + l * NN);
        fb.push_back(p.Af + mm * NN);
        fc.push_back(p.Ytf + (long)y * NN);
      } else {
        ya.push_back(p.A + l * NN);
        yb.push_back(p.A + mm * NN);
        yc.push_back(p.Yt + (long)y * NN);
      }
    }
  if (m.prec == RMHMC_MIXED) {
    p.Yapf = (const float**)p.meta.alloc<float*>(fa.size());
    p.Ybpf = (const float**)p.meta.alloc<float*>(fb.size());
    p.Ycpf = p.meta.alloc<float*>(fc.size());
    RM_HIP(hipMemcpy((void*)p.Yapf, fa.data(), fa.size() * sizeof(void*), hipMemcpyHostToDevice));
    RM_HIP(hipMemcpy((void*)p.Ybpf, fb.data(), fb.size() * sizeof(void*), hipMemcpyHostToDevice));
    RM_HIP(hipMemcpy((void*)p.Ycpf, fc.data(), fc.size() * sizeof(void*), hipMemcpyHostToDevice));
  } else {
    p.Yap = (const double**)p.meta.alloc<double*>(ya.size());
    p.Ybp = (const double**)p.meta.alloc<double*>(yb.size());
    p.Ycp = p.meta.alloc<double*>(yc.size());
    RM_HIP(hipMemcpy((void*)p.Yap, ya.data(), ya.size() * sizeof(void*), hipMemcpyHostToDevice));
    RM_HIP(hipMemcpy((void*)p.Ybp, yb.data(), yb.size() * sizeof(void*), hipMemcpyHostToDevice));
    RM_HIP(hipMemcpy((void*)p.Ycp, yc.data(), yc.size() * sizeof(void*), hipMemcpyHostToDevice));
  }
  RM_REQUIRE((int)la.size() == m.nyl && (int)ra.size() == m.nyr, "internal: low-rank Y pairs");
  if (m.nyl + m.nyr > 0) {
    auto upload = [&](auto& v) {
      using E = typename std::decay_t<decltype(v)>::value_type;
      E* d = p.meta.alloc<E>(std::max<size_t>(v.size(), 1));
      if (!v.empty()) RM_HIP(hipMemcpy((void*)d, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice));
      return d;
    };
    p.YLa = upload(la); p.YLb = upload(lb); p.YLc = upload(lc);
    p.YRa = upload(ra); p.YRb = upload(rb); p.YRc = upload(rc);
    // the outer products of both cases run as one batch
    a2l.insert(a2l.end(), a2r.begin(), a2r.end());
    b2l.insert(b2l.end(), b2r.begin(), b2r.end());
    c2l.insert(c2l.end(), c2r.begin(), c2r.end());
    c2lf.insert(c2lf.end(), c2rf.begin(), c2rf.end());
    p.Y2a = upload(a2l); p.Y2b = upload(b2l);
    if (m.prec == RMHMC_MIXED) p.Y2cf = upload(c2lf);
    else p.Y2c = upload(c2l);
  }
  RM_HIP(hipMemset(p.data, 0, p.data_bytes));
  return pt;
}

void check_flag_nonfinite(Model& m, const double* x, long n, hipStream_t st, const char* what) {
  fill_int(m.dflag, 1, 0, st);
  hipLaunchKernelGGL(any_nonfinite_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, x, m.dflag);
  RM_CHECK_LAUNCH();
  RM_HIP(hipMemcpyAsync(m.hflag, m.dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  RM_HIP(hipStreamSynchronize(st));
  if (*m.hflag) throw Error(RMHMC_E_NONFINITE, std::string("non-finite values in ") + what);
}

// U, grad U, H at pt.q.  fail == nullptr: a non-positive-definite K is
// reported at once (reads the Cholesky flag, synchronises the stream);
// otherwise the flag is folded into *fail on the device.
void compute_hessian(Model& m, Point& pt, hipStream_t st, int* fail) {
  if (m.basis) {
    // no factorisation can fail here: a hyperparameter outside (0, inf)
    // leaves non-finite values, which the eigensolver reports
    pt.have_pre = pt.have_vW2 = pt.have_eig = false;
    basis_hessian(m.bd, m.lik, m.noise_var, m.beta, m.y, pt.q, pt.alpha, pt.lik, pt.H, m.Dp,
                  pt.gradU, pt.scal, m.bwork, st);
    (void)fail;
    return;
  }
  const int N = m.N, P = m.P;
  const long NN = (long)N * N;
  const double* eta = pt.q + N;
  pt.have_pre = pt.have_vW2 = pt.have_eig = false;
  kgen(m.md, eta, pt.K, pt.K1, st);
  chol_inverse(N, pt.K, pt.Kinv, pt.scal + 0, m.chol, nullptr, st);
  // K^-1 and K_l are symmetric: A x = A' x, and the column-dot kernel is the
  // well-parallelised one
  gemv(N, N, 1.0, pt.Kinv, N, true, 0, pt.q, 0, 0.0, pt.alpha, 0, 1, st);
  lik_derivs(N, m.lik, m.noise_var, m.delta, pt.q, m.y, pt.lik, st);
  const bool mixed = m.prec == RMHMC_MIXED;
  const long ncol = (long)m.nlr * m.rl;
  if (m.nlr > 0) {  // [Z | Zc] = K^-1 [U | U C]
    hipLaunchKernelGGL(lr_scale_kernel, dim3(cdiv((long)N * ncol, 256)), dim3(256), 0, st, N,
                       (int)ncol, m.rl, m.UU, (const int*)m.lr_param, (const int*)m.lr_kind, eta);
    RM_CHECK_LAUNCH();
    Gemm<double> z;
    z.m = N; z.n = (int)(2 * ncol); z.k = N;
    z.A = pt.Kinv; z.lda = N;
    z.B = m.UU; z.ldb = N;
    z.C = pt.ZZ; z.ldc = N;
    thin_gemm(m, z, st);
  }
  for (const auto& run : m.runs_h) {  // A_l = K^-1 K_l, and the transposed copies
    // A_l stays FP64 in both modes: K^-1 reaches 1/jitter while A_l is O(1),
    // so its entries come from heavy cancellation that FP32 operands and
    // accumulation cannot resolve.  Mixed mode takes the FP32 operands of the
    // later products (A_l, A_l' for the traces) from the same epilogue.
    const int l0 = run.first, s0 = m.lr_slot_h[l0];
    Gemm<double> g;
    g.m = N; g.n = N;
    if (s0 < 0) {
      g.k = N;
      g.A = pt.Kinv; g.lda = N;
      g.B = pt.K1 + l0 * NN; g.ldb = N; g.sB = NN;
    } else {  // A_l = Zc_l U_l'
      g.k = m.rl;
      g.A = pt.ZZ + (ncol + (long)s0 * m.rl) * N; g.lda = N; g.sA = (long)m.rl * N;
      g.B = m.UU + (long)s0 * m.rl * N; g.ldb = N; g.tB = true; g.sB = (long)m.rl * N;
    }
    g.C = pt.A + l0 * NN; g.ldc = N; g.sC = NN;
    g.batch = run.second;
    if (!mixed) {
      g.C2 = pt.At + l0 * NN; g.ldc2 = N; g.sC2 = NN;
    } else {
      g.Co = pt.Af + l0 * NN; g.sCo = NN;
      g.ldc2 = N; g.C2o = pt.Atf + l0 * NN; g.sC2o = NN;
    }
    gemm(g, st);
  }
  gemv(N, N, 1.0, pt.K1, N, true, NN, pt.alpha, 0, 0.0, pt.k1a, N, P, st);
  gemv(N, N, 1.0, pt.Kinv, N, true, 0, pt.k1a, N, 0.0, pt.a, N, P, st);   // A_l a = K^-1 (K_l a)
  multi_dot(N, N, pt.Kinv, N, pt.K1, N, NN, P, pt.trK1, m.mdwork, st);
  pair_dots(N, pt.k1a, N, P, pt.a, N, P, pt.kla, st);
  pair_dots(N, pt.alpha, 0, 1, pt.k1a, N, P, pt.ak, st);
  kd_wsum(m.md, eta, m.pairs, m.pairs_h.data(), m.npairs, 0, pt.Kinv, pt.alpha, nullptr, 1,
          pt.phiK2, m.kdwork, st);
  if (!mixed)
    gemm_tallk(P, P, NN, pt.A, NN, pt.At, NN, pt.trAA, P, tall_space(m, P, P), tallk_splits(NN), st);
  else
    gemm_tallk(P, P, NN, pt.Af, NN, pt.Atf, NN, pt.trAA, P, tall_space(m, P, P), tallk_splits(NN), st);
  vsum(N, pt.lik, pt.scal + 3, st);
  vdot(N, pt.q, pt.alpha, pt.scal + 4, st);
  hipLaunchKernelGGL(assemble_H_kernel, dim3(cdiv((long)m.Dp * m.Dp, 256)), dim3(256), 0, st, N, P,
                     m.Dp, m.R, m.beta, (const double*)pt.Kinv, (const double*)pt.lik,
                     (const double*)pt.a, (const double*)pt.kla, (const double*)pt.phiK2,
                     (const double*)pt.trAA, (const int*)m.pidx, pt.H);
  RM_CHECK_LAUNCH();
  hipLaunchKernelGGL(grad_U_kernel, dim3(1), dim3(256), 0, st, N, P, m.beta, (const double*)pt.q,
                     (const double*)pt.alpha, (const double*)pt.lik, (const double*)pt.ak,
                     (const double*)pt.trK1, pt.gradU, pt.scal);
  RM_CHECK_LAUNCH();
  if (fail) {
    hipLaunchKernelGGL(fold_flag_kernel, dim3(1), dim3(64), 0, st, (const int*)m.chol.info, fail,
                       (int)FAIL_NOT_PD);
    RM_CHECK_LAUNCH();
  } else {
    RM_HIP(hipMemcpyAsync(m.hflag, m.chol.info, sizeof(int), hipMemcpyDeviceToHost, st));
    RM_HIP(hipStreamSynchronize(st));
    if (*m.hflag) throw Error(RMHMC_E_NOT_PD, "kernel matrix K is not positive definite");
  }
}

// Softabs eigen-state of pt.H; warm == nullptr: static, else dynamic from
// warm->Psi (Sec. 2.4).  The warm basis is copied before anything touches it
// (a move's start point stays as it was); with `reorth` the copy is first
// re-orthonormalised.
JacobiResult compute_eig(Model& m, Point& pt, const Point* warm, double alpha, const EigCfg& ec,
                         bool reorth, hipStream_t st) {
  const int D = m.D, Dp = m.Dp;
  if (!warm) {
    eig_load_matrix(D, pt.H, Dp, m.eig, st);
    eig_load_basis(D, nullptr, Dp, m.eig, st);
  } else {
    copy(m.eig.Psi, warm->Psi, (long)Dp * Dp, st);
    if (reorth) orthonormalise(D, Dp, m.eig.Psi, m.Wt1, m.Wt2, st, m.gsplit, m.gsplit_layers);
    // M = Psi_w' H Psi_w
    Gemm<double> g;
    g.m = Dp; g.n = Dp; g.k = Dp;
    g.A = pt.H; g.lda = Dp;
    g.B = m.eig.Psi; g.ldb = Dp;
    g.C = m.Wt1; g.ldc = Dp;
    gemm_splitk(g, m.gsplit, m.gsplit_layers, st);
    Gemm<double> h;
    h.m = Dp; h.n = Dp; h.k = Dp;
    h.A = m.eig.Psi; h.lda = Dp; h.tA = true;
    h.B = m.Wt1; h.ldb = Dp;
    h.C = m.eig.M; h.ldc = Dp;
    gemm_splitk(h, m.gsplit, m.gsplit_layers, st);
    symmetrize(Dp, m.eig.M, Dp, st);
  }
  const JacobiResult r0 =
      jacobi_eig(D, m.eig, ec.zeta, 1.0 / alpha, ec.max_sweeps,
                 warm ? JACOBI_INNER_DYNAMIC : JACOBI_INNER_STATIC, ec.blind, ec.host_check,
                 ec.host_check ? nullptr : ec.fail, ec.dstats, st, ec.zeta_s);
  const JacobiResult& r = r0;
  if (warm && ec.host_check && ec.max_seen && r.sweeps > *ec.max_seen) *ec.max_seen = r.sweeps;
  // a static solve accumulates one rounding per rotation into Psi: restore
  // orthogonality before the eigenvalues are refined against H
  if (!warm) orthonormalise(D, Dp, m.eig.Psi, m.Wt1, m.Wt2, st, m.gsplit, m.gsplit_layers);
  rayleigh_refine(D, pt.H, Dp, m.eig, m.Wt2, st, m.gsplit, m.gsplit_layers);
  copy(pt.Psi, m.eig.Psi, (long)Dp * Dp, st);
  softabs_finalize(D, m.eig.M, Dp, alpha, ec.softabs, pt.lam, pt.g, pt.gp, pt.scal + 2, st);
  pt.have_eig = true;
  pt.have_vW2 = false;
  return r;
}

// W-independent pieces of v(W) at pt (needs compute_hessian first).
void compute_precompute(Model& m, Point& pt, hipStream_t st) {
  if (pt.have_pre || m.basis) return;
  const int N = m.N, P = m.P;
  const long NN = (long)N * N;
  const double* eta = pt.q + N;
  const bool mixed = m.prec == RMHMC_MIXED;
  const long ncol = (long)m.nlr * m.rl;
  // B_l = A_l K^-1, FP64 in both modes: the product of an O(1) matrix with
  // K^-1 (entries up to 1/jitter) cancels as heavily as A_l does.  For a
  // low-rank l, B_l = K^-1 U_l C_l U_l' K^-1 = Zc_l Z_l'.
  for (const auto& run : m.runs_h) {
    const int l0 = run.first, s0 = m.lr_slot_h[l0];
    Gemm<double> g;
    g.m = N; g.n = N;
    if (s0 < 0) {
      g.k = N;
      g.A = pt.A + l0 * NN; g.lda = N; g.sA = NN;
      g.B = pt.Kinv; g.ldb = N;
    } else {
      g.k = m.rl;
      g.A = pt.ZZ + (ncol + (long)s0 * m.rl) * N; g.lda = N; g.sA = (long)m.rl * N;
      g.B = pt.ZZ + (long)s0 * m.rl * N; g.ldb = N; g.tB = true; g.sB = (long)m.rl * N;
    }
    g.C = pt.B + l0 * NN; g.ldc = N; g.sC = NN;
    g.batch = run.second;
    gemm(g, st);
  }
  // Y_lm = A_l A_m (formed pairs l <= m), stored transposed: pairs of two
  // full-rank parameters by N^3 products (FP32 operands in mixed mode),
  // the others by the thin products (FP64, rounded to FP32 in mixed mode)
  if (m.nyf > 0) {
    if (!mixed) {
      Gemm<double> g;
      g.m = N; g.n = N; g.k = N;
      g.Ap = pt.Yap; g.lda = N;
      g.Bp = pt.Ybp; g.ldb = N;
      g.C2p = pt.Ycp; g.ldc2 = N;
      g.batch = m.nyf;
      gemm(g, st);
    } else {
      Gemm<float> g;
      g.m = N; g.n = N; g.k = N;
      g.Ap = pt.Yapf; g.lda = N;
      g.Bp = pt.Ybpf; g.ldb = N;
      g.C2p = pt.Ycpf; g.ldc2 = N;
      g.batch = m.nyf;
      gemm(g, st);
    }
  }
  if (m.nyl > 0) {  // G = A_m' U_l
    Gemm<double> g;
    g.m = N; g.n = m.rl; g.k = N;
    g.Ap = pt.YLa; g.lda = N; g.tA = true;
    g.Bp = pt.YLb; g.ldb = N;
    g.Cp = pt.YLc; g.ldc = N;
    g.batch = m.nyl;
    gemm(g, st);
  }
  if (m.nyr > 0) {  // G = A_l Zc_m
    Gemm<double> g;
    g.m = N; g.n = m.rl; g.k = N;
    g.Ap = pt.YRa; g.lda = N;
    g.Bp = pt.YRb; g.ldb = N;
    g.Cp = pt.YRc; g.ldc = N;
    g.batch = m.nyr;
    gemm(g, st);
  }
  if (m.nyl + m.nyr > 0) {  // Y' = G Zc_l' (l low rank), U_m G' (only m low rank)
    Gemm<double> g;
    g.m = N; g.n = N; g.k = m.rl;
    g.Ap = pt.Y2a; g.lda = N;
    g.Bp = pt.Y2b; g.ldb = N; g.tB = true;
    g.ldc = N;
    if (!mixed) g.Cp = pt.Y2c;
    else g.Cop = reinterpret_cast<void* const*>(pt.Y2cf);
    g.batch = m.nyl + m.nyr;
    gemm(g, st);
  }
  // tau[n, y] = tr(A_n A_l A_m) = <A_n, Y_lm'> for the formed pairs y = (l, m)
  if (!mixed)
    gemm_tallk(P, m.nyy, NN, pt.A, NN, pt.Yt, NN, m.tau, P, tall_space(m, P, m.nyy), tallk_splits(NN), st);
  else
    gemm_tallk(P, m.nyy, NN, pt.Af, NN, pt.Ytf, NN, m.tau, P, tall_space(m, P, m.nyy), tallk_splits(NN), st);
  kd_matvec(m.md, eta, m.pairs, m.pairs_h.data(), m.npairs, pt.alpha, 1, pt.k2a, m.mvwork, st);
  {
    Gemm<double> g;  // ik2a = K^-1 [K_lm alpha]
    g.m = N; g.n = m.npairs; g.k = N;
    g.A = pt.Kinv; g.lda = N;
    g.B = pt.k2a; g.ldb = N;
    g.C = pt.ik2a; g.ldc = N;
    thin_gemm(m, g, st);
  }
  {
    Gemm<double> g;  // c1a[l] = K_l [a_0 .. a_P-1]
    g.m = N; g.n = P; g.k = N;
    g.A = pt.K1; g.lda = N; g.sA = NN;
    g.B = pt.a; g.ldb = N;
    g.C = pt.c1a; g.ldc = N; g.sC = (long)N * P;
    g.batch = P;
    gemm(g, st);
    Gemm<double> h = g;  // Aam[l] = A_l [a_0 .. a_P-1]
    h.A = pt.A;
    h.C = pt.Aam;
    gemm(h, st);
  }
  kd_wsum_stack(m.md, eta, m.pairs, m.pairs_h.data(), m.npairs, pt.B, P, m.tB, m.ktbuf,
                tall_space(m, std::min(m.npairs, MAX_TUPLES), P), st);
  kd_wsum(m.md, eta, m.triples, m.triples_h.data(), m.ntriples, 0, pt.Kinv, pt.alpha, nullptr, 1,
          m.t3, m.kdwork, st);
  pair_dots(N, pt.k1a, N, P, pt.Aam, N, P * P, m.D1, st);
  pair_dots(N, pt.k2a, N, m.npairs, pt.a, N, P, m.D2, st);
  pair_dots(N, pt.k1a, N, P, pt.ik2a, N, m.npairs, m.D3, st);
  hipLaunchKernelGGL(dHe_kernel, dim3(cdiv(P * P * P, 256)), dim3(256), 0, st, P,
                     (const double*)m.D1, (const double*)m.D2, (const double*)m.D3,
                     (const double*)m.t3, (const double*)m.tB, (const double*)m.tau,
                     (const int*)m.pidx, (const int*)m.tidx, (const int*)m.tauidx, m.npairs,
                     pt.dHe);
  RM_CHECK_LAUNCH();
  pt.have_pre = true;
}

// v = tr(W dH/dq_i) for a symmetric W (Dp x Dp, ld Dp).
void contract(Model& m, Point& pt, const double* W, double* v, hipStream_t st) {
  if (m.basis) {
    basis_contract(m.bd, m.beta, pt.q, pt.lik, W, m.Dp, v, m.bwork, st);
    return;
  }
  compute_precompute(m, pt, st);
  const int N = m.N, P = m.P, Dp = m.Dp;
  const long NN = (long)N * N;
  multi_dot(N, N, W, Dp, pt.B, N, NN, P, m.wB, m.mdwork, st);
  {
    Gemm<double> g;  // u = K^-1 W[f, eta]
    g.m = N; g.n = P; g.k = N;
    g.A = pt.Kinv; g.lda = N;
    g.B = W + (long)N * Dp; g.ldb = Dp;
    g.C = m.u; g.ldc = N;
    thin_gemm(m, g, st);
  }
  gemv(N, N, 1.0, pt.K1, N, true, NN, m.u, N, 0.0, m.Ku, N, P, st);      // K_l u_l
  gemv(N, N, 1.0, pt.Kinv, N, true, 0, m.Ku, N, 0.0, m.Au, N, P, st);     // A_l u_l = K^-1 K_l u_l
  pair_dots(N, m.u, N, P, pt.c1a, N, P * P, m.E1, st);
  pair_dots(N, m.u, N, P, pt.k2a, N, m.npairs, m.E2, st);
  hipLaunchKernelGGL(zvec_kernel, dim3(cdiv(N, 64)), dim3(64 * ZV_WAVES), 0, st, N, P, Dp, W,
                     (const double*)pt.c1a, (const double*)pt.k2a, (const int*)m.pidx, m.z);
  RM_CHECK_LAUNCH();
  gemv(N, N, 1.0, pt.Kinv, N, true, 0, m.z, 0, 0.0, m.Kz, 0, 1, st);
  hipLaunchKernelGGL(contract_final_kernel, dim3(cdiv(N, 256)), dim3(256), 0, st, N, P, Dp,
                     m.R, m.beta, W, (const double*)pt.lik, (const double*)m.Au, (const double*)m.Kz, v);
  RM_CHECK_LAUNCH();
  if (P > 0) {
    hipLaunchKernelGGL(contract_eta_kernel, dim3(P), dim3(64), 0, st, N, P, Dp, W,
                       (const double*)m.wB, (const double*)m.E1, (const double*)m.E2,
                       (const double*)pt.dHe, (const int*)m.pidx, m.npairs, v);
    RM_CHECK_LAUNCH();
  }
}

void compute_vW2(Model& m, Point& pt, hipStream_t st) {
  if (pt.have_vW2) return;
  const int D = m.D, Dp = m.Dp;
  fill(m.W, (long)Dp * Dp, 0.0, st);
  scale_cols(D, D, pt.Psi, Dp, pt.gp, pt.g, m.Wt1, Dp, st);   // Psi diag(g'/g)
  Gemm<double> g;
  g.m = D; g.n = D; g.k = D;
  g.A = m.Wt1; g.lda = Dp;
  g.B = pt.Psi; g.ldb = Dp; g.tB = true;
  g.C = m.W; g.ldc = Dp;
  gemm_splitk(g, m.gsplit, m.gsplit_layers, st);
  contract(m, pt, m.W, pt.vW2, st);
  pt.have_vW2 = true;
}

// c = Psi'p, b = c / g, dHdp = Psi b (= G^-1 p), ham (optional, device scalar)
void metric_vectors(Model& m, Point& pt, const double* p, double* dHdp, double* ham, hipStream_t st) {
  const int D = m.D, Dp = m.Dp;
  gemv(D, D, 1.0, pt.Psi, Dp, true, 0, p, 0, 0.0, m.vc, 0, 1, st);
  vec_scale(D, m.vc, nullptr, pt.g, false, m.vb, st);
  if (dHdp) gemv_split(D, D, 1.0, pt.Psi, Dp, m.vb, 0.0, dHdp, m.gvwork, st);
  if (ham) {
    hipLaunchKernelGGL(ham_kernel, dim3(1), dim3(256), 0, st, D, (const double*)m.vc,
                       (const double*)pt.g, (const double*)(pt.scal + 1),
                       (const double*)(pt.scal + 2), ham);
    RM_CHECK_LAUNCH();
  }
}

// dH/dq = grad U + v(W2)/2 - v(W1)/2 at pt for momentum p.  Also dH/dp, ham.
void grad_q(Model& m, Point& pt, const double* p, double alpha, int kind, double* dHdq,
            double* dHdp, double* ham, hipStream_t st) {
  const int D = m.D, Dp = m.Dp;
  compute_vW2(m, pt, st);
  metric_vectors(m, pt, p, dHdp, ham, st);
  fill(m.W, (long)Dp * Dp, 0.0, st);
  t_bb(D, pt.lam, m.vb, alpha, kind, m.Wt1, Dp, st);       // T o b b'
  // the D x D products leave about one wave per SIMD with 64 x 64 tiles:
  // their k range is split over the model's layers, as for the warm start
  Gemm<double> g;                                            // Wt2 = (T o bb') Psi'
  g.m = D; g.n = D; g.k = D;
  g.A = m.Wt1; g.lda = Dp;
  g.B = pt.Psi; g.ldb = Dp; g.tB = true;
  g.C = m.Wt2; g.ldc = Dp;
  gemm_splitk(g, m.gsplit, m.gsplit_layers, st);
  Gemm<double> h;                                            // W1 = Psi Wt2
  h.m = D; h.n = D; h.k = D;
  h.A = pt.Psi; h.lda = Dp;
  h.B = m.Wt2; h.ldb = Dp;
  h.C = m.W; h.ldc = Dp;
  gemm_splitk(h, m.gsplit, m.gsplit_layers, st);
  contract(m, pt, m.W, m.v1, st);
  lincomb3(D, pt.gradU, 0.5, pt.vW2, -0.5, m.v1, dHdq, st);
}

// Metric at a new point: Hessian, then the eigen-state (static when warm is
// null).  A warm start whose Jacobi sweeps run out is redone statically
// (counted in *fallbacks) when the host checks convergence; without host
// checks the failure word records it.  A non-finite eigenproblem marks the
// failure word (host-checked mode: also returns false).
bool full_point(Model& m, Point& pt, const Point* warm, double alpha, const EigCfg& ec, bool reorth,
                hipStream_t st, int* fail, long* fallbacks) {
  compute_hessian(m, pt, st, fail);
  JacobiResult r = compute_eig(m, pt, warm, alpha, ec, reorth, st);
  if (!ec.host_check) return true;
  if (!r.converged && !r.nonfinite && warm) {
    if (fallbacks) ++*fallbacks;
    r = compute_eig(m, pt, nullptr, alpha, ec, false, st);
  }
  if (r.nonfinite || !r.converged) {
    if (!fail) {
      if (r.nonfinite) throw Error(RMHMC_E_NONFINITE, "non-finite values in the Hessian");
      throw Error(RMHMC_E_EIG_NOCONV, "softabs_eig: Jacobi did not converge");
    }
    hipLaunchKernelGGL(or_flag_kernel, dim3(1), dim3(64), 0, st, fail,
                       r.nonfinite ? (int)FAIL_NONFINITE : (int)FAIL_NOCONV);
    RM_CHECK_LAUNCH();
    return false;
  }
  return true;
}

std::unique_ptr<struct State> make_state(Model& m, double alpha);

void build_model(Model& m, const rmhmc_model_desc* d, rmhmc_precision prec) {
  RM_REQUIRE(d != nullptr, "model descriptor is NULL");
  RM_REQUIRE(d->N >= 2 && d->dx >= 1, "need N >= 2 and dx >= 1");
  RM_REQUIRE(d->X && d->y, "X and y are required");
  RM_REQUIRE(d->nterms >= 1 && d->nterms <= MAX_TERMS && d->terms, "1..8 kernel terms required");
  RM_REQUIRE(d->jitter > 0.0 && std::isfinite(d->jitter), "jitter must be positive");
  RM_REQUIRE(d->beta >= 0.0 && std::isfinite(d->beta), "beta must be finite and >= 0");
  RM_REQUIRE(d->lik == RMHMC_LIK_BERNOULLI_LOGIT || d->lik == RMHMC_LIK_GAUSSIAN ||
                 d->lik == RMHMC_LIK_GAUSSIAN_MV,
             "unknown likelihood");
  if (d->lik == RMHMC_LIK_GAUSSIAN) RM_REQUIRE(d->noise_var > 0.0, "noise_var must be positive");
  RM_REQUIRE(prec == RMHMC_FP64 || prec == RMHMC_MIXED, "unknown precision");
  const bool two = d->n_fns == 2;
  RM_REQUIRE(d->n_fns >= 0 && d->n_fns <= 2, "n_fns must be 0, 1 or 2");
  RM_REQUIRE(two == (d->lik == RMHMC_LIK_GAUSSIAN_MV),
             "two latent functions go with the mean/variance likelihood and only with it");
  if (two) {
    RM_REQUIRE(d->N % 2 == 0, "two latent functions need N = 2R points");
    RM_REQUIRE(d->fn_col >= 0 && d->fn_col < d->dx, "fn_col out of range");
    RM_REQUIRE(d->delta > 0.0 && std::isfinite(d->delta), "delta must be positive");
    for (int i = 0; i < d->N; ++i)
      RM_REQUIRE(d->X[(long)i * d->dx + d->fn_col] == (i < d->N / 2 ? 0.0 : 1.0),
                 "the function column must be 0 for the first R points and 1 for the last R");
  }
  m.N = d->N; m.dx = d->dx; m.lik = d->lik; m.noise_var = d->noise_var;
  m.jitter = d->jitter; m.beta = d->beta; m.prec = prec;
  m.R = two ? d->N / 2 : 0;
  m.delta = two ? d->delta : 0.0;
  int P = 0;
  ModelDev& md = m.md;
  md.N = m.N; md.dx = m.dx; md.nterms = d->nterms; md.jitter = d->jitter;
  md.fn_col = two ? d->fn_col : -1;
  for (int t = 0; t < d->nterms; ++t) {
    const rmhmc_kernel_term& tt = d->terms[t];
    RM_REQUIRE(tt.ncols >= 1 && tt.ncols <= RMHMC_MAX_TERM_COLS, "term ncols out of range");
    for (int c = 0; c < tt.ncols; ++c)
      RM_REQUIRE(tt.cols[c] >= 0 && tt.cols[c] < d->dx, "term column out of range");
    int np;
    switch (tt.kind) {
      case RMHMC_K_SE_ISO: np = 2; break;
      case RMHMC_K_SE_ARD: np = 1 + tt.ncols; break;
      case RMHMC_K_LINEAR_ARD: np = tt.ncols; break;
      case RMHMC_K_BINARY_SAME:
        RM_REQUIRE(tt.ncols == 1, "BINARY_SAME takes one column");
        np = 1;
        break;
      default: throw Error(RMHMC_E_ARG, "unknown kernel kind");
    }
    if (two) RM_REQUIRE(tt.fn >= -1 && tt.fn <= 1, "term fn must be -1, 0 or 1");
    TermDev& T = md.terms[t];
    T.kind = tt.kind; T.ncols = tt.ncols; T.p0 = P; T.np = np;
    T.fn = two ? tt.fn : -1;
    for (int c = 0; c < RMHMC_MAX_TERM_COLS; ++c) T.cols[c] = c < tt.ncols ? tt.cols[c] : 0;
    RM_REQUIRE(P + np <= MAX_P, "too many hyperparameters");
    for (int a = 0; a < np; ++a) md.param_term[P + a] = t;
    P += np;
  }
  m.P = P; md.P = P;
  m.D = m.N + P;
  m.Dp = eig_padded_dim(m.D);
  for (long i = 0; i < (long)m.N * m.dx; ++i)
    RM_REQUIRE(std::isfinite(d->X[i]), "X contains a non-finite value");
  for (int i = 0; i < m.N; ++i) RM_REQUIRE(std::isfinite(d->y[i]), "y contains a non-finite value");
  // derivative tuples: pairs l <= m and triples l <= m <= n within a term
  m.pidx_h.assign(P * P, -1);
  m.tidx_h.assign(P * P * P, -1);
  m.yidx_h.assign(P * P, -1);
  // a derivative tuple is structurally non-zero only within one term, and
  // for linear-ARD and same-value terms only when all indices coincide
  auto nonzero = [&](int a, int b, int c) {
    const int t = md.param_term[a];
    if (md.param_term[b] != t || md.param_term[c] != t) return false;
    const int kind = md.terms[t].kind;
    if (kind == RMHMC_K_SE_ISO || kind == RMHMC_K_SE_ARD) return true;
    return a == b && b == c;
  };
  // low-rank derivatives: U columns per slot (parameter order)
  m.lr_slot_h.assign(P, -1);
  std::vector<std::vector<std::vector<double>>> lr_cols;
  std::vector<int> lr_param_h, lr_kind_h;
  for (int t = 0; t < md.nterms; ++t) {
    const TermDev& T = md.terms[t];
    auto xv = [&](int i, int c) { return d->X[(long)i * m.dx + c]; };
    auto in_fn = [&](int i) { return T.fn < 0 || xv(i, md.fn_col) == (double)T.fn; };
    if (T.kind == RMHMC_K_LINEAR_ARD) {
      for (int a = 0; a < T.np; ++a) {
        std::vector<double> u(m.N);
        for (int i = 0; i < m.N; ++i) u[i] = in_fn(i) ? xv(i, T.cols[a]) : 0.0;
        m.lr_slot_h[T.p0 + a] = (int)lr_cols.size();
        lr_cols.push_back({u});
        lr_param_h.push_back(T.p0 + a);
        lr_kind_h.push_back(0);
      }
    } else if (T.kind == RMHMC_K_BINARY_SAME) {
      std::vector<double> vals;
      for (int i = 0; i < m.N && (int)vals.size() <= LR_MAX_RANK; ++i)
        if (in_fn(i) && std::find(vals.begin(), vals.end(), xv(i, T.cols[0])) == vals.end())
          vals.push_back(xv(i, T.cols[0]));
      if ((int)vals.size() <= LR_MAX_RANK) {
        std::vector<std::vector<double>> us;
        for (double v : vals) {
          std::vector<double> u(m.N);
          for (int i = 0; i < m.N; ++i) u[i] = (in_fn(i) && xv(i, T.cols[0]) == v) ? 1.0 : 0.0;
          us.push_back(u);
        }
        m.lr_slot_h[T.p0] = (int)lr_cols.size();
        lr_cols.push_back(us);
        lr_param_h.push_back(T.p0);
        lr_kind_h.push_back(1);
      }
    }
  }
  m.nlr = (int)lr_cols.size();
  m.rl = 0;
  for (auto& c : lr_cols) m.rl = std::max(m.rl, (int)c.size());
  for (int l = 0; l < P;) {
    int e = l + 1;
    while (e < P && (m.lr_slot_h[e] >= 0) == (m.lr_slot_h[l] >= 0)) ++e;
    m.runs_h.push_back({l, e - l});
    l = e;
  }
  // tau_nlm = tr(A_n A_l A_m) is symmetric in all three indices (the trace
  // is cyclic, and transposing A_n A_l A_m with A_i = K^-1 K_i reverses the
  // order), so Y_lm = A_l A_m is formed only for pairs within one of two
  // sides of a split of the parameters: of any three indices two share a
  // side.  The full-rank parameters alternate between the sides (and so do
  // the low-rank ones), so the N^3 products (pairs of two full-rank
  // parameters) split evenly: 12 of them for 6 full-rank parameters.
  std::vector<int> side(P);
  {
    int nf = 0, nl = 0;
    for (int l = 0; l < P; ++l) side[l] = (m.lr_slot_h[l] < 0 ? nf++ : nl++) & 1;
  }
  int ny = 0;
  m.nyf = m.nyl = m.nyr = 0;
  for (int l = 0; l < P; ++l)
    for (int mm = l; mm < P; ++mm)
      if (side[l] == side[mm]) {
        m.yidx_h[l * P + mm] = m.yidx_h[mm * P + l] = ny++;
        if (m.lr_slot_h[l] >= 0) ++m.nyl;
        else if (m.lr_slot_h[mm] >= 0) ++m.nyr;
        else ++m.nyf;
      }
  m.nyy = ny;
  m.tauidx_h.assign(P * P * P, -1);
  for (int n = 0; n < P; ++n)
    for (int l = 0; l < P; ++l)
      for (int mm = 0; mm < P; ++mm) {
        int& t = m.tauidx_h[(n * P + l) * P + mm];
        if (m.yidx_h[l * P + mm] >= 0) t = n + P * m.yidx_h[l * P + mm];
        else if (m.yidx_h[n * P + l] >= 0) t = mm + P * m.yidx_h[n * P + l];
        else t = l + P * m.yidx_h[n * P + mm];
        RM_REQUIRE(t >= 0 && t < P * m.nyy, "internal: tau index table");
      }
  for (int l = 0; l < P; ++l)
    for (int mm = l; mm < P; ++mm) {
      if (!nonzero(l, mm, mm)) continue;
      const int idx = (int)m.pairs_h.size();
      m.pairs_h.push_back({2, l, mm, 0});
      m.pidx_h[l * P + mm] = m.pidx_h[mm * P + l] = idx;
    }
  for (int l = 0; l < P; ++l)
    for (int mm = l; mm < P; ++mm)
      for (int n = mm; n < P; ++n) {
        if (!nonzero(l, mm, n)) continue;
        const int idx = (int)m.triples_h.size();
        m.triples_h.push_back({3, l, mm, n});
        const int perm[6][3] = {{l, mm, n}, {l, n, mm}, {mm, l, n}, {mm, n, l}, {n, l, mm}, {n, mm, l}};
        for (auto& pp : perm) m.tidx_h[(pp[0] * P + pp[1]) * P + pp[2]] = idx;
      }
  m.npairs = (int)m.pairs_h.size();
  m.ntriples = (int)m.triples_h.size();
  Pool& pl = m.pool;
  const long N = m.N, NN = N * N, Dp = m.Dp;
  // data, column-major on the device
  std::vector<double> Xc((size_t)m.dx * m.N);
  for (int i = 0; i < m.N; ++i)
    for (int c = 0; c < m.dx; ++c) Xc[(size_t)c * m.N + i] = d->X[(size_t)i * m.dx + c];
  double* Xd = pl.alloc<double>(Xc.size());
  RM_HIP(hipMemcpy(Xd, Xc.data(), Xc.size() * sizeof(double), hipMemcpyHostToDevice));
  md.X = Xd;
  m.y = pl.alloc<double>(N);
  RM_HIP(hipMemcpy(m.y, d->y, N * sizeof(double), hipMemcpyHostToDevice));
  m.pairs = pl.alloc<Tuple>(std::max(m.npairs, 1));
  m.triples = pl.alloc<Tuple>(std::max(m.ntriples, 1));
  if (m.npairs) RM_HIP(hipMemcpy(m.pairs, m.pairs_h.data(), m.npairs * sizeof(Tuple), hipMemcpyHostToDevice));
  if (m.ntriples) RM_HIP(hipMemcpy(m.triples, m.triples_h.data(), m.ntriples * sizeof(Tuple), hipMemcpyHostToDevice));
  m.pidx = pl.alloc<int>(P * P);
  m.tidx = pl.alloc<int>(P * P * P);
  m.tauidx = pl.alloc<int>(P * P * P);
  RM_HIP(hipMemcpy(m.pidx, m.pidx_h.data(), P * P * sizeof(int), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(m.tidx, m.tidx_h.data(), P * P * P * sizeof(int), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(m.tauidx, m.tauidx_h.data(), P * P * P * sizeof(int), hipMemcpyHostToDevice));
  if (m.nlr > 0) {
    const long ncol = (long)m.nlr * m.rl;
    std::vector<double> U((size_t)(N * ncol), 0.0);
    for (int sl = 0; sl < m.nlr; ++sl)
      for (size_t c = 0; c < lr_cols[sl].size(); ++c)
        std::copy(lr_cols[sl][c].begin(), lr_cols[sl][c].end(), U.begin() + (sl * m.rl + c) * N);
    m.UU = pl.alloc<double>(2 * N * ncol);
    RM_HIP(hipMemcpy(m.UU, U.data(), U.size() * sizeof(double), hipMemcpyHostToDevice));
    m.lr_param = pl.alloc<int>(m.nlr);
    m.lr_kind = pl.alloc<int>(m.nlr);
    RM_HIP(hipMemcpy(m.lr_param, lr_param_h.data(), m.nlr * sizeof(int), hipMemcpyHostToDevice));
    RM_HIP(hipMemcpy(m.lr_kind, lr_kind_h.data(), m.nlr * sizeof(int), hipMemcpyHostToDevice));
    m.Gy = pl.alloc<double>(std::max(1L, (long)(m.nyl + m.nyr) * N * m.rl));
  }
  // scratch
  m.chol.L = pl.alloc<double>(NN);
  m.chol.Linv = pl.alloc<double>(NN);
  m.chol.tmp = pl.alloc<double>(NN);
  m.chol.diagLogs = pl.alloc<double>(N);
  m.chol.info = pl.alloc<int>(1);
  m.eig.M = pl.alloc<double>(Dp * Dp);
  m.eig.M2 = pl.alloc<double>(Dp * Dp);
  m.eig.Psi = pl.alloc<double>(Dp * Dp);
  m.eig.V = pl.alloc<double>(eig_rotation_doubles(Dp));
  m.eig.part = pl.alloc<double>(eig_part_doubles(Dp));
  m.eig.ctrl = pl.alloc<double>(EIG_CTRL_DOUBLES);
  m.eig.ctrl_host = pl.alloc_host<double>(EIG_CTRL_DOUBLES);
  const int spl = tallk_splits(NN);
  // the tall-K products: P x P traces, P x nyy traces against the Y stack,
  // and the second-derivative tuples (up to MAX_TUPLES at a time) against P
  // weights
  m.tallwork_n = (long)spl * std::max<long>((long)P * std::max(P, m.nyy),
                                            (long)std::min(m.npairs, MAX_TUPLES) * P);
  m.tallwork = pl.alloc<double>(m.tallwork_n + 64);
  m.kdwork = pl.alloc<double>(512L * MAX_P * MAX_TUPLES + (long)MAX_P * std::max(m.ntriples, m.npairs) + 64);
  m.mvwork = pl.alloc<double>((long)KD_MV_SPLIT * std::min(m.npairs, MAX_TUPLES) * N + 64);
  m.ktbuf = pl.alloc<double>((long)std::min(m.npairs, MAX_TUPLES) * N * N + 64);
  m.mdwork = pl.alloc<double>(multi_dot_work(std::max<long>(N, Dp)) + 64);
  m.gsplit = pl.alloc<double>((long)GSPLIT_MAX * std::max<long>(Dp * Dp, NN) + 64);
  m.chol.split = m.gsplit;   // same stream, never live at the same time
  m.chol.nsplit = GSPLIT_DEFAULT;
  m.W = pl.alloc<double>(Dp * Dp);
  m.Wt1 = pl.alloc<double>(Dp * Dp);
  m.Wt2 = pl.alloc<double>(Dp * Dp);
  m.vc = pl.alloc<double>(Dp);
  m.vb = pl.alloc<double>(Dp);
  m.vtmp = pl.alloc<double>(Dp);
  m.vtmp2 = pl.alloc<double>(Dp);
  m.v1 = pl.alloc<double>(Dp);
  m.u = pl.alloc<double>(N * P);
  m.Au = pl.alloc<double>(N * P);
  m.Ku = pl.alloc<double>(N * P);
  m.gvwork = pl.alloc<double>(64L * Dp);
  m.z = pl.alloc<double>(N);
  m.Kz = pl.alloc<double>(N);
  m.wB = pl.alloc<double>(P);
  m.E1 = pl.alloc<double>(P * P * P);
  m.E2 = pl.alloc<double>(P * std::max(m.npairs, 1));
  m.D1 = pl.alloc<double>(P * P * P);
  m.D2 = pl.alloc<double>(std::max(m.npairs, 1) * P);
  m.D3 = pl.alloc<double>(P * std::max(m.npairs, 1));
  m.t3 = pl.alloc<double>(std::max(m.ntriples, 1));
  m.tB = pl.alloc<double>(P * std::max(m.npairs, 1));
  m.tau = pl.alloc<double>(P * m.nyy);
  m.dflag = pl.alloc<int>(1);
  m.hflag = pl.alloc_host<int>(1);
  m.api_pt_own = new_point(m);
  m.api_pt = m.api_pt_own.get();
}

// The reduced-rank basis model (Sec. 2.1; features in the appendix on the
// reduced-rank representation): features on the device, FP64 throughout.
void build_basis_model(Model& m, const rmhmc_basis_desc* d) {
  RM_REQUIRE(d != nullptr, "basis descriptor is NULL");
  RM_REQUIRE(d->N >= 1 && d->dx >= 1 && d->X && d->y && d->kinds, "need N >= 1, dx >= 1, X, y, kinds");
  RM_REQUIRE(d->lik == RMHMC_LIK_BERNOULLI_LOGIT || d->lik == RMHMC_LIK_GAUSSIAN,
             "the basis model takes the logit or Gaussian likelihood");
  if (d->lik == RMHMC_LIK_GAUSSIAN) RM_REQUIRE(d->noise_var > 0.0, "noise_var must be positive");
  RM_REQUIRE(d->M >= 1 && d->L > 0.0 && d->bias_var > 0.0, "need M >= 1, L > 0, bias_var > 0");
  RM_REQUIRE(d->beta >= 0.0 && std::isfinite(d->beta), "beta must be finite and >= 0");
  for (int h = 0; h < 3; ++h)
    RM_REQUIRE(d->ig_alpha[h] > 0.0 && d->ig_beta[h] > 0.0, "inverse-Gamma parameters must be positive");
  std::vector<int> col, freq, kind;
  for (int c = 0; c < d->dx; ++c) {
    RM_REQUIRE(d->kinds[c] == RMHMC_BASIS_GAUSS || d->kinds[c] == RMHMC_BASIS_LINEAR,
               "unknown basis kernel kind");
    const int nf = d->kinds[c] == RMHMC_BASIS_GAUSS ? d->M : 1;
    for (int mm = 1; mm <= nf; ++mm) {
      col.push_back(c);
      freq.push_back(d->kinds[c] == RMHMC_BASIS_GAUSS ? mm : 0);
      kind.push_back(d->kinds[c] == RMHMC_BASIS_GAUSS ? 0 : 1);
    }
  }
  const int F = (int)col.size();
  for (long i = 0; i < (long)d->N * d->dx; ++i)
    RM_REQUIRE(std::isfinite(d->X[i]), "X contains a non-finite value");
  for (int i = 0; i < d->N; ++i) RM_REQUIRE(std::isfinite(d->y[i]), "y contains a non-finite value");
  m.basis = true;
  m.N = d->N; m.dx = d->dx; m.lik = d->lik; m.noise_var = d->noise_var;
  m.beta = d->beta; m.prec = RMHMC_FP64;
  m.P = 3;
  m.D = F + 4;
  m.Dp = eig_padded_dim(m.D);
  BasisDev& bd = m.bd;
  bd.N = m.N; bd.F = F; bd.Fa = F + 1;
  bd.bias_var = d->bias_var;
  for (int h = 0; h < 3; ++h) {
    bd.ig_a[h] = d->ig_alpha[h];
    bd.ig_b[h] = d->ig_beta[h];
  }
  Pool& pl = m.pool;
  const long N = m.N, Dp = m.Dp;
  std::vector<double> Xc((size_t)m.dx * m.N), kap(F);
  for (int i = 0; i < m.N; ++i)
    for (int c = 0; c < m.dx; ++c) Xc[(size_t)c * m.N + i] = d->X[(size_t)i * m.dx + c];
  for (int j = 0; j < F; ++j)
    kap[j] = kind[j] == 0 ? M_PI * M_PI * freq[j] * freq[j] / (16.0 * d->L * d->L) : 0.0;
  double* Xd = pl.alloc<double>(Xc.size());
  int* cold = pl.alloc<int>(F);
  int* freqd = pl.alloc<int>(F);
  bd.kind = pl.alloc<int>(F);
  bd.kappa = pl.alloc<double>(F);
  bd.Phi = pl.alloc<double>(N * bd.Fa);
  RM_HIP(hipMemcpy(Xd, Xc.data(), Xc.size() * sizeof(double), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(cold, col.data(), F * sizeof(int), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(freqd, freq.data(), F * sizeof(int), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(bd.kind, kind.data(), F * sizeof(int), hipMemcpyHostToDevice));
  RM_HIP(hipMemcpy(bd.kappa, kap.data(), F * sizeof(double), hipMemcpyHostToDevice));
  basis_features(bd, Xd, cold, freqd, d->L, nullptr);
  m.y = pl.alloc<double>(N);
  RM_HIP(hipMemcpy(m.y, d->y, N * sizeof(double), hipMemcpyHostToDevice));
  m.bwork = pl.alloc<double>(N * bd.Fa + N + 64);
  m.eig.M = pl.alloc<double>(Dp * Dp);
  m.eig.M2 = pl.alloc<double>(Dp * Dp);
  m.eig.Psi = pl.alloc<double>(Dp * Dp);
  m.eig.V = pl.alloc<double>(eig_rotation_doubles(Dp));
  m.eig.part = pl.alloc<double>(eig_part_doubles(Dp));
  m.eig.ctrl = pl.alloc<double>(EIG_CTRL_DOUBLES);
  m.eig.ctrl_host = pl.alloc_host<double>(EIG_CTRL_DOUBLES);
  m.gsplit = pl.alloc<double>((long)GSPLIT_MAX * Dp * Dp + 64);
  m.W = pl.alloc<double>(Dp * Dp);
  m.Wt1 = pl.alloc<double>(Dp * Dp);
  m.Wt2 = pl.alloc<double>(Dp * Dp);
  m.vc = pl.alloc<double>(Dp);
  m.vb = pl.alloc<double>(Dp);
  m.vtmp = pl.alloc<double>(Dp);
  m.vtmp2 = pl.alloc<double>(Dp);
  m.v1 = pl.alloc<double>(Dp);
  m.gvwork = pl.alloc<double>(64L * Dp);
  m.dflag = pl.alloc<int>(1);
  m.hflag = pl.alloc_host<int>(1);
  RM_HIP(hipDeviceSynchronize());
  m.api_pt_own = new_point(m);
  m.api_pt = m.api_pt_own.get();
}

// ------------------------------------------------------------ integrator state

}  // namespace

struct State {
  Pool pool;
  Model* m;
  std::unique_ptr<Point> own[3];
  Point* pts[3];     // pts[0] = current point
  double alpha;
  EigCfg ec;         // eigensolver control (fail / dstats point into this state)
  long reorth_every = 10;
  long updates_since_reorth = 0;   // dynamic eigen-updates since the last re-orthonormalisation
  // Captured moves: the sweep budget of the eigen-solve at each position of
  // the position iteration (0 = none set); the tuner records the most sweeps
  // each position needed in its host-checked probe leapfrogs.
  int budget_pos[MAX_FP_BUDGETS] = {};
  int seen_pos[MAX_FP_BUDGETS] = {};
  bool track_pos = false;
  double *p, *ph, *v0, *vk, *gq, *qk, *ham, *z;
  int* fail = nullptr;     // failure word of the current move or step
  int* acc = nullptr;      // accept decision of the current move
  long long* dmove = nullptr;   // index of the chain's next move (device)
  double* dstats = nullptr;   // ST_N device statistics
  double* hstats = nullptr;   // pinned mirror
  int* hfail = nullptr;       // pinned mirror of fail
  long leapfrogs = 0, fallbacks = 0;
};

namespace {

std::unique_ptr<State> make_state(Model& m, double alpha) {
  auto s = std::make_unique<State>();
  s->m = &m;
  s->alpha = alpha;
  for (int i = 0; i < 3; ++i) {
    s->own[i] = new_point(m);
    s->pts[i] = s->own[i].get();
  }
  Pool& pl = s->pool;
  s->p = pl.alloc<double>(m.D);
  s->ph = pl.alloc<double>(m.D);
  s->v0 = pl.alloc<double>(m.D);
  s->vk = pl.alloc<double>(m.D);
  s->gq = pl.alloc<double>(m.D);
  s->qk = pl.alloc<double>(m.D);
  s->z = pl.alloc<double>(m.D);
  s->ham = pl.alloc<double>(2);
  s->fail = pl.alloc<int>(2);
  s->acc = s->fail + 1;
  s->dmove = pl.alloc<long long>(1);
  RM_HIP(hipMemset(s->dmove, 0, sizeof(long long)));
  s->dstats = pl.alloc<double>(ST_N);
  s->hstats = pl.alloc_host<double>(ST_N);
  s->hfail = pl.alloc_host<int>(1);
  RM_HIP(hipMemset(s->fail, 0, 2 * sizeof(int)));
  RM_HIP(hipMemset(s->dstats, 0, ST_N * sizeof(double)));
  s->ec.fail = s->fail;
  s->ec.dstats = s->dstats;
  return s;
}

void reset_stats(State& S, hipStream_t st) {
  fill(S.dstats, ST_N, 0.0, st);
  fill_int(S.fail, 2, 0, st);
  S.leapfrogs = S.fallbacks = 0;
}

void read_stats(State& S, rmhmc_chain_stats* out, hipStream_t st) {
  RM_HIP(hipMemcpyAsync(S.hstats, S.dstats, ST_N * sizeof(double), hipMemcpyDeviceToHost, st));
  RM_HIP(hipStreamSynchronize(st));
  const double* h = S.hstats;
  *out = rmhmc_chain_stats{};
  out->accepted = (int)h[ST_ACC_KEPT];
  out->accepted_all = (int)h[ST_ACC];
  out->failures = (int)h[ST_FAIL];
  out->fail_not_pd = (int)h[ST_NOTPD];
  out->fail_nonfinite = (int)h[ST_NONFINITE];
  out->fail_noconv = (int)h[ST_NOCONV];
  out->leapfrogs = S.leapfrogs;
  out->eig_calls = (long long)h[ST_EIG];
  out->sweeps = (long long)h[ST_SWEEPS];
  out->eig_fallbacks = (int)S.fallbacks;
  out->max_res_p = h[ST_RESP];
  out->max_res_q = h[ST_RESQ];
}

}  // namespace

Model::~Model() = default;

namespace {

// p = G^{1/2} z = Psi diag(sqrt g) Psi' z: p ~ N(0, G(q)) for z ~ N(0, I)
// (Algorithm 1's momentum draw).  The symmetric square root depends on G
// alone, not on the signs or the in-cluster rotation of the eigenvectors.
void draw_momentum(Model& m, State& S, Point& pt, const double* z, hipStream_t st) {
  gemv(m.D, m.D, 1.0, pt.Psi, m.Dp, true, 0, z, 0, 0.0, S.v0, 0, 1, st);
  vec_scale(m.D, S.v0, pt.g, nullptr, true, S.vk, st);
  gemv_split(m.D, m.D, 1.0, pt.Psi, m.Dp, S.vk, 0.0, S.p, m.gvwork, st);
}

void fp_update(int n, const double* base, double c1, const double* x, double c2, const double* y,
               double* dst, double* res, hipStream_t st) {
  hipLaunchKernelGGL(fp_update_kernel, dim3(1), dim3(1024), 0, st, n, base, c1, x, c2, y, dst, res);
  RM_CHECK_LAUNCH();
}

// One generalized leapfrog (Eq. leapfrog) from cur with momentum s.p; trial
// points alternate among the two non-current Points, never touching `keep`
// (if given), which is left exactly as it was.  Both implicit equations are
// solved by K plain fixed-point iterations; the relative residual of the last
// iteration of each goes into the state's statistics.  Failures land in the
// state's failure word; returns false when the host already knows this
// leapfrog failed (the rest of the move can be skipped).
Point* leapfrog(State& s, Point* cur, Point* keep, double eps, int K, hipStream_t st, bool* ok) {
  Model& m = *s.m;
  const int D = m.D;
  Point* trial = nullptr;
  for (int i = 0; i < 3; ++i)
    if (s.pts[i] != cur && s.pts[i] != keep) { trial = s.pts[i]; break; }
  // implicit momentum half step at fixed q: ph <- p - eps/2 dH/dq(q, ph)
  copy(s.ph, s.p, D, st);
  for (int k = 0; k < K; ++k) {
    grad_q(m, *cur, s.ph, s.alpha, s.ec.softabs, s.gq, nullptr, nullptr, st);
    fp_update(D, s.p, -0.5 * eps, s.gq, 0.0, s.gq, s.ph, k == K - 1 ? s.dstats + ST_RESP : nullptr, st);
  }
  // implicit position step: qk <- q + eps/2 (G(q)^-1 ph + G(qk)^-1 ph)
  metric_vectors(m, *cur, s.ph, s.v0, nullptr, st);
  copy(s.qk, cur->q, D, st);
  fp_update(D, cur->q, eps, s.v0, 0.0, s.v0, s.qk, K == 1 ? s.dstats + ST_RESQ : nullptr, st);
  const Point* warm = cur;
  bool good = true;
  int pos = 0;
  auto eval = [&](Point& pt) {
    copy(pt.q, s.qk, D, st);
    const bool reorth = ++s.updates_since_reorth >= s.reorth_every;
    if (reorth) s.updates_since_reorth = 0;
    EigCfg ec = s.ec;
    if (pos < K - 2) {
      ec.zeta = std::max(ec.zeta, LOOSE_ZETA);
      ec.zeta_s = LOOSE_ZETA_S;
    }
    int seen = 0;
    const int slot = std::min(pos, MAX_FP_BUDGETS - 1);
    if (!ec.host_check && s.budget_pos[slot] > 0) ec.blind = s.budget_pos[slot];
    if (s.track_pos) ec.max_seen = &seen;
    good = full_point(m, pt, warm, s.alpha, ec, reorth, st, s.fail, &s.fallbacks) && good;
    if (s.track_pos) s.seen_pos[slot] = std::max(s.seen_pos[slot], seen);
    ++pos;
    warm = &pt;
  };
  for (int k = 1; k < K; ++k) {
    eval(*trial);
    metric_vectors(m, *trial, s.ph, s.vk, nullptr, st);
    fp_update(D, cur->q, 0.5 * eps, s.v0, 0.5 * eps, s.vk, s.qk,
              k == K - 1 ? s.dstats + ST_RESQ : nullptr, st);
  }
  eval(*trial);
  // explicit momentum half step
  grad_q(m, *trial, s.ph, s.alpha, s.ec.softabs, s.gq, nullptr, nullptr, st);
  lincomb3(D, s.ph, -0.5 * eps, s.gq, 0.0, s.gq, s.p, st);
  s.leapfrogs += 1;
  if (ok) *ok = good;
  return trial;
}

}  // namespace
}  // namespace rmhmc

namespace rmhmc {
namespace {

// ------------------------------------------------------------ chain (Algorithm 1)

void check_chain_cfg(const Model& m, const rmhmc_chain_cfg* cfg) {
  RM_REQUIRE(cfg != nullptr, "NULL chain configuration");
  RM_REQUIRE(cfg->n_leapfrog >= 1 && cfg->n_fixed_point >= 1,
             "n_leapfrog and n_fixed_point must be >= 1");
  RM_REQUIRE(cfg->n_moves >= 1 && cfg->n_burnin >= 0 && cfg->n_burnin < cfg->n_moves,
             "need n_moves >= 1 and 0 <= n_burnin < n_moves");
  RM_REQUIRE(std::isfinite(cfg->eps) && cfg->eps > 0.0, "eps must be positive");
  RM_REQUIRE(std::isfinite(cfg->alpha) && cfg->alpha > 0.0, "alpha must be positive");
  RM_REQUIRE(cfg->precision == m.prec, "chain precision differs from the model's");
  RM_REQUIRE(cfg->softabs == RMHMC_SOFTABS_COTH || cfg->softabs == RMHMC_SOFTABS_SQRT,
             "unknown softabs map");
}

// Chain set-up: the configuration into the state, statistics and move
// counter cleared, q0 loaded and its eigen-state solved statically (this
// first solve must succeed; its failure is an error, not a rejection).
void chain_begin(Model& m, State& S, const rmhmc_chain_cfg* cfg, const double* q0,
                 hipStream_t st) {
  const int D = m.D;
  S.alpha = cfg->alpha;
  S.ec.softabs = cfg->softabs;
  S.ec.zeta = cfg->zeta > 0.0 ? cfg->zeta : 1e-13;
  S.ec.max_sweeps = cfg->max_sweeps > 0 ? cfg->max_sweeps : 60;
  S.ec.blind = 0;
  S.ec.host_check = true;
  S.reorth_every = cfg->reorth_every > 0 ? cfg->reorth_every : 10;
  reset_stats(S, st);
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, st, S.dmove, 0LL);
  RM_CHECK_LAUNCH();
  Point* start = S.pts[0];
  copy(start->q, q0, D, st);
  check_flag_nonfinite(m, start->q, D, st, "q0");
  EigCfg ec0 = S.ec;
  ec0.fail = nullptr;
  full_point(m, *start, nullptr, S.alpha, ec0, false, st, nullptr, nullptr);
}

// One move of Algorithm 1 from the state's current point pts[0]: momentum
// from the move's normals (move index read from the device counter), C
// leapfrogs, Metropolis-Hastings on the device, the accepted end point copied
// over the start point, the sample stored.  With host checks off (S.ec) it
// reads nothing back and can be captured into a graph.
void chain_move(Model& m, State& S, const rmhmc_chain_cfg* cfg, double* samples, double* logpost,
                int* accepted, hipStream_t st) {
  const int D = m.D;
  Point* start = S.pts[0];
  const size_t words = start->data_bytes / sizeof(double2);
  const unsigned copy_grid = (unsigned)std::min<size_t>(cdiv((long)words, 256), 2048);
  // p ~ N(0, G(q)) from the move's normals
  hipLaunchKernelGGL(normals_kernel, dim3(cdiv(cdiv(D, 4), 64)), dim3(64), 0, st, D, cfg->seed,
                     cfg->stream_id, 0ull, (const long long*)S.dmove, S.z);
  RM_CHECK_LAUNCH();
  draw_momentum(m, S, *start, S.z, st);
  metric_vectors(m, *start, S.p, nullptr, S.ham, st);
  S.updates_since_reorth = 0;
  Point* cur = start;
  bool ok = true;
  for (int c = 0; c < cfg->n_leapfrog && ok; ++c)
    cur = leapfrog(S, cur, start, cfg->eps, cfg->n_fixed_point, st, &ok);
  metric_vectors(m, *cur, S.p, nullptr, S.ham + 1, st);
  hipLaunchKernelGGL(mh_kernel, dim3(1), dim3(64), 0, st, cfg->seed, cfg->stream_id,
                     (const long long*)S.dmove, cfg->n_burnin, (const double*)S.ham, S.fail,
                     S.acc, S.dstats, accepted);
  RM_CHECK_LAUNCH();
  hipLaunchKernelGGL(copy_if_kernel, dim3(copy_grid), dim3(256), 0, st, (long)words,
                     (double2*)start->data, (const double2*)cur->data, (const int*)S.acc);
  RM_CHECK_LAUNCH();
  hipLaunchKernelGGL(store_sample_kernel, dim3(1), dim3(1024), 0, st, D, (const double*)start->q,
                     (const double*)(start->scal + 1), S.dmove, cfg->n_burnin, samples, logpost);
  RM_CHECK_LAUNCH();
}

void chain_impl(Model& m, const rmhmc_chain_cfg* cfg, const double* q0, double* samples,
                double* logpost, int* accepted, rmhmc_chain_stats* stats, hipStream_t st) {
  check_chain_cfg(m, cfg);
  RM_REQUIRE(q0 && samples && logpost && accepted, "NULL argument");
  State& S = *m.chain_state;
  chain_begin(m, S, cfg, q0, st);
  for (int ell = 0; ell < cfg->n_moves; ++ell) chain_move(m, S, cfg, samples, logpost, accepted, st);
  rmhmc_chain_stats tmp;
  read_stats(S, &tmp, st);
  if (stats) *stats = tmp;
}

// ------------------------------------------------------------ launch-shape tuner
// For a class of chains (padded dimension and precision) the tuner picks, on
// the first model of the class it sees, (a) the number of k-range layers of
// the single Dp x Dp products and of K^-1 = L^-T L^-1 (1, 2, 4 or 8), by
// timing a few leapfrogs with each, and (b) the Jacobi sweep budget of the
// graph-captured moves: one more than the most sweeps a warm start needed in
// those leapfrogs.  The result is kept per class for the process, so every
// chain of a class runs the same launch shapes wherever it is admitted.
struct TunedShape {
  int gsplit = GSPLIT_DEFAULT;
  int sweep_budget = 6;               // the largest of budget_pos
  int budget_pos[MAX_FP_BUDGETS] = {};
  double ms_per_leapfrog = 0.0;
  bool valid = false;
};

std::mutex g_tune_mu;
std::map<std::pair<int, int>, TunedShape> g_tuned;

void apply_shape(Model& m, const TunedShape& t) {
  m.gsplit_layers = t.gsplit;
  m.chol.nsplit = t.gsplit;
}

TunedShape tune_class(Model& m, const rmhmc_chain_cfg* cfg, const double* q0, hipStream_t st) {
  const std::pair<int, int> key(m.Dp, (int)m.prec);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  State& S = *m.chain_state;
  const int probe = std::max(1, std::min(cfg->n_leapfrog, 3));
  hipEvent_t e0, e1;
  RM_HIP(hipEventCreate(&e0));
  RM_HIP(hipEventCreate(&e1));
  TunedShape best;
  int seen = 0;
  for (int& v : S.seen_pos) v = 0;
  for (int layers : {1, 2, 4, 8}) {
    TunedShape t;
    t.gsplit = layers;
    apply_shape(m, t);
    chain_begin(m, S, cfg, q0, st);
    hipLaunchKernelGGL(normals_kernel, dim3(cdiv(cdiv(m.D, 4), 64)), dim3(64), 0, st, m.D,
                       cfg->seed, cfg->stream_id, 0ull, (const long long*)S.dmove, S.z);
    RM_CHECK_LAUNCH();
    draw_momentum(m, S, *S.pts[0], S.z, st);
    S.updates_since_reorth = 0;
    S.track_pos = true;
    Point* cur = S.pts[0];
    // one untimed leapfrog: it also computes the start point's precompute
    cur = leapfrog(S, cur, S.pts[0], cfg->eps, cfg->n_fixed_point, st, nullptr);
    RM_HIP(hipEventRecord(e0, st));
    for (int c = 0; c < probe; ++c)
      cur = leapfrog(S, cur, S.pts[0], cfg->eps, cfg->n_fixed_point, st, nullptr);
    RM_HIP(hipEventRecord(e1, st));
    RM_HIP(hipEventSynchronize(e1));
    S.track_pos = false;
    float ms = 0.f;
    RM_HIP(hipEventElapsedTime(&ms, e0, e1));
    t.ms_per_leapfrog = ms / probe;
    if (!best.valid || t.ms_per_leapfrog < best.ms_per_leapfrog) {
      best = t;
      best.valid = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // one sweep of margin over the most each position of the position
  // iteration needed in the probe
  best.sweep_budget = 0;
  for (int k = 0; k < MAX_FP_BUDGETS; ++k) {
    best.budget_pos[k] = S.seen_pos[k] > 0 ? S.seen_pos[k] + 1 : 2;
    best.sweep_budget = std::max(best.sweep_budget, best.budget_pos[k]);
  }
  (void)seen;
  if (eig_trace()) {
    std::fprintf(stderr, "[tune] Dp=%d prec=%d gsplit=%d ms/leapfrog=%.3f budgets", m.Dp,
                 (int)m.prec, best.gsplit, best.ms_per_leapfrog);
    for (int k = 0; k < cfg->n_fixed_point && k < MAX_FP_BUDGETS; ++k)
      std::fprintf(stderr, " %d", best.budget_pos[k]);
    std::fprintf(stderr, "\n");
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;   // tuned meanwhile by another thread
    g_tuned[key] = best;
  }
  return best;
}

// The move of a chain captured into a graph: set up eagerly (static first
// solve and the start point's contraction precompute), then one move with
// host checks off is recorded on the stream and instantiated.  Replaying the
// graph advances the chain by one move: the move index lives in the state's
// device counter and the trial points are chosen in the same order every
// move, so the recorded launches are the same for every move.
hipGraphExec_t capture_move(Model& m, const rmhmc_chain_cfg* cfg, const double* q0,
                            double* samples, double* logpost, int* accepted,
                            const TunedShape& shape, hipStream_t st, hipGraph_t* graph_out) {
  RM_REQUIRE(!timing_enabled(), "kernel timing must be off while a move is captured");
  State& S = *m.chain_state;
  chain_begin(m, S, cfg, q0, st);
  compute_vW2(m, *S.pts[0], st);   // precompute and v(W2) of the start point
  RM_HIP(hipStreamSynchronize(st));
  const EigCfg saved = S.ec;
  S.ec.host_check = false;
  S.ec.blind = shape.sweep_budget;
  for (int k = 0; k < MAX_FP_BUDGETS; ++k) S.budget_pos[k] = shape.budget_pos[k];
  hipGraph_t graph = nullptr;
  RM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    chain_move(m, S, cfg, samples, logpost, accepted, st);
  } catch (...) {
    (void)hipStreamEndCapture(st, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    S.ec = saved;
    throw;
  }
  RM_HIP(hipStreamEndCapture(st, &graph));
  S.ec = saved;
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    throw Error(RMHMC_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  *graph_out = graph;
  return exec;
}

}  // namespace
}  // namespace rmhmc

// ------------------------------------------------------------ batch of graph-captured chains

struct rmhmc_batch {
  struct Slot {
    rmhmc_model* m = nullptr;
    rmhmc_chain_cfg cfg{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t st = nullptr;
    int launched = 0;
    bool active = false;
    rmhmc::TunedShape shape;
  };
  std::vector<hipStream_t> streams;
  std::vector<Slot> slots;
  std::mutex mu;
};

// ------------------------------------------------------------ worker pool
// Chains (Algorithm 1) run concurrently on a fixed set of worker threads,
// one HIP stream each.  A job submitted while others run starts as soon as
// a worker is free and no other job holds its model (continuous admission);
// results are read back with rmhmc_pool_poll.

struct rmhmc_model {
  rmhmc::Model impl;
};

namespace rmhmc {
namespace {

struct PoolJob {
  long long id = 0;
  rmhmc_model* m = nullptr;
  rmhmc_chain_cfg cfg{};
  const double* q0 = nullptr;
  double *samples = nullptr, *logpost = nullptr;
  int* accepted = nullptr;
  rmhmc_chain_stats stats{};
  rmhmc_status status = RMHMC_OK;
  std::string err;
  int state = 0;   // 0 queued, 1 running, 2 done
  double t_submit = 0, t_start = 0, t_end = 0;
};

}  // namespace
}  // namespace rmhmc

struct rmhmc_pool {
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::deque<std::shared_ptr<rmhmc::PoolJob>> queue;
  std::map<long long, std::shared_ptr<rmhmc::PoolJob>> jobs;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  bool stop = false;
  long long next_id = 0;
  std::chrono::steady_clock::time_point t0;
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace rmhmc {
namespace {

void pool_worker(rmhmc_pool* pool, int w) {
  hipStream_t st = pool->streams[w];
  for (;;) {
    std::shared_ptr<PoolJob> job;
    {
      std::unique_lock<std::mutex> lk(pool->mu);
      for (;;) {
        if (pool->stop) return;
        // first queued job whose model is free
        for (auto it = pool->queue.begin(); it != pool->queue.end(); ++it) {
          if ((*it)->m->impl.busy.try_lock()) {
            job = *it;
            pool->queue.erase(it);
            break;
          }
        }
        if (job) break;
        pool->cv.wait_for(lk, std::chrono::milliseconds(2));
      }
      job->state = 1;
      job->t_start = pool->now_ms();
    }
    rmhmc_status status = RMHMC_OK;
    std::string err;
    try {
      RM_REQUIRE(!job->m->impl.in_batch, "the model is admitted to a batch");
      chain_impl(job->m->impl, &job->cfg, job->q0, job->samples, job->logpost, job->accepted,
                 &job->stats, st);
    } catch (const Error& e) {
      status = e.status;
      err = e.what();
    } catch (const std::exception& e) {
      status = RMHMC_E_HIP;
      err = e.what();
    }
    job->m->impl.busy.unlock();
    {
      std::lock_guard<std::mutex> lk(pool->mu);
      job->status = status;
      job->err = err;
      job->t_end = pool->now_ms();
      job->state = 2;
    }
    pool->cv_done.notify_all();
    pool->cv.notify_all();
  }
}

}  // namespace
}  // namespace rmhmc

// ================================================================ no-allocation eigensolver workspace
// A file-scope device array holds the whole workspace of the stand-alone
// eigensolver for D <= NOALLOC_MAX_D (M, M2, Psi, the rotation sets, the
// convergence partials and control block), so rmhmc_softabs_eig_noalloc
// needs no device allocation.  Each device holds its own copy for the life
// of the process; its address is resolved once per device and used from
// then on (the array's name is not a device address on the host).
namespace rmhmc {
namespace {
constexpr int NOALLOC_MAX_D = 1088;
constexpr int NOALLOC_DP = NOALLOC_MAX_D;   // already a multiple of 64
constexpr long NOALLOC_DOUBLES = 3L * NOALLOC_DP * NOALLOC_DP + 2L * (NOALLOC_DP / 32) * 32 * 32 +
                                 5L * (NOALLOC_DP / 8 + 1) + EIG_CTRL_DOUBLES + 64;
static_assert(NOALLOC_DP % 64 == 0, "padded maximum must be a multiple of 64");
}  // namespace
}  // namespace rmhmc

static __device__ __align__(256) double scratch[rmhmc::NOALLOC_DOUBLES];

namespace rmhmc {
namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex g_noalloc_call_mu[NOALLOC_MAX_DEVICES];

// The current device's copy of `scratch` (resolved on its first use there).
double* noalloc_scratch(int dev) {
  RM_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    RM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    RM_REQUIRE(ptr != nullptr, "no device address for the eigensolver scratch array");
    g_noalloc_ptr[dev] = static_cast<double*>(ptr);
  }
  return g_noalloc_ptr[dev];
}

// Carve an EigWork for padded dimension Dp out of the scratch array.
EigWork noalloc_work(double* base, int Dp, double* ctrl_host) {
  EigWork w;
  long off = 0;
  auto take = [&](long n) {
    double* p = base + off;
    off += (n + 31) / 32 * 32;   // 256-byte steps
    return p;
  };
  w.M = take((long)Dp * Dp);
  w.M2 = take((long)Dp * Dp);
  w.Psi = take((long)Dp * Dp);
  w.V = take(eig_rotation_doubles(Dp));
  w.part = take(eig_part_doubles(Dp));
  w.ctrl = take(EIG_CTRL_DOUBLES);
  w.ctrl_host = ctrl_host;
  RM_REQUIRE(off <= NOALLOC_DOUBLES, "internal: eigensolver scratch layout exceeds the array");
  return w;
}
}  // namespace
}  // namespace rmhmc

// ================================================================ C ABI

using namespace rmhmc;

struct rmhmc_state {
  std::unique_ptr<State> impl;
};

namespace {

template <class F>
rmhmc_status guard(F&& f) {
  try {
    f();
    g_last_error.clear();
    return RMHMC_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return RMHMC_E_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return RMHMC_E_HIP;
  }
}

// Workspace of the stand-alone eigensolver, one per device, sized by the
// largest dimension reserved or solved so far.  A call holds its mutex until
// its stream has drained, so calls from several threads never share it.
struct EigWorkspace {
  std::mutex mu;
  int Dp = 0;
  std::unique_ptr<Pool> pool;
  EigWork w;
};

EigWorkspace& eig_workspace() {
  static std::mutex gmu;
  static std::map<int, std::unique_ptr<EigWorkspace>> per_device;
  int dev = 0;
  RM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(gmu);
  auto& p = per_device[dev];
  if (!p) p = std::make_unique<EigWorkspace>();
  return *p;
}

// Caller holds ws.mu; every earlier use of the buffers has completed.
void eig_workspace_grow(EigWorkspace& ws, int D) {
  const int Dp = eig_padded_dim(D);
  if (ws.Dp >= Dp) return;
  auto pool = std::make_unique<Pool>();
  EigWork w;
  w.M = pool->alloc<double>((long)Dp * Dp);
  w.M2 = pool->alloc<double>((long)Dp * Dp);
  w.Psi = pool->alloc<double>((long)Dp * Dp);
  w.V = pool->alloc<double>(eig_rotation_doubles(Dp));
  w.part = pool->alloc<double>(eig_part_doubles(Dp));
  w.ctrl = pool->alloc<double>(EIG_CTRL_DOUBLES);
  w.ctrl_host = pool->alloc_host<double>(EIG_CTRL_DOUBLES);
  ws.pool = std::move(pool);
  ws.w = w;
  ws.Dp = Dp;
}

template <typename T>
rmhmc_status gemm_entry(int m, int n, int k, T alpha, const T* A, int lda, int transA,
                               const T* B, int ldb, int transB, T beta, T* C, int ldc,
                               hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(m >= 0 && n >= 0 && k >= 0, "negative dimension");
    RM_REQUIRE(A && B && C, "NULL matrix");
    RM_REQUIRE(lda >= std::max(1, transA ? k : m), "lda too small");
    RM_REQUIRE(ldb >= std::max(1, transB ? n : k), "ldb too small");
    RM_REQUIRE(ldc >= std::max(1, m), "ldc too small");
    Gemm<T> g;
    g.m = m; g.n = n; g.k = k; g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.tA = transA != 0;
    g.B = B; g.ldb = ldb; g.tB = transB != 0;
    g.C = C; g.ldc = ldc;
    gemm(g, st);
  });
}

void check_eig_args(int D, const double* H, int ldh, double alpha, int softabs, const double* Q,
                    const double* lam, const double* g, const double* gp, const double* logdetG) {
  RM_REQUIRE(softabs == RMHMC_SOFTABS_COTH || softabs == RMHMC_SOFTABS_SQRT, "unknown softabs map");
  RM_REQUIRE(D >= 1 && H && Q && lam && g && gp && logdetG, "bad argument");
  RM_REQUIRE(ldh >= D, "ldh < D");
  RM_REQUIRE(alpha > 0.0 && std::isfinite(alpha), "alpha must be positive");
  RM_REQUIRE(eig_padded_dim(D) <= 4096, "D too large");
}

// The stand-alone eigensolve on workspace w (sized for D); synchronises `st`.
void softabs_eig_impl(EigWork& w, int D, const double* H, int ldh, double alpha, int softabs,
                      double zeta,
                      int max_sweeps, const double* Q_warm, double* Q, double* lam, double* g,
                      double* gp, double* logdetG, int* sweeps, hipStream_t st) {
  if (zeta <= 0.0) zeta = 1e-13;
  if (max_sweeps <= 0) max_sweeps = 60;
  const int Dp = eig_padded_dim(D);
  eig_load_matrix(D, H, ldh, w, st);
  if (Q_warm) {
    // M = Qw' H Qw computed through padded copies
    eig_load_basis(D, Q_warm, D, w, st);
    Gemm<double> a;
    a.m = Dp; a.n = Dp; a.k = Dp;
    a.A = w.M; a.lda = Dp;
    a.B = w.Psi; a.ldb = Dp;
    a.C = w.M2; a.ldc = Dp;
    gemm(a, st);
    Gemm<double> b;
    b.m = Dp; b.n = Dp; b.k = Dp;
    b.A = w.Psi; b.lda = Dp; b.tA = true;
    b.B = w.M2; b.ldb = Dp;
    b.C = w.M; b.ldc = Dp;
    gemm(b, st);
    symmetrize(Dp, w.M, Dp, st);
  } else {
    eig_load_basis(D, nullptr, D, w, st);
  }
  const JacobiResult r = jacobi_eig(D, w, zeta, 1.0 / alpha, max_sweeps,
                                    Q_warm ? JACOBI_INNER_DYNAMIC : JACOBI_INNER_STATIC, 0, true,
                                    nullptr, nullptr, st);
  if (r.nonfinite) {
    RM_HIP(hipStreamSynchronize(st));
    throw Error(RMHMC_E_NONFINITE, "softabs_eig: non-finite entries in the matrix");
  }
  // static solve: restore orthogonality (M's off-diagonal part is free now)
  if (!Q_warm) orthonormalise(D, Dp, w.Psi, w.M2, w.M, st);
  rayleigh_refine(D, H, ldh, w, w.M2, st);
  copy_matrix(D, D, w.Psi, Dp, Q, D, st);
  softabs_finalize(D, w.M, Dp, alpha, softabs, lam, g, gp, logdetG, st);
  RM_HIP(hipStreamSynchronize(st));
  if (sweeps) *sweeps = r.sweeps;
  if (!r.converged) throw Error(RMHMC_E_EIG_NOCONV, "softabs_eig: Jacobi did not converge");
}

}  // namespace

template <typename T>
rmhmc_status tallk_entry(int m, int n, long k, const T* A, long lda, const T* B, long ldb,
                         double* C, int ldc, T* work, int splits, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(m >= 0 && n >= 0 && k >= 0, "negative dimension");
    RM_REQUIRE(A && B && C && work, "NULL matrix or workspace");
    RM_REQUIRE(splits >= 1 && splits <= 1024, "splits must be in [1, 1024]");
    RM_REQUIRE(k < (1L << 31), "k too large");
    RM_REQUIRE(lda >= std::max(1L, k) && ldb >= std::max(1L, k), "lda or ldb too small");
    RM_REQUIRE(ldc >= std::max(1, m), "ldc too small");
    gemm_tallk(m, n, k, A, lda, B, ldb, C, ldc, reinterpret_cast<double*>(work), splits, st);
  });
}

extern "C" {

const char* rmhmc_last_error(void) { return g_last_error.c_str(); }

rmhmc_status rmhmc_gemm_f64(int m, int n, int k, double alpha, const double* A, int lda, int transA,
                            const double* B, int ldb, int transB, double beta, double* C, int ldc,
                            hipStream_t st) {
  return gemm_entry<double>(m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc, st);
}
rmhmc_status rmhmc_gemm_f32(int m, int n, int k, float alpha, const float* A, int lda, int transA,
                            const float* B, int ldb, int transB, float beta, float* C, int ldc,
                            hipStream_t st) {
  return gemm_entry<float>(m, n, k, alpha, A, lda, transA, B, ldb, transB, beta, C, ldc, st);
}
rmhmc_status rmhmc_gemm_f64_splitk(int m, int n, int k, const double* A, int lda, int transA,
                                   const double* B, int ldb, int transB, double* C, int ldc,
                                   double* work, int splits, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(m >= 0 && n >= 0 && k >= 0, "negative dimension");
    RM_REQUIRE(A && B && C && work, "NULL matrix or workspace");
    RM_REQUIRE(splits >= 1 && splits <= 64, "splits must be in [1, 64]");
    RM_REQUIRE(lda >= std::max(1, transA ? k : m), "lda too small");
    RM_REQUIRE(ldb >= std::max(1, transB ? n : k), "ldb too small");
    RM_REQUIRE(ldc >= std::max(1, m), "ldc too small");
    Gemm<double> g;
    g.m = m; g.n = n; g.k = k;
    g.A = A; g.lda = lda; g.tA = transA != 0;
    g.B = B; g.ldb = ldb; g.tB = transB != 0;
    g.C = C; g.ldc = ldc;
    gemm_splitk(g, work, splits, st);
  });
}

rmhmc_status rmhmc_gemm_tallk_f64(int m, int n, long k, const double* A, long lda,
                                  const double* B, long ldb, double* C, int ldc, double* work,
                                  int splits, hipStream_t st) {
  return tallk_entry<double>(m, n, k, A, lda, B, ldb, C, ldc, work, splits, st);
}
rmhmc_status rmhmc_gemm_tallk_f32(int m, int n, long k, const float* A, long lda, const float* B,
                                  long ldb, double* C, int ldc, float* work, int splits,
                                  hipStream_t st) {
  return tallk_entry<float>(m, n, k, A, lda, B, ldb, C, ldc, work, splits, st);
}

rmhmc_status rmhmc_model_create(const rmhmc_model_desc* desc, rmhmc_precision prec,
                                rmhmc_model** out) {
  return guard([&] {
    RM_REQUIRE(out != nullptr, "out is NULL");
    auto m = std::make_unique<rmhmc_model>();
    Model& md = m->impl;
    build_model(md, desc, prec);
    md.chain_state = make_state(md, 1e6);
    md.device_bytes = md.pool.bytes + md.api_pt->meta.bytes + md.chain_state->pool.bytes;
    for (int i = 0; i < 3; ++i) md.device_bytes += md.chain_state->pts[i]->meta.bytes;
    RM_HIP(hipDeviceSynchronize());
    *out = m.release();
  });
}

rmhmc_status rmhmc_basis_model_create(const rmhmc_basis_desc* desc, rmhmc_model** out) {
  return guard([&] {
    RM_REQUIRE(out != nullptr, "out is NULL");
    auto m = std::make_unique<rmhmc_model>();
    Model& md = m->impl;
    build_basis_model(md, desc);
    md.chain_state = make_state(md, 1.0);
    md.device_bytes = md.pool.bytes + md.api_pt->meta.bytes + md.chain_state->pool.bytes;
    for (int i = 0; i < 3; ++i) md.device_bytes += md.chain_state->pts[i]->meta.bytes;
    RM_HIP(hipDeviceSynchronize());
    *out = m.release();
  });
}

rmhmc_status rmhmc_model_dims(const rmhmc_model* m, int* N, int* P, int* D) {
  return guard([&] {
    RM_REQUIRE(m != nullptr, "model is NULL");
    if (N) *N = m->impl.N;
    if (P) *P = m->impl.P;
    if (D) *D = m->impl.D;
  });
}

rmhmc_status rmhmc_model_bytes(const rmhmc_model* m, long long* bytes) {
  return guard([&] {
    RM_REQUIRE(m && bytes, "NULL argument");
    *bytes = (long long)m->impl.device_bytes;
  });
}

rmhmc_status rmhmc_model_set_beta(rmhmc_model* mh, double beta) {
  return guard([&] {
    RM_REQUIRE(mh != nullptr, "model is NULL");
    RM_REQUIRE(beta >= 0.0 && std::isfinite(beta), "beta must be finite and >= 0");
    Model& m = mh->impl;
    std::lock_guard<std::mutex> lk(m.busy);
    RM_REQUIRE(!m.in_batch, "the model is admitted to a batch");
    m.beta = beta;
  });
}

rmhmc_status rmhmc_log_likelihood(rmhmc_model* mh, const double* q, double* ll, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(mh && q && ll, "NULL argument");
    Model& m = mh->impl;
    std::lock_guard<std::mutex> lk(m.busy);
    RM_REQUIRE(!m.in_batch, "the model is admitted to a batch");
    Point& pt = *m.api_pt;
    const double* f = q;
    if (m.basis) {   // f = Phi (a, b)
      gemv(m.N, m.bd.Fa, 1.0, m.bd.Phi, m.N, false, 0, q, 0, 0.0, pt.alpha, 0, 1, st);
      f = pt.alpha;
    }
    lik_derivs(m.N, m.lik, m.noise_var, m.delta, f, m.y, pt.lik, st);   // l_i = -ln P(X_i | f_i)
    vsum(m.N, pt.lik, ll, st);
    axpby(1, 0.0, ll, -1.0, ll, st);
    RM_HIP(hipStreamSynchronize(st));
  });
}

rmhmc_status rmhmc_model_destroy(rmhmc_model* m) {
  return guard([&] {
    if (m) {
      (void)hipDeviceSynchronize();
      delete m;
    }
  });
}

rmhmc_status rmhmc_hessian(rmhmc_model* mh, const double* q, double* U, double* gradU, double* H,
                           int ldh, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(mh && q && U && gradU && H, "NULL argument");
    Model& m = mh->impl;
    RM_REQUIRE(ldh >= m.D, "ldh < D");
    std::lock_guard<std::mutex> lk(m.busy);
    RM_REQUIRE(!m.in_batch, "the model is admitted to a batch");
    Point& pt = *m.api_pt;
    copy(pt.q, q, m.D, st);
    check_flag_nonfinite(m, pt.q, m.D, st, "q");
    compute_hessian(m, pt, st, nullptr);
    copy(U, pt.scal + 1, 1, st);
    copy(gradU, pt.gradU, m.D, st);
    copy_matrix(m.D, m.D, pt.H, m.Dp, H, ldh, st);
    RM_HIP(hipStreamSynchronize(st));   // the model's scratch is free on return
  });
}

rmhmc_status rmhmc_softabs_eig_reserve(int D) {
  return guard([&] {
    RM_REQUIRE(D >= 1, "D must be >= 1");
    RM_REQUIRE(eig_padded_dim(D) <= 4096, "D too large");
    EigWorkspace& ws = eig_workspace();
    std::lock_guard<std::mutex> lk(ws.mu);
    eig_workspace_grow(ws, D);
  });
}

rmhmc_status rmhmc_softabs_eig(int D, const double* H, int ldh, double alpha, int softabs,
                               double zeta, int max_sweeps, const double* Q_warm, double* Q,
                               double* lam, double* g, double* gp, double* logdetG, int* sweeps,
                               hipStream_t st) {
  return guard([&] {
    check_eig_args(D, H, ldh, alpha, softabs, Q, lam, g, gp, logdetG);
    EigWorkspace& ws = eig_workspace();
    std::lock_guard<std::mutex> lk(ws.mu);
    eig_workspace_grow(ws, D);
    softabs_eig_impl(ws.w, D, H, ldh, alpha, softabs, zeta, max_sweeps, Q_warm, Q, lam, g, gp,
                     logdetG, sweeps, st);
  });
}

rmhmc_status rmhmc_softabs_eig_noalloc(int D, const double* H, int ldh, double alpha,
                                       int softabs, double zeta, int max_sweeps,
                                       const double* Q_warm, double* Q, double* lam, double* g,
                                       double* gp, double* logdetG, int* sweeps,
                                       hipStream_t st) {
  return guard([&] {
    check_eig_args(D, H, ldh, alpha, softabs, Q, lam, g, gp, logdetG);
    RM_REQUIRE(D <= NOALLOC_MAX_D, "softabs_eig_noalloc: D exceeds the scratch maximum (1088)");
    int dev = 0;
    RM_HIP(hipGetDevice(&dev));
    double* base = noalloc_scratch(dev);
    std::lock_guard<std::mutex> lk(g_noalloc_call_mu[dev]);
    double ctrl_host[EIG_CTRL_DOUBLES];
    EigWork w = noalloc_work(base, eig_padded_dim(D), ctrl_host);
    softabs_eig_impl(w, D, H, ldh, alpha, softabs, zeta, max_sweeps, Q_warm, Q, lam, g, gp,
                     logdetG, sweeps, st);
  });
}

rmhmc_status rmhmc_metric_grad(rmhmc_model* mh, const double* q, const double* p, const double* Q,
                               const double* lam, double alpha, int softabs, double* dHdq,
                               double* dHdp, double* ham, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(mh && q && p && Q && lam && dHdq && dHdp && ham, "NULL argument");
    RM_REQUIRE(alpha > 0.0 && std::isfinite(alpha), "alpha must be positive");
    Model& m = mh->impl;
    std::lock_guard<std::mutex> lk(m.busy);
    RM_REQUIRE(!m.in_batch, "the model is admitted to a batch");
    Point& pt = *m.api_pt;
    copy(pt.q, q, m.D, st);
    compute_hessian(m, pt, st, nullptr);
    // eigen-state supplied by the caller
    eig_load_basis(m.D, Q, m.D, m.eig, st);
    copy(pt.Psi, m.eig.Psi, (long)m.Dp * m.Dp, st);
    fill(m.eig.M, (long)m.Dp * m.Dp, 0.0, st);
    copy_matrix(1, m.D, lam, 1, m.eig.M, m.Dp + 1, st);   // diag(lam)
    RM_REQUIRE(softabs == RMHMC_SOFTABS_COTH || softabs == RMHMC_SOFTABS_SQRT,
               "unknown softabs map");
    softabs_finalize(m.D, m.eig.M, m.Dp, alpha, softabs, pt.lam, pt.g, pt.gp, pt.scal + 2, st);
    pt.have_eig = true;
    grad_q(m, pt, p, alpha, softabs, dHdq, dHdp, ham, st);
    RM_HIP(hipStreamSynchronize(st));
  });
}

rmhmc_status rmhmc_state_create(rmhmc_model* mh, const double* q0, const double* p0, double alpha,
                                int softabs, hipStream_t st, rmhmc_state** out) {
  return guard([&] {
    RM_REQUIRE(mh && q0 && p0 && out, "NULL argument");
    RM_REQUIRE(alpha > 0.0 && std::isfinite(alpha), "alpha must be positive");
    Model& m = mh->impl;
    std::lock_guard<std::mutex> lk(m.busy);
    RM_REQUIRE(!m.in_batch, "the model is admitted to a batch");
    auto s = std::make_unique<rmhmc_state>();
    RM_REQUIRE(softabs == RMHMC_SOFTABS_COTH || softabs == RMHMC_SOFTABS_SQRT,
               "unknown softabs map");
    s->impl = make_state(m, alpha);
    State& S = *s->impl;
    S.ec.softabs = softabs;
    copy(S.pts[0]->q, q0, m.D, st);
    copy(S.p, p0, m.D, st);
    check_flag_nonfinite(m, S.pts[0]->q, m.D, st, "q0");
    full_point(m, *S.pts[0], nullptr, alpha, S.ec, false, st, nullptr, nullptr);
    RM_HIP(hipStreamSynchronize(st));
    *out = s.release();
  });
}

rmhmc_status rmhmc_state_get(const rmhmc_state* sh, double* q, double* p, double* ham,
                             hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(sh && q && p, "NULL argument");
    State& S = *sh->impl;
    Model& m = *S.m;
    std::lock_guard<std::mutex> lk(m.busy);
    RM_REQUIRE(!m.in_batch, "the model is admitted to a batch");
    copy(q, S.pts[0]->q, m.D, st);
    copy(p, S.p, m.D, st);
    if (ham) metric_vectors(m, *S.pts[0], S.p, nullptr, ham, st);
    RM_HIP(hipStreamSynchronize(st));
  });
}

rmhmc_status rmhmc_state_set_momentum(rmhmc_state* sh, const double* p, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(sh && p, "NULL argument");
    copy(sh->impl->p, p, sh->impl->m->D, st);
  });
}

rmhmc_status rmhmc_state_draw_momentum(rmhmc_state* sh, const double* z, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(sh && z, "NULL argument");
    State& S = *sh->impl;
    std::lock_guard<std::mutex> lk(S.m->busy);
    draw_momentum(*S.m, S, *S.pts[0], z, st);
    RM_HIP(hipStreamSynchronize(st));
  });
}

rmhmc_status rmhmc_state_stats(const rmhmc_state* sh, rmhmc_chain_stats* out) {
  return guard([&] {
    RM_REQUIRE(sh && out, "NULL argument");
    State& S = *sh->impl;
    read_stats(S, out, nullptr);
  });
}

rmhmc_status rmhmc_chain_randoms(int D, unsigned long long seed, unsigned long long stream_id,
                                 unsigned long long move, double* z, double* u,
                                 hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(D >= 1 && z && u, "bad argument");
    hipLaunchKernelGGL(normals_kernel, dim3(cdiv(cdiv(D, 4), 64)), dim3(64), 0, st, D, seed,
                       stream_id, move, (const long long*)nullptr, z);
    RM_CHECK_LAUNCH();
    hipLaunchKernelGGL(uniform_kernel, dim3(1), dim3(64), 0, st, seed, stream_id, move, u);
    RM_CHECK_LAUNCH();
  });
}

rmhmc_status rmhmc_timing_enable(unsigned mask) {
  return guard([&] {
    RM_HIP(hipDeviceSynchronize());
    timing_set(mask);
  });
}

rmhmc_status rmhmc_timing_read(int kind, long long* launches, double* ms, double* flops,
                               double* bytes) {
  return guard([&] {
    RM_REQUIRE(kind >= 0 && kind < TK_COUNT, "unknown timer kind");
    RM_REQUIRE(launches && ms && flops && bytes, "NULL argument");
    timing_read(kind, launches, ms, flops, bytes);
  });
}

rmhmc_status rmhmc_state_destroy(rmhmc_state* sh) {
  return guard([&] {
    (void)hipDeviceSynchronize();
    delete sh;
  });
}

rmhmc_status rmhmc_glf_step(rmhmc_model* mh, rmhmc_state* sh, double eps, int n_fixed_point,
                            hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(mh && sh, "NULL argument");
    RM_REQUIRE(sh->impl->m == &mh->impl, "state belongs to another model");
    RM_REQUIRE(n_fixed_point >= 1, "n_fixed_point must be >= 1");
    RM_REQUIRE(std::isfinite(eps) && eps > 0.0, "eps must be positive");
    State& S = *sh->impl;
    std::lock_guard<std::mutex> lk(mh->impl.busy);
    RM_REQUIRE(!mh->impl.in_batch, "the model is admitted to a batch");
    Point* nxt = leapfrog(S, S.pts[0], nullptr, eps, n_fixed_point, st, nullptr);
    // one read of the failure word per step; a failed step leaves the state
    // at its start point
    RM_HIP(hipMemcpyAsync(S.hfail, S.fail, sizeof(int), hipMemcpyDeviceToHost, st));
    RM_HIP(hipStreamSynchronize(st));
    const int f = *S.hfail;
    if (f) {
      fill_int(S.fail, 1, 0, st);
      RM_HIP(hipStreamSynchronize(st));
      if (f & FAIL_NOT_PD) throw Error(RMHMC_E_NOT_PD, "kernel matrix K is not positive definite");
      if (f & FAIL_NONFINITE) throw Error(RMHMC_E_NONFINITE, "non-finite values in the leapfrog");
      throw Error(RMHMC_E_EIG_NOCONV, "softabs_eig: Jacobi did not converge");
    }
    for (int i = 1; i < 3; ++i)
      if (S.pts[i] == nxt) std::swap(S.pts[0], S.pts[i]);
  });
}

rmhmc_status rmhmc_chain(rmhmc_model* mh, const rmhmc_chain_cfg* cfg, const double* q0,
                         double* samples, double* logpost, int* accepted,
                         rmhmc_chain_stats* stats, hipStream_t st) {
  return guard([&] {
    RM_REQUIRE(mh != nullptr, "NULL model");
    std::lock_guard<std::mutex> lk(mh->impl.busy);
    RM_REQUIRE(!mh->impl.in_batch, "the model is admitted to a batch");
    chain_impl(mh->impl, cfg, q0, samples, logpost, accepted, stats, st);
  });
}

rmhmc_status rmhmc_batch_create(int n_streams, rmhmc_batch** out) {
  return guard([&] {
    RM_REQUIRE(out != nullptr, "out is NULL");
    RM_REQUIRE(n_streams >= 1 && n_streams <= 64, "n_streams must be in 1..64");
    auto b = std::make_unique<rmhmc_batch>();
    for (int i = 0; i < n_streams; ++i) {
      hipStream_t s;
      RM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      b->streams.push_back(s);
    }
    *out = b.release();
  });
}

rmhmc_status rmhmc_batch_admit(rmhmc_batch* b, rmhmc_model* mh, const rmhmc_chain_cfg* cfg,
                               const double* q0, double* samples, double* logpost, int* accepted,
                               int* slot) {
  return guard([&] {
    RM_REQUIRE(b && mh && cfg && q0 && samples && logpost && accepted && slot, "NULL argument");
    Model& m = mh->impl;
    check_chain_cfg(m, cfg);
    std::lock_guard<std::mutex> blk(b->mu);
    std::lock_guard<std::mutex> lk(m.busy);
    RM_REQUIRE(!m.in_batch, "the model is already admitted to a batch");
    int k = 0;
    while (k < (int)b->slots.size() && b->slots[k].active) ++k;
    if (k == (int)b->slots.size()) b->slots.emplace_back();
    rmhmc_batch::Slot& sl = b->slots[k];
    sl = rmhmc_batch::Slot{};
    sl.m = mh;
    sl.cfg = *cfg;
    sl.st = b->streams[k % b->streams.size()];
    sl.shape = tune_class(m, cfg, q0, sl.st);
    apply_shape(m, sl.shape);
    sl.exec = capture_move(m, cfg, q0, samples, logpost, accepted, sl.shape, sl.st, &sl.graph);
    m.in_batch = true;
    sl.active = true;
    *slot = k;
  });
}

rmhmc_status rmhmc_batch_step(rmhmc_batch* b, int n_moves) {
  return guard([&] {
    RM_REQUIRE(b != nullptr, "NULL batch");
    RM_REQUIRE(n_moves >= 0, "n_moves must be >= 0");
    std::lock_guard<std::mutex> blk(b->mu);
    // one move of every active chain in turn, so the streams stay busy together
    for (int k = 0; k < n_moves; ++k)
      for (auto& sl : b->slots) {
        if (!sl.active || sl.launched >= sl.cfg.n_moves) continue;
        RM_HIP(hipGraphLaunch(sl.exec, sl.st));
        ++sl.launched;
      }
  });
}

rmhmc_status rmhmc_batch_sync(rmhmc_batch* b) {
  return guard([&] {
    RM_REQUIRE(b != nullptr, "NULL batch");
    for (hipStream_t s : b->streams) RM_HIP(hipStreamSynchronize(s));
  });
}

rmhmc_status rmhmc_batch_retire(rmhmc_batch* b, int slot, int* moves_done,
                                rmhmc_chain_stats* stats, int* sweep_budget, int* gsplit) {
  return guard([&] {
    RM_REQUIRE(b != nullptr, "NULL batch");
    std::lock_guard<std::mutex> blk(b->mu);
    RM_REQUIRE(slot >= 0 && slot < (int)b->slots.size() && b->slots[slot].active, "no such slot");
    rmhmc_batch::Slot& sl = b->slots[slot];
    RM_HIP(hipStreamSynchronize(sl.st));
    Model& m = sl.m->impl;
    State& S = *m.chain_state;
    S.leapfrogs = (long)sl.launched * sl.cfg.n_leapfrog;
    S.fallbacks = 0;
    rmhmc_chain_stats st{};
    read_stats(S, &st, sl.st);
    if (stats) *stats = st;
    if (moves_done) *moves_done = sl.launched;
    if (sweep_budget) *sweep_budget = sl.shape.sweep_budget;
    if (gsplit) *gsplit = sl.shape.gsplit;
    (void)hipGraphExecDestroy(sl.exec);
    (void)hipGraphDestroy(sl.graph);
    {
      std::lock_guard<std::mutex> lk(m.busy);
      m.in_batch = false;
    }
    sl = rmhmc_batch::Slot{};
  });
}

rmhmc_status rmhmc_batch_destroy(rmhmc_batch* b) {
  return guard([&] {
    if (!b) return;
    for (hipStream_t s : b->streams) (void)hipStreamSynchronize(s);
    for (auto& sl : b->slots) {
      if (!sl.active) continue;
      (void)hipGraphExecDestroy(sl.exec);
      (void)hipGraphDestroy(sl.graph);
      std::lock_guard<std::mutex> lk(sl.m->impl.busy);
      sl.m->impl.in_batch = false;
    }
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    delete b;
  });
}

rmhmc_status rmhmc_pool_create(int n_workers, rmhmc_pool** out) {
  return guard([&] {
    RM_REQUIRE(out != nullptr, "out is NULL");
    RM_REQUIRE(n_workers >= 1 && n_workers <= 64, "n_workers must be in 1..64");
    auto p = std::make_unique<rmhmc_pool>();
    p->t0 = std::chrono::steady_clock::now();
    for (int w = 0; w < n_workers; ++w) {
      hipStream_t s;
      RM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      p->streams.push_back(s);
    }
    rmhmc_pool* raw = p.get();
    for (int w = 0; w < n_workers; ++w) raw->workers.emplace_back([raw, w] { pool_worker(raw, w); });
    *out = p.release();
  });
}

rmhmc_status rmhmc_pool_submit(rmhmc_pool* pool, rmhmc_model* m, const rmhmc_chain_cfg* cfg,
                               const double* q0, double* samples, double* logpost, int* accepted,
                               long long* ticket) {
  return guard([&] {
    RM_REQUIRE(pool && m && cfg && q0 && samples && logpost && accepted && ticket,
               "NULL argument");
    check_chain_cfg(m->impl, cfg);
    auto j = std::make_shared<PoolJob>();
    j->m = m;
    j->cfg = *cfg;
    j->q0 = q0;
    j->samples = samples; j->logpost = logpost; j->accepted = accepted;
    {
      std::lock_guard<std::mutex> lk(pool->mu);
      j->id = ++pool->next_id;
      j->t_submit = pool->now_ms();
      pool->jobs[j->id] = j;
      pool->queue.push_back(j);
    }
    pool->cv.notify_all();
    *ticket = j->id;
  });
}

rmhmc_status rmhmc_pool_poll(rmhmc_pool* pool, long long ticket, int wait, int* done,
                             rmhmc_chain_stats* stats, double* times_ms) {
  return guard([&] {
    RM_REQUIRE(pool && done, "NULL argument");
    std::unique_lock<std::mutex> lk(pool->mu);
    auto it = pool->jobs.find(ticket);
    RM_REQUIRE(it != pool->jobs.end(), "unknown ticket");
    std::shared_ptr<PoolJob> j = it->second;
    if (wait) pool->cv_done.wait(lk, [&] { return j->state == 2; });
    if (j->state != 2) {
      *done = 0;
      return;
    }
    *done = j->status == RMHMC_OK ? 1 : (int)j->status;
    if (stats) *stats = j->stats;
    if (times_ms) {
      times_ms[0] = j->t_submit;
      times_ms[1] = j->t_start;
      times_ms[2] = j->t_end;
    }
    if (j->status != RMHMC_OK) g_last_error = j->err;
    pool->jobs.erase(it);
  });
}

rmhmc_status rmhmc_pool_destroy(rmhmc_pool* pool) {
  return guard([&] {
    if (!pool) return;
    {
      std::lock_guard<std::mutex> lk(pool->mu);
      pool->stop = true;
    }
    pool->cv.notify_all();
    for (auto& t : pool->workers) t.join();
    for (hipStream_t s : pool->streams) (void)hipStreamDestroy(s);
    delete pool;
  });
}

}  // extern "C"
