// Small dense linear-algebra building blocks: GEMV, multi-dot reductions,
// blocked Cholesky with explicit inverse, and vector utilities.  Every
// reduction runs in a fixed order (no atomics), so results are bitwise
// reproducible run to run.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.h"

namespace rmhmc {

// ---------------------------------------------------------------- timing
namespace {
struct TRec {
  int kind;
  hipEvent_t a, b;
  double flops, bytes;
  long long launches;   // back-to-back launches of the kind between a and b
};
std::mutex g_tmu;
unsigned g_tmask = 0;
std::vector<TRec> g_recs;
std::vector<hipEvent_t> g_evpool;
hipEvent_t take_event() {
  if (!g_evpool.empty()) {
    hipEvent_t e = g_evpool.back();
    g_evpool.pop_back();
    return e;
  }
  hipEvent_t e;
  RM_HIP(hipEventCreate(&e));
  return e;
}
}  // namespace

bool timing_enabled() { return g_tmask != 0; }

int timing_begin(int kind, hipStream_t st) {
  if (!((g_tmask >> kind) & 1u)) return -1;
  std::lock_guard<std::mutex> lk(g_tmu);
  TRec r{kind, take_event(), take_event(), 0.0, 0.0, 1};
  RM_HIP(hipEventRecord(r.a, st));
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}

void timing_end(int slot, hipStream_t st, double flops, double bytes, long long launches) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_tmu);
  TRec& r = g_recs[slot];
  RM_HIP(hipEventRecord(r.b, st));
  r.flops = flops;
  r.bytes = bytes;
  r.launches = launches;
}

void timing_set(unsigned mask) {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& r : g_recs) {
    g_evpool.push_back(r.a);
    g_evpool.push_back(r.b);
  }
  g_recs.clear();
  g_tmask = mask;
}

void timing_read(int kind, long long* launches, double* ms, double* flops, double* bytes) {
  std::lock_guard<std::mutex> lk(g_tmu);
  long long n = 0;
  double t = 0, f = 0, b = 0;
  for (auto& r : g_recs) {
    if (r.kind != kind) continue;
    RM_HIP(hipEventSynchronize(r.b));
    float e = 0.f;
    RM_HIP(hipEventElapsedTime(&e, r.a, r.b));
    n += r.launches;
    t += e;
    f += r.flops;
    b += r.bytes;
  }
  *launches = n;
  *ms = t;
  *flops = f;
  *bytes = b;
}

namespace {

constexpr int CB = 64;   // Cholesky block

__device__ __forceinline__ double block_sum(double v, double* sh) {
  // 256-thread deterministic sum (tree in LDS)
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- GEMV
// y = alpha A x + beta y: 64 rows x 4 column groups per workgroup.
__global__ __launch_bounds__(256) void gemv_n_kernel(int m, int n, double alpha, const double* A,
                                                     long lda, long sA, const double* x, long sx,
                                                     double beta, double* y, long sy) {
  __shared__ double sh[4][64];
  const int b = blockIdx.y;
  A += (long)b * sA; x += (long)b * sx; y += (long)b * sy;
  const int r = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + r;
  double s = 0;
  if (i < m) {
#pragma unroll 8
    for (int j = g; j < n; j += 4) s += A[i + (long)j * lda] * x[j];
  }
  sh[g][r] = s;
  __syncthreads();
  if (g == 0 && i < m) {
    double t = sh[0][r] + sh[1][r] + sh[2][r] + sh[3][r];
    y[i] = alpha * t + (beta != 0.0 ? beta * y[i] : 0.0);
  }
}

// y = alpha A x + beta y with the columns split over gridDim.y chunks:
// each thread owns a row of a 256-row block and sums its column chunk;
// partials are reduced in a fixed order by gemv_reduce_kernel.
__global__ __launch_bounds__(256) void gemv_n_split_kernel(int m, int n, const double* A, long lda,
                                                           const double* x, int chunk,
                                                           double* part) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * chunk, c1 = min(n, c0 + chunk);
  if (i >= m) return;
  double s = 0.0;
#pragma unroll 8
  for (int j = c0; j < c1; ++j) s += A[i + (long)j * lda] * x[j];
  part[(long)blockIdx.y * m + i] = s;
}

__global__ void gemv_reduce_kernel(int m, int nsplit, const double* part, double alpha,
                                   double beta, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
#pragma unroll 8
  for (int c = 0; c < nsplit; ++c) s += part[(long)c * m + i];
  y[i] = alpha * s + (beta != 0.0 ? beta * y[i] : 0.0);
}

// y = alpha A' x + beta y: one wave per output column.
__global__ __launch_bounds__(256) void gemv_t_kernel(int m, int n, double alpha, const double* A,
                                                     long lda, long sA, const double* x, long sx,
                                                     double beta, double* y, long sy) {
  const int b = blockIdx.y;
  A += (long)b * sA; x += (long)b * sx; y += (long)b * sy;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  double s = 0;
#pragma unroll 8
  for (int i = lane; i < m; i += 64) s += A[i + (long)j * lda] * x[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) y[j] = alpha * s + (beta != 0.0 ? beta * y[j] : 0.0);
}

// ---------------------------------------------------------------- multi-dot
// out[b] = sum_ij A(i, j) B_b(i, j) for up to MD_MAX matrices B_b.  One
// workgroup per column j; its 256 threads stride over the rows, so every
// load is coalesced and a launch holds n workgroups (several per CU, enough
// loads in flight to stream the nb + 1 matrices from HBM).  Each wave sums
// its lanes with a shuffle tree and writes one partial per matrix:
// part[(4 j + wave) * nb + b].
constexpr int MD_MAX = 32;
constexpr int MD_WAVES = 4;
__global__ __launch_bounds__(256) void multi_dot_kernel(int m, const double* A, long lda,
                                                        const double* B, long ldb, long sB,
                                                        int nb, double* part) {
  double acc[MD_MAX];
#pragma unroll
  for (int b = 0; b < MD_MAX; ++b) acc[b] = 0;
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double a = A[i + (long)j * lda];
#pragma unroll
    for (int b = 0; b < MD_MAX; ++b)
      if (b < nb) acc[b] += a * B[(long)b * sB + i + (long)j * ldb];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double mine = 0;
#pragma unroll
  for (int b = 0; b < MD_MAX; ++b) {
    if (b < nb) {
      double s = acc[b];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == b) mine = s;
    }
  }
  if (lane < nb) part[((long)j * MD_WAVES + wave) * nb + lane] = mine;
}

// out[b] = sum over the partials of matrix b.  One wave per matrix: lanes
// take every 64th partial and a shuffle tree adds the lane sums, so the
// order is fixed and the result deterministic.
__global__ __launch_bounds__(64) void reduce_parts_kernel(int nparts, int nb, const double* part,
                                                          double* out) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0;
#pragma unroll 8
  for (int p = lane; p < nparts; p += 64) s += part[(long)p * nb + b];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[b] = s;
}

// Panel of the blocked Cholesky factorisation: P = B L_kk^-T for the rows
// below the diagonal block, i.e. the triangular solve X L_kk' = B, in place,
// by forward substitution, which is backward stable; multiplying B by the
// explicit inverse of L_kk instead loses accuracy in proportion to cond(L_kk)
// (measured 13x on a 1024-point kernel matrix with jitter 1e-6).  One lane
// per row: x_c = (b_c - sum_{j<c} x_j L_kk[c][j]) / L_kk[c][c] over four
// interleaved partial sums, x in registers, L_kk and the reciprocals of its
// diagonal in LDS (every lane reads the same entry).  Measured at D = 1038:
// 22.6 us a launch; one wave per workgroup (49.7 us), a column-oriented
// update (33.1 us), scalar loads of L_kk (114 us) and eight lanes per row
// with a shuffle reduction (27.8 us) were all slower.
__global__ __launch_bounds__(256) void trsm_panel_kernel(int n, int k0, int bw, int r0,
                                                         double* __restrict__ L) {
  __shared__ double sL[CB * CB];   // sL[c * CB + j] = L_kk[c][j], row c
  __shared__ double rd[CB];
  const double* Dk = L + k0 + (long)k0 * n;
  for (int e = threadIdx.x; e < CB * CB; e += blockDim.x) {
    const int r = e / CB, c = e % CB;
    sL[e] = (r < bw && c <= r) ? Dk[r + (long)c * n] : 0.0;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < CB; c += blockDim.x) rd[c] = c < bw ? 1.0 / sL[c * CB + c] : 0.0;
  __syncthreads();
  const int row = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double* B = L + row + (long)k0 * n;   // element c of this row at B[c * n]
  double x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = c < bw ? B[(long)c * n] : 0.0;
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    if (c < bw) {
      const double* Lc = sL + c * CB;
      double s0 = x[c], s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int j = 0;
#pragma unroll
      for (; j + 3 < c; j += 4) {
        s0 -= Lc[j] * x[j];
        s1 -= Lc[j + 1] * x[j + 1];
        s2 -= Lc[j + 2] * x[j + 2];
        s3 -= Lc[j + 3] * x[j + 3];
      }
#pragma unroll
      for (; j < c; ++j) s0 -= Lc[j] * x[j];
      x[c] = ((s0 + s1) + (s2 + s3)) * rd[c];
    }
  }
#pragma unroll
  for (int c = 0; c < CB; ++c)
    if (c < bw) B[(long)c * n] = x[c];
}

// ---------------------------------------------------------------- Cholesky
// Factor one CB x CB diagonal block in one workgroup (right-looking,
// unscaled columns): thread (row i = lane, wave g) keeps S[i][k] for
// k = g + 4m in registers.  At step j the wave owning column j publishes it
// to LDS (double-buffered, one barrier per column) and every thread applies
// S_ik -= (S_ij / d_j) S_kj to its k > j.  Then L_ij = S_ij / sqrt(d_j),
// L_jj = sqrt(d_j).  Padding rows/columns of a partial block start as the
// identity, so they factor trivially.  The inverse of the triangle is not
// needed until the factorisation is complete and is formed afterwards for
// every diagonal block at once (trtri_diag_kernel), off this chain.
// (The block comes from registers: potrf_block is shared with the fused
// trailing update below, which factors the next diagonal block in place.)
// All 256 threads call it; sv[m] = S[i][g + 4m] on entry, only the lower
// triangle of S is used.
__device__ __forceinline__ void potrf_block(int n, int k0, double (&sv)[CB / 4], double* L,
                                            long ldl, double* diagLogs, int* info) {
  constexpr int NM = CB / 4;
  __shared__ double col[2][CB];
  __shared__ double dg[CB];
  const int w = min(CB, n - k0);
  const int tid = threadIdx.x;
  const int i = tid & (CB - 1);
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  __builtin_assume(g >= 0 && g < 4);
  bool bad = false;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int b = j & 1;
    if (g == (j & 3)) col[b][i] = sv[j >> 2];
    __syncthreads();
    const double d = col[b][j];
    bad = bad || !(d > 0.0);
    if (tid == 0) dg[j] = d;
    const double f = col[b][i] * (1.0 / d);
#pragma unroll
    for (int m = 0; m < NM; ++m)
      if (g + 4 * m > j) sv[m] -= f * col[b][g + 4 * m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int k = g + 4 * m;
    if (i < w && k < w) {
      const double dk = dg[k];
      L[(k0 + i) + (long)(k0 + k) * ldl] = i > k ? sv[m] * rsqrt(dk) : (i == k ? sqrt(dk) : 0.0);
    }
  }
  if (tid < w) diagLogs[k0 + tid] = 0.5 * log(dg[tid]);
  if (tid == 0 && bad) *info = k0 + 1;
}

__global__ __launch_bounds__(256) void potrf_diag_kernel(int n, int k0, double* L, long ldl,
                                                         double* diagLogs, int* info) {
  constexpr int NM = CB / 4;
  const int w = min(CB, n - k0);
  const int i = threadIdx.x & (CB - 1);
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double sv[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int k = g + 4 * m;
    sv[m] = (i < w && k < w) ? L[(k0 + i) + (long)(k0 + k) * ldl] : (i == k ? 1.0 : 0.0);
  }
  potrf_block(n, k0, sv, L, ldl, diagLogs, info);
}

// Trailing update of the blocked Cholesky after the panel of block k0:
// S[r0:, r0:] -= P P' (P = L[r0:, k0:k0+CB], solved), lower 64 x 64 tiles
// only (the upper triangle of L is cleared at the end), one workgroup per
// tile (I >= J) on v_mfma_f64_16x16x4f64 (a 32 x 32 quadrant per wave, both
// 64 x 64 panel pieces in LDS).  Workgroup 0 owns the next diagonal block:
// it keeps its updated tile on chip and factors it at once (potrf_block),
// so the factorisation of block r0 needs no launch of its own.
__global__ __launch_bounds__(256) void chol_update_kernel(int n, int k0, double* L,
                                                          double* diagLogs, int* info) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int PAD = 4;
  __shared__ double Ps[2][CB][CB + PAD];   // Ps[0][k][m] = P[64 I + m][k], Ps[1]: P_J
  const int r0 = k0 + CB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // tile (I, J), I >= J, from the workgroup index b = I (I + 1) / 2 + J
  const int b = blockIdx.x;
  int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= b) ++I;
  while (I * (I + 1) / 2 > b) --I;
  const int J = b - I * (I + 1) / 2;
  const int ri = r0 + CB * I, rj = r0 + CB * J;
  // P pieces: rows ri.. and rj.., columns k0..k0+63 (coalesced down columns)
  for (int e = tid; e < CB * CB; e += 256) {
    const int m = e % CB, k = e / CB;
    const double* Pc = L + (long)(k0 + k) * n;
    Ps[0][k][m] = ri + m < n ? Pc[ri + m] : 0.0;
    Ps[1][k][m] = rj + m < n ? Pc[rj + m] : 0.0;
  }
  __syncthreads();
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = d4{0, 0, 0, 0};
#pragma unroll 4
  for (int kq = 0; kq < CB / 4; ++kq) {
    const int kr = 4 * kq + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      av[t] = Ps[0][kr][wm * 32 + t * 16 + (lane & 15)];
      bv[t] = Ps[1][kr][wn * 32 + t * 16 + (lane & 15)];
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[tj], av[ti], acc[ti][tj], 0, 0, 0);
  }
  // acc[ti][tj][r] = (P_I P_J')(m, c), m = wm 32 + ti 16 + lane % 16,
  // c = wn 32 + tj 16 + lane / 16 + 4 r
  if (b != 0) {
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = ri + wm * 32 + ti * 16 + (lane & 15);
          const int gc = rj + wn * 32 + tj * 16 + (lane >> 4) + 4 * r;
          if (gm < n && gc < n) L[gm + (long)gc * n] -= acc[ti][tj][r];
        }
    return;
  }
  // workgroup 0: the next diagonal block, updated on chip, then factored
  double (*S)[CB + PAD] = Ps[0];
  __syncthreads();   // every wave is done reading Ps
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = wm * 32 + ti * 16 + (lane & 15);
        const int c = wn * 32 + tj * 16 + (lane >> 4) + 4 * r;
        const double v = (r0 + m < n && r0 + c < n) ? L[(r0 + m) + (long)(r0 + c) * n] : 0.0;
        S[m][c] = v - acc[ti][tj][r];
      }
  __syncthreads();
  constexpr int NM = CB / 4;
  const int w = min(CB, n - r0);
  const int i = tid & (CB - 1);
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  double sv[NM];
#pragma unroll
  for (int m = 0; m < NM; ++m) {
    const int k = g + 4 * m;
    sv[m] = (i < w && k < w) ? S[i][k] : (i == k ? 1.0 : 0.0);
  }
  potrf_block(n, r0, sv, L, (long)n, diagLogs, info);
}

// Inverse of every diagonal block's triangle (one workgroup per block):
// wave 0, one lane per column c, right-looking forward substitution: once
// X[r][c] is final (scaled by 1/L[r][r]) it is removed from every later row,
// a[i] -= L[i][r] X[r][c], so the updates of a step are independent of each
// other.  a stays in registers; L is read from LDS at the same address in
// every lane.
__global__ __launch_bounds__(256) void trtri_diag_kernel(int n, const double* __restrict__ L,
                                                         long ldl, double* __restrict__ Linv) {
  __shared__ double Ls[CB][CB + 1];
  __shared__ double Xs[CB][CB + 1];
  __shared__ double rl[CB];   // 1 / L[k][k]
  const int k0 = blockIdx.x * CB;
  const int w = min(CB, n - k0);
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += 256) {
    const int r = e % CB, c = e / CB;
    Ls[r][c] = (r < w && c < w) ? (r >= c ? L[(k0 + r) + (long)(k0 + c) * ldl] : 0.0)
                                : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < CB) rl[tid] = 1.0 / Ls[tid][tid];
  __syncthreads();
  if (tid < CB) {
    const int c = tid;
    double a[CB];
#pragma unroll
    for (int r = 0; r < CB; ++r) a[r] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int r = 0; r < CB; ++r) {
      a[r] *= rl[r];
#pragma unroll
      for (int i = r + 1; i < CB; ++i) a[i] -= Ls[i][r] * a[r];
    }
#pragma unroll
    for (int r = 0; r < CB; ++r) Xs[r][c] = a[r];
  }
  __syncthreads();
  for (int e = tid; e < CB * CB; e += 256) {
    const int r = e % CB, c = e / CB;
    if (r < w && c < w) Linv[(k0 + r) + (long)(k0 + c) * ldl] = Xs[r][c];
  }
}

__global__ void zero_upper_kernel(int n, double* A, long lda) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  if (j > i) A[i + (long)j * lda] = 0.0;
}

__global__ void fill_kernel(double* x, long n, double v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void fill_int_kernel(int* x, long n, int v) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void copy_kernel(double* d, const double* s, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}
__global__ void axpby_kernel(long n, double a, const double* x, double b, double* y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
__global__ void lincomb3_kernel(long n, const double* base, double c1, const double* x, double c2,
                                const double* y, double* dst) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = base[i] + c1 * x[i] + c2 * y[i];
}
__global__ void symmetrize_kernel(int n, double* A, long lda) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  if (i > j) {
    const double v = 0.5 * (A[i + (long)j * lda] + A[j + (long)i * lda]);
    A[i + (long)j * lda] = v;
    A[j + (long)i * lda] = v;
  }
}
__global__ __launch_bounds__(256) void vsum_kernel(long n, const double* x, const double* y,
                                                   double* out) {
  __shared__ double sh[256];
  double s = 0;
  for (long i = threadIdx.x; i < n; i += 256) s += y ? x[i] * y[i] : x[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = s;
}
__global__ void set_identity_kernel(int n, double* A, long lda) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int i = (int)(e % n), j = (int)(e / n);
  A[i + (long)j * lda] = (i == j) ? 1.0 : 0.0;
}
__global__ void copy_matrix_kernel(int m, int n, const double* A, long lda, double* B, long ldb) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  B[i + (long)j * ldb] = A[i + (long)j * lda];
}
__global__ void cast_kernel(long n, const double* x, float* y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ void widen_kernel(long n, const float* x, double* y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

}  // namespace

void gemv_split(int m, int n, double alpha, const double* A, long lda, const double* x,
                double beta, double* y, double* work, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  const int nsplit = std::max(1, std::min(64, n / 16));
  const int chunk = cdiv(n, nsplit);
  hipLaunchKernelGGL(gemv_n_split_kernel, dim3(cdiv(m, 256), nsplit), dim3(256), 0, st, m, n, A,
                     lda, x, chunk, work);
  RM_CHECK_LAUNCH();
  hipLaunchKernelGGL(gemv_reduce_kernel, dim3(cdiv(m, 256)), dim3(256), 0, st, m, nsplit,
                     (const double*)work, alpha, beta, y);
  RM_CHECK_LAUNCH();
}

void gemv(int m, int n, double alpha, const double* A, long lda, bool tA, long sA,
          const double* x, long sx, double beta, double* y, long sy, int batch, hipStream_t st) {
  if (m <= 0 || n <= 0 || batch <= 0) return;
  if (!tA)
    hipLaunchKernelGGL(gemv_n_kernel, dim3(cdiv(m, 64), batch), dim3(256), 0, st, m, n, alpha, A,
                       lda, sA, x, sx, beta, y, sy);
  else
    hipLaunchKernelGGL(gemv_t_kernel, dim3(cdiv(n, 4), batch), dim3(256), 0, st, m, n, alpha, A,
                       lda, sA, x, sx, beta, y, sy);
  RM_CHECK_LAUNCH();
}

void multi_dot(int m, int n, const double* A, long lda, const double* B, long ldb, long sB,
               int nb, double* out, double* work, hipStream_t st) {
  if (nb <= 0) return;
  RM_REQUIRE(nb <= MD_MAX, "multi_dot: too many matrices");
  if (m <= 0 || n <= 0) {
    fill(out, nb, 0.0, st);
    return;
  }
  hipLaunchKernelGGL(multi_dot_kernel, dim3(n), dim3(256), 0, st, m, A, lda, B, ldb, sB, nb, work);
  RM_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(nb), dim3(64), 0, st, n * MD_WAVES, nb,
                     (const double*)work, out);
  RM_CHECK_LAUNCH();
}

void chol_inverse(int n, const double* K, double* Kinv, double* logdet, CholWork& w,
                  double* redwork, hipStream_t st) {
  const long nn = (long)n * n;
  copy(w.L, K, nn, st);
  fill(w.Linv, nn, 0.0, st);
  fill_int(w.info, 1, 0, st);
  const int nb = cdiv(n, CB);
  // block 0 on its own; every later diagonal block is factored by the
  // trailing update that precedes it (chol_update_kernel, workgroup 0)
  hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, n, 0, w.L, (long)n, w.diagLogs,
                     w.info);
  RM_CHECK_LAUNCH();
  for (int kb = 0; kb + 1 < nb; ++kb) {
    const int k0 = kb * CB, r0 = k0 + CB, rm = n - r0;
    // panel: L[r0:, k0:k0+CB] <- L[r0:, k0:k0+CB] L_kk^-T by substitution
    hipLaunchKernelGGL(trsm_panel_kernel, dim3(cdiv(rm, 256)), dim3(256), 0, st, n, k0, CB, r0,
                       w.L);
    RM_CHECK_LAUNCH();
    // trailing: L[r0:, r0:] -= P P' (lower tiles), then block r0 factored
    const int T = cdiv(rm, CB);
    hipLaunchKernelGGL(chol_update_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, st, n, k0, w.L,
                       w.diagLogs, w.info);
    RM_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(zero_upper_kernel, dim3(cdiv(nn, 256)), dim3(256), 0, st, n, w.L, (long)n);
  RM_CHECK_LAUNCH();
  hipLaunchKernelGGL(trtri_diag_kernel, dim3(nb), dim3(256), 0, st, n, (const double*)w.L, (long)n,
                     w.Linv);
  RM_CHECK_LAUNCH();
  // Linv by doubling: for two inverted diagonal blocks X11 = L11^-1 (s x s)
  // and X22 = L22^-1 (s2 x s2, s2 <= s) of [L11 0; L21 L22], the block below
  // X11 is X21 = -X22 (L21 X11).  Level s pairs the blocks starting at
  // multiples of 2s; those pairs are independent and lie at a constant
  // stride 2s(n + 1) along the diagonal, so each level is two batched
  // products (plus a ragged last pair when n is not a power-of-two multiple
  // of CB).
  // the upper levels have few output tiles and a long k: split k so that
  // about 256 workgroups run (partials in w.split, which holds at least
  // GSPLIT_MAX n^2 doubles when present)
  auto level_splits = [&](int m, int nn, int k, int batch) {
    if (!w.split) return 1;
    const long tiles = (long)cdiv(m, 64) * cdiv(nn, 64) * batch;
    int sp = (int)std::max(1L, std::min(8L, 256 / std::max(tiles, 1L)));
    while (sp > 1 && (long)k < 2L * 16 * sp) --sp;
    return sp;
  };
  for (int s = CB; s < n; s *= 2) {
    const int full = n / (2 * s);                  // pairs with s2 = s
    const long stride = 2L * s * (n + 1);
    auto level = [&](int b0, int s2, int batch) {
      const long off21 = (b0 + s) + (long)b0 * n;
      Gemm<double> a;                                // T = L21 X11
      a.m = s2; a.n = s; a.k = s;
      a.A = w.L + off21; a.lda = n; a.sA = stride;
      a.B = w.Linv + b0 + (long)b0 * n; a.ldb = n; a.sB = stride;
      a.C = w.tmp + off21; a.ldc = n; a.sC = stride;
      a.batch = batch;
      gemm_splitk(a, w.split, level_splits(s2, s, s, batch), st);
      Gemm<double> b;                                // X21 = -X22 T
      b.m = s2; b.n = s; b.k = s2; b.alpha = -1.0;
      b.A = w.Linv + (b0 + s) + (long)(b0 + s) * n; b.lda = n; b.sA = stride;
      b.B = w.tmp + off21; b.ldb = n; b.sB = stride;
      b.C = w.Linv + off21; b.ldc = n; b.sC = stride;
      b.batch = batch;
      gemm_splitk(b, w.split, level_splits(s2, s, s2, batch), st);
    };
    if (full > 0) level(0, s, full);
    const int b0 = full * 2 * s;
    if (b0 + s < n) level(b0, n - b0 - s, 1);
  }
  // K^-1 = Linv' Linv
  Gemm<double> c;
  c.m = n; c.n = n; c.k = n;
  c.A = w.Linv; c.lda = n; c.tA = true;
  c.B = w.Linv; c.ldb = n;
  c.C = Kinv; c.ldc = n;
  gemm_splitk(c, w.split, w.nsplit, st);
  symmetrize(n, Kinv, n, st);
  vsum(n, w.diagLogs, logdet, st);
  axpby(1, 0.0, logdet, 2.0, logdet, st);  // log|K| = 2 sum log L_ii
  (void)redwork;
}

void fill(double* x, long n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, x, n, v);
  RM_CHECK_LAUNCH();
}
void fill_int(int* x, long n, int v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_int_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, x, n, v);
  RM_CHECK_LAUNCH();
}
void copy(double* dst, const double* src, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, dst, src, n);
  RM_CHECK_LAUNCH();
}
void axpby(long n, double a, const double* x, double b, double* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, a, x, b, y);
  RM_CHECK_LAUNCH();
}
void lincomb3(long n, const double* base, double c1, const double* x, double c2, const double* y,
              double* dst, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(lincomb3_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, base, c1, x, c2, y,
                     dst);
  RM_CHECK_LAUNCH();
}
void symmetrize(int n, double* A, long lda, hipStream_t st) {
  const long nn = (long)n * n;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(cdiv(nn, 256)), dim3(256), 0, st, n, A, lda);
  RM_CHECK_LAUNCH();
}
void vsum(long n, const double* x, double* out, hipStream_t st) {
  hipLaunchKernelGGL(vsum_kernel, dim3(1), dim3(256), 0, st, n, x, (const double*)nullptr, out);
  RM_CHECK_LAUNCH();
}
void vdot(long n, const double* x, const double* y, double* out, hipStream_t st) {
  hipLaunchKernelGGL(vsum_kernel, dim3(1), dim3(256), 0, st, n, x, y, out);
  RM_CHECK_LAUNCH();
}
void set_identity(int n, double* A, long lda, hipStream_t st) {
  const long nn = (long)n * n;
  hipLaunchKernelGGL(set_identity_kernel, dim3(cdiv(nn, 256)), dim3(256), 0, st, n, A, lda);
  RM_CHECK_LAUNCH();
}
void copy_matrix(int m, int n, const double* A, long lda, double* B, long ldb, hipStream_t st) {
  const long mn = (long)m * n;
  if (mn <= 0) return;
  hipLaunchKernelGGL(copy_matrix_kernel, dim3(cdiv(mn, 256)), dim3(256), 0, st, m, n, A, lda, B,
                     ldb);
  RM_CHECK_LAUNCH();
}
void cast_to_float(long n, const double* x, float* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cast_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, x, y);
  RM_CHECK_LAUNCH();
}
void widen_to_double(long n, const float* x, double* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(widen_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, x, y);
  RM_CHECK_LAUNCH();
}

}  // namespace rmhmc
