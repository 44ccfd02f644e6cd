// Shared declarations of the librmhmc device code (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/rmhmc.h"

namespace rmhmc {

// Error carried from deep inside the library to the ABI boundary, where it
// becomes an rmhmc_status and a thread-local message.
struct Error : std::runtime_error {
  rmhmc_status status;
  Error(rmhmc_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

#define RM_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::rmhmc::Error(RMHMC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define RM_CHECK_LAUNCH() RM_HIP(hipGetLastError())

#define RM_REQUIRE(cond, msg)                                           \
  do {                                                                  \
    if (!(cond)) throw ::rmhmc::Error(RMHMC_E_ARG, msg);                \
  } while (0)

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ live kernel timing
// Off by default.  When on, instrumented launch sites bracket the launch with
// HIP events on the launch stream and record the algorithmic flops / bytes
// of that launch; rmhmc_timing_read() sums them per kernel family.
enum TimerKind {
  TK_GEMM_F64 = 0, TK_GEMM_F32, TK_JACOBI_DYNAMIC, TK_JACOBI_STATIC, TK_KD_WSUM, TK_KD_MATVEC,
  TK_POTRF, TK_COUNT
};
bool timing_enabled();
int timing_begin(int kind, hipStream_t st);
// flops and bytes are the algorithmic work of everything between begin and
// end, which may be several back-to-back launches of one kernel family
void timing_end(int slot, hipStream_t st, double flops, double bytes, long long launches = 1);

// ------------------------------------------------------------------ GEMM
// C = alpha * op(A) op(B) + beta * C, column-major.  op(A) is m x k, op(B)
// is k x n.  Batches use strides or per-batch pointer arrays (device
// arrays; when given they override base + stride).  If C2 is set, the same
// result is also stored transposed (C2[j + i*ldc2]).
template <typename T>
struct Gemm {
  int m = 0, n = 0, k = 0;
  T alpha = 1, beta = 0;
  const T* A = nullptr; long lda = 0; bool tA = false; long sA = 0;
  const T* B = nullptr; long ldb = 0; bool tB = false; long sB = 0;
  T* C = nullptr; long ldc = 0; long sC = 0;
  T* C2 = nullptr; long ldc2 = 0; long sC2 = 0;
  int batch = 1;
  const T* const* Ap = nullptr;
  const T* const* Bp = nullptr;
  T* const* Cp = nullptr;
  T* const* C2p = nullptr;
  // Copies of the result in the other precision (float for a double GEMM,
  // double for a float one), written by the same epilogue: Co in C's layout
  // (ldc, stride sCo), C2o transposed (ldc2, stride sC2o).
  void* Co = nullptr; long sCo = 0;
  void* C2o = nullptr; long sC2o = 0;
  // pointer-array batches: Co per batch item (C's layout, ldc)
  void* const* Cop = nullptr;
};

void gemm(const Gemm<double>& g, hipStream_t st);
void gemm(const Gemm<float>& g, hipStream_t st);

// C (m x n) = op(A)' B over a very long inner dimension k, split across
// workgroups and summed in a fixed order (deterministic).  A is k x m (lda),
// B is k x n (ldb), both column-major.  `work` must hold splits*m*n values.
// A plain product C = alpha op(A) op(B) (beta 0, C only; a strided batch
// allowed) with its k range split over `splits` layers; `work` holds
// batch * splits * m * n doubles.  Anything else goes to gemm().
void gemm_splitk(const Gemm<double>& g, double* work, int splits, hipStream_t st);
void gemm_tallk(int m, int n, long k, const double* A, long lda, const double* B, long ldb,
                double* C, long ldc, double* work, int splits, hipStream_t st);
void gemm_tallk(int m, int n, long k, const float* A, long lda, const float* B, long ldb,
                double* C, long ldc, double* work, int splits, hipStream_t st);
int tallk_splits(long k);

// ------------------------------------------------------------------ misc linear algebra
// y_b = alpha * op(A_b) x_b + beta * y_b for b < batch (A_b = A + b*sA, x_b = x + b*sx, ...).
void gemv(int m, int n, double alpha, const double* A, long lda, bool tA, long sA,
          const double* x, long sx, double beta, double* y, long sy, int batch, hipStream_t st);

// y = alpha A x + beta y for one well-parallelised GEMV: columns split over
// workgroups, partials (<= 64 m) in `work`, reduced in a fixed order.
void gemv_split(int m, int n, double alpha, const double* A, long lda, const double* x,
                double beta, double* y, double* work, hipStream_t st);

// out[b] = sum_ij A(i,j) * B_b(i,j) for an m x n A (lda) and B_b = B + b*sB (ldb).
// `work` holds multi_dot_work(n) doubles; nb <= 32.
inline long multi_dot_work(long n) { return n * 4 * 32; }
void multi_dot(int m, int n, const double* A, long lda, const double* B, long ldb, long sB,
               int nb, double* out, double* work, hipStream_t st);

// Cholesky K = L L' (lower, in place on a copy), log|K|, L^-1 and K^-1.
// `info` (device int) is set to a positive value if K is not positive definite.
struct CholWork {
  double* L = nullptr;      // n x n
  double* Linv = nullptr;   // n x n
  double* tmp = nullptr;    // n x n
  double* diagLogs = nullptr;  // n
  int* info = nullptr;
  double* split = nullptr;  // optional: nsplit * n * n partials for K^-1 = Linv' Linv
  int nsplit = 0;
};
void chol_inverse(int n, const double* K, double* Kinv, double* logdet, CholWork& w,
                  double* redwork, hipStream_t st);

void fill(double* x, long n, double v, hipStream_t st);
void fill_int(int* x, long n, int v, hipStream_t st);
void copy(double* dst, const double* src, long n, hipStream_t st);
// y = a*x + b*y (vectors)
void axpby(long n, double a, const double* x, double b, double* y, hipStream_t st);
// dst = x + c*(y + z) style updates used by the integrator: dst = base + c1*x + c2*y
void lincomb3(long n, const double* base, double c1, const double* x, double c2, const double* y,
              double* dst, hipStream_t st);
// 0.5*(A + A') in place for an n x n matrix
void symmetrize(int n, double* A, long lda, hipStream_t st);
// sum of x (length n) into out[0] (deterministic, single workgroup)
void vsum(long n, const double* x, double* out, hipStream_t st);
// out[0] = sum x_i * y_i
void vdot(long n, const double* x, const double* y, double* out, hipStream_t st);
void set_identity(int n, double* A, long lda, hipStream_t st);
void copy_matrix(int m, int n, const double* A, long lda, double* B, long ldb, hipStream_t st);
void cast_to_float(long n, const double* x, float* y, hipStream_t st);
void widen_to_double(long n, const float* x, double* y, hipStream_t st);

}  // namespace rmhmc
