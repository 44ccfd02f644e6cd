// Dense GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64 and
// v_mfma_f32_16x16x4f32), column-major, with strided / pointer-array
// batches and split-K for the very tall inner products used by the
// trace terms.
//
// Tiling: 256 threads (4 wave64), a 64x64 output tile per workgroup, each
// wave owns a 32x32 quadrant = 2x2 MFMA tiles of 16x16; k advances 16 per
// LDS stage with register double-buffering of the next stage.  The MFMA
// "row" operand is fed from the B tile and the "column" operand from the A
// tile, so each lane's accumulators hold consecutive rows m of C and the
// column-major stores coalesce.
#include "common.h"

namespace rmhmc {
namespace {

constexpr int BK = 16, PADL = 4;

template <typename T> struct Mfma;
// Accumulator layout of a 16x16 output tile: lane l, register r holds
// D[row(l, r)][l % 16].  The FP32 instruction keeps four consecutive rows
// per lane; the FP64 one interleaves them (row = l/16 + 4r).
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T> struct OtherPrec;
template <> struct OtherPrec<double> { typedef float type; };
template <> struct OtherPrec<float> { typedef double type; };

template <typename T>
struct Params {
  typedef typename OtherPrec<T>::type OT;
  OT* Co; long sCo;     // result in the other precision, C's layout
  OT* C2o; long sC2o;   // and transposed (ldc2)
  int m, n, k;
  T alpha, beta;
  const T* A; long lda; long sA;
  const T* B; long ldb; long sB;
  T* C; long ldc; long sC;
  T* C2; long ldc2; long sC2;
  const T* const* Ap; const T* const* Bp; T* const* Cp; T* const* C2p;
  OT* const* Cop;       // per batch item: Co (pointer-array batches)
  int ksplit; long kchunk;
  T* part;          // split-K partials: part[kc * m * n + i + j * m]
};

// BT: the output tile (BT x BT per workgroup, a BT/2 x BT/2 quadrant per
// wave = (BT/32)^2 MFMA tiles).  BT = 128 halves the operand traffic per
// flop of BT = 64 and doubles the MFMAs per LDS read; it needs about twice
// the registers and LDS, so it serves large outputs, where the grid still
// fills the chip.
template <typename T, bool TA, bool TB, int BT>
__global__ __launch_bounds__(256) void gemm_kernel(Params<T> p) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int TW = BT / 32;            // MFMA tiles per wave and dimension
  constexpr int LPT = BT * BK / 256;     // operand elements a thread stages per stage
  constexpr int LG = BT == 64 ? 6 : 7;   // log2(BT)
  const int bz = blockIdx.z;
  const int batch = bz / p.ksplit, kc = bz % p.ksplit;
  const T* __restrict__ A = p.Ap ? p.Ap[batch] : p.A + (long)batch * p.sA;
  const T* __restrict__ B = p.Bp ? p.Bp[batch] : p.B + (long)batch * p.sB;
  const long kbeg = (long)kc * p.kchunk;
  const long kend = min((long)p.k, kbeg + p.kchunk);
  // XCD-aware tile order.  Workgroups are handed to the eight XCDs in
  // turn, so workgroup ids j, j + 8, j + 16, ... of a batch item share an
  // XCD and its L2.  Those ids get one compact block of tiles (a quarter of
  // the row bands times half of the column bands) instead of two row bands
  // against every column band, so each XCD streams less of A and B.  The
  // map is a bijection whenever gx % 4 == 0 and gy % 2 == 0 (then gx * gy is
  // a multiple of 8); other grids keep the plain order.
  int bx = blockIdx.x, by = blockIdx.y;
  {
    const int gx = gridDim.x, gy = gridDim.y;
    if (gx % 4 == 0 && gy % 2 == 0) {
      const int lin = blockIdx.x + gx * blockIdx.y;
      const int j = lin % 8, k = lin / 8;
      const int rw = gx / 4, cw = gy / 2;
      bx = (j % 4) * rw + k % rw;
      by = (j / 4) * cw + k / rw;
    }
  }
  const int m0 = bx * BT, n0 = by * BT;
  const int M = p.m, N = p.n;
  const long lda = p.lda, ldb = p.ldb;

  __shared__ T As[2][BK][BT + PADL];
  __shared__ T Bs[2][BK][BT + PADL];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  v4 acc[TW][TW];
#pragma unroll
  for (int a = 0; a < TW; ++a)
#pragma unroll
    for (int b = 0; b < TW; ++b) acc[a][b] = v4{0, 0, 0, 0};

  // staging map: k-major operands (A', B) by 16-long k columns, the others
  // by BT-long m / n rows, LPT elements a thread
  auto mapA = [&](int r, int& ml, int& kl) {
    if (!TA) { ml = tid & (BT - 1); kl = (tid >> LG) + (256 >> LG) * r; }
    else     { kl = tid & 15; ml = (tid >> 4) + 16 * r; }
  };
  auto mapB = [&](int r, int& nl, int& kl) {
    if (!TB) { kl = tid & 15; nl = (tid >> 4) + 16 * r; }
    else     { nl = tid & (BT - 1); kl = (tid >> LG) + (256 >> LG) * r; }
  };
  T ra[LPT], rb[LPT];
  auto loadA = [&](long k0) {
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      int ml, kl;
      mapA(r, ml, kl);
      const long gm = m0 + ml, gk = k0 + kl;
      T v = 0;
      if (gm < M && gk < kend) v = TA ? A[gk + gm * lda] : A[gm + gk * lda];
      ra[r] = v;
    }
  };
  auto loadB = [&](long k0) {
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      int nl, kl;
      mapB(r, nl, kl);
      const long gn = n0 + nl, gk = k0 + kl;
      T v = 0;
      if (gn < N && gk < kend) v = TB ? B[gn + gk * ldb] : B[gk + gn * ldb];
      rb[r] = v;
    }
  };
  auto storeAB = [&](int buf) {
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      int ml, kl, nl, kl2;
      mapA(r, ml, kl);
      As[buf][kl][ml] = ra[r];
      mapB(r, nl, kl2);
      Bs[buf][kl2][nl] = rb[r];
    }
  };

  if (kbeg < kend) {
    loadA(kbeg);
    loadB(kbeg);
    storeAB(0);
  }
  __syncthreads();
  int cur = 0;
  for (long k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) { loadA(k0 + BK); loadB(k0 + BK); }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = 4 * kk + (lane >> 4);
      T av[TW], bv[TW];
#pragma unroll
      for (int t = 0; t < TW; ++t) {
        av[t] = As[cur][kr][wm * (BT / 2) + t * 16 + (lane & 15)];
        bv[t] = Bs[cur][kr][wn * (BT / 2) + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int ti = 0; ti < TW; ++ti)
#pragma unroll
        for (int tj = 0; tj < TW; ++tj) acc[ti][tj] = Mfma<T>::op(bv[tj], av[ti], acc[ti][tj]);
    }
    if (more) storeAB(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  // Epilogue.  acc[ti][tj][r] = C(m, n) with m = mbase + lane%16,
  // n = nbase + row(lane, r) (the MFMA row index is our n).
  if (p.part) {
    T* part = p.part + ((long)batch * p.ksplit + kc) * M * N;
#pragma unroll
    for (int ti = 0; ti < TW; ++ti)
#pragma unroll
      for (int tj = 0; tj < TW; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gm = m0 + wm * (BT / 2) + ti * 16 + (lane & 15);
          const int gn = n0 + wn * (BT / 2) + tj * 16 + Mfma<T>::row(lane, r);
          if (gm < M && gn < N) part[gm + (long)gn * M] = acc[ti][tj][r];
        }
    return;
  }
  typedef typename OtherPrec<T>::type OT;
  T* C = p.Cp ? p.Cp[batch] : (p.C ? p.C + (long)batch * p.sC : nullptr);
  T* C2 = p.C2p ? p.C2p[batch] : (p.C2 ? p.C2 + (long)batch * p.sC2 : nullptr);
  OT* Co = p.Cop ? p.Cop[batch] : (p.Co ? p.Co + (long)batch * p.sCo : nullptr);
  OT* C2o = p.C2o ? p.C2o + (long)batch * p.sC2o : nullptr;
#pragma unroll
  for (int ti = 0; ti < TW; ++ti)
#pragma unroll
    for (int tj = 0; tj < TW; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * (BT / 2) + ti * 16 + (lane & 15);
        const int gn = n0 + wn * (BT / 2) + tj * 16 + Mfma<T>::row(lane, r);
        if (gm < M && gn < N) {
          T v = p.alpha * acc[ti][tj][r];
          if (C) {
            T* c = C + gm + (long)gn * p.ldc;
            if (p.beta != T(0)) v += p.beta * *c;
            *c = v;
          }
          if (C2) C2[gn + (long)gm * p.ldc2] = v;
          if (Co) Co[gm + (long)gn * p.ldc] = (OT)v;
          if (C2o) C2o[gn + (long)gm * p.ldc2] = (OT)v;
        }
      }
}

// C = sum over the split-K partials.  One wave per output element: its
// lanes take every 64th split and a shuffle tree adds the lane sums (a fixed
// order, so the result is deterministic).  With a few hundred outputs and
// hundreds of splits, a thread per output would leave the loads serial.
template <typename T>
__global__ __launch_bounds__(256) void splitk_reduce(int m, int n, int splits,
                                                     const T* __restrict__ part,
                                                     double* __restrict__ C, long ldc) {
  const long mn = (long)m * n;
  const long idx = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  double s = 0;
  if (idx < mn) {
#pragma unroll 4
    for (int kc = lane; kc < splits; kc += 64) s += (double)part[(long)kc * mn + idx];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0 && idx < mn) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    C[i + (long)j * ldc] = s;
  }
}

// Tall-k products with a small output (m <= 16, n <= 16 NT): partials of
// C = A' B over one k chunk per workgroup, for the traces of products of
// N x N matrices (k = N^2).  One 16 x 16 MFMA tile per 16 output columns, no
// LDS staging: lane l streams four consecutive k of operand row l mod 16
// (one 16- or 32-byte load), and the four MFMAs of a 16-long k step take one
// of those k each, so that each chunk of A and B is read once.  The waves
// take interleaved 16-long steps of the chunk; their sums are added in a
// fixed order (deterministic).  Partials as the tiled kernel's split-K:
// part[kc * m * n + i + j * m].
template <typename T, int NT>
__global__ __launch_bounds__(256) void tallk_small_kernel(int m, int n, long k,
                                                          const T* __restrict__ A, long lda,
                                                          const T* __restrict__ B, long ldb,
                                                          long kchunk, T* __restrict__ part) {
  typedef typename Mfma<T>::v4 v4;
  typedef T t4 __attribute__((ext_vector_type(4)));
  __shared__ v4 red[3][NT][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, q = lane >> 4;
  const long kbeg = (long)blockIdx.x * kchunk, kend = min(k, kbeg + kchunk);
  v4 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = v4{0, 0, 0, 0};
  const bool am = r16 < m;
  const T* Ar = A + (long)(am ? r16 : 0) * lda;
  const T* Br[NT];
  bool bn[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    bn[j] = 16 * j + r16 < n;
    Br[j] = B + (long)(bn[j] ? 16 * j + r16 : 0) * ldb;
  }
  long k0 = kbeg + 16L * wave;
  for (; k0 + 16 <= kend; k0 += 64) {
    const long kk = k0 + 4 * q;
    const t4 a = am ? *reinterpret_cast<const t4*>(Ar + kk) : t4{0, 0, 0, 0};
    t4 b[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = bn[j] ? *reinterpret_cast<const t4*>(Br[j] + kk) : t4{0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[j] = Mfma<T>::op(b[j][t], a[t], acc[j]);
  }
  if (k0 < kend) {   // a last step shorter than 16
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const long kt = k0 + 4 * q + t;
      const bool in = kt < kend;
      const T a = (am && in) ? Ar[kt] : T(0);
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[j] = Mfma<T>::op((bn[j] && in) ? Br[j][kt] : T(0), a, acc[j]);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int j = 0; j < NT; ++j) red[wave - 1][j][lane] = acc[j];
  }
  __syncthreads();
  if (wave > 0) return;
  T* out = part + (long)blockIdx.x * m * n;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const v4 s = ((acc[j] + red[0][j][lane]) + red[1][j][lane]) + red[2][j][lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jn = 16 * j + Mfma<T>::row(lane, r);
      if (am && jn < n) out[r16 + (long)jn * m] = s[r];
    }
  }
}

// C = sum over a few split-K partials, one thread per output element, the
// splits added in order (deterministic).  For wide outputs with few splits.
// (blockIdx.y: batch item; its partials follow the previous item's.)
__global__ __launch_bounds__(256) void splitk_sum(int m, int n, int splits, double alpha,
                                                  const double* __restrict__ part,
                                                  double* __restrict__ C, long ldc, long sC) {
  const long mn = (long)m * n;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mn) return;
  const double* pb = part + (long)blockIdx.y * splits * mn;
  double s = 0;
#pragma unroll 4
  for (int kc = 0; kc < splits; ++kc) s += pb[(long)kc * mn + idx];
  const int i = (int)(idx % m), j = (int)(idx / m);
  C[(long)blockIdx.y * sC + i + (long)j * ldc] = alpha * s;
}

template <typename T, int BT>
void launch_tiles(const Params<T>& p, bool tA, bool tB, int batch, hipStream_t st) {
  dim3 grid(cdiv(p.m, BT), cdiv(p.n, BT), batch * p.ksplit);
  RM_REQUIRE(grid.z <= 65535, "gemm: batch*ksplit too large");
  if (!tA && !tB) hipLaunchKernelGGL((gemm_kernel<T, false, false, BT>), grid, dim3(256), 0, st, p);
  else if (!tA && tB) hipLaunchKernelGGL((gemm_kernel<T, false, true, BT>), grid, dim3(256), 0, st, p);
  else if (tA && !tB) hipLaunchKernelGGL((gemm_kernel<T, true, false, BT>), grid, dim3(256), 0, st, p);
  else hipLaunchKernelGGL((gemm_kernel<T, true, true, BT>), grid, dim3(256), 0, st, p);
  RM_CHECK_LAUNCH();
}

// 64 x 64 tiles throughout.  128 x 128 tiles (223 registers a lane, one
// wave per SIMD) were measured slower on the large batched products: 888
// against 687 us for the 14 products K^-1 K_l at N = 1024, 3026 against
// 2737 us for the 56 products A_l A_m.
template <typename T>
void launch(const Params<T>& p, bool tA, bool tB, int batch, hipStream_t st) {
  const int slot = timing_begin(sizeof(T) == 8 ? TK_GEMM_F64 : TK_GEMM_F32, st);
  launch_tiles<T, 64>(p, tA, tB, batch, st);
  if (slot >= 0) {
    const double mnk = (double)p.m * p.n * p.k * batch;
    const double io = ((double)p.m * p.k + (double)p.k * p.n + (double)p.m * p.n) * batch * sizeof(T);
    timing_end(slot, st, 2.0 * mnk, io);
  }
}

template <typename T>
void gemm_impl(const Gemm<T>& g, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return;
  Params<T> p{};
  p.m = g.m; p.n = g.n; p.k = g.k; p.alpha = g.alpha; p.beta = g.beta;
  p.A = g.A; p.lda = g.lda; p.sA = g.sA;
  p.B = g.B; p.ldb = g.ldb; p.sB = g.sB;
  p.C = g.C; p.ldc = g.ldc; p.sC = g.sC;
  p.C2 = g.C2; p.ldc2 = g.ldc2; p.sC2 = g.sC2;
  p.Ap = g.Ap; p.Bp = g.Bp; p.Cp = g.Cp; p.C2p = g.C2p;
  p.Co = static_cast<typename Params<T>::OT*>(g.Co); p.sCo = g.sCo;
  p.C2o = static_cast<typename Params<T>::OT*>(g.C2o); p.sC2o = g.sC2o;
  p.Cop = reinterpret_cast<typename Params<T>::OT* const*>(g.Cop);
  RM_REQUIRE(!(g.Co || g.C2o) || (!g.Cp && !g.C2p), "gemm: other-precision copies need strided C");
  p.ksplit = 1; p.kchunk = g.k > 0 ? g.k : 1; p.part = nullptr;
  launch(p, g.tA, g.tB, g.batch, st);
}

template <typename T>
void tallk_impl(int m, int n, long k, const T* A, long lda, const T* B, long ldb, double* C,
                long ldc, double* work, int splits, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  const uintptr_t align = 4 * sizeof(T);
  if (m <= 16 && n <= 64 && lda % 4 == 0 && ldb % 4 == 0 && (uintptr_t)A % align == 0 &&
      (uintptr_t)B % align == 0) {
    // small output: the streaming kernel, k chunks of a multiple of 64
    long chunk = ((k + splits - 1) / splits + 63) / 64 * 64;
    if (chunk < 64) chunk = 64;
    const int sp = (int)((k + chunk - 1) / chunk);
    T* part = reinterpret_cast<T*>(work);
    const int nt = cdiv(n, 16);
    const int slot = timing_begin(sizeof(T) == 8 ? TK_GEMM_F64 : TK_GEMM_F32, st);
    if (nt == 1)
      hipLaunchKernelGGL((tallk_small_kernel<T, 1>), dim3(sp), dim3(256), 0, st, m, n, k, A, lda, B, ldb, chunk, part);
    else if (nt == 2)
      hipLaunchKernelGGL((tallk_small_kernel<T, 2>), dim3(sp), dim3(256), 0, st, m, n, k, A, lda, B, ldb, chunk, part);
    else
      hipLaunchKernelGGL((tallk_small_kernel<T, 4>), dim3(sp), dim3(256), 0, st, m, n, k, A, lda, B, ldb, chunk, part);
    RM_CHECK_LAUNCH();
    if (slot >= 0) timing_end(slot, st, 2.0 * m * n * (double)k, (double)(m + n) * k * sizeof(T));
    const long mn = (long)m * n;
    hipLaunchKernelGGL((splitk_reduce<T>), dim3(cdiv(mn, 4)), dim3(256), 0, st, m, n, sp,
                       (const T*)part, C, ldc);
    RM_CHECK_LAUNCH();
    return;
  }
  Params<T> p{};
  p.m = m; p.n = n; p.k = (int)k; p.alpha = 1; p.beta = 0;
  RM_REQUIRE(k < (1L << 31), "gemm_tallk: k too large");
  p.A = A; p.lda = lda; p.B = B; p.ldb = ldb;
  long chunk = ((k + splits - 1) / splits + BK - 1) / BK * BK;
  if (chunk < BK) chunk = BK;
  int sp = (int)((k + chunk - 1) / chunk);
  if (sp < 1) sp = 1;
  p.ksplit = sp; p.kchunk = chunk;
  p.part = reinterpret_cast<T*>(work);
  launch(p, true, false, 1, st);
  const long mn = (long)m * n;
  hipLaunchKernelGGL((splitk_reduce<T>), dim3(cdiv(mn, 4)), dim3(256), 0, st, m, n, sp,
                     (const T*)p.part, C, ldc);
  RM_CHECK_LAUNCH();
}

// A plain product C = alpha op(A) op(B) (or a strided batch of them) with
// its k range split over `splits` workgroup layers.  A single square
// product near 1000 has only a few hundred 64 x 64 tiles, about one wave per
// SIMD; the layers multiply the waves in flight, and a second pass adds them
// in order.  work: batch * splits * m * n partials.
void gemm_splitk_impl(const Gemm<double>& g, double* work, int splits, hipStream_t st) {
  const bool plain = g.batch >= 1 && g.beta == 0.0 && !g.C2 && !g.C2p && !g.Ap && !g.Bp &&
                     !g.Cp && !g.Co && !g.C2o && !g.Cop && g.C && work;
  if (!plain || splits <= 1 || g.k < 2 * BK * splits) {
    gemm_impl(g, st);
    return;
  }
  if (g.m <= 0 || g.n <= 0) return;
  Params<double> p{};
  p.m = g.m; p.n = g.n; p.k = g.k; p.alpha = 1; p.beta = 0;
  p.A = g.A; p.lda = g.lda; p.sA = g.sA; p.B = g.B; p.ldb = g.ldb; p.sB = g.sB;
  long chunk = ((long)g.k + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  const int sp = (int)(((long)g.k + chunk - 1) / chunk);
  p.ksplit = sp; p.kchunk = chunk;
  p.part = work;
  launch(p, g.tA, g.tB, g.batch, st);
  const long mn = (long)g.m * g.n;
  hipLaunchKernelGGL(splitk_sum, dim3(cdiv(mn, 256), g.batch), dim3(256), 0, st, g.m, g.n, sp,
                     g.alpha, (const double*)work, g.C, g.ldc, g.sC);
  RM_CHECK_LAUNCH();
}

}  // namespace

void gemm(const Gemm<double>& g, hipStream_t st) { gemm_impl(g, st); }
void gemm(const Gemm<float>& g, hipStream_t st) { gemm_impl(g, st); }
void gemm_splitk(const Gemm<double>& g, double* work, int splits, hipStream_t st) {
  gemm_splitk_impl(g, work, splits, st);
}

int tallk_splits(long k) {
  long s = k / 2048;
  if (s < 1) s = 1;
  if (s > 1024) s = 1024;
  return (int)s;
}

void gemm_tallk(int m, int n, long k, const double* A, long lda, const double* B, long ldb,
                double* C, long ldc, double* work, int splits, hipStream_t st) {
  tallk_impl<double>(m, n, k, A, lda, B, ldb, C, ldc, work, splits, st);
}
void gemm_tallk(int m, int n, long k, const float* A, long lda, const float* B, long ldb,
                double* C, long ldc, double* work, int splits, hipStream_t st) {
  tallk_impl<float>(m, n, k, A, lda, B, ldb, C, ldc, work, splits, st);
}

}  // namespace rmhmc
