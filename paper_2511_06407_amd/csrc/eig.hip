// Softabs eigendecomposition (Sec. 2.2) by cyclic two-sided Jacobi, static
// or warm-started (Sec. 2.4: Jacobi on Psi_prev' H Psi_prev, then
// Psi = Psi_prev Q).
//
// Block Jacobi on the padded Dp x Dp matrix (Dp a multiple of 64): the
// nb = Dp/16 column blocks play a round-robin tournament, nb-1 rounds per
// sweep.  In a round every pair of blocks (I, J) forms a 32 x 32 symmetric
// subproblem that one workgroup diagonalises in LDS with an inner cyclic
// Jacobi (its own round-robin over 32 indices; most rounds rotate only the
// pairs between the two blocks); the resulting 32 x 32
// rotations are then applied to M (one wave per 32 x 32 tile on the FP64
// matrix cores, double-buffered M) and to the columns of Psi (fused into
// the next round's solve launch).  Padding rows/columns are zero and never
// rotate (their off-diagonal entries stay exactly zero).  Each rotation
// takes the smaller angle (|angle| <= pi/4) and annihilates its pair
// exactly (Rutishauser's update of the diagonal).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <utility>

#include "common.h"
#include "eig.h"

namespace rmhmc {
namespace {

constexpr int JSB = 32, JHB = 16;   // subproblem size of the block Jacobi and its block width
// A full inner sweep (all pairs of the subproblem) in every
// JACOBI_FULL_PERIOD-th round of an outer sweep, only the pairs between the
// two blocks in the others.  Measured on the Hessians of the D = 1038 model,
// warm-started from a nearby point and from the identity, the outer sweeps
// converge as with a full inner sweep in every round (also at a period of
// 16; a full sweep in the first round alone converges more slowly).
constexpr int JACOBI_FULL_PERIOD = 8;
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int rr_player(int r, int k, int n) {
  // round r of a round-robin over n players: player at seat k (seat 0 fixed)
  return k == 0 ? 0 : 1 + ((k - 1 + r) % (n - 1));
}

// Hand LDS data between lanes of one wave: every LDS access of this wave
// before the call is ordered before every access after it.  The hardware
// runs a wave's LDS instructions in order, but without this the compiler may
// move an access past another one it can prove is to a different address
// for the same lane, which breaks data exchange between lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// rr_player over the SB local indices of a subproblem, branch-free:
// k - 1 + r <= 2 SB - 4, so one conditional subtraction replaces the modulo.
template <int SB>
__device__ __forceinline__ int rr_local(int r, int k) {
  const int x = k - 1 + r;
  return k == 0 ? 0 : 1 + (x >= SB - 1 ? x - (SB - 1) : x);
}

// Pair u of inner round ir.  Full rounds: the round-robin over all SB local
// indices (SB - 1 rounds cover every pair).  Cross rounds: u in the first
// block against HB + (u + ir) mod HB in the second (HB rounds cover the HB^2
// pairs between the two blocks and none inside one).
template <int SB>
__device__ __forceinline__ void inner_pair(bool cross, int ir, int u, int& p, int& q) {
  constexpr int HB = SB / 2;
  if (cross) {
    p = u;
    q = HB + ((u + ir) & (HB - 1));
  } else {
    p = rr_local<SB>(ir, u);
    q = rr_local<SB>(ir, SB - 1 - u);
  }
}

// The SB global indices of a slot in a round: local x < HB in block I,
// x >= HB in block J (computed once per workgroup or wave).
template <int HB>
struct SlotCols {
  int I0, J0;
  __device__ __forceinline__ int col(int x) const { return x < HB ? I0 + x : J0 + (x - HB); }
};
template <int HB>
__device__ __forceinline__ SlotCols<HB> slot_cols(int r, int slot, int nb) {
  return SlotCols<HB>{rr_player(r, slot, nb) * HB, rr_player(r, nb - 1 - slot, nb) * HB};
}

// An SB x SB rotation V is stored in MFMA operand order: element
// (k, c) = (4 kq + l / 16, 16 cb + l % 16) sits at cb * 16 SB + kq * 64 + l, so
// the 64 lanes of a wave read the operand of one v_mfma_f64_16x16x4f64 step
// (rows k0 .. k0+3, 16 columns) as 64 consecutive doubles.
template <int SB>
__device__ __forceinline__ int vfrag_index(int cb, int kq, int lane) {
  return cb * 16 * SB + kq * 64 + lane;
}

// Round-r position of block X: its slot and its half (0: first 16 columns).
__device__ __forceinline__ void rr_locate(int X, int r, int nb, int& slot, int& half) {
  const int m = nb - 1;
  const int k = X == 0 ? 0 : 1 + (((X - 1 - r) % m) + m) % m;   // seat of X
  if (k < nb / 2) { slot = k; half = 0; } else { slot = nb - 1 - k; half = 1; }
}

// The subproblem of `slot` in round `round` >= 1 assembled from the previous
// round's matrix Mprev and rotations Vprev, without waiting for the full M
// update: with its blocks I', J' at (slot A, half hA) and (B, hB) of the
// previous round and V~_X = V_X[:, 16 h_X ..] (32 x 16),
//   S = [V~_A' Mprev[A,A] V~_A, V~_A' Mprev[A,B] V~_B; (.)', V~_B' Mprev[B,B] V~_B].
// Waves 0..2 form the three distinct 16 x 16 blocks on the matrix cores
// (T = Mprev tile x V~_Y, then V~_X' T).  The tiles are staged in T0..T2
// (scratch of the caller) and S is written to Sout, each diagonal block from
// its upper triangle (so S is exactly symmetric).  T2 is then set to the
// identity and red[w] receives this wave's part of ||S||_F^2.  All threads of
// the workgroup call this; it ends with a barrier.
__device__ __forceinline__ void jacobi_compose_subproblem(
    int Dp, int round, int slot, const double* __restrict__ Mprev,
    const double* __restrict__ Vprev, double (*T0)[JSB + 1], double (*T1)[JSB + 1],
    double (*T2)[JSB + 1], double (*Tw)[JSB][17], double (*Sout)[JSB + 1], double* red) {
  const int nb = Dp / JHB;
  const int tid = threadIdx.x, lane = tid & 63, lm = lane & 15, lk = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Ip = rr_player(round, slot, nb), Jp = rr_player(round, nb - 1 - slot, nb);
  int sA, hA, sB, hB;
  rr_locate(Ip, round - 1, nb, sA, hA);
  rr_locate(Jp, round - 1, nb, sB, hB);
  const SlotCols<JHB> ca = slot_cols<JHB>(round - 1, sA, nb), cb = slot_cols<JHB>(round - 1, sB, nb);
  // the three tiles Mprev[A,A], Mprev[A,B], Mprev[B,B]: 12 loads per thread, issued together
  double ld[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const int t = i / 4, e = tid + 256 * (i % 4), x = e % JSB, y = e / JSB;
    const SlotCols<JHB>& cr = t == 2 ? cb : ca;
    const SlotCols<JHB>& cc = t == 0 ? ca : cb;
    ld[i] = Mprev[cr.col(x) + (long)cc.col(y) * Dp];
  }
  // this wave's rotation halves (w = 0: (A, A), 1: (A, B), 2: (B, B))
  const int sX = w == 2 ? sB : sA, hX = w == 2 ? hB : hA;
  const int sY = w == 0 ? sA : sB, hY = w == 0 ? hA : hB;
  double fx[JSB / 4], fy[JSB / 4];
  if (w < 3) {
    const double* VX = Vprev + (long)sX * JSB * JSB + hX * (JSB / 4) * 64;
    const double* VY = Vprev + (long)sY * JSB * JSB + hY * (JSB / 4) * 64;
#pragma unroll
    for (int kq = 0; kq < JSB / 4; ++kq) {
      fx[kq] = VX[kq * 64 + lane];
      fy[kq] = VY[kq * 64 + lane];
    }
  }
  __builtin_amdgcn_sched_barrier(0);   // keep every load issued before the first use
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    const int t = i / 4, e = tid + 256 * (i % 4), x = e % JSB, y = e / JSB;
    double(*T)[JSB + 1] = t == 0 ? T0 : (t == 1 ? T1 : T2);
    T[x][y] = ld[i];
  }
  __syncthreads();
  d4 s2 = d4{0, 0, 0, 0};
  if (w < 3) {
    double(*Mt)[JSB + 1] = w == 0 ? T0 : (w == 1 ? T1 : T2);
    // T = Mt V~_Y (32 x 16): two row tiles
    d4 t1[2] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
#pragma unroll
    for (int kq = 0; kq < JSB / 4; ++kq)
#pragma unroll
      for (int t = 0; t < 2; ++t)
        t1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fy[kq], Mt[16 * t + lm][4 * kq + lk], t1[t], 0, 0, 0);
    double(*Tt)[17] = Tw[w];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) Tt[16 * t + lm][lk + 4 * r] = t1[t][r];
    wave_lds_sync();   // T is read back by other lanes
    // S_XY = V~_X' T (16 x 16); A(m, k) = V~_X(k, m) is this lane's fragment
#pragma unroll
    for (int kq = 0; kq < JSB / 4; ++kq)
      s2 = __builtin_amdgcn_mfma_f64_16x16x4f64(Tt[4 * kq + lk][lm], fx[kq], s2, 0, 0, 0);
  }
  __syncthreads();   // every wave is done with T0..T2
  double ss = 0.0;
  if (w < 3) {
    // lane, register r hold S_XY(m = lm, n = lk + 4 r)
    const int r0 = w == 2 ? JHB : 0, c0 = w == 0 ? 0 : JHB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = lk + 4 * r;
      const double v = s2[r];
      if (w == 1 || lm <= n) {
        Sout[r0 + lm][c0 + n] = v;
        Sout[c0 + n][r0 + lm] = v;
        ss += (w != 1 && lm == n) ? v * v : 2.0 * v * v;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < JSB * JSB / 256; ++i) {
    const int e = tid + 256 * i, x = e % JSB, y = e / JSB;
    T2[x][y] = (x == y) ? 1.0 : 0.0;
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_down(ss, o, 64);
  if (lane == 0) red[w] = ss;
  __syncthreads();
}

// One workgroup diagonalises the SB x SB subproblem of its slot with an inner
// cyclic Jacobi (round-robin over SB indices, SB/2 disjoint rotations a round,
// at most max_inner sweeps) and writes the accumulated rotation V.
//
// Every wave computes the round's SB/2 rotations itself (lane l holds pair
// l mod SB/2; the computation is identical in every wave, so the decisions
// taken from it are uniform over the workgroup).  S is double-buffered: a round reads one
// copy and writes the other, so one barrier per rotating round orders
// everything.  Thread t updates the 2 x 2 blocks (u, v) = (t mod SB/2, ...)
// of S, whose row pair u is the pair it computed itself, and the entries
// (v, u) and (v + SB/2, u) of V, so V only needs its own rotation; the
// rotation of column pair v comes from lane v of the wave by a shuffle.
//
// The subproblem is read from M directly when Vprev is null, else composed
// from the previous round's M and rotations (see the round kernel).  A solve
// whose stop flag (ctrl[1]) is set returns once the subproblem is loaded: the
// flag is read together with the subproblem instead of before it.
//
// cross: one sweep of cross rounds only (pairs between the two blocks).  Each
// block comes from a subproblem that the previous round rotated, so the
// coupling inside a block is what that solve left; a later full round removes
// it, and every pair of indices still meets once per outer sweep.
__device__ __forceinline__ void jacobi_solve_block(int Dp, int round, int slot,
                                                   const double* __restrict__ M,
                                                   const double* __restrict__ Vprev,
                                                   double* __restrict__ Vbuf, int max_inner,
                                                   bool cross, const double* __restrict__ ctrl) {
  constexpr int SB = JSB;
  constexpr int HB = SB / 2;                  // block width; also the number of pairs
  // one 2 x 2 block of S and two entries of V per thread
  static_assert(HB * HB == 256, "the thread mapping needs a 32 x 32 subproblem");
  __shared__ double Sb[2][SB][SB + 1];
  __shared__ double V[SB][SB + 1];
  __shared__ double Tw[3][SB][17];  // per-wave intermediates of the composition
  __shared__ double red[4];
  const double stop = ctrl[1];
  const int nb = Dp / HB;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int NLD = SB * SB / 256;
  if (Vprev == nullptr) {
    const SlotCols<HB> sc = slot_cols<HB>(round, slot, nb);
    double ld[NLD];
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int e = tid + 256 * i, x = e % SB, y = e / SB;
      ld[i] = M[sc.col(x) + (long)sc.col(y) * Dp];
    }
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int e = tid + 256 * i, x = e % SB, y = e / SB;
      Sb[0][x][y] = ld[i];
      V[x][y] = (x == y) ? 1.0 : 0.0;
      ss += ld[i] * ld[i];
    }
    for (int o = 32; o > 0; o >>= 1) ss += __shfl_down(ss, o, 64);
    if (lane == 0) red[w] = ss;
    __syncthreads();
  } else {
    jacobi_compose_subproblem(Dp, round, slot, M, Vprev, Sb[0], Sb[1], V, Tw, Sb[0], red);
  }
  if (stop != 0.0) return;   // uniform: every thread of the workgroup returns
  // Skip a rotation when |a_pq| <= 1e-15 sqrt(|a_pp a_qq|) (relative
  // criterion, so eigenvectors of small eigenvalues stay accurate next to
  // large ones), with an absolute floor of 1e-30 ||S||_F; entries below
  // 1e-150 never rotate, so every square below stays a normal number.
  const double thr = fmax(1e-30 * sqrt(red[0] + red[1] + red[2] + red[3]), 1e-150);
  const double thr2 = thr * thr;
  const int u = tid % HB, v = tid / HB;
  int cur = 0;
  const int n_inner = cross ? HB : SB - 1;
  for (int sweep = 0; sweep < max_inner; ++sweep) {
    bool significant = false;
    for (int ir = 0; ir < n_inner; ++ir) {
      double(*S)[SB + 1] = Sb[cur];
      double(*T)[SB + 1] = Sb[cur ^ 1];
      // rotation of pair u (the smaller angle, |angle| <= pi/4)
      int pu, qu;
      inner_pair<SB>(cross, ir, u, pu, qu);
      const double app = S[pu][pu], aqq = S[qu][qu], apq = S[pu][qu];
      // this thread's 2 x 2 block of S and entries of V, read before the
      // rotations are known so that the reads overlap their arithmetic
      int pv, qv;
      inner_pair<SB>(cross, ir, v, pv, qv);
      const double x0 = S[pu][pv], x1 = S[pu][qv], x2 = S[qu][pv], x3 = S[qu][qv];
      const double vp0 = V[v][pu], vq0 = V[v][qu], vp1 = V[v + HB][pu], vq1 = V[v + HB][qu];
      // The rotation is kept as (s, tau), tau = s / (1 + c) = tan(angle / 2),
      // and applied as x' = x - s (y + tau x), y' = y + s (x - tau y): c
      // never appears rounded.  With c = fl(1 / sqrt(1 + t^2)), every small
      // angle (t^2 below the unit roundoff, where c rounds to 1) would grow
      // both columns' norms by t^2, always upwards, and a warm-started solve
      // applies thousands of such angles to each column.
      double sn = 0.0, tau = 0.0, t = 0.0;
      const double apq2 = apq * apq;
      if (apq2 > fmax(thr2, 1e-30 * fabs(app * aqq))) {
        // The smaller angle with tan(2 angle) = 2 a_pq / d, d = a_qq - a_pp
        // (sgn(0) = +1), from two rsqrt and one reciprocal, with no division
        // on the chain: rho = 1 / sqrt(d^2 + 4 a_pq^2), cos^2 = (1 + |d| rho) / 2,
        // sin = sgn(d) a_pq rho / cos, t = tan = sin / cos.  1 + c lies in
        // [1 + 1/sqrt 2, 2], so the hardware reciprocal refined by two Newton
        // steps is accurate to rounding.
        const double d = aqq - app;
        const double rho = rsqrt(d * d + 4.0 * apq2);
        const double x = fma(0.5 * fabs(d), rho, 0.5);
        const double ic = rsqrt(x);
        const double c = x * ic;
        sn = ((d >= 0.0 ? apq : -apq) * rho) * ic;
        t = sn * ic;
        const double y = 1.0 + c;
        double ry = __builtin_amdgcn_rcp(y);
        ry = fma(ry, fma(-y, ry, 1.0), ry);
        ry = fma(ry, fma(-y, ry, 1.0), ry);
        tau = sn * ry;
      }
      if (__ballot(t != 0.0) == 0) continue;   // no pair rotates: S and V stay
      // significant: an angle above 1e-8.  Inside a tight cluster the entries
      // are tiny next to the diagonal but the angles are not, and the
      // subproblem must still be diagonalised for the outer sweeps to
      // converge quadratically.
      significant = significant || (__ballot(fabs(t) > 1e-8) != 0);
      // the rotation of column pair v: lane v of this wave computed it
      const double sv = __shfl(sn, v, 64), tv = __shfl(tau, v, 64);

      // S' = J' S J on the 2 x 2 block (u, v)
      const double y11 = x0 - sn * (x2 + tau * x0);
      const double y12 = x1 - sn * (x3 + tau * x1);
      const double y21 = x2 + sn * (x0 - tau * x2);
      const double y22 = x3 + sn * (x1 - tau * x3);
      double z11 = y11 - sv * (y12 + tv * y11), z12 = y12 + sv * (y11 - tv * y12);
      double z21 = y21 - sv * (y22 + tv * y21), z22 = y22 + sv * (y21 - tv * y22);
      if (v == u && t != 0.0) {
        // the pair's own block: exact annihilation (Rutishauser update)
        z11 = x0 - t * x1;
        z22 = x3 + t * x1;
        z12 = 0.0;
        z21 = 0.0;
      }
      T[pu][pv] = z11;
      T[pu][qv] = z12;
      T[qu][pv] = z21;
      T[qu][qv] = z22;
      // V <- V J: rows v and v + HB of the columns of pair u
      V[v][pu] = vp0 - sn * (vq0 + tau * vp0);
      V[v][qu] = vq0 + sn * (vp0 - tau * vq0);
      V[v + HB][pu] = vp1 - sn * (vq1 + tau * vp1);
      V[v + HB][qu] = vq1 + sn * (vp1 - tau * vq1);
      __syncthreads();
      cur ^= 1;
    }
    // start another inner sweep only after a significant rotation; smaller
    // residues are removed by later outer sweeps
    if (!significant) break;
  }
  // V in MFMA operand order (see vfrag_index)
  double* out = Vbuf + (long)slot * SB * SB;
  for (int e = tid; e < SB * SB; e += 256) {
    const int l = e & 63, kq = (e >> 6) % (SB / 4), cb = e / (16 * SB);
    out[e] = V[4 * kq + (l >> 4)][16 * cb + (l & 15)];
  }
}



// C (32 x 32, one wave) = sum_k A(m, k) B(k, n) on v_mfma_f64_16x16x4f64:
// 2 x 2 tiles, lane l, register r of tile (ti, tj) holding
// (m = 16 ti + l % 16, n = 16 tj + l / 16 + 4 r).  Aat(t, kq) returns this
// lane's A(16 t + l % 16, 4 kq + l / 16), Bat(kq, t) its B(4 kq + l / 16,
// 16 t + l % 16).
template <class FA, class FB>
__device__ __forceinline__ void mm32_wave(FA Aat, FB Bat, d4 acc[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
#pragma unroll
  for (int kq = 0; kq < JSB / 4; ++kq) {
    double av[2], bv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      av[t] = Aat(t, kq);
      bv[t] = Bat(kq, t);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[tj], av[ti], acc[ti][tj], 0, 0, 0);
  }
}

__device__ __forceinline__ void mm32_to_lds(const d4 acc[2][2], double (*X)[JSB + 1]) {
  const int lane = threadIdx.x & 63, lm = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) X[ti * 16 + lm][tj * 16 + lk + 4 * r] = acc[ti][tj][r];
}

// This lane's operand fragments of a stored rotation (all JSB/4 k-steps, both
// 16-column halves), loaded together so their latencies overlap.
__device__ __forceinline__ void load_vfrag(const double* __restrict__ V, double f[JSB / 4][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int kq = 0; kq < JSB / 4; ++kq)
#pragma unroll
    for (int t = 0; t < 2; ++t) f[kq][t] = V[vfrag_index<JSB>(t, kq, lane)];
}

// A 32 x 32 tile (rows from rowcol, columns from colcol) into registers:
// element e = lane + 64 i, x = e % 32, y = e / 32.
template <class FR, class FC>
__device__ __forceinline__ void load_tile32(const double* __restrict__ A, long lda, FR rowidx,
                                            FC colidx, double v[JSB * JSB / 64]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < JSB * JSB / 64; ++i) {
    const int e = lane + 64 * i, x = e % JSB, y = e / JSB;
    v[i] = A[rowidx(x) + (long)colidx(y) * lda];
  }
}

__device__ __forceinline__ void tile32_to_lds(const double v[JSB * JSB / 64], double (*X)[JSB + 1]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < JSB * JSB / 64; ++i) {
    const int e = lane + 64 * i;
    X[e % JSB][e / JSB] = v[i];
  }
}

// M tile of a round (one wave per 32 x 32 tile (P, R), P <= R, tiles in row
// order): M_out[P,R] = V_P' M_in[P,R] V_R, stored with its mirror
// M_out[R,P] = M_out[P,R]' (M stays exactly symmetric; diagonal tiles are
// symmetrised).  Every global load of the wave (its tile and both rotations
// in their stored MFMA order) is issued before the first is used; the wave
// stages its tile in its own LDS region X, with wavefront-scope fences
// between the lanes' writes and reads (no workgroup barrier).  The tiles
// (and Psi's) are written with streaming stores: the next launch reads them
// from other XCDs, and a round leaves less dirty data in the L2s to write
// back at the launch boundary (17.7 -> 17.1 us per launch at Dp = 1088).
__device__ __forceinline__ void jacobi_m_tile(int Dp, int round, int tile,
                                              const double* __restrict__ Min,
                                              double* __restrict__ Mout,
                                              const double* __restrict__ Vbuf,
                                              double (*X)[JSB + 1]) {
  const int nb = Dp / JHB, ns = nb / 2;
  const int lane = threadIdx.x & 63, lm = lane & 15, lk = lane >> 4;
  int P = 0, rowlen = ns;
  while (tile >= rowlen) { tile -= rowlen; ++P; --rowlen; }
  const int R = P + tile;
  const SlotCols<JHB> cp = slot_cols<JHB>(round, P, nb), cr = slot_cols<JHB>(round, R, nb);
  double tv[JSB * JSB / 64], vp[JSB / 4][2], vr[JSB / 4][2];
  load_tile32(Min, Dp, [&](int x) { return cp.col(x); }, [&](int y) { return cr.col(y); }, tv);
  load_vfrag(Vbuf + (long)P * JSB * JSB, vp);
  load_vfrag(Vbuf + (long)R * JSB * JSB, vr);
  __builtin_amdgcn_sched_barrier(0);   // keep every load issued before the first use
  // X is written and read by different lanes of this wave: order every
  // hand-over (and every rewrite after reads) explicitly
  tile32_to_lds(tv, X);
  wave_lds_sync();
  d4 acc[2][2];
  // Y = VP' X:  A(m, k) = VP(k, m)
  mm32_wave([&](int t, int kq) { return vp[kq][t]; },
            [&](int kq, int t) { return X[4 * kq + lk][16 * t + lm]; }, acc);
  wave_lds_sync();
  mm32_to_lds(acc, X);
  wave_lds_sync();
  // Z = Y VR
  mm32_wave([&](int t, int kq) { return X[16 * t + lm][4 * kq + lk]; },
            [&](int kq, int t) { return vr[kq][t]; }, acc);
  wave_lds_sync();
  mm32_to_lds(acc, X);
  wave_lds_sync();
  if (P == R) {
#pragma unroll 4
    for (int e = lane; e < JSB * JSB; e += 64) {
      const int x = e % JSB, y = e / JSB;
      __builtin_nontemporal_store(0.5 * (X[x][y] + X[y][x]), &Mout[cp.col(x) + (long)cp.col(y) * Dp]);
    }
  } else {
#pragma unroll 4
    for (int e = lane; e < JSB * JSB; e += 64) {
      const int x = e % JSB, y = e / JSB;
      __builtin_nontemporal_store(X[x][y], &Mout[cp.col(x) + (long)cr.col(y) * Dp]);
      __builtin_nontemporal_store(X[y][x], &Mout[cr.col(x) + (long)cp.col(y) * Dp]);
    }
  }
}

// Psi tile k of a round (one wave): rows 32 (k / ns) .., columns of slot
// k mod ns:  Psi[:, P] <- Psi[:, P] V_P.
__device__ __forceinline__ void jacobi_psi_tile(int Dp, int round, int k, double* __restrict__ Psi,
                                                const double* __restrict__ Vbuf,
                                                double (*X)[JSB + 1]) {
  const int nb = Dp / JHB, ns = nb / 2;
  const int lane = threadIdx.x & 63, lm = lane & 15, lk = lane >> 4;
  const int P = k % ns, row0 = (k / ns) * JSB;
  const SlotCols<JHB> cp = slot_cols<JHB>(round, P, nb);
  double tv[JSB * JSB / 64], vp[JSB / 4][2];
  load_tile32(Psi, Dp, [&](int x) { return row0 + x; }, [&](int y) { return cp.col(y); }, tv);
  load_vfrag(Vbuf + (long)P * JSB * JSB, vp);
  __builtin_amdgcn_sched_barrier(0);   // keep every load issued before the first use
  tile32_to_lds(tv, X);
  wave_lds_sync();
  d4 acc[2][2];
  mm32_wave([&](int t, int kq) { return X[16 * t + lm][4 * kq + lk]; },
            [&](int kq, int t) { return vp[kq][t]; }, acc);
  wave_lds_sync();
  mm32_to_lds(acc, X);
  wave_lds_sync();
#pragma unroll 4
  for (int e = lane; e < JSB * JSB; e += 64) {
    const int x = e % JSB, y = e / JSB;
    __builtin_nontemporal_store(X[x][y], &Psi[(row0 + x) + (long)cp.col(y) * Dp]);
  }
}

// One launch per round r (apply_round = r >= 0):
//   workgroups [0, nsolve)        solve the subproblems of round r + 1, each
//                                 assembled from M_r (Min) and V_r (Vprev),
//                                 writing V_{r+1} (Vnew);
//   the next ceil(ntri / 4)       M_{r+1} = J_r' M_r J_r (Mout), one wave per tile;
//   the rest                      Psi <- Psi J_r, one wave per 32 x 32 tile.
// The three parts read M_r and V_r and write different buffers, so they run
// side by side.  With apply_round < 0 the launch only solves round 0 from Min.
// MAX_INNER is the number of inner sweeps per subproblem (1 for every solve).
template <int MAX_INNER>
__global__ __launch_bounds__(256) void jacobi_round_kernel(int Dp, int apply_round, int nsolve,
                                                           const double* __restrict__ Min,
                                                           double* __restrict__ Mout,
                                                           const double* __restrict__ Vprev,
                                                           double* __restrict__ Vnew,
                                                           const double* __restrict__ ctrl,
                                                           int ntri, int npsi,
                                                           double* __restrict__ Psi) {
  const int b = blockIdx.x;
  // ctrl[1]: stop flag, set by the convergence check after a sweep and
  // constant within one; every part of a launch of a stopped solve exits
  // (sweeps launched ahead of the check cost only their launch and the
  // subproblem loads)
  if (b < nsolve) {
    // the full inner sweep every JACOBI_FULL_PERIOD-th round, cross rounds
    // in between
    const int round = apply_round + 1;
    const bool cross = MAX_INNER == JACOBI_INNER_DYNAMIC && round % JACOBI_FULL_PERIOD != 0;
    if (apply_round < 0)
      jacobi_solve_block(Dp, 0, b, Min, nullptr, Vnew, MAX_INNER, false, ctrl);
    else
      jacobi_solve_block(Dp, round, b, Min, Vprev, Vnew, MAX_INNER, cross, ctrl);
    return;
  }
  if (ctrl[1] != 0.0) return;
  __shared__ double Xs[4][JSB][JSB + 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nmwg = (ntri + 3) / 4;
  if (b < nsolve + nmwg) {
    const int tile = (b - nsolve) * 4 + wave;
    if (tile < ntri) jacobi_m_tile(Dp, apply_round, tile, Min, Mout, Vprev, Xs[wave]);
    return;
  }
  const int k = (b - nsolve - nmwg) * 4 + wave;
  if (k < npsi) jacobi_psi_tile(Dp, apply_round, k, Psi, Vprev, Xs[wave]);
}

// Per OFF_COLS-column chunk: off-diagonal squares, all squares, the largest
// relative off-diagonal |m_ij| / sqrt(|m_ii m_jj|), and the same squares
// scaled by 1 / (s_i s_j) with s_i = max(|m_ii|, gfloor), together with the
// sum of 1 / s_i^2 over the chunk's diagonal.
constexpr int OFF_COLS = 8;   // columns per workgroup of the convergence check
constexpr int OFF_MAXDP = 4096;
constexpr int OFF_PARTS = 5;  // partials per chunk
constexpr int OFF_BATCH = 18; // loads in flight per thread
constexpr int CTRL_N = EIG_CTRL_DOUBLES;

__global__ __launch_bounds__(256) void offnorm_kernel(int Dp, const double* __restrict__ M,
                                                      double* __restrict__ part, double gfloor,
                                                      const double* __restrict__ ctrl) {
  __shared__ double sh[OFF_PARTS][4];
  __shared__ double rdg[OFF_MAXDP];   // 1 / sqrt|m_ii| (inf for a zero diagonal)
  __shared__ double rs[OFF_MAXDP];    // 1 / max(|m_ii|, gfloor)
  if (ctrl[1] != 0.0) return;
  // every load of a thread is issued before the first is used: the diagonal
  // (at most OFF_MAXDP / 256 entries a thread), then the chunk in batches of
  // OFF_BATCH elements a thread (two batches at Dp = 1088)
  {
    constexpr int ND = OFF_MAXDP / 256;
    double dv[ND];
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const int i = threadIdx.x + 256 * t;
      dv[t] = i < Dp ? M[i + (long)i * Dp] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < ND; ++t) {
      const int i = threadIdx.x + 256 * t;
      if (i < Dp) {
        const double d = fabs(dv[t]);
        rdg[i] = d > 0.0 ? rsqrt(d) : INFINITY;
        rs[i] = 1.0 / fmax(d, gfloor);
      }
    }
  }
  __syncthreads();
  const int c0 = blockIdx.x * OFF_COLS;
  // columns c0 .. c0 + OFF_COLS - 1 (ld Dp) are one contiguous range
  const double* chunk = M + (long)c0 * Dp;
  const int ne = OFF_COLS * Dp;
  double off = 0.0, tot = 0.0, rel = 0.0, soff = 0.0, sdiag = 0.0;
  for (int e0 = 0; e0 < ne; e0 += 256 * OFF_BATCH) {
    double v[OFF_BATCH];
#pragma unroll
    for (int t = 0; t < OFF_BATCH; ++t) {
      const int e = e0 + threadIdx.x + 256 * t;
      v[t] = e < ne ? chunk[e] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < OFF_BATCH; ++t) {
      const int e = e0 + threadIdx.x + 256 * t;
      if (e < ne) {
        const int j = c0 + e / Dp, i = e - (j - c0) * Dp;
        const double x = v[t];
        tot += x * x;
        if (i != j) {
          if (x != 0.0) {
            off += x * x;
            rel = fmax(rel, fabs(x) * rdg[i] * rdg[j]);
            const double w = x * rs[i] * rs[j];
            soff += w * w;
          }
        } else if (x != 0.0) {
          sdiag += rs[j] * rs[j];
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    off += __shfl_down(off, o, 64);
    tot += __shfl_down(tot, o, 64);
    rel = fmax(rel, __shfl_down(rel, o, 64));
    soff += __shfl_down(soff, o, 64);
    sdiag += __shfl_down(sdiag, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    sh[0][w] = off;
    sh[1][w] = tot;
    sh[2][w] = rel;
    sh[3][w] = soff;
    sh[4][w] = sdiag;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + OFF_PARTS * blockIdx.x;
    o[0] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    o[1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    o[2] = fmax(fmax(sh[2][0], sh[2][1]), fmax(sh[2][2], sh[2][3]));
    o[3] = sh[3][0] + sh[3][1] + sh[3][2] + sh[3][3];
    o[4] = sh[4][0] + sh[4][1] + sh[4][2] + sh[4][3];
  }
}

// Control block of one solve (doubles):
//   [0] ||M||_F (set on the first check)     [1] stop flag (converged or non-finite)
//   [2] last off/||M|| ratio                  [3] checks made
//   [4] the norm-wise test held at the previous check
//   [5] non-finite entries found              [6] buffer holding M when stopped (0: M, 1: M2)
//   [7] sweeps applied before the stop
//   [8 + c], [16 + c], [24 + c] for checks c < 8: the norm-wise ratio, the
//   scaled ratio and the largest relative off-diagonal (convergence history)
// Two stopping rules:
//   EIG_STOP_POLISH: off(M)_F <= zeta ||M||_F (the stated tolerance) and
//     either every off-diagonal is below 1e-12 of the geometric mean of its
//     diagonals or the norm-wise test also held one sweep earlier;
//   EIG_STOP_METRIC: off(M)_F <= zeta ||M||_F and off(S M S)_F <= zeta_s
//     ||diag(S)||_F with S = diag(1 / max(|m_ii|, 1/alpha)).  To first order
//     an off-diagonal E left in M moves G by at most ||E|| (|g'| <= 1) and
//     G^-1 by E_ij / (g_i g_j) with g >= max(|lambda|, 1/alpha), so the two
//     tests bound the relative errors of G and of G^-1 (hence of G^-1 p and
//     of the trace terms) by zeta and zeta_s.  Off-diagonals between two
//     eigenvalues of the cluster near 1/jitter are then left at their
//     harmless size instead of being resolved to 1e-12 of 1/jitter.
__global__ void offnorm_finish_kernel(int nparts, const double* __restrict__ part, double zeta,
                                      double zeta_s, int rule, double* __restrict__ ctrl,
                                      int first, int cur_buf) {
  // One wave: lanes take every 64th partial, then a shuffle tree combines
  // the lane sums and maxima in a fixed order.
  if (ctrl[1] != 0.0) return;
  const int lane = threadIdx.x;
  double off = 0.0, tot = 0.0, rel = 0.0, soff = 0.0, sdiag = 0.0;
  for (int p = lane; p < nparts; p += 64) {
    const double* o = part + OFF_PARTS * p;
    off += o[0];
    tot += o[1];
    rel = fmax(rel, o[2]);
    soff += o[3];
    sdiag += o[4];
  }
  for (int o = 32; o > 0; o >>= 1) {
    off += __shfl_xor(off, o, 64);
    tot += __shfl_xor(tot, o, 64);
    rel = fmax(rel, __shfl_xor(rel, o, 64));
    soff += __shfl_xor(soff, o, 64);
    sdiag += __shfl_xor(sdiag, o, 64);
  }
  if (lane != 0) return;
  const double nrm = sqrt(tot);
  const double sweeps = ctrl[3];   // checks before this one = sweeps applied
  ctrl[3] = sweeps + 1.0;
  ctrl[6] = (double)cur_buf;
  ctrl[7] = sweeps;
  if (!isfinite(nrm) || !isfinite(off) || !isfinite(soff)) {
    ctrl[5] = 1.0;
    ctrl[1] = 1.0;
    return;
  }
  if (first) ctrl[0] = nrm;
  const double r = nrm > 0.0 ? sqrt(off) / nrm : 0.0;
  const double rs = sdiag > 0.0 ? sqrt(soff / sdiag) : 0.0;
  ctrl[2] = r;
  const int c = (int)sweeps;
  if (c < 8) {
    ctrl[8 + c] = r;
    ctrl[16 + c] = rs;
    ctrl[24 + c] = rel;
  }
  const bool normwise = sqrt(off) <= zeta * nrm || !(nrm > 0.0);
  bool done;
  if (rule == EIG_STOP_METRIC) {
    done = normwise && rs <= zeta_s;
  } else {
    done = normwise && (rel <= 1e-12 || off == 0.0 || ctrl[4] != 0.0);
  }
  ctrl[4] = normwise ? 1.0 : 0.0;
  ctrl[1] = done ? 1.0 : 0.0;
}

// After the last sweep: keep the converged matrix in M (copy it from M2 when
// the stop came there), tally the sweeps and flag a solve that did not
// converge.  fail |= 4 (no convergence) or 8 (non-finite); stats[0] counts
// solves and stats[1] their sweeps.  One workgroup per 256 x 16 chunk.
__global__ __launch_bounds__(256) void jacobi_collect_kernel(long n, double* __restrict__ M,
                                                             const double* __restrict__ M2,
                                                             const double* __restrict__ ctrl,
                                                             int last_buf, int* __restrict__ fail,
                                                             double* __restrict__ stats) {
  const bool stopped = ctrl[1] != 0.0;
  const int buf = stopped ? (int)ctrl[6] : last_buf;
  if (buf == 1) {
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
      M[i] = M2[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const bool nonfinite = ctrl[5] != 0.0;
    if (fail && (!stopped || nonfinite)) *fail |= nonfinite ? 8 : 4;
    if (stats) {
      stats[0] += 1.0;
      stats[1] += stopped ? ctrl[7] : ctrl[3] - 1.0;
    }
  }
}

__global__ void fill_ctrl_kernel(double* __restrict__ ctrl) {
  if (threadIdx.x < CTRL_N) ctrl[threadIdx.x] = 0.0;
}

// ------------------------------------------------------------ softabs g, g'
// h(x) = x coth x with x = alpha * lambda; g = h / alpha, g' = h'(x).
// |x| >= 20: h = |x| (coth 20 - 1 < 2^-53); |x| < 1/2: Taylor series in x^2
// (radius pi) with 12 terms; otherwise the closed forms.
__device__ const double kCoth[12] = {1.0,
                                     1.0 / 3.0,
                                     -1.0 / 45.0,
                                     2.0 / 945.0,
                                     -1.0 / 4725.0,
                                     2.0 / 93555.0,
                                     -1382.0 / 638512875.0,
                                     4.0 / 18243225.0,
                                     -3617.0 / 162820783125.0,
                                     87734.0 / 38979295480125.0,
                                     -349222.0 / 1531329465290625.0,
                                     310732.0 / 13447856940643125.0};

__device__ double h0(double x) {
  const double ax = fabs(x);
  if (ax >= 20.0) return ax;
  if (ax < 0.5) {
    const double z = x * x;
    double s = kCoth[11];
    for (int n = 10; n >= 0; --n) s = s * z + kCoth[n];
    return s;
  }
  return x / tanh(x);
}

__device__ double h1(double x) {
  const double ax = fabs(x);
  if (ax >= 20.0) return x > 0 ? 1.0 : -1.0;
  if (ax < 0.5) {
    const double z = x * x;
    double s = 22.0 * kCoth[11];
    for (int n = 10; n >= 1; --n) s = s * z + 2.0 * n * kCoth[n];
    return s * x;
  }
  const double sh = sinh(x);
  return (0.5 * sinh(2.0 * x) - x) / (sh * sh);
}

__device__ double h3(double x) {
  const double ax = fabs(x);
  if (ax >= 20.0) return 0.0;
  if (ax < 0.5) {
    const double z = x * x;
    double s = 0.0;
    for (int n = 11; n >= 2; --n) {
      const double k = 2.0 * n;
      s = s * z + k * (k - 1.0) * (k - 2.0) * kCoth[n];
    }
    return s * x;
  }
  const double sh = sinh(x), ct = 1.0 / tanh(x);
  return 2.0 / (sh * sh) * (3.0 * ct - 3.0 * x * ct * ct + x);
}

}  // namespace

// The softabs map (rmhmc_softabs): g = lam coth(alpha lam) (COTH) or
// g = sqrt(kappa^2 + lam^2) with kappa = 1 / alpha (SQRT, the form of the
// paper's own runs, Sec. 2.5).  For SQRT, g' = lam / g and the divided
// difference (g_j - g_l) / (lam_j - lam_l) equals (lam_j + lam_l) / (g_j + g_l),
// which has no cancellation.
__device__ __forceinline__ double sqrt_g(double l, double alpha) {
  const double kappa = 1.0 / alpha;
  return sqrt(fma(l, l, kappa * kappa));
}

__device__ double divided_difference(double lj, double ll, double alpha, int kind) {
  if (kind == RMHMC_SOFTABS_SQRT) return (lj + ll) / (sqrt_g(lj, alpha) + sqrt_g(ll, alpha));
  const double xj = alpha * lj, xl = alpha * ll;
  if (fabs(xj) >= 20.0 && fabs(xl) >= 20.0) {
    if ((xj > 0) == (xl > 0)) return xj > 0 ? 1.0 : -1.0;
    return (fabs(lj) - fabs(ll)) / (lj - ll);
  }
  const double d = xj - xl;
  if (fabs(d) < 1e-3) {
    const double m = 0.5 * (xj + xl);
    return h1(m) + h3(m) * d * d / 24.0;
  }
  return (h0(xj) - h0(xl)) / d;
}

namespace {

__global__ __launch_bounds__(256) void softabs_finalize_kernel(int D, const double* __restrict__ M,
                                                               long ldm, double alpha, int kind,
                                                               double* __restrict__ lam,
                                                               double* __restrict__ g,
                                                               double* __restrict__ gp,
                                                               double* __restrict__ logdetG) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < D; i += 256) {
    const double l = M[i + (long)i * ldm];
    double gi, gpi;
    if (kind == RMHMC_SOFTABS_SQRT) {
      gi = sqrt_g(l, alpha);
      gpi = l / gi;
    } else {
      const double x = alpha * l;
      gi = h0(x) / alpha;
      gpi = h1(x);
    }
    lam[i] = l;
    g[i] = gi;
    gp[i] = gpi;
    s += log(gi);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) logdetG[0] = sh[0] + sh[1] + sh[2] + sh[3];
}

// M1(j,k) = T_jk b_j b_k  (T from Eq. d3_transform), D x D with ld.
__global__ void t_bb_kernel(int D, const double* __restrict__ lam, const double* __restrict__ b,
                            double alpha, int kind, double* __restrict__ M1, long ld) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)D * D) return;
  const int j = (int)(e % D), k = (int)(e / D);
  double t;
  if (j == k)
    t = kind == RMHMC_SOFTABS_SQRT ? lam[j] / sqrt_g(lam[j], alpha) : h1(alpha * lam[j]);
  else
    t = divided_difference(lam[j], lam[k], alpha, kind);
  M1[j + (long)k * ld] = t * b[j] * b[k];
}

__global__ void scale_cols_kernel(int m, int n, const double* __restrict__ A, long lda,
                                  const double* __restrict__ num, const double* __restrict__ den,
                                  double* __restrict__ B, long ldb) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)m * n) return;
  const int i = (int)(e % m), j = (int)(e / m);
  double s = num ? num[j] : 1.0;
  if (den) s /= den[j];
  B[i + (long)j * ldb] = A[i + (long)j * lda] * s;
}

__global__ void vec_scale_kernel(int n, const double* __restrict__ x, const double* __restrict__ num,
                                 const double* __restrict__ den, int sqrt_num, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = x[i];
  if (num) s *= sqrt_num ? sqrt(num[i]) : num[i];
  if (den) s /= den[i];
  y[i] = s;
}

// lam_i = psi_i' H psi_i from Z = H Psi (column dots), overwriting diag(M).
__global__ __launch_bounds__(256) void rayleigh_kernel(int D, int Dp, const double* __restrict__ Psi,
                                                       const double* __restrict__ Z,
                                                       double* __restrict__ M) {
  __shared__ double sh[4];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < D; k += 256) s += Psi[k + (long)j * Dp] * Z[k + (long)j * Dp];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) M[j + (long)j * Dp] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void pad_copy_kernel(int D, int Dp, const double* __restrict__ H, long ldh,
                                double* __restrict__ M) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)Dp * Dp) return;
  const int i = (int)(e % Dp), j = (int)(e / Dp);
  M[e] = (i < D && j < D) ? 0.5 * (H[i + (long)j * ldh] + H[j + (long)i * ldh]) : 0.0;
}

__global__ void pad_identity_kernel(int D, int Dp, const double* __restrict__ Q, long ldq,
                                    double* __restrict__ Psi) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)Dp * Dp) return;
  const int i = (int)(e % Dp), j = (int)(e / Dp);
  double v;
  if (i < D && j < D) v = Q ? Q[i + (long)j * ldq] : (i == j ? 1.0 : 0.0);
  else v = (i == j) ? 1.0 : 0.0;
  Psi[e] = v;
}

}  // namespace

// padded to a multiple of 64 (whole 64 x 64 tiles for every kernel)
int eig_padded_dim(int D) { return ((D + 63) / 64) * 64; }

void eig_workspace_sizes(int D, long* doubles) {
  const int Dp = eig_padded_dim(D);
  const int nb = Dp / JHB;
  // M, M2, Psi; two rotation sets (double-buffered); convergence partials; ctrl
  *doubles = 3L * Dp * Dp + 2L * (nb / 2) * JSB * JSB + eig_part_doubles(Dp) + CTRL_N;
}

// Unused dynamic LDS reserved by the update-and-solve launches: it lifts a
// workgroup's LDS above half of the CU's 160 KB, so each CU holds one
// workgroup.  The solves are a latency-bound chain of dependent FP64 steps;
// without this, tile workgroups of the same launch share their CU and delay
// the chain (measured: 1.5 us of a 29.9 us launch at Dp = 1088).
constexpr int ROUND_LDS_RESERVE = 12288;

bool eig_trace() {
  static const bool on = std::getenv("RMHMC_EIG_TRACE") != nullptr;
  return on;
}

long eig_part_doubles(int Dp) { return (long)OFF_PARTS * (Dp / OFF_COLS + 1); }

int eig_stop_rule() {
  static const int rule = [] {
    const char* e = std::getenv("RMHMC_EIG_STOP");
    return (e && std::string(e) == "polish") ? EIG_STOP_POLISH : EIG_STOP_METRIC;
  }();
  return rule;
}
double eig_stop_zeta_scaled() { return 1e-12; }

JacobiResult jacobi_eig(int D, EigWork& w, double zeta, double gfloor, int max_sweeps,
                        int max_inner, int blind, bool host_check, int* fail, double* dstats,
                        hipStream_t st, double zeta_s) {
  if (!(zeta_s > 0.0)) zeta_s = eig_stop_zeta_scaled();
  // Input: w.M (Dp x Dp symmetric, padded) and w.Psi (Dp x Dp, padded with identity).
  const int Dp = eig_padded_dim(D);
  const int nb = Dp / JHB, ns = nb / 2;
  RM_REQUIRE(Dp % JSB == 0 && nb % 2 == 0, "softabs_eig: padded dimension does not fit the blocks");
  RM_REQUIRE(Dp <= OFF_MAXDP, "softabs_eig: dimension too large for the convergence check");
  RM_REQUIRE(max_inner == JACOBI_INNER_DYNAMIC || max_inner == JACOBI_INNER_STATIC,
             "softabs_eig: unsupported number of inner sweeps");
  const int nparts = Dp / OFF_COLS;
  double* Mb[2] = {w.M, w.M2};
  int cur = 0;   // buffer holding the current M
  hipLaunchKernelGGL(fill_ctrl_kernel, dim3(1), dim3(64), 0, st, w.ctrl);
  RM_CHECK_LAUNCH();
  auto check = [&](int first) {
    hipLaunchKernelGGL(offnorm_kernel, dim3(nparts), dim3(256), 0, st, Dp, (const double*)Mb[cur],
                       w.part, gfloor, (const double*)w.ctrl);
    RM_CHECK_LAUNCH();
    hipLaunchKernelGGL(offnorm_finish_kernel, dim3(1), dim3(64), 0, st, nparts,
                       (const double*)w.part, zeta, zeta_s, eig_stop_rule(),
                       w.ctrl, first, cur);
    RM_CHECK_LAUNCH();
  };
  const int ntri = ns * (ns + 1) / 2;
  const int npsi = (Dp / JSB) * ns;
  double* Vb[2] = {w.V, w.V + (long)ns * JSB * JSB};
  // per inner round of a subproblem; rounds per solve: JSB - 1 (full), JHB (cross)
  const double inner_flops = (double)ns * (JHB * JHB * 24.0 + JSB * JHB * 6.0);
  auto solve_flops = [&](int round) {
    const bool cross = round % JACOBI_FULL_PERIOD != 0;
    return inner_flops * (cross ? JHB : JSB - 1);
  };
  const double compose_flops = (double)ns * 3.0 * (2.0 * JSB * JSB * JHB + 2.0 * JHB * JSB * JHB);
  const double sb3 = (double)JSB * JSB * JSB;
  const double vset = (double)ns * JSB * JSB * sizeof(double);
  const double tile = (double)JSB * JSB * sizeof(double);
  // static and warm solves run the same rounds (one inner sweep, the cross
  // schedule); max_inner only picks the timing family
  auto round_kernel = jacobi_round_kernel<1>;
  auto sweep = [&]() {
    // launch 0 solves round 0 from M; launch r + 1 applies round r to M and
    // Psi and solves round r + 1 from M_r and V_r.  One event pair brackets
    // the sweep's nb back-to-back launches, so the per-launch average carries
    // no event overhead of its own.
    const int slot =
        timing_begin(max_inner == JACOBI_INNER_DYNAMIC ? TK_JACOBI_DYNAMIC : TK_JACOBI_STATIC, st);
    hipLaunchKernelGGL(round_kernel, dim3(ns), dim3(256), 0, st, Dp, -1, ns,
                       (const double*)Mb[cur], Mb[cur ^ 1], (const double*)nullptr, Vb[0],
                       (const double*)w.ctrl, 0, 0, w.Psi);
    RM_CHECK_LAUNCH();
    // algorithmic bytes: subproblems read, rotations written
    double flops = solve_flops(0), bytes = 2.0 * vset;
    for (int r = 0; r < nb - 1; ++r) {
      const bool more = r + 1 < nb - 1;
      const int nsolve = more ? ns : 0;
      hipLaunchKernelGGL(round_kernel, dim3(nsolve + cdiv(ntri, 4) + cdiv(npsi, 4)), dim3(256),
                         ROUND_LDS_RESERVE, st, Dp, r, nsolve, (const double*)Mb[cur], Mb[cur ^ 1],
                         (const double*)Vb[r & 1], Vb[(r + 1) & 1], (const double*)w.ctrl, ntri,
                         npsi, w.Psi);
      RM_CHECK_LAUNCH();
      // algorithmic work: M update (upper tiles read, all of M written), Psi
      // read and written, rotations V_r read once; solves: three tiles of
      // M_r read per subproblem, V_{r+1} written
      flops += 4.0 * sb3 * ntri + 2.0 * sb3 * npsi + (more ? solve_flops(r + 1) + compose_flops : 0.0);
      bytes += (double)ntri * tile + 3.0 * (double)Dp * Dp * sizeof(double) + vset +
               (more ? 3.0 * ns * tile + vset : 0.0);
      cur ^= 1;
    }
    timing_end(slot, st, flops, bytes, nb);
    check(0);
  };
  check(1);
  JacobiResult res;
  int launched = 0;
  // sweeps launched before the host first looks (all of them without host checks)
  const int ahead = std::min(max_sweeps, host_check ? std::max(blind, 0) : std::max(blind, 1));
  for (; launched < ahead; ++launched) sweep();
  if (host_check) {
    for (;;) {
      RM_HIP(hipMemcpyAsync(w.ctrl_host, w.ctrl, CTRL_N * sizeof(double), hipMemcpyDeviceToHost, st));
      RM_HIP(hipStreamSynchronize(st));
      if (w.ctrl_host[1] != 0.0 || launched >= max_sweeps) break;
      sweep();
      ++launched;
    }
    res.nonfinite = w.ctrl_host[5] != 0.0;
    res.converged = w.ctrl_host[1] != 0.0 && !res.nonfinite;
    res.sweeps = w.ctrl_host[1] != 0.0 ? (int)w.ctrl_host[7] : launched;
    if (eig_trace()) {
      std::fprintf(stderr, "[eig] D=%d sweeps=%d converged=%d", D, res.sweeps, (int)res.converged);
      for (int c = 0; c < 8 && c <= res.sweeps; ++c)
        std::fprintf(stderr, " | %.1e %.1e %.1e", w.ctrl_host[8 + c], w.ctrl_host[16 + c],
                     w.ctrl_host[24 + c]);
      std::fprintf(stderr, "\n");
    }
  }
  const long n = (long)Dp * Dp;
  hipLaunchKernelGGL(jacobi_collect_kernel, dim3((unsigned)std::min<long>(cdiv(n, 256 * 16), 1024)),
                     dim3(256), 0, st, n, w.M, (const double*)w.M2, (const double*)w.ctrl, cur,
                     fail, dstats);
  RM_CHECK_LAUNCH();
  return res;
}

namespace {
// G <- (3I - G) / 2 on the D x D block.
__global__ void ns_coeff_kernel(int D, int Dp, double* __restrict__ G) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)D * D) return;
  const int i = (int)(e % D), j = (int)(e / D);
  double* x = G + i + (long)j * Dp;
  *x = (i == j ? 1.5 : 0.0) - 0.5 * *x;
}
}  // namespace

void orthonormalise(int D, int Dp, double* Psi, double* T1, double* T2, hipStream_t st,
                    double* split, int nsplit) {
  Gemm<double> g;
  g.m = D; g.n = D; g.k = D;
  g.A = Psi; g.lda = Dp; g.tA = true;
  g.B = Psi; g.ldb = Dp;
  g.C = T1; g.ldc = Dp;
  gemm_splitk(g, split, split ? nsplit : 1, st);
  hipLaunchKernelGGL(ns_coeff_kernel, dim3(cdiv((long)D * D, 256)), dim3(256), 0, st, D, Dp, T1);
  RM_CHECK_LAUNCH();
  Gemm<double> h;
  h.m = D; h.n = D; h.k = D;
  h.A = Psi; h.lda = Dp;
  h.B = T1; h.ldb = Dp;
  h.C = T2; h.ldc = Dp;
  gemm_splitk(h, split, split ? nsplit : 1, st);
  copy_matrix(D, D, T2, Dp, Psi, Dp, st);
}

void eig_load_matrix(int D, const double* H, long ldh, EigWork& w, hipStream_t st) {
  const int Dp = eig_padded_dim(D);
  const long n = (long)Dp * Dp;
  hipLaunchKernelGGL(pad_copy_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, D, Dp, H, ldh, w.M);
  RM_CHECK_LAUNCH();
}

void eig_load_basis(int D, const double* Q, long ldq, EigWork& w, hipStream_t st) {
  const int Dp = eig_padded_dim(D);
  const long n = (long)Dp * Dp;
  hipLaunchKernelGGL(pad_identity_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, D, Dp, Q, ldq, w.Psi);
  RM_CHECK_LAUNCH();
}

void rayleigh_refine(int D, const double* H, long ldh, EigWork& w, double* Z, hipStream_t st,
                     double* split, int nsplit) {
  // Z = H Psi on the leading D x D block, then diag(M) <- column dots
  const int Dp = eig_padded_dim(D);
  Gemm<double> g;
  g.m = D; g.n = D; g.k = D;
  g.A = H; g.lda = ldh;
  g.B = w.Psi; g.ldb = Dp;
  g.C = Z; g.ldc = Dp;
  gemm_splitk(g, split, split ? nsplit : 1, st);
  hipLaunchKernelGGL(rayleigh_kernel, dim3(D), dim3(256), 0, st, D, Dp, (const double*)w.Psi,
                     (const double*)Z, w.M);
  RM_CHECK_LAUNCH();
}

void softabs_finalize(int D, const double* M, long ldm, double alpha, int kind, double* lam,
                      double* g, double* gp, double* logdetG, hipStream_t st) {
  hipLaunchKernelGGL(softabs_finalize_kernel, dim3(1), dim3(256), 0, st, D, M, ldm, alpha, kind,
                     lam, g, gp, logdetG);
  RM_CHECK_LAUNCH();
}

void t_bb(int D, const double* lam, const double* b, double alpha, int kind, double* M1, long ld,
          hipStream_t st) {
  const long n = (long)D * D;
  hipLaunchKernelGGL(t_bb_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, D, lam, b, alpha, kind, M1,
                     ld);
  RM_CHECK_LAUNCH();
}

void scale_cols(int m, int n, const double* A, long lda, const double* num, const double* den,
                double* B, long ldb, hipStream_t st) {
  const long mn = (long)m * n;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(cdiv(mn, 256)), dim3(256), 0, st, m, n, A, lda, num,
                     den, B, ldb);
  RM_CHECK_LAUNCH();
}

void vec_scale(int n, const double* x, const double* num, const double* den, bool sqrt_num,
               double* y, hipStream_t st) {
  hipLaunchKernelGGL(vec_scale_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, n, x, num, den,
                     (int)sqrt_num, y);
  RM_CHECK_LAUNCH();
}

}  // namespace rmhmc
