// Band LU of M(omega) = i omega I - L on MFMA (the solves are in rr_solve.hip).
//
// The paper factors the shifted operator once and reuses the LU in the three
// linear solves of Algorithm 1 (Section 3.1).  Here the band (kl = ku = b =
// 2*ny) is cut into T x T tiles: block row s holds tiles (s, s-B) .. (s, s+B)
// with B = ceil(b / T), so the band becomes block-banded with B blocks on each
// side.  Without pivoting (element growth of the shifted operator stays O(1);
// the oracle's probe measures it) the block LU is
//   A_rt -= sum_s L_rs U_st             (updates, complex GEMMs on MFMA)
//   A_mm  = L_mm U_mm                    (T x T LU in LDS)
//   L_rm  = A_rm U_mm^-1,  U_mt = L_mm^-1 A_mt
// The diagonal step publishes the LU with its 16 x 16 diagonal blocks
// inverted first; the off-diagonal finalisations are triangular solves with
// it (wave-local, on MFMA).  The full inverses follow off the dependency
// chain, and the diagonal tile is stored as [U_mm^-1 (upper, diagonal
// included) | L_mm^-1 (strictly lower, unit diagonal implied)] for the
// solves, where applying D^-1 is a GEMM.
//
// Storage: L tiles (r > t) and diagonal tiles are column-major, U tiles
// (r < t) row-major, so that in the update L_rs U_st both MFMA operands are
// read with consecutive lanes on consecutive addresses.
//
// Scheduling: one persistent launch per factorisation; a global ticket counter
// hands out tasks in an order where every task only waits on smaller tickets,
// so the launch cannot deadlock whatever the residency.  Per tile (r, t) with
// m = min(r, t) there are two tasks:
//   E(r, t)  the early updates s <= m-2 (inputs final long before), written
//            back as a partial tile (flag 1); issued one step ahead
//   F(r, t)  the last update s = m-1 (before waiting on the diagonal tile m)
//            and the finalisation (flag 2; the diagonal tile 2, then 3 once
//            its full inverses are stored)
// so the chain from one diagonal block to the next carries one update GEMM,
// one triangular solve and one T x T LU.  A diagonal tile's early updates are
// split once more, so that no long task sits on that chain either:
//   E'(m, m)  s <= m-3, issued two block steps ahead (flag 1)
//   G(m, m)   s = m-2 on top of E'(m, m), issued one step ahead (flag 2)
// and the diagonal worker adds s = m-1 before its LU.  With the superblock
// solve (no chain tiles) the worker publishes only the block-inverse LU; the
// full inverses of the diagonal tiles follow in a launch of their own.  The tile of M itself is generated
// from the stencil in registers: the band is never read before it is final.
// Every tile store is device-coherent (st_coherent) and goes through LDS so
// that each store instruction writes whole lines: a tile is written twice
// per launch, from different XCDs in general, and read from others.
//
// Chain tiles.  In each sweep of a solve, block s depends on the blocks t
// within B of it through x_s = D^-1 (b_s - sum_t T_st x_t), D^-1 a triangle of
// the diagonal inverse.  For the nearest neighbours (distance d = 1 .. 3) the
// factorisation stores the products G_s,d = D^-1 T_s,s-+d, so that a solve
// step applies D^-1 to the far terms, four or more blocks back, long before
// the neighbours are ready, and every product left is a register MFMA with no
// LDS round trip:  x_s = D^-1 (b_s - sum_far) - sum_{d <= 3} G_s,d x_s-+d.
//   CH_FWD_L,d = L_ss^-1 L_s,s-d   (column-major)   forward, L sweep
//   CH_FWD_U,d = U_ss^-1 U_s,s+d   (column-major)   forward, U sweep
//   CH_ADJ_U,d = U_s-d,s U_ss^-1   (row-major)      adjoint, U^H sweep (used as ^H)
//   CH_ADJ_L,d = L_s+d,s L_ss^-1   (row-major)      adjoint, L^H sweep (used as ^H)
// F(s, s) forms CH_FWD_L and CH_ADJ_U after publishing D_s; F(s+d, s) and
// F(s, s+d) form CH_ADJ_L,d and CH_FWD_U,d after publishing their tile (and
// waiting for D_s).  Nothing in the launch waits on chain tiles.
#include "rr_mfma.h"

namespace rr {

template <int T>
struct FGeom {
  static constexpr int NW = (T / 16) * (T / 16) / 2;  // waves: two 16x16 blocks each
  static constexpr int NT = 64 * NW;
  static constexpr int CPR = T / 32;                  // column-block pairs per row block
  static constexpr int LDT = T + 1;                   // padded LDS leading dimension
};

struct FactorParams {
  OpDesc op;
  BandGeom g;
  const double* omega;  // 2 * n_omega
  int n_omega;
  void* tiles;
  int* flags;           // per tile: 1 = partial (E done), 2 = final
  uint32_t* ticket;     // [0] task tickets, [1] diagonal-worker roles
  uint32_t* status;
  int slots;            // tickets per step and shift
  int64_t total;        // n_omega * NB * slots
};

// Entry (gi, gj) of M = i omega I - L from the 12-point stencil; padding rows
// and columns beyond n carry the identity.
__device__ __forceinline__ double2 m_entry(const OpDesc& op, double om_r, double om_i, int64_t gi,
                                           int64_t gj) {
  if (gi >= op.n || gj >= op.n) return make_double2(gi == gj ? 1.0 : 0.0, 0.0);
  int p = (int)(gi >> 1), c = (int)(gi & 1), q = (int)(gj >> 1), d = (int)(gj & 1);
  const double* cf = op.coef + 12 * (int64_t)p + 6 * c;
  double lv = 0.0;
  if (q == p) {
    lv = (d == c) ? cf[0] : cf[5];
  } else if (d == c) {
    int ny = op.ny, jj = p % ny;
    if (q == p + op.ny) lv = cf[1];
    else if (q == p - op.ny) lv = cf[2];
    else if (q == p + 1 && jj < ny - 1) lv = cf[3];
    else if (q == p - 1 && jj > 0) lv = cf[4];
  }
  double re = -lv, im = 0.0;
  if (gi == gj) { re -= om_i; im += om_r; }
  return make_double2(re, im);
}

// Triangular masks on a stored tile's own indices (row, col).
enum { MK_NONE = 0, MK_UNIT_LOWER = 1, MK_UPPER = 2 };

template <typename R>
__device__ __forceinline__ cplx<R> apply_mask(cplx<R> v, int mask, int row, int col) {
  if (mask == MK_UNIT_LOWER && row <= col) return cplx<R>{row == col ? (R)1 : (R)0, (R)0};
  if (mask == MK_UPPER && row > col) return cplx<R>{(R)0, (R)0};
  return v;
}

// Value of lane `src` (wave-uniform) in every lane.
__device__ __forceinline__ float bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename R>
__device__ __forceinline__ cplx<R> bcast(cplx<R> v, int src) {
  return cplx<R>{bcast(v.re, src), bcast(v.im, src)};
}

__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <typename R>
__device__ __forceinline__ void csub_mul(cplx<R>& x, cplx<R> a, cplx<R> b) {  // x -= a b
  x.re = fmaR(-a.re, b.re, fmaR(a.im, b.im, x.re));
  x.im = fmaR(-a.re, b.im, fmaR(-a.im, b.re, x.im));
}

// (re, im) (+/-)= A * B for one 16 x 16 output block with K = 4q terms, both
// operands column-major in LDS: A[i][k] at (ac + k) * lda + ar + i, B[k][j] at
// (bc + j) * ldb + br + k.  Masks apply to each operand's own coordinates.
template <typename R, bool SUB>
__device__ __forceinline__ void lds_blk_gemm(typename Mf<R>::v4& re, typename Mf<R>::v4& im,
                                             const cplx<R>* A, int lda, int ar, int ac, int amask,
                                             const cplx<R>* Bm, int ldb, int br, int bc, int bmask,
                                             int K) {
  const int l = threadIdx.x & 63;
#pragma unroll 1
  for (int q = 0; q < K / 4; q++) {
    const int k = 4 * q + (l >> 4);
    cplx<R> a = apply_mask(A[(ac + k) * lda + ar + (l & 15)], amask, ar + (l & 15), ac + k);
    cplx<R> b = apply_mask(Bm[(bc + (l & 15)) * ldb + br + k], bmask, br + k, bc + (l & 15));
    cmfma<R, false, SUB>(re, im, a, b);
  }
}

template <typename R>
__device__ __forceinline__ void blk_load(typename Mf<R>::v4& re, typename Mf<R>::v4& im,
                                         const cplx<R>* S, int ld, int r0, int c0) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    cplx<R> v = S[(c0 + (l & 15)) * ld + r0 + Mf<R>::row(l, e)];
    re[e] = v.re;
    im[e] = v.im;
  }
}
template <typename R>
__device__ __forceinline__ void blk_store(const typename Mf<R>::v4& re,
                                          const typename Mf<R>::v4& im, cplx<R>* S, int ld,
                                          int r0, int c0) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 4; e++)
    S[(c0 + (l & 15)) * ld + r0 + Mf<R>::row(l, e)] = cplx<R>{re[e], im[e]};
}

// Inverse of the 16 x 16 diagonal block at (b0, b0) of an LU held in LDS
// (column-major, leading dimension LD), in place: unit-lower L (its strictly
// lower part is rewritten) or upper U (the upper part with the diagonal).
// Lane c computes column c of the inverse by substitution in registers,
// reading the triangle's entries as wave-uniform (broadcast) LDS loads; lanes
// 16 .. 63 compute copies and store nothing.  The other triangle of the block is
// neither read nor written, so the L and U inversions of one block may run
// in two waves at once.
// No-pivot LU of the T x T tile S (LDS, column-major, leading dimension LD),
// then in-place inversion of its 16 x 16 diagonal blocks:
//   S <- L (strictly lower, unit diagonal implied) and U (upper, diagonal
//        included), each diagonal block L_jj, U_jj replaced by its inverse
// (the block-inverse LU: enough for the triangular solves of the
// off-diagonal finalisations).  Blocked so that the sequential part is short
// and wave-local: per 16-column panel one wave factors the panel in registers
// (lane = row, the pivot row broadcast lane to lane); then U12 = L11^-1 A12
// and L11^-1 by forward substitution (thread = column, in registers) while
// another wave forms U11^-1 by back substitution; then A22 -= L21 U12 on MFMA.
// A zero or non-finite pivot latches ST_SINGULAR and is replaced by 1.
template <typename R, int T, int NW>
__device__ void lu_blockinv(cplx<R>* S, int LD, uint32_t* status) {
  typedef typename Mf<R>::v4 v4;
  constexpr int P = 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const cplx<R> one{(R)1, (R)0}, zero{(R)0, (R)0};
  auto at = [&](int i, int c) -> cplx<R>& { return S[c * LD + i]; };
#pragma unroll 1
  for (int c0 = 0; c0 < T; c0 += P) {
    // panel: lane = row c0 + lane.  Lanes at or above the pivot row get a
    // zero multiplier, which leaves their row unchanged (no per-element select).
    if (wave == 0) {
      const int r = c0 + lane;
      const bool act = r < T;
      cplx<R> a[P];
#pragma unroll
      for (int c = 0; c < P; c++) a[c] = act ? at(r, c0 + c) : zero;
#pragma unroll
      for (int j = 0; j < P; j++) {
        cplx<R> p = bcast(a[j], j);
        const R mag = p.re * p.re + p.im * p.im;
        if (!(mag > (R)0) || !isfinite(mag)) {
          if (lane == 0) latch(status, ST_SINGULAR);
          if (lane == j) a[j] = one;
          p = one;
        }
        const bool below = act && lane > j;
        const cplx<R> l = below ? cmul(a[j], cinv(p)) : zero;
        if (below) a[j] = l;
#pragma unroll
        for (int c = j + 1; c < P; c++) csub_mul(a[c], l, bcast(a[c], j));
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int c = 0; c < P; c++)
        if (act) at(r, c0 + c) = a[c];
    }
    __syncthreads();
    // Wave 0: U12 = L11^-1 A12 by forward substitution, thread t owning
    // column c0 + P + t, and L11^-1 in the next 16 threads (identity columns).
    // Wave 1: U11^-1 by back substitution, lane t < 16 owning column t.
    // Both inverses are kept in registers until the barrier (L11 and U11
    // are read until then) and written over the diagonal block after it.
    const int nu = T - c0 - P;  // columns of U12
    cplx<R> x[P];
    const bool lsolve = threadIdx.x < nu + P;
    const bool uinv = wave == 1 && lane < P;
    if (lsolve) {
      const int t = threadIdx.x;
#pragma unroll
      for (int i = 0; i < P; i++)
        x[i] = t < nu ? at(c0 + i, c0 + P + t) : cplx<R>{i == t - nu ? (R)1 : (R)0, (R)0};
#pragma unroll
      for (int j = 0; j < P - 1; j++) {
#pragma unroll
        for (int i = j + 1; i < P; i++) csub_mul(x[i], at(c0 + i, c0 + j), x[j]);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (t < nu) {
#pragma unroll
        for (int i = 0; i < P; i++) at(c0 + i, c0 + P + t) = x[i];
      }
    } else if (uinv) {
      // the 16 reciprocals of the diagonal at once (lane j: 1 / U_jj), so
      // that no division sits on the substitution's dependency chain
      const cplx<R> dinv = cinv(at(c0 + lane, c0 + lane));
#pragma unroll
      for (int i = 0; i < P; i++) x[i] = cplx<R>{i == lane ? (R)1 : (R)0, (R)0};
#pragma unroll
      for (int j = P - 1; j >= 0; j--) {
        x[j] = cmul(x[j], bcast(dinv, j));
#pragma unroll
        for (int i = 0; i < j; i++) csub_mul(x[i], at(c0 + i, c0 + j), x[j]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
    if (lsolve && threadIdx.x >= nu) {  // L11^-1, strictly lower part
      const int cc = threadIdx.x - nu;
#pragma unroll
      for (int i = 1; i < P; i++)
        if (i > cc) at(c0 + i, c0 + cc) = x[i];
    } else if (uinv) {                  // U11^-1, upper part with the diagonal
#pragma unroll
      for (int i = 0; i < P; i++)
        if (i <= lane) at(c0 + i, c0 + lane) = x[i];
    }
    if (nu == 0) break;
    // A22 -= L21 U12 in 16 x 16 blocks (disjoint from the diagonal block)
    const int nb = nu / 16;
    for (int b = wave; b < nb * nb; b += NW) {
      const int bi = c0 + P + 16 * (b % nb), bj = c0 + P + 16 * (b / nb);
      v4 re, im;
      blk_load<R>(re, im, S, LD, bi, bj);
      lds_blk_gemm<R, true>(re, im, S, LD, bi, c0, MK_NONE, S, LD, c0, bj, MK_NONE, P);
      blk_store<R>(re, im, S, LD, bi, bj);
    }
    __syncthreads();
  }
  __syncthreads();
}

// Block-inverse LU (lu_blockinv) -> [U^-1 on and above the diagonal | L^-1
// strictly below], in place, by doubling: [[A, 0], [C, D]]^-1 has lower-left
// -D^-1 C A^-1 and [[A, B], [0, D]]^-1 upper-right -A^-1 B D^-1, two MFMA
// products per level (tmp: T*T/2 complex of LDS for the intermediate products).
template <typename R, int T, int NW>
__device__ void inv_doubling(cplx<R>* S, int LD, cplx<R>* tmp) {
  typedef typename Mf<R>::v4 v4;
  const int wave = threadIdx.x >> 6;
  // blocks of 2h along the diagonal; kind 0 = L, 1 = U
#pragma unroll 1
  for (int h = 16; h < T; h *= 2) {
    const int nblk = T / (2 * h), nsub = (h / 16) * (h / 16);
    const int ntask = 2 * nblk * nsub;
    for (int tsk = wave; tsk < ntask; tsk += NW) {
      const int kind = tsk / (nblk * nsub), rem = tsk % (nblk * nsub);
      const int blk = rem / nsub, sub = rem % nsub;
      const int b0 = 2 * h * blk, si = 16 * (sub % (h / 16)), sj = 16 * (sub / (h / 16));
      cplx<R>* t1 = tmp + (kind * nblk + blk) * h * h;
      v4 re, im;
#pragma unroll
      for (int e = 0; e < 4; e++) { re[e] = 0; im[e] = 0; }
      if (kind == 0)  // L21 L11^-1
        lds_blk_gemm<R, false>(re, im, S, LD, b0 + h + si, b0, MK_NONE, S, LD, b0, b0 + sj,
                               MK_UNIT_LOWER, h);
      else            // U12 U22^-1
        lds_blk_gemm<R, false>(re, im, S, LD, b0 + si, b0 + h, MK_NONE, S, LD, b0 + h,
                               b0 + h + sj, MK_UPPER, h);
      blk_store<R>(re, im, t1, h, si, sj);
    }
    __syncthreads();
    for (int tsk = wave; tsk < ntask; tsk += NW) {
      const int kind = tsk / (nblk * nsub), rem = tsk % (nblk * nsub);
      const int blk = rem / nsub, sub = rem % nsub;
      const int b0 = 2 * h * blk, si = 16 * (sub % (h / 16)), sj = 16 * (sub / (h / 16));
      const cplx<R>* t1 = tmp + (kind * nblk + blk) * h * h;
      v4 re, im;
#pragma unroll
      for (int e = 0; e < 4; e++) { re[e] = 0; im[e] = 0; }
      if (kind == 0) {  // lower-left <- -L22^-1 (L21 L11^-1)
        lds_blk_gemm<R, true>(re, im, S, LD, b0 + h + si, b0 + h, MK_UNIT_LOWER, t1, h, 0, sj,
                              MK_NONE, h);
        blk_store<R>(re, im, S, LD, b0 + h + si, b0 + sj);
      } else {          // upper-right <- -U11^-1 (U12 U22^-1)
        lds_blk_gemm<R, true>(re, im, S, LD, b0 + si, b0, MK_UPPER, t1, h, 0, sj, MK_NONE, h);
        blk_store<R>(re, im, S, LD, b0 + si, b0 + h + sj);
      }
    }
    __syncthreads();
  }
}

// Triangular solves with a block-inverse LU Db (LDS, column-major, leading
// dimension LDD), in place on the T x T tile S (LDS, column-major, leading
// dimension LD).  Both are wave-local (no barriers): the waves below T/16
// each own one 16-row (right solve) or 16-column (left solve) strip and walk
// its blocks in dependency order; the other waves return at once.
//   right, upper:      S <- S U^-1:  X_j = (A_j - sum_{i<j} X_i U_ij) U_jj^-1
//   left, unit lower:  S <- L^-1 S:  X_i = L_ii^-1 (A_i - sum_{k<i} L_ik X_k)
template <typename R, int T>
__device__ __forceinline__ void trsm_right_upper(cplx<R>* S, int LD, const cplx<R>* Db, int LDD) {
  typedef typename Mf<R>::v4 v4;
  const int wave = threadIdx.x >> 6;
  if (wave >= T / 16) return;
  const int r0 = 16 * wave;
#pragma unroll 1
  for (int j = 0; j < T / 16; j++) {
    v4 re, im;
    blk_load<R>(re, im, S, LD, r0, 16 * j);
    if (j > 0)
      lds_blk_gemm<R, true>(re, im, S, LD, r0, 0, MK_NONE, Db, LDD, 0, 16 * j, MK_NONE, 16 * j);
    blk_store<R>(re, im, S, LD, r0, 16 * j);
#pragma unroll
    for (int e = 0; e < 4; e++) { re[e] = 0; im[e] = 0; }
    lds_blk_gemm<R, false>(re, im, S, LD, r0, 16 * j, MK_NONE, Db, LDD, 16 * j, 16 * j, MK_UPPER,
                           16);
    blk_store<R>(re, im, S, LD, r0, 16 * j);
  }
}
template <typename R, int T>
__device__ __forceinline__ void trsm_left_lower(cplx<R>* S, int LD, const cplx<R>* Db, int LDD) {
  typedef typename Mf<R>::v4 v4;
  const int wave = threadIdx.x >> 6;
  if (wave >= T / 16) return;
  const int c0 = 16 * wave;
#pragma unroll 1
  for (int i = 0; i < T / 16; i++) {
    v4 re, im;
    blk_load<R>(re, im, S, LD, 16 * i, c0);
    if (i > 0)
      lds_blk_gemm<R, true>(re, im, Db, LDD, 16 * i, 0, MK_NONE, S, LD, 0, c0, MK_NONE, 16 * i);
    blk_store<R>(re, im, S, LD, 16 * i, c0);
#pragma unroll
    for (int e = 0; e < 4; e++) { re[e] = 0; im[e] = 0; }
    lds_blk_gemm<R, false>(re, im, Db, LDD, 16 * i, 16 * i, MK_UNIT_LOWER, S, LD, 16 * i, c0,
                           MK_NONE, 16);
    blk_store<R>(re, im, S, LD, 16 * i, c0);
  }
}

// A wave's two 16x16 accumulator blocks of a T x T tile: row block rb,
// column blocks 2cp and 2cp+1.
template <typename R>
struct Acc2 {
  typename Mf<R>::v4 re[2], im[2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int e = 0; e < 4; e++) { re[b][e] = 0; im[b][e] = 0; }
  }
};

// Element address of (i, j) in a stored tile: column-major or row-major.
__device__ __forceinline__ int tix(int i, int j, int T, bool rowmajor) {
  return rowmajor ? i * T + j : j * T + i;
}

// acc (+/-)= A * B for T x T tiles.  A: column-major (A[i][k] at k*lda + i)
// or row-major (at i*lda + k); B: row-major (B[k][j] at k*ldb + j) or
// column-major (at j*ldb + k); either may live in LDS or global memory.
// Optional triangular masks apply to each stored tile's own indices.
// Fragments of KQ k-steps are loaded before use.  G3: Gauss's three real
// products per complex one (a_r b_r, a_i b_i, (a_r + a_i)(b_r + b_i)),
// summed apart and combined at the end.
template <typename R>
struct Gauss3 {
  typename Mf<R>::v4 p1[2], p2[2], p3[2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int e = 0; e < 4; e++) { p1[b][e] = 0; p2[b][e] = 0; p3[b][e] = 0; }
  }
  __device__ __forceinline__ void mma(cplx<R> a, cplx<R> b, int c) {
    p1[c] = Mf<R>::op(a.re, b.re, p1[c]);
    p2[c] = Mf<R>::op(a.im, b.im, p2[c]);
    p3[c] = Mf<R>::op(a.re + a.im, b.re + b.im, p3[c]);
  }
  template <bool SUB>
  __device__ __forceinline__ void add_to(Acc2<R>& acc) const {
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const R re = p1[b][e] - p2[b][e], im = p3[b][e] - p1[b][e] - p2[b][e];
        acc.re[b][e] += SUB ? -re : re;
        acc.im[b][e] += SUB ? -im : im;
      }
  }
};

template <typename R, int T, int KQ, bool SUB, bool G3 = false>
__device__ __forceinline__ void tile_gemm(Acc2<R>& acc, const cplx<R>* A, int lda, bool a_rowmajor,
                                          int amask, const cplx<R>* Bm, int ldb, bool b_colmajor,
                                          int bmask, int rb, int cp) {
  const int l = threadIdx.x & 63;
  const int i = 16 * rb + (l & 15);
  const int j0 = 32 * cp + (l & 15), j1 = j0 + 16;
  Gauss3<R> g;
  if constexpr (G3) g.zero();
#pragma unroll 1
  for (int kq = 0; kq < T / 4; kq += KQ) {
    cplx<R> a[KQ], b0[KQ], b1[KQ];
#pragma unroll
    for (int q = 0; q < KQ; q++) {
      const int k = 4 * (kq + q) + (l >> 4);
      a[q] = a_rowmajor ? A[i * lda + k] : A[k * lda + i];
      b0[q] = b_colmajor ? Bm[j0 * ldb + k] : Bm[k * ldb + j0];
      b1[q] = b_colmajor ? Bm[j1 * ldb + k] : Bm[k * ldb + j1];
    }
    if (amask != MK_NONE || bmask != MK_NONE) {
#pragma unroll
      for (int q = 0; q < KQ; q++) {
        const int k = 4 * (kq + q) + (l >> 4);
        a[q] = apply_mask(a[q], amask, i, k);
        b0[q] = apply_mask(b0[q], bmask, k, j0);
        b1[q] = apply_mask(b1[q], bmask, k, j1);
      }
    }
#pragma unroll
    for (int q = 0; q < KQ; q++) {
      if constexpr (G3) {
        g.mma(a[q], b0[q], 0);
        g.mma(a[q], b1[q], 1);
      } else {
        cmfma<R, false, SUB>(acc.re[0], acc.im[0], a[q], b0[q]);
        cmfma<R, false, SUB>(acc.re[1], acc.im[1], a[q], b1[q]);
      }
    }
  }
  if constexpr (G3) g.template add_to<SUB>(acc);
}

// The diagonal tiles are not in the ticket order: the first n_omega
// workgroups to start (a second counter) each own the diagonal chain of one
// shift and factor its diagonal tiles m = 0, 1, ... in turn, so a diagonal
// step starts the moment its inputs are final instead of when a workgroup
// frees up for its ticket.  Its inputs all come from earlier block steps of
// the ticket order (below), so a ticket task waiting on a diagonal tile
// cannot block it.
//
// Task decoding: slot -> (kind, r, t) for block step m.  Kinds: 0 = F,
// 1 = E (off-diagonal), 2 / 3 = the chain tiles of diagonal tile m (column /
// row side), 4 = E' and 5 = G of a diagonal tile.
//   slot 0: G(m+1, m+1) (it feeds the next diagonal tile)
//   slot 1: E'(m+2, m+2)
//   slots 2 .. 2B-3: E of the off-diagonal tiles finalised at step m+1
//     (distance <= B-2)
//   slots 2B-2, 2B-1: F(m+1, m), F(m, m+1)
//   slots 2B .. 4B-3: F at distance 2 .. B
//   slots 4B-2, 4B-1: the chain tiles of diagonal tile m
// (B = 1: F(m+1, m), F(m, m+1) and the two chain tasks.)
struct Task {
  int kind, r, t;
};
enum { TK_F = 0, TK_E = 1, TK_CHAIN_L = 2, TK_CHAIN_U = 3, TK_EDIAG = 4, TK_GDIAG = 5 };

__host__ __device__ inline int factor_slots(int B) { return B >= 2 ? 4 * B : 4; }

__host__ __device__ inline Task decode(int slot, int m, int B) {
  if (B < 2) {
    if (slot == 0) return {TK_F, m + 1, m};
    if (slot == 1) return {TK_F, m, m + 1};
    return {slot == 2 ? TK_CHAIN_L : TK_CHAIN_U, m, m};
  }
  if (slot == 0) return {TK_GDIAG, m + 1, m + 1};
  if (slot == 1) return {TK_EDIAG, m + 2, m + 2};
  if (slot < 2 * B - 2) {
    const int mm = m + 1, d = slot >> 1;  // slots 2d, 2d+1 hold distance d
    return (slot & 1) ? Task{TK_E, mm, mm + d} : Task{TK_E, mm + d, mm};
  }
  if (slot == 2 * B - 2) return {TK_F, m + 1, m};
  if (slot == 2 * B - 1) return {TK_F, m, m + 1};
  if (slot < 4 * B - 2) {
    const int f = slot - 2 * B, d = 2 + (f >> 1);
    return (f & 1) ? Task{TK_F, m, m + d} : Task{TK_F, m + d, m};
  }
  return {slot == 4 * B - 2 ? TK_CHAIN_L : TK_CHAIN_U, m, m};
}

// Update ranges s in [lo, hi] of the tasks of tile (r, t), m = min(r, t),
// mx = max(r, t): all of them together cover [max(0, mx - B), m - 1].
//   E (off-diagonal):  [max(0, mx - B), m - 2]
//   E' (diagonal):     [max(0, m - B), m - 3]
//   G (diagonal):      m - 2 alone, when in the band
// F and the diagonal worker take s = m - 1.
__host__ __device__ inline bool has_early(int r, int t, int B) {  // E or G
  int m = min(r, t), d = abs(r - t);
  return m >= 2 && d <= B - 2;
}
__host__ __device__ inline bool has_ediag(int m, int B) { return m >= 3 && B >= 3; }

// Test hook (host only): the factor launch's ticket tasks of one shift, in
// ticket order, as (kind, r, t) triples with the decoder above; tasks that
// fall outside the matrix or have no work are skipped, as the kernel skips
// them.  Writes at most `cap` triples and returns the count (or -1 if B or
// NB is not positive).
extern "C" int64_t rr_factor_schedule(int32_t B, int32_t NB, int32_t* out, int64_t cap) {
  if (B <= 0 || NB <= 0) return -1;
  const int slots = factor_slots(B);
  int64_t n = 0;
  for (int m = 0; m < NB; m++)
    for (int slot = 0; slot < slots; slot++) {
      const Task tk = decode(slot, m, B);
      if (tk.r < 0 || tk.r >= NB || tk.t >= NB) continue;
      if (tk.kind == TK_E && !has_early(tk.r, tk.t, B)) continue;
      if (tk.kind == TK_GDIAG && !has_early(tk.r, tk.r, B)) continue;
      if (tk.kind == TK_EDIAG && !has_ediag(tk.r, B)) continue;
      if ((tk.kind == TK_CHAIN_L || tk.kind == TK_CHAIN_U) && tk.r == 0) continue;
      if (n < cap) {
        out[3 * n] = tk.kind;
        out[3 * n + 1] = tk.r;
        out[3 * n + 2] = tk.t;
      }
      n++;
    }
  return n;
}

template <typename R, int T>
__device__ __forceinline__ cplx<R>* tile_ptr(const FactorParams& P, int w, int r, int t) {
  int64_t idx = ((int64_t)w * P.g.NB + r) * P.g.row_tiles() + (t - r + P.g.B);
  return reinterpret_cast<cplx<R>*>(P.tiles) + idx * (T * T);
}
// Chain tile `c` of block row s (CH_* below).
template <typename R, int T>
__device__ __forceinline__ cplx<R>* chain_ptr(const FactorParams& P, int w, int s, int c) {
  int64_t idx = ((int64_t)w * P.g.NB + s) * P.g.row_tiles() + 2 * P.g.B + 1 + c;
  return reinterpret_cast<cplx<R>*>(P.tiles) + idx * (T * T);
}
__device__ __forceinline__ int* flag_ptr(const FactorParams& P, int w, int r, int t) {
  const int W = 2 * P.g.B + 1;
  return P.flags + ((int64_t)w * P.g.NB + r) * W + (t - r + P.g.B);
}

// acc -= sum_{s = s0 .. s1} L_rs U_st for the tile (r, t), operands straight
// from global memory (L tiles column-major, U tiles row-major).  The KQ-step
// chunks of all the products form one sequence, loaded one chunk ahead of
// the MFMAs (two register buffers), so that only the first load's latency is
// exposed; the chunk count per product is even, so the loop needs no tail.
// G3: Gauss's three real MFMAs per complex product (the FP32 factor's early
// updates; the last update of every tile and the diagonal worker's keep four).
template <typename R, int T, int KQ>
struct UpdChunk {
  cplx<R> a[KQ], b0[KQ], b1[KQ];
};

template <typename R, int T, int KQ, bool G3 = false>
__device__ __forceinline__ void update_gemms(Acc2<R>& acc, const FactorParams& P, int w, int r,
                                             int t, int s0, int s1, int rb, int cp) {
  constexpr int NKC = T / 4 / KQ;  // chunks per product
  static_assert(NKC % 2 == 0, "even chunk count");
  const int N = (s1 - s0 + 1) * NKC;
  if (N <= 0) return;
  const int l = threadIdx.x & 63;
  const int i = 16 * rb + (l & 15), j0 = 32 * cp + (l & 15);
  auto load = [&](UpdChunk<R, T, KQ>& c, int idx) {
    const int s = s0 + idx / NKC, kq = (idx % NKC) * KQ;
    const cplx<R>* A = tile_ptr<R, T>(P, w, r, s);
    const cplx<R>* Bm = tile_ptr<R, T>(P, w, s, t);
#pragma unroll
    for (int q = 0; q < KQ; q++) {
      const int k = 4 * (kq + q) + (l >> 4);
      c.a[q] = A[k * T + i];
      c.b0[q] = Bm[k * T + j0];
      c.b1[q] = Bm[k * T + j0 + 16];
    }
  };
  Gauss3<R> g;
  if constexpr (G3) g.zero();
  auto mma = [&](const UpdChunk<R, T, KQ>& c) {
#pragma unroll
    for (int q = 0; q < KQ; q++) {
      if constexpr (G3) {
        g.mma(c.a[q], c.b0[q], 0);
        g.mma(c.a[q], c.b1[q], 1);
      } else {
        cmfma<R, false, true>(acc.re[0], acc.im[0], c.a[q], c.b0[q]);
        cmfma<R, false, true>(acc.re[1], acc.im[1], c.a[q], c.b1[q]);
      }
    }
  };
  UpdChunk<R, T, KQ> c0, c1;
  load(c0, 0);
#pragma unroll 1
  for (int idx = 0; idx < N; idx += 2) {
    load(c1, idx + 1);
    mma(c0);
    load(c0, min(idx + 2, N - 1));  // the last one reloads a chunk (unused)
    mma(c1);
  }
  if constexpr (G3) g.template add_to<true>(acc);
}

// Tile flags.  Off-diagonal: 1 = partial (E done), 3 = final.  Diagonal:
// 1 = E' done, 2 = G done, 3 = block-inverse LU published, 4 = [U^-1 | L^-1]
// published (only when chain tiles are formed).
enum { FL_PARTIAL = 1, FL_PARTIAL2 = 2, FL_FINAL = 3, FL_DIAG_INV = 4 };

// Wave 0 polls one optional flag (to extra_want) and the flags of tiles
// (r, s) and (s, t), s in [s0, s1] (to FL_FINAL), one flag per lane so that
// the round trips of the atomic polls overlap (lane q takes flags q, q + 64,
// ...), then lane 0 issues one acquire fence and the barrier hands the result
// to every wave.
__device__ __forceinline__ void wait_inputs(const FactorParams& P, int w, int r, int t, int s0,
                                            int s1, int* extra, int extra_want) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int nq = 1 + 2 * max(0, s1 - s0 + 1);  // q = 0: extra, then (r, s), (s, t) pairs
    bool live =
        !(__hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_TIMEOUT);
    uint64_t t0 = wall_clock64();
    uint32_t polls = 0;
    for (int q0 = 0; q0 < nq; q0 += 64) {
      const int q = q0 + lane;
      int* f = nullptr;
      int want = FL_FINAL;
      if (q == 0) {
        f = extra;
        want = extra_want;
      } else if (q < nq) {
        const int s = s0 + ((q - 1) >> 1);
        f = ((q - 1) & 1) ? flag_ptr(P, w, s, t) : flag_ptr(P, w, r, s);
      }
      bool done = f == nullptr;
      for (;;) {
        if (!done)
          done = __hip_atomic_fetch_add(f, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want;
        if (__all(done) || !live) break;
        __builtin_amdgcn_s_sleep(1);
        if (++polls > kWaitPolls || wall_clock64() - t0 > kWaitTicks) {
          if (lane == 0) latch(P.status, ST_TIMEOUT);
          live = false;
        }
      }
    }
    if (lane == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Every thread's stores are complete, then thread 0 releases and sets the
// flag; barriers close the interval on both sides.  Everything a task hands
// over is stored device-coherent (written through), so the stores' completion
// is the whole release: no L2 write-back precedes the flag, and the release
// fence is at workgroup scope.
__device__ __forceinline__ void publish(int* flag, int value) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

template <typename R, int T>
__device__ __forceinline__ void acc_to_lds(const Acc2<R>& acc, cplx<R>* lds, bool rowmajor, int rb,
                                           int cp) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int b = 0; b < 2; b++) {
    const int c = 32 * cp + 16 * b + (l & 15);
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int rr = 16 * rb + Mf<R>::row(l, e);
      lds[rowmajor ? rr * FGeom<T>::LDT + c : c * FGeom<T>::LDT + rr] =
          cplx<R>{acc.re[b][e], acc.im[b][e]};
    }
  }
}

// Copy of the T x T tile held column-major in LDS (leading dimension LDT) to
// the stored tile X (column-major, or row-major when rowmajor): consecutive
// threads write consecutive 8-byte words, so every store instruction covers
// whole cache lines.  CO: device-coherent stores (written through), for
// tiles other workgroups of the launch read; the kernels after the
// factorisation, whose tiles only the same workgroup or later launches
// read, store plainly and keep them in the L2.
template <typename R, int T, bool CO = true>
__device__ __forceinline__ void lds_to_tile(const cplx<R>* S, cplx<R>* X, bool rowmajor) {
  typedef FGeom<T> G;
  constexpr int WPE = sizeof(cplx<R>) / 8;  // 8-byte words per element
  constexpr int N = T * T * WPE / G::NT;
#pragma unroll 4
  for (int q = 0; q < N; q++) {
    const int wi = threadIdx.x + q * G::NT;
    const int idx = wi / WPE, o = idx / T, i = idx % T;
    const int e = rowmajor ? i * G::LDT + o : o * G::LDT + i;
    if constexpr (!CO) {
      if constexpr (WPE == 2)
        reinterpret_cast<double*>(X)[wi] = reinterpret_cast<const double*>(S)[2 * e + (wi & 1)];
      else
        X[idx] = S[e];
    } else if constexpr (WPE == 2) {
      const double v = reinterpret_cast<const double*>(S)[2 * e + (wi & 1)];
      __hip_atomic_store(reinterpret_cast<double*>(X) + wi, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      st_coherent(&X[idx], S[e]);
    }
  }
}

// The column-major stored tile X into LDS (column-major, leading dimension LDT).
template <typename R, int T>
__device__ __forceinline__ void tile_to_lds(const cplx<R>* X, cplx<R>* S) {
  typedef FGeom<T> G;
#pragma unroll
  for (int q = 0; q < T * T / G::NT; q++) {
    const int idx = threadIdx.x + q * G::NT;
    S[(idx / T) * G::LDT + idx % T] = X[idx];
  }
}

// acc -> stored tile X through the LDS staging area `stage` (T x LDT).
template <typename R, int T, bool CO = true>
__device__ __forceinline__ void stage_store(const Acc2<R>& acc, cplx<R>* stage, cplx<R>* X,
                                            bool rowmajor, int rb, int cp) {
  __syncthreads();  // earlier readers of the staging area are done
  acc_to_lds<R, T>(acc, stage, false, rb, cp);
  __syncthreads();
  lds_to_tile<R, T, CO>(stage, X, rowmajor);
}

// Block-inverse LU of diagonal tile s (lu_blockinv), kept beside the chain tiles.
template <typename R, int T>
__device__ __forceinline__ cplx<R>* lub_ptr(const FactorParams& P, int w, int s) {
  int64_t idx = ((int64_t)w * P.g.NB + s) * P.g.row_tiles() + P.g.lub_index();
  return reinterpret_cast<cplx<R>*>(P.tiles) + idx * (T * T);
}


// The tile (r, t) into the accumulators: the partial whose flag reaches
// `partial` (> 0), or the tile of M generated from the stencil (0).
template <typename R, int T>
__device__ __forceinline__ void load_tile(const FactorParams& P, Acc2<R>& acc, int w, int r,
                                          int t, int partial, int rb, int cp) {
  const int l = threadIdx.x & 63;
  const bool rowmajor = r < t;
  if (partial > 0) {
    const cplx<R>* X = tile_ptr<R, T>(P, w, r, t);
    wait_inputs(P, w, r, t, 0, -1, flag_ptr(P, w, r, t), partial);
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int c = 32 * cp + 16 * b + (l & 15);
#pragma unroll
      for (int e = 0; e < 4; e++) {
        cplx<R> v = X[tix(16 * rb + Mf<R>::row(l, e), c, T, rowmajor)];
        acc.re[b][e] = v.re;
        acc.im[b][e] = v.im;
      }
    }
  } else {
    const double om_r = P.omega[2 * w], om_i = P.omega[2 * w + 1];
#pragma unroll
    for (int b = 0; b < 2; b++) {
      const int c = 32 * cp + 16 * b + (l & 15);
#pragma unroll
      for (int e = 0; e < 4; e++) {
        double2 v = m_entry(P.op, om_r, om_i, (int64_t)r * T + 16 * rb + Mf<R>::row(l, e),
                            (int64_t)t * T + c);
        acc.re[b][e] = (R)v.x;
        acc.im[b][e] = (R)v.y;
      }
    }
  }
}

template <typename R, int T>
__global__ __launch_bounds__(FGeom<T>::NT) void k_factor(FactorParams P) {
  typedef FGeom<T> G;
  constexpr int KQ = sizeof(R) == 8 ? 4 : 8;
  constexpr int KU = (T / 4) / KQ >= 2 ? KQ : KQ / 2;  // update chunks: an even count
  extern __shared__ __align__(16) char smem_raw[];
  cplx<R>* lds = reinterpret_cast<cplx<R>*>(smem_raw);  // T x LDT: the task's tile
  cplx<R>* aux = lds + T * G::LDT;  // T x LDT: staging, the block-inverse LU, scratch
  __shared__ uint32_t s_ticket;
  const int B = P.g.B, NB = P.g.NB;
  const int wave = threadIdx.x >> 6;
  const int rb = wave / G::CPR, cp = wave % G::CPR;
  Acc2<R> acc;

  // diagonal worker of shift w: F(m, m) for m = 0 .. NB-1
  const int64_t role = wg_ticket(P.ticket + 1, &s_ticket);
  if (role < P.n_omega) {
    const int w = (int)role;
#pragma unroll 1
    for (int m = 0; m < NB; m++) {
      cplx<R>* X = tile_ptr<R, T>(P, w, m, m);
      int* dflag = flag_ptr(P, w, m, m);
      load_tile<R, T>(P, acc, w, m, m, has_early(m, m, B) ? FL_PARTIAL2 : 0, rb, cp);
      if (m >= 1) wait_inputs(P, w, m, m, m - 1, m - 1, nullptr, FL_FINAL);
      update_gemms<R, T, KU>(acc, P, w, m, m, max(0, m - 1), m - 1, rb, cp);
      acc_to_lds<R, T>(acc, lds, false, rb, cp);
      __syncthreads();
      // LU with inverted diagonal blocks: published first (the step's other
      // finalisations wait on it), then the full inverses
      lu_blockinv<R, T, G::NW>(lds, G::LDT, P.status);
      lds_to_tile<R, T>(lds, lub_ptr<R, T>(P, w, m), false);
      publish(dflag, FL_FINAL);
      if (P.g.P > 0) continue;  // the full inverse follows in k_diaginv
      inv_doubling<R, T, G::NW>(lds, G::LDT, aux);
      lds_to_tile<R, T>(lds, X, false);
      publish(dflag, FL_DIAG_INV);
    }
    return;
  }

  for (;;) {
    const int64_t ticket = wg_ticket(P.ticket, &s_ticket);
    if (ticket >= P.total) break;
    const int w = (int)(ticket % P.n_omega);
    const int64_t task = ticket / P.n_omega;
    const int m0 = (int)(task / P.slots), slot = (int)(task % P.slots);
    const Task tk = decode(slot, m0, B);
    const int r = tk.r, t = tk.t;
    if (r < 0 || r >= NB || t >= NB) continue;
    const int m = min(r, t), mx = max(r, t);
    int* dflag = flag_ptr(P, w, m, m);
    if (tk.kind == TK_CHAIN_L || tk.kind == TK_CHAIN_U) {
      // chain tiles of diagonal tile m: L_mm^-1 L_m,m-dd (kind 2) or
      // U_m-dd,m U_mm^-1 (kind 3), dd = 1 .. kChainD, with D_m in LDS; only
      // the tile-by-tile solve reads them
      if (m == 0 || P.g.P > 0) continue;
      wait_inputs(P, w, m, m, 0, -1, dflag, FL_DIAG_INV);
      tile_to_lds<R, T>(tile_ptr<R, T>(P, w, m, m), lds);
      __syncthreads();
      for (int dd = 1; dd <= BandGeom::kChainD && dd <= B && m - dd >= 0; dd++) {
        acc.zero();
        if (tk.kind == TK_CHAIN_L) {
          tile_gemm<R, T, KQ, false>(acc, lds, G::LDT, false, MK_UNIT_LOWER,
                                     tile_ptr<R, T>(P, w, m, m - dd), T, true, MK_NONE, rb, cp);
          stage_store<R, T>(acc, aux, chain_ptr<R, T>(P, w, m, chain_index(CH_FWD_L, dd)),
                            false, rb, cp);
        } else {
          tile_gemm<R, T, KQ, false>(acc, tile_ptr<R, T>(P, w, m - dd, m), T, true, MK_NONE, lds,
                                     G::LDT, true, MK_UPPER, rb, cp);
          stage_store<R, T>(acc, aux, chain_ptr<R, T>(P, w, m, chain_index(CH_ADJ_U, dd)), true,
                            rb, cp);
        }
      }
      continue;
    }
    const bool early = tk.kind != TK_F;  // E, E' or G: a partial tile
    if (tk.kind == TK_E && !has_early(r, t, B)) continue;
    if (tk.kind == TK_GDIAG && !has_early(r, t, B)) continue;
    if (tk.kind == TK_EDIAG && !has_ediag(m, B)) continue;
    const bool rowmajor = r < t;  // U tiles
    cplx<R>* X = tile_ptr<R, T>(P, w, r, t);
    // 1. the tile: E and E' start from the stencil, G from E' (if any), F
    // from E (if any); 2. their updates A_rt -= L_rs U_st over the ranges
    // above (F: s = m-1, whose inputs are final a block step before tile m)
    int partial = 0, s_lo, s_hi, done = FL_PARTIAL;
    if (tk.kind == TK_E) {
      s_lo = max(0, mx - B);
      s_hi = m - 2;
    } else if (tk.kind == TK_EDIAG) {
      s_lo = max(0, m - B);
      s_hi = m - 3;
    } else if (tk.kind == TK_GDIAG) {
      partial = has_ediag(m, B) ? FL_PARTIAL : 0;
      s_lo = s_hi = m - 2;
      done = FL_PARTIAL2;
    } else {
      partial = has_early(r, t, B) ? FL_PARTIAL : 0;
      s_lo = max(max(0, mx - B), m - 1);
      s_hi = m - 1;
    }
    load_tile<R, T>(P, acc, w, r, t, partial, rb, cp);
    if (s_lo <= s_hi) wait_inputs(P, w, r, t, s_lo, s_hi, nullptr, FL_FINAL);
    if (sizeof(R) == 4 && early)  // FP32 early updates: Gauss products
      update_gemms<R, T, KU, true>(acc, P, w, r, t, s_lo, s_hi, rb, cp);
    else
      update_gemms<R, T, KU>(acc, P, w, r, t, s_lo, s_hi, rb, cp);
    acc_to_lds<R, T>(acc, lds, false, rb, cp);  // column-major in every case
    if (early) {
      __syncthreads();
      lds_to_tile<R, T>(lds, X, rowmajor);
      publish(flag_ptr(P, w, r, t), done);
      continue;
    }
    // 3. finalise: a triangular solve with the block-inverse LU of tile m
    const int d = mx - m;
    wait_inputs(P, w, r, t, 0, -1, dflag, FL_FINAL);  // its barrier also covers acc_to_lds
    tile_to_lds<R, T>(lub_ptr<R, T>(P, w, m), aux);
    __syncthreads();
    if (r > t)
      trsm_right_upper<R, T>(lds, G::LDT, aux, G::LDT);  // L_rm = A_rm U_mm^-1
    else
      trsm_left_lower<R, T>(lds, G::LDT, aux, G::LDT);   // U_mt = L_mm^-1 A_mt
    __syncthreads();
    lds_to_tile<R, T>(lds, X, rowmajor);
    publish(flag_ptr(P, w, r, t), FL_FINAL);
    if (d > BandGeom::kChainD || P.g.P > 0) continue;
    // 4. chain tile with the full inverse D of tile m (the new tile is in LDS)
    const cplx<R>* D = tile_ptr<R, T>(P, w, m, m);
    wait_inputs(P, w, r, t, 0, -1, dflag, FL_DIAG_INV);
    acc.zero();
    if (r > t) {  // L_m+d,m L_mm^-1
      tile_gemm<R, T, KQ, false>(acc, lds, G::LDT, false, MK_NONE, D, T, true, MK_UNIT_LOWER, rb,
                                 cp);
      stage_store<R, T>(acc, aux, chain_ptr<R, T>(P, w, m, chain_index(CH_ADJ_L, d)), true, rb,
                        cp);
    } else {      // U_mm^-1 U_m,m+d
      tile_gemm<R, T, KQ, false>(acc, D, T, false, MK_UPPER, lds, G::LDT, true, MK_NONE, rb, cp);
      stage_store<R, T>(acc, aux, chain_ptr<R, T>(P, w, m, chain_index(CH_FWD_U, d)), false, rb,
                        cp);
    }
  }
}

// Full inverses [U^-1 | L^-1] of the diagonal tiles from their published
// block-inverse LUs (inv_doubling), one workgroup per (shift, block row),
// after the factorisation: the superblock solve's diagonal blocks.
template <typename R, int T>
__global__ __launch_bounds__(FGeom<T>::NT) void k_diaginv(FactorParams P) {
  typedef FGeom<T> G;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<R>* lds = reinterpret_cast<cplx<R>*>(smem_raw);  // T x LDT
  cplx<R>* aux = lds + T * G::LDT;
  const int64_t id = blockIdx.x;
  const int m = (int)(id % P.g.NB), w = (int)(id / P.g.NB);
  tile_to_lds<R, T>(lub_ptr<R, T>(P, w, m), lds);
  __syncthreads();
  inv_doubling<R, T, G::NW>(lds, G::LDT, aux);
  lds_to_tile<R, T, false>(lds, tile_ptr<R, T>(P, w, m, m), false);
}

// Tile `slot` of block row r's superblock-inverse area (BandGeom::sb_slot).
template <typename R, int T>
__device__ __forceinline__ cplx<R>* sb_ptr(const FactorParams& P, int w, int r, int slot) {
  int64_t idx = ((int64_t)w * P.g.NB + r) * P.g.row_tiles() + P.g.sb_index(slot);
  return reinterpret_cast<cplx<R>*>(P.tiles) + idx * (T * T);
}

// acc += sum_{l = lo .. hi} A_il X_lj for the superblock inverse's block
// substitution (k_sbinv): A_il the factor's tile (s0+i, s0+l) (L column-major,
// or U row-major when upper), X_lj the inverse's tile already formed (stored
// column-major, or row-major when upper).  The KQ-step chunks of all the
// products form one sequence loaded a chunk ahead of the MFMAs.
template <typename R, int T, int KQ, bool G3>
__device__ __forceinline__ void sb_chain(Acc2<R>& acc, const FactorParams& P, int w, int s0, int i,
                                         int lo, int hi, int j, bool upper, int rb, int cp) {
  constexpr int NKC = T / 4 / KQ;  // chunks per product
  static_assert(NKC % 2 == 0, "even chunk count");
  const int N = (hi - lo + 1) * NKC;
  if (N <= 0) return;
  const int l = threadIdx.x & 63;
  const int ii = 16 * rb + (l & 15), j0 = 32 * cp + (l & 15), j1 = j0 + 16;
  Gauss3<R> g;
  if constexpr (G3) g.zero();
  auto load = [&](UpdChunk<R, T, KQ>& c, int idx) {
    const int ll = lo + idx / NKC, kq = (idx % NKC) * KQ;
    const cplx<R>* A = tile_ptr<R, T>(P, w, s0 + i, s0 + ll);
    const cplx<R>* X = sb_ptr<R, T>(P, w, s0 + ll, sb_slot(ll, j));
#pragma unroll
    for (int q = 0; q < KQ; q++) {
      const int k = 4 * (kq + q) + (l >> 4);
      c.a[q] = upper ? A[ii * T + k] : A[k * T + ii];
      c.b0[q] = upper ? X[k * T + j0] : X[j0 * T + k];
      c.b1[q] = upper ? X[k * T + j1] : X[j1 * T + k];
    }
  };
  auto mma = [&](const UpdChunk<R, T, KQ>& c) {
#pragma unroll
    for (int q = 0; q < KQ; q++) {
      if constexpr (G3) {
        g.mma(c.a[q], c.b0[q], 0);
        g.mma(c.a[q], c.b1[q], 1);
      } else {
        cmfma<R, false, false>(acc.re[0], acc.im[0], c.a[q], c.b0[q]);
        cmfma<R, false, false>(acc.re[1], acc.im[1], c.a[q], c.b1[q]);
      }
    }
  };
  UpdChunk<R, T, KQ> c0, c1;
  load(c0, 0);
#pragma unroll 1
  for (int idx = 0; idx < N; idx += 2) {
    load(c1, idx + 1);
    mma(c0);
    load(c0, min(idx + 2, N - 1));  // the last one reloads a chunk (unused)
    mma(c1);
  }
  if constexpr (G3) g.template add_to<false>(acc);
}

// Off-diagonal tiles of the inverses of each superblock's diagonal block (the
// block triangles L-hat and U-hat of P block rows), after the factorisation:
//   L-hat^-1:  X_jj = L_jj^-1,  X_ij = -L_ii^-1 sum_{l=j}^{i-1} L_il X_lj   (i > j)
//   U-hat^-1:  X_jj = U_jj^-1,  X_ij = -U_ii^-1 sum_{l=i+1}^{j} U_il X_lj   (i < j)
// (block forward / back substitution on the identity).  One workgroup per
// (shift, superblock, triangle, column j) walks its column outward from the
// diagonal; each tile it writes is read back by the later ones after a
// barrier (same workgroup, same CU).  Products are T x T tile GEMMs on MFMA
// with operands from memory (the ones with formed inverse tiles in one
// pipelined sequence, sb_chain); the sum is staged in LDS for the product
// with the diagonal inverse.  In FP32 the complex products are Gauss's three
// real MFMAs: these inverses only serve the superblock solves, whose FP32
// errors the FP64-residual refinement removes (the factor itself, which is
// also the GMRES-IR preconditioner, keeps four).
template <typename R, int T>
__global__ __launch_bounds__(FGeom<T>::NT) void k_sbinv(FactorParams P) {
  typedef FGeom<T> G;
  constexpr int KQ = sizeof(R) == 8 ? 4 : 8;
  constexpr bool G3 = sizeof(R) == 4;    // Gauss products in FP32
  // FP32: sb_chain; FP64 loads each product's chunks in turn (a second
  // chunk buffer would cost the FP64 kernel its second workgroup per CU)
  constexpr bool PIPE = sizeof(R) == 4;
  constexpr int KS = PIPE ? KQ / 2 : KQ;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<R>* sacc = reinterpret_cast<cplx<R>*>(smem_raw);  // T x LDT, column-major
  cplx<R>* stage = sacc + T * G::LDT;
  const int PS = P.g.P, NB = P.g.NB, NS = P.g.NS(), B = P.g.B;
  const int wave = threadIdx.x >> 6;
  const int rb = wave / G::CPR, cp = wave % G::CPR;
  int64_t id = blockIdx.x;
  const int c = (int)(id % (PS - 1));
  id /= PS - 1;
  const int upper = (int)(id % 2);
  id /= 2;
  const int S = (int)(id % NS), w = (int)(id / NS);
  const int s0 = S * PS;
  Acc2<R> acc;
  if (!upper) {
    const int j = c;
    if (s0 + j >= NB) return;
    const cplx<R>* Djj = tile_ptr<R, T>(P, w, s0 + j, s0 + j);
    for (int i = j + 1; i < PS && s0 + i < NB; i++) {
      acc.zero();
      if constexpr (PIPE) {
        if (i - j <= B)  // L_ij X_jj, X_jj = L_jj^-1 (outside the band L_il = 0)
          tile_gemm<R, T, KQ, false, G3>(acc, tile_ptr<R, T>(P, w, s0 + i, s0 + j), T, false,
                                         MK_NONE, Djj, T, true, MK_UNIT_LOWER, rb, cp);
        sb_chain<R, T, KS, G3>(acc, P, w, s0, i, max(j + 1, i - B), i - 1, j, false, rb, cp);
      } else {
        for (int l = j; l < i; l++) {
          if (i - l > B) continue;  // outside the band: L_il = 0
          const cplx<R>* X = l == j ? Djj : sb_ptr<R, T>(P, w, s0 + l, sb_slot(l, j));
          tile_gemm<R, T, KQ, false>(acc, tile_ptr<R, T>(P, w, s0 + i, s0 + l), T, false, MK_NONE,
                                     X, T, true, l == j ? MK_UNIT_LOWER : MK_NONE, rb, cp);
        }
      }
      __syncthreads();
      acc_to_lds<R, T>(acc, sacc, false, rb, cp);
      __syncthreads();
      acc.zero();
      tile_gemm<R, T, KQ, true, G3>(acc, tile_ptr<R, T>(P, w, s0 + i, s0 + i), T, false,
                                    MK_UNIT_LOWER, sacc, G::LDT, true, MK_NONE, rb, cp);
      stage_store<R, T, false>(acc, stage, sb_ptr<R, T>(P, w, s0 + i, sb_slot(i, j)), false, rb,
                               cp);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  } else {
    const int j = c + 1;
    if (s0 + j >= NB) return;
    const cplx<R>* Djj = tile_ptr<R, T>(P, w, s0 + j, s0 + j);
    for (int i = j - 1; i >= 0; i--) {
      acc.zero();
      if constexpr (PIPE) {
        sb_chain<R, T, KS, G3>(acc, P, w, s0, i, i + 1, min(j - 1, i + B), j, true, rb, cp);
        if (j - i <= B)  // U_ij X_jj, X_jj = U_jj^-1 (outside the band U_il = 0)
          tile_gemm<R, T, KQ, false, G3>(acc, tile_ptr<R, T>(P, w, s0 + i, s0 + j), T, true,
                                         MK_NONE, Djj, T, true, MK_UPPER, rb, cp);
      } else {
        for (int l = i + 1; l <= j; l++) {
          if (l - i > B) continue;  // outside the band: U_il = 0
          const cplx<R>* X = l == j ? Djj : sb_ptr<R, T>(P, w, s0 + l, sb_slot(l, j));
          tile_gemm<R, T, KQ, false>(acc, tile_ptr<R, T>(P, w, s0 + i, s0 + l), T, true, MK_NONE,
                                     X, T, l == j, l == j ? MK_UPPER : MK_NONE, rb, cp);
        }
      }
      __syncthreads();
      acc_to_lds<R, T>(acc, sacc, false, rb, cp);
      __syncthreads();
      acc.zero();
      tile_gemm<R, T, KQ, true, G3>(acc, tile_ptr<R, T>(P, w, s0 + i, s0 + i), T, false, MK_UPPER,
                                    sacc, G::LDT, true, MK_NONE, rb, cp);
      stage_store<R, T, false>(acc, stage, sb_ptr<R, T>(P, w, s0 + i, sb_slot(i, j)), true, rb,
                               cp);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }
}

template <typename R, int T>
constexpr size_t factor_lds() {
  return sizeof(cplx<R>) * 2 * (size_t)T * FGeom<T>::LDT;
}

template <typename R, int T>
static hipError_t launch_factor_t(const FactorParams& P, int grid, hipStream_t s,
                                  const hipEvent_t* ev) {
  const size_t lds = factor_lds<R, T>();
  if (ev && ev[0]) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL((k_factor<R, T>), dim3(grid), dim3(FGeom<T>::NT), lds, s, P);
  if (ev && ev[1]) (void)hipEventRecord(ev[1], s);
  if (P.g.P > 0)  // the diagonal tiles' full inverses
    hipLaunchKernelGGL((k_diaginv<R, T>), dim3((unsigned)((int64_t)P.n_omega * P.g.NB)),
                       dim3(FGeom<T>::NT), lds, s, P);
  if (P.g.P > 1) {  // the superblocks' diagonal inverses, for the superblock solve
    const int64_t nblk = (int64_t)P.n_omega * P.g.NS() * 2 * (P.g.P - 1);
    hipLaunchKernelGGL((k_sbinv<R, T>), dim3((unsigned)nblk), dim3(FGeom<T>::NT), lds, s, P);
  }
  return hipGetLastError();
}

// Dynamic-LDS limit of the factor kernel (a host call, kept out of the launch
// path so that launches can be captured into a graph).
hipError_t prepare_factor(int T, bool fp32) {
  auto set = [](const void* fn, size_t lds) {
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  };
  hipError_t e = hipErrorInvalidValue;
  if (fp32) {
    if (T == 64) {
      e = set((const void*)k_factor<float, 64>, factor_lds<float, 64>());
      if (e == hipSuccess) e = set((const void*)k_sbinv<float, 64>, factor_lds<float, 64>());
      if (e == hipSuccess) e = set((const void*)k_diaginv<float, 64>, factor_lds<float, 64>());
    } else if (T == 32) {
      e = set((const void*)k_factor<float, 32>, factor_lds<float, 32>());
      if (e == hipSuccess) e = set((const void*)k_sbinv<float, 32>, factor_lds<float, 32>());
      if (e == hipSuccess) e = set((const void*)k_diaginv<float, 32>, factor_lds<float, 32>());
    }
  } else {
    if (T == 64) {
      e = set((const void*)k_factor<double, 64>, factor_lds<double, 64>());
      if (e == hipSuccess) e = set((const void*)k_sbinv<double, 64>, factor_lds<double, 64>());
      if (e == hipSuccess) e = set((const void*)k_diaginv<double, 64>, factor_lds<double, 64>());
    } else if (T == 32) {
      e = set((const void*)k_factor<double, 32>, factor_lds<double, 32>());
      if (e == hipSuccess) e = set((const void*)k_sbinv<double, 32>, factor_lds<double, 32>());
      if (e == hipSuccess) e = set((const void*)k_diaginv<double, 32>, factor_lds<double, 32>());
    }
  }
  return e;
}

// Shifts per launch: every shift of a launch holds one diagonal worker for the
// whole launch, so their number stays well below the resident workgroups (one
// per CU) and more shifts are factored by consecutive launches.
constexpr int kMaxShiftsPerLaunch = 64;

hipError_t launch_factor(const OpDesc& op, const BandGeom& g, const double* omega, int n_omega,
                         bool fp32, void* tiles, int* flags, uint32_t* counters,
                         uint32_t* status, int grid, hipStream_t s, const hipEvent_t* ev) {
  const int slots = factor_slots(g.B);
  const size_t tile_bytes = (size_t)g.T * g.T * (fp32 ? 8 : 16);
  hipError_t e = launch_fill_u32((uint32_t*)flags, 0u, (int64_t)n_omega * g.tiles_per_omega(), s);
  for (int w0 = 0; e == hipSuccess && w0 < n_omega; w0 += kMaxShiftsPerLaunch) {
    const int nw = n_omega - w0 < kMaxShiftsPerLaunch ? n_omega - w0 : kMaxShiftsPerLaunch;
    FactorParams P{op, g, omega + 2 * w0, nw,
                   static_cast<char*>(tiles) + (size_t)w0 * g.tiles_per_omega() * tile_bytes,
                   flags + (size_t)w0 * g.NB * (2 * g.B + 1), counters, status, slots,
                   (int64_t)nw * g.NB * slots};
    e = launch_fill_u32(counters, 0u, 2, s);  // tickets and worker roles
    if (e != hipSuccess) break;
    int gr = grid > P.total ? (int)P.total : grid;
    gr += nw;  // the diagonal workers
    if (fp32) {
      if (g.T == 64) e = launch_factor_t<float, 64>(P, gr, s, w0 == 0 ? ev : nullptr);
      else if (g.T == 32) e = launch_factor_t<float, 32>(P, gr, s, w0 == 0 ? ev : nullptr);
      else e = hipErrorInvalidValue;
    } else {
      if (g.T == 64) e = launch_factor_t<double, 64>(P, gr, s, w0 == 0 ? ev : nullptr);
      else if (g.T == 32) e = launch_factor_t<double, 32>(P, gr, s, w0 == 0 ? ev : nullptr);
      else e = hipErrorInvalidValue;
    }
  }
  return e;
}

}  // namespace rr
