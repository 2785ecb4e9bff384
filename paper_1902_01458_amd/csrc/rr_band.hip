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
// The diagonal tile is stored as [U_mm^-1 (upper, diagonal included) |
// L_mm^-1 (strictly lower, unit diagonal implied)], so the solves and the
// off-diagonal finalisations are GEMMs too.
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
//   F(r, t)  the last update s = m-1 and the finalisation (flag 2)
// so the chain from one diagonal block to the next carries one update GEMM,
// one finalisation GEMM and one T x T LU.  The tile of M itself is generated
// from the stencil in registers: the band is never read before it is final.
// Every tile store is device-coherent (st_coherent): a tile is written twice
// per launch, from different XCDs in general, and read from others.
//
// Chain tiles.  In each sweep of a solve, block s depends on the blocks t
// within B of it through x_s = D^-1 (b_s - sum_t T_st x_t), D^-1 a triangle of
// the diagonal inverse.  For the two nearest neighbours (distance d = 1, 2)
// the factorisation stores the products G_s,d = D^-1 T_s,s-+d, so that a solve
// step applies D^-1 to the far terms three or more blocks back, before either
// neighbour is ready, and the two products left after that are register MFMAs
// with no LDS round trip:  x_s = D^-1 (b_s - sum_far) - G_s,2 x_s-+2 - G_s,1 x_s-+1.
//   CH_FWD_L,d = L_ss^-1 L_s,s-d   (column-major)   forward, L sweep
//   CH_FWD_U,d = U_ss^-1 U_s,s+d   (column-major)   forward, U sweep
//   CH_ADJ_U,d = U_s-d,s U_ss^-1   (row-major)      adjoint, U^H sweep (used as ^H)
//   CH_ADJ_L,d = L_s+d,s L_ss^-1   (row-major)      adjoint, L^H sweep (used as ^H)
// F(s, s) forms CH_FWD_L and CH_ADJ_U after publishing D_s; F(s+d, s) and
// F(s, s+d) form CH_ADJ_L,d and CH_FWD_U,d after publishing their tile.
// Nothing in the launch waits on chain tiles.
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
  uint32_t* ticket;
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

// In-LDS no-pivot LU of the T x T tile S (column-major, leading dimension
// LD), then in-place inversion of both triangles:
//   S <- [U^-1 on and above the diagonal | L^-1 strictly below].
template <typename R, int T, int NT>
__device__ void lu_inv_tile(cplx<R>* S, int LD, cplx<R>* tmpL, cplx<R>* tmpU, uint32_t* status) {
  auto at = [&](int i, int j) -> cplx<R>& { return S[j * LD + i]; };
  for (int j = 0; j < T; j++) {
    cplx<R> piv = at(j, j);
    R mag = piv.re * piv.re + piv.im * piv.im;
    bool bad = !(mag > (R)0) || !isfinite(mag);
    if (bad) {
      if (threadIdx.x == 0) latch(status, ST_SINGULAR);
      piv = cplx<R>{(R)1, (R)0};
    }
    cplx<R> ip = cinv(piv);
    __syncthreads();
    if (bad && threadIdx.x == 0) at(j, j) = piv;
    for (int i = j + 1 + threadIdx.x; i < T; i += NT) at(i, j) = cmul(at(i, j), ip);
    __syncthreads();
    int w = T - 1 - j;
    for (int idx = threadIdx.x; idx < w * w; idx += NT) {
      int i = j + 1 + idx % w, c = j + 1 + idx / w;
      cplx<R> l = at(i, j), u = at(j, c), x = at(i, c);
      x.re -= l.re * u.re - l.im * u.im;
      x.im -= l.re * u.im + l.im * u.re;
      at(i, c) = x;
    }
    __syncthreads();
  }
  // L^-1 (ascending j) and U^-1 (descending jj = T-1-j) touch disjoint
  // triangles, so both advance in the same loop.
  for (int j = 0; j < T; j++) {
    int jj = T - 1 - j;
    cplx<R> iu = cinv(at(jj, jj));
    for (int i = threadIdx.x; i < T; i += NT) {
      if (i > j) tmpL[i] = at(i, j);      // multipliers L[i][j]
      if (i < jj) tmpU[i] = at(i, jj);    // multipliers U[i][jj]
    }
    __syncthreads();
    // U: finalise row jj: X[jj][c] = acc[jj][c] / U[jj][jj]
    for (int c = jj + 1 + threadIdx.x; c < T; c += NT) at(jj, c) = cmul(at(jj, c), iu);
    if (threadIdx.x == 0) at(jj, jj) = iu;
    __syncthreads();
    // L: rows i > j, columns c <= j:  X[i][c] -= L[i][j] X[j][c]  (X[j][j] = 1)
    int wl = T - 1 - j, hl = j + 1;
    for (int idx = threadIdx.x; idx < wl * hl; idx += NT) {
      int i = j + 1 + idx % wl, c = idx / wl;
      cplx<R> m = tmpL[i];
      cplx<R> xj = (c == j) ? cplx<R>{(R)1, (R)0} : at(j, c);
      cplx<R> x = (c == j) ? cplx<R>{(R)0, (R)0} : at(i, c);
      x.re -= m.re * xj.re - m.im * xj.im;
      x.im -= m.re * xj.im + m.im * xj.re;
      at(i, c) = x;
    }
    // U: rows i < jj, columns c >= jj:  acc[i][c] -= U[i][jj] X[jj][c]
    int hu = jj, wu = T - jj;
    for (int idx = threadIdx.x; idx < hu * wu; idx += NT) {
      int i = idx % hu, c = jj + idx / hu;
      cplx<R> m = tmpU[i];
      cplx<R> xj = at(jj, c);
      cplx<R> x = (c == jj) ? cplx<R>{(R)0, (R)0} : at(i, c);
      x.re -= m.re * xj.re - m.im * xj.im;
      x.im -= m.re * xj.im + m.im * xj.re;
      at(i, c) = x;
    }
    __syncthreads();
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
// Fragments of KQ k-steps are loaded before use.
enum { MK_NONE = 0, MK_UNIT_LOWER = 1, MK_UPPER = 2 };

template <typename R>
__device__ __forceinline__ cplx<R> apply_mask(cplx<R> v, int mask, int row, int col) {
  if (mask == MK_UNIT_LOWER && row <= col) return cplx<R>{row == col ? (R)1 : (R)0, (R)0};
  if (mask == MK_UPPER && row > col) return cplx<R>{(R)0, (R)0};
  return v;
}

template <typename R, int T, int KQ, bool SUB>
__device__ __forceinline__ void tile_gemm(Acc2<R>& acc, const cplx<R>* A, int lda, bool a_rowmajor,
                                          int amask, const cplx<R>* Bm, int ldb, bool b_colmajor,
                                          int bmask, int rb, int cp) {
  const int l = threadIdx.x & 63;
  const int i = 16 * rb + (l & 15);
  const int j0 = 32 * cp + (l & 15), j1 = j0 + 16;
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
      cmfma<R, false, SUB>(acc.re[0], acc.im[0], a[q], b0[q]);
      cmfma<R, false, SUB>(acc.re[1], acc.im[1], a[q], b1[q]);
    }
  }
}

// Task decoding: slot -> (kind, r, t) for step m.  kind 0 = F, 1 = E.
//   slot 0: F(m, m); 1: F(m+1, m); 2: F(m, m+1)
//   slots 3 .. 2B-1: E of the tiles finalised at step m+1 (distance <= B-2)
//   slots 2B .. 4B-3: F at distance 2 .. B
struct Task {
  int kind, r, t;
};

__device__ __forceinline__ Task decode(int slot, int m, int B) {
  if (slot == 0) return {0, m, m};
  if (slot == 1) return {0, m + 1, m};
  if (slot == 2) return {0, m, m + 1};
  if (B < 2) return {0, -1, -1};
  int e = slot - 3;
  if (e < 2 * B - 3) {
    int mm = m + 1;
    if (e == 0) return {1, mm, mm};
    int d = (e + 1) >> 1;
    return (e & 1) ? Task{1, mm + d, mm} : Task{1, mm, mm + d};
  }
  int f = slot - 2 * B;
  int d = 2 + (f >> 1);
  return (f & 1) ? Task{0, m, m + d} : Task{0, m + d, m};
}

// E(r, t) has work when its early range s in [mx-B, m-2] is non-empty.
__device__ __forceinline__ bool has_early(int r, int t, int B) {
  int m = min(r, t), d = abs(r - t);
  return m >= 2 && d <= B - 2;
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

// Thread 0 polls one optional flag (to extra_want) and the flags of tiles
// (r, s) and (s, t), s in [s0, s1] (to 2 = final), then one acquire fence.
__device__ __forceinline__ void wait_inputs(const FactorParams& P, int w, int r, int t, int s0,
                                            int s1, int* extra, int extra_want) {
  if (threadIdx.x == 0) {
    bool live =
        !(__hip_atomic_load(P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_TIMEOUT);
    uint64_t t0 = wall_clock64();
    uint32_t polls = 0;
    for (int q = -1; q < 2 * (s1 - s0 + 1); q++) {
      int* f;
      int want = 2;
      if (q < 0) {
        if (!extra) continue;
        f = extra;
        want = extra_want;
      } else {
        int s = s0 + (q >> 1);
        f = (q & 1) ? flag_ptr(P, w, s, t) : flag_ptr(P, w, r, s);
      }
      while (live &&
             __hip_atomic_fetch_add(f, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        __builtin_amdgcn_s_sleep(1);
        if (++polls > kWaitPolls || wall_clock64() - t0 > kWaitTicks) {
          latch(P.status, ST_TIMEOUT);
          live = false;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Every thread's stores are complete, then thread 0 releases (L2 write-back)
// and sets the flag; barriers close the interval on both sides.
__device__ __forceinline__ void publish(int* flag, int value) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
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

template <typename R, int T>
__device__ __forceinline__ void acc_to_tile(const Acc2<R>& acc, cplx<R>* X, bool rowmajor, int rb,
                                            int cp) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int b = 0; b < 2; b++) {
    const int c = 32 * cp + 16 * b + (l & 15);
#pragma unroll
    for (int e = 0; e < 4; e++)
      st_coherent(&X[tix(16 * rb + Mf<R>::row(l, e), c, T, rowmajor)],
                  cplx<R>{acc.re[b][e], acc.im[b][e]});
  }
}

template <typename R, int T>
__global__ __launch_bounds__(FGeom<T>::NT) void k_factor(FactorParams P) {
  typedef FGeom<T> G;
  constexpr int KQ = sizeof(R) == 8 ? 4 : 8;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<R>* lds = reinterpret_cast<cplx<R>*>(smem_raw);  // T x LDT
  __shared__ uint32_t s_ticket;
  __shared__ cplx<R> tmpL[T], tmpU[T];
  const int B = P.g.B, NB = P.g.NB;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int rb = wave / G::CPR, cp = wave % G::CPR;
  Acc2<R> acc;
  for (;;) {
    const int64_t ticket = wg_ticket(P.ticket, &s_ticket);
    if (ticket >= P.total) break;
    const int w = (int)(ticket % P.n_omega);
    const int64_t task = ticket / P.n_omega;
    const int m0 = (int)(task / P.slots), slot = (int)(task % P.slots);
    const Task tk = decode(slot, m0, B);
    const int r = tk.r, t = tk.t;
    if (r < 0 || r >= NB || t >= NB) continue;
    const bool early = tk.kind == 1;
    if (early && !has_early(r, t, B)) continue;
    const int m = min(r, t), mx = max(r, t);
    const bool rowmajor = r < t;  // U tiles
    cplx<R>* X = tile_ptr<R, T>(P, w, r, t);
    // 1. the tile: the partial left by E(r, t), or generated from the stencil
    if (!early && has_early(r, t, B)) {
      wait_inputs(P, w, r, t, 0, -1, flag_ptr(P, w, r, t), 1);
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
    // 2. updates A_rt -= L_rs U_st: E takes s in [mx-B, m-2], F takes s = m-1
    const int s_lo = early ? max(0, mx - B) : max(max(0, mx - B), m - 1);
    const int s_hi = early ? m - 2 : m - 1;
    int* dflag = (!early && r != t) ? flag_ptr(P, w, m, m) : nullptr;
    if (s_lo <= s_hi || dflag) wait_inputs(P, w, r, t, s_lo, s_hi, dflag, 2);
    for (int s = s_lo; s <= s_hi; s++)
      tile_gemm<R, T, KQ, true>(acc, tile_ptr<R, T>(P, w, r, s), T, false, MK_NONE,
                                tile_ptr<R, T>(P, w, s, t), T, false, MK_NONE, rb, cp);
    if (early) {
      acc_to_tile<R, T>(acc, X, rowmajor, rb, cp);
      publish(flag_ptr(P, w, r, t), 1);
      continue;
    }
    // 3. finalise
    const cplx<R>* D = tile_ptr<R, T>(P, w, m, m);
    if (r == t) {
      acc_to_lds<R, T>(acc, lds, false, rb, cp);
      __syncthreads();
      lu_inv_tile<R, T, G::NT>(lds, G::LDT, tmpL, tmpU, P.status);
      for (int idx = threadIdx.x; idx < T * T; idx += G::NT)
        st_coherent(&X[idx], lds[(idx / T) * G::LDT + idx % T]);
    } else if (r > t) {
      // L_rm = A_rm U_mm^-1: A from LDS (column-major), U^-1 = upper part of D
      acc_to_lds<R, T>(acc, lds, false, rb, cp);
      __syncthreads();
      acc.zero();
      tile_gemm<R, T, KQ, false>(acc, lds, G::LDT, false, MK_NONE, D, T, true, MK_UPPER, rb, cp);
      acc_to_tile<R, T>(acc, X, false, rb, cp);
    } else {
      // U_mt = L_mm^-1 A_mt: L^-1 = unit-lower part of D, A from LDS (row-major)
      acc_to_lds<R, T>(acc, lds, true, rb, cp);
      __syncthreads();
      acc.zero();
      tile_gemm<R, T, KQ, false>(acc, D, T, false, MK_UNIT_LOWER, lds, G::LDT, false, MK_NONE, rb,
                                 cp);
      acc_to_tile<R, T>(acc, X, true, rb, cp);
    }
    publish(flag_ptr(P, w, r, t), 2);
    // 4. chain tiles (off the dependency chain: published data first)
    const int d = mx - m;
    if (r == t) {
      for (int dd = 1; dd <= 2 && dd <= B && m - dd >= 0; dd++) {
        // L_mm^-1 L_m,m-dd and U_m-dd,m U_mm^-1, with D still in LDS
        acc.zero();
        tile_gemm<R, T, KQ, false>(acc, lds, G::LDT, false, MK_UNIT_LOWER,
                                   tile_ptr<R, T>(P, w, m, m - dd), T, true, MK_NONE, rb, cp);
        acc_to_tile<R, T>(acc, chain_ptr<R, T>(P, w, m, chain_index(CH_FWD_L, dd)), false, rb,
                          cp);
        acc.zero();
        tile_gemm<R, T, KQ, false>(acc, tile_ptr<R, T>(P, w, m - dd, m), T, true, MK_NONE, lds,
                                   G::LDT, true, MK_UPPER, rb, cp);
        acc_to_tile<R, T>(acc, chain_ptr<R, T>(P, w, m, chain_index(CH_ADJ_U, dd)), true, rb, cp);
      }
    } else if (d <= 2 && r > t) {
      // L_m+d,m L_mm^-1: the new L tile (still in acc) goes to LDS
      acc_to_lds<R, T>(acc, lds, false, rb, cp);
      __syncthreads();
      acc.zero();
      tile_gemm<R, T, KQ, false>(acc, lds, G::LDT, false, MK_NONE, D, T, true, MK_UNIT_LOWER, rb,
                                 cp);
      acc_to_tile<R, T>(acc, chain_ptr<R, T>(P, w, m, chain_index(CH_ADJ_L, d)), true, rb, cp);
    } else if (d <= 2) {
      // U_mm^-1 U_m,m+d: the new U tile (still in acc) goes to LDS
      acc_to_lds<R, T>(acc, lds, true, rb, cp);
      __syncthreads();
      acc.zero();
      tile_gemm<R, T, KQ, false>(acc, D, T, false, MK_UPPER, lds, G::LDT, false, MK_NONE, rb, cp);
      acc_to_tile<R, T>(acc, chain_ptr<R, T>(P, w, m, chain_index(CH_FWD_U, d)), false, rb, cp);
    }
  }
}

template <typename R, int T>
static hipError_t launch_factor_t(const FactorParams& P, int grid, hipStream_t s) {
  size_t lds = sizeof(cplx<R>) * (size_t)T * FGeom<T>::LDT;
  hipError_t e = hipFuncSetAttribute((const void*)k_factor<R, T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_factor<R, T>), dim3(grid), dim3(FGeom<T>::NT), lds, s, P);
  return hipGetLastError();
}

hipError_t launch_factor(const OpDesc& op, const BandGeom& g, const double* omega, int n_omega,
                         bool fp32, void* tiles, int* flags, uint32_t* ticket, uint32_t* status,
                         int grid, hipStream_t s) {
  const int slots = g.B >= 2 ? 4 * g.B - 2 : 3;
  FactorParams P{op, g, omega, n_omega, tiles, flags, ticket, status, slots,
                 (int64_t)n_omega * g.NB * slots};
  hipError_t e = launch_fill_u32((uint32_t*)flags, 0u, (int64_t)n_omega * g.tiles_per_omega(), s);
  if (e == hipSuccess) e = launch_fill_u32(ticket, 0u, 1, s);
  if (e != hipSuccess) return e;
  if (grid > P.total) grid = (int)P.total;
  if (fp32) {
    if (g.T == 64) return launch_factor_t<float, 64>(P, grid, s);
    if (g.T == 32) return launch_factor_t<float, 32>(P, grid, s);
  } else {
    if (g.T == 64) return launch_factor_t<double, 64>(P, grid, s);
    if (g.T == 32) return launch_factor_t<double, 32>(P, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace rr
