// Band LU of M(omega) = i omega I - L on MFMA (the solves are in rr_solve.hip).
//
// The paper factors the shifted operator once and reuses the LU in the three
// linear solves of Algorithm 1 (Section 3.1).  Here the band (kl = ku = b =
// 2*ny) is cut into T x T tiles: block row s holds tiles (s, s-B) .. (s, s+B)
// with B = ceil(b / T), so the band becomes block-banded with B blocks on each
// side.  Without pivoting (the shifted operator is only mildly non-normal in
// the sense that matters here: element growth stays O(1); the design doc records
// the measured growth) the block LU is
//   A_rt -= sum_s L_rs U_st             (updates, complex GEMMs on MFMA)
//   A_mm  = L_mm U_mm                    (T x T LU in LDS)
//   L_rm  = A_rm U_mm^-1,  U_mt = L_mm^-1 A_mt
// The diagonal tile is stored as [U_mm^-1 (upper, diagonal included) |
// L_mm^-1 (strictly lower, unit diagonal implied)], so the solves and the
// off-diagonal finalisations are GEMMs too.
//
// Scheduling: one persistent launch per factorisation.  Work
// is handed out by a global ticket counter in a dependency-respecting order
// (every task only waits on tasks with smaller tickets), so the launch cannot
// deadlock whatever the residency; dependencies are per-tile flags published
// with agent-scope release and awaited with acquire.  Left-looking: a task
// owns one tile, generates it from the stencil (the band is never read from
// memory before it is final), accumulates all its updates in MFMA registers,
// finalises it and writes it exactly once.
#include "rr_internal.h"

namespace rr {

constexpr int kThreads = 256;  // 4 waves of 64
constexpr int KC = 16;         // k-chunk staged through LDS

template <typename R>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element e of lane l sits at row (l/16) + 4e, column l%16
  static __device__ __forceinline__ int row(int l, int e) { return (l >> 4) + 4 * e; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element e of lane l sits at row 4(l/16) + e, column l%16
  static __device__ __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
};

// A wave's share of an MxN complex accumulator in 16x16 blocks: block
// b = wave + 4*q (q < NPW) covers rows 16*(b / NCB) and columns 16*(b % NCB).
template <typename R, int MB, int NCB>
struct Acc {
  static constexpr int NBLK = MB * NCB;
  static constexpr int NPW = (NBLK + 3) / 4;
  typename Mfma<R>::v4 re[NPW], im[NPW];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int q = 0; q < NPW; q++)
#pragma unroll
      for (int e = 0; e < 4; e++) { re[q][e] = 0; im[q][e] = 0; }
  }
  static __device__ __forceinline__ int blk(int q) { return (threadIdx.x >> 6) + 4 * q; }
  static __device__ __forceinline__ bool valid(int q) { return blk(q) < NBLK; }
  static __device__ __forceinline__ int row(int q, int e) {
    return 16 * (blk(q) / NCB) + Mfma<R>::row(threadIdx.x & 63, e);
  }
  static __device__ __forceinline__ int col(int q) { return 16 * (blk(q) % NCB) + (threadIdx.x & 15); }
};

// Masks applied to a stored tile X before it is used as an operand.
enum { MASK_NONE = 0, MASK_UNIT_LOWER = 1, MASK_UPPER = 2 };

template <typename R>
__device__ __forceinline__ cplx<R> masked(const cplx<R>* X, int T, int a, int b, int mask) {
  // element (a, b) of a column-major T x T tile after masking
  if (mask == MASK_UNIT_LOWER) {
    if (a == b) return cplx<R>{(R)1, (R)0};
    if (a < b) return cplx<R>{(R)0, (R)0};
  } else if (mask == MASK_UPPER) {
    if (a > b) return cplx<R>{(R)0, (R)0};
  }
  return X[(int64_t)b * T + a];
}

// Stage rows k0..k0+KC-1 of op(X) viewed as the "k" index into S[kk][m]
// (row length LD) for m < M.  role_a: the operand is A (element (m, k));
// otherwise B (element (k, m)).  conj_t: op = conjugate transpose.
template <typename R, int T>
__device__ __forceinline__ void stage_tile(cplx<R>* S, int LD, const cplx<R>* X, int k0,
                                           bool role_a, bool conj_t, int mask) {
  // X-index of element (m, k): A-role N: (m, k); A-role C: (k, m) conj;
  // B-role N: (k, m); B-role C: (m, k) conj.  Contiguous direction of X is
  // its row index, so map threads along whichever of m, k is X's row.
  bool m_is_row = (role_a && !conj_t) || (!role_a && conj_t);
  for (int idx = threadIdx.x; idx < KC * T; idx += kThreads) {
    int m, kk;
    if (m_is_row) { kk = idx / T; m = idx % T; } else { m = idx / KC; kk = idx % KC; }
    int k = k0 + kk;
    cplx<R> v = m_is_row ? masked(X, T, m, k, mask) : masked(X, T, k, m, mask);
    if (conj_t) v.im = -v.im;
    S[kk * LD + m] = v;
  }
}

// Stage rows k0..k0+KC-1 of an RHS block (B-role, element (k, j) at
// V[j*ld + row0 + k], zero beyond nrows / ncols) into S[kk][j].
template <typename R>
__device__ __forceinline__ void stage_rhs(cplx<R>* S, int LD, const double2* V, int64_t ld,
                                          int64_t row0, int64_t nrows, int ncols, int NP, int k0) {
  for (int idx = threadIdx.x; idx < KC * NP; idx += kThreads) {
    int j = idx / KC, kk = idx % KC;
    int64_t r = row0 + k0 + kk;
    cplx<R> v{(R)0, (R)0};
    if (j < ncols && r < nrows) {
      double2 d = V[(int64_t)j * ld + r];
      v.re = (R)d.x;
      v.im = (R)d.y;
    }
    S[kk * LD + j] = v;
  }
}

// acc (+/-)= A_chunk * B_chunk for one staged chunk: As[kk][m] (m < 16*MB),
// Bs[kk][j] (j < 16*NCB).
template <typename R, int MB, int NCB>
__device__ __forceinline__ void mma_chunk(Acc<R, MB, NCB>& acc, const cplx<R>* As, int lda,
                                          const cplx<R>* Bs, int ldb, bool subtract) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int ks = 0; ks < KC; ks += 4) {
    const int kk = ks + (l >> 4);
#pragma unroll
    for (int q = 0; q < Acc<R, MB, NCB>::NPW; q++) {
      if (!Acc<R, MB, NCB>::valid(q)) continue;
      int b = Acc<R, MB, NCB>::blk(q);
      cplx<R> a = As[kk * lda + 16 * (b / NCB) + (l & 15)];
      cplx<R> bb = Bs[kk * ldb + 16 * (b % NCB) + (l & 15)];
      R ar = subtract ? -a.re : a.re, ai = subtract ? -a.im : a.im;
      acc.re[q] = Mfma<R>::op(ar, bb.re, acc.re[q]);
      acc.re[q] = Mfma<R>::op(-ai, bb.im, acc.re[q]);
      acc.im[q] = Mfma<R>::op(ar, bb.im, acc.im[q]);
      acc.im[q] = Mfma<R>::op(ai, bb.re, acc.im[q]);
    }
  }
}

// acc (+/-)= op(XA) * op(XB), both T x T tiles in global memory.
template <typename R, int T>
__device__ void gemm_tt(Acc<R, T / 16, T / 16>& acc, cplx<R>* lds, const cplx<R>* XA, bool ca,
                        int ma, const cplx<R>* XB, bool cb, int mb, bool subtract) {
  constexpr int LD = T + 1;
  cplx<R>* As = lds;
  cplx<R>* Bs = lds + KC * LD;
  for (int k0 = 0; k0 < T; k0 += KC) {
    stage_tile<R, T>(As, LD, XA, k0, true, ca, ma);
    stage_tile<R, T>(Bs, LD, XB, k0, false, cb, mb);
    __syncthreads();
    mma_chunk<R, T / 16, T / 16>(acc, As, LD, Bs, LD, subtract);
    __syncthreads();
  }
}

// acc (+/-)= op(XA) * V where XA is a T x T tile and V an RHS block (T x NP).
template <typename R, int T, int NP>
__device__ void gemm_tv(Acc<R, T / 16, NP / 16>& acc, cplx<R>* lds, const cplx<R>* XA, bool ca,
                        int ma, const double2* V, int64_t ld, int64_t row0, int64_t nrows,
                        int ncols, bool subtract) {
  constexpr int LDA = T + 1, LDB = NP + 1;
  cplx<R>* As = lds;
  cplx<R>* Bs = lds + KC * LDA;
  for (int k0 = 0; k0 < T; k0 += KC) {
    stage_tile<R, T>(As, LDA, XA, k0, true, ca, ma);
    stage_rhs<R>(Bs, LDB, V, ld, row0, nrows, ncols, NP, k0);
    __syncthreads();
    mma_chunk<R, T / 16, NP / 16>(acc, As, LDA, Bs, LDB, subtract);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The factorisation
// ---------------------------------------------------------------------------
struct FactorParams {
  OpDesc op;
  BandGeom g;
  const double* omega;  // 2 * n_omega
  int n_omega;
  void* tiles;
  int* flags;
  uint32_t* ticket;
  uint32_t* status;
  int64_t total;        // tickets = n_omega * NB * (2B+1)
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

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return cplx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cplx<R> cinv(cplx<R> a) {
  R d = a.re * a.re + a.im * a.im;
  return cplx<R>{a.re / d, -a.im / d};
}

// In-LDS no-pivot LU of the T x T tile S (column-major, leading dimension
// LD), then in-place inversion of both triangles:
//   S <- [U^-1 on and above the diagonal | L^-1 strictly below].
template <typename R, int T>
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
    for (int i = j + 1 + threadIdx.x; i < T; i += kThreads) at(i, j) = cmul(at(i, j), ip);
    __syncthreads();
    int w = T - 1 - j;
    for (int idx = threadIdx.x; idx < w * w; idx += kThreads) {
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
    // U: finalise row jj: X[jj][c] = acc[jj][c] / U[jj][jj]
    cplx<R> ujj = at(jj, jj);
    cplx<R> iu = cinv(ujj);
    for (int i = threadIdx.x; i < T; i += kThreads) {
      if (i > j) tmpL[i] = at(i, j);      // multipliers L[i][j]
      if (i < jj) tmpU[i] = at(i, jj);    // multipliers U[i][jj]
    }
    __syncthreads();
    for (int c = jj + 1 + threadIdx.x; c < T; c += kThreads) at(jj, c) = cmul(at(jj, c), iu);
    if (threadIdx.x == 0) at(jj, jj) = iu;
    __syncthreads();
    // L: rows i > j, columns c <= j:  X[i][c] -= L[i][j] X[j][c]  (X[j][j] = 1)
    int wl = T - 1 - j, hl = j + 1;
    for (int idx = threadIdx.x; idx < wl * hl; idx += kThreads) {
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
    for (int idx = threadIdx.x; idx < hu * wu; idx += kThreads) {
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

template <typename R, int T>
__device__ __forceinline__ cplx<R>* tile_ptr(const FactorParams& P, int w, int r, int t) {
  const int W = 2 * P.g.B + 1;
  int64_t idx = ((int64_t)w * P.g.NB + r) * W + (t - r + P.g.B);
  return reinterpret_cast<cplx<R>*>(P.tiles) + idx * (T * T);
}
__device__ __forceinline__ int* flag_ptr(const FactorParams& P, int w, int r, int t) {
  const int W = 2 * P.g.B + 1;
  return P.flags + ((int64_t)w * P.g.NB + r) * W + (t - r + P.g.B);
}

template <typename R, int T>
__device__ void store_acc_tile(const Acc<R, T / 16, T / 16>& acc, cplx<R>* X) {
#pragma unroll
  for (int q = 0; q < Acc<R, T / 16, T / 16>::NPW; q++) {
    int c = Acc<R, T / 16, T / 16>::col(q);
#pragma unroll
    for (int e = 0; e < 4; e++) {
      int r = Acc<R, T / 16, T / 16>::row(q, e);
      X[c * T + r] = cplx<R>{acc.re[q][e], acc.im[q][e]};
    }
  }
}

template <typename R, int T>
__global__ __launch_bounds__(kThreads) void k_factor(FactorParams P) {
  extern __shared__ __align__(16) char smem_raw[];
  cplx<R>* lds = reinterpret_cast<cplx<R>*>(smem_raw);
  __shared__ uint32_t s_ticket;
  __shared__ cplx<R> tmpL[T], tmpU[T];
  const int B = P.g.B, NB = P.g.NB, W = 2 * B + 1;
  typedef Acc<R, T / 16, T / 16> A;
  A acc;
  for (;;) {
    const int64_t ticket = wg_ticket(P.ticket, &s_ticket);
    if (ticket >= P.total) break;
    const int w = (int)(ticket % P.n_omega);
    const int64_t task = ticket / P.n_omega;
    const int m = (int)(task / W), slot = (int)(task % W);
    int r = m, t = m;
    if (slot) {
      int d = (slot + 1) >> 1;
      if (slot & 1) r = m + d; else t = m + d;
    }
    if (r >= NB || t >= NB) continue;  // no such tile: the next ticket
    // 1. the tile of M, generated from the stencil into the accumulator
    const double om_r = P.omega[2 * w], om_i = P.omega[2 * w + 1];
#pragma unroll
    for (int q = 0; q < A::NPW; q++) {
      int c = A::col(q);
#pragma unroll
      for (int e = 0; e < 4; e++) {
        int rr = A::row(q, e);
        double2 v = m_entry(P.op, om_r, om_i, (int64_t)r * T + rr, (int64_t)t * T + c);
        acc.re[q][e] = (R)v.x;
        acc.im[q][e] = (R)v.y;
      }
    }
    // 2. left-looking updates A_rt -= L_rs U_st
    int s0 = max(0, max(r, t) - B);
    for (int s = s0; s < m; s++) {
      wg_wait_flag(flag_ptr(P, w, r, s), 1, P.status);
      wg_wait_flag(flag_ptr(P, w, s, t), 1, P.status);
      gemm_tt<R, T>(acc, lds, tile_ptr<R, T>(P, w, r, s), false, MASK_NONE,
                    tile_ptr<R, T>(P, w, s, t), false, MASK_NONE, true);
    }
    // 3. finalise
    cplx<R>* X = tile_ptr<R, T>(P, w, r, t);
    if (r == t) {
      constexpr int LD = T + 1;
#pragma unroll
      for (int q = 0; q < A::NPW; q++) {
        int c = A::col(q);
#pragma unroll
        for (int e = 0; e < 4; e++) lds[c * LD + A::row(q, e)] = cplx<R>{acc.re[q][e], acc.im[q][e]};
      }
      __syncthreads();
      lu_inv_tile<R, T>(lds, LD, tmpL, tmpU, P.status);
      for (int idx = threadIdx.x; idx < T * T; idx += kThreads) {
        int i = idx % T, c = idx / T;
        X[idx] = lds[c * LD + i];
      }
      __syncthreads();
    } else {
      wg_wait_flag(flag_ptr(P, w, m, m), 1, P.status);
      const cplx<R>* D = tile_ptr<R, T>(P, w, m, m);
      store_acc_tile<R, T>(acc, X);
      __threadfence_block();
      __syncthreads();
      acc.zero();
      if (r > t)  // L_rm = A_rm U_mm^-1
        gemm_tt<R, T>(acc, lds, X, false, MASK_NONE, D, false, MASK_UPPER, false);
      else        // U_mt = L_mm^-1 A_mt
        gemm_tt<R, T>(acc, lds, D, false, MASK_UNIT_LOWER, X, false, MASK_NONE, false);
      store_acc_tile<R, T>(acc, X);
    }
    wg_publish(flag_ptr(P, w, r, t), 1);
  }
}

template <typename R, int T>
static hipError_t launch_factor_t(const FactorParams& P, int grid, hipStream_t s) {
  size_t lds = sizeof(cplx<R>) * (size_t)T * (T + 1);
  size_t stage = sizeof(cplx<R>) * (size_t)2 * KC * (T + 1);
  if (stage > lds) lds = stage;
  hipError_t e = hipFuncSetAttribute((const void*)k_factor<R, T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_factor<R, T>), dim3(grid), dim3(kThreads), lds, s, P);
  return hipGetLastError();
}

hipError_t launch_factor(const OpDesc& op, const BandGeom& g, const double* omega, int n_omega,
                         bool fp32, void* tiles, int* flags, uint32_t* ticket, uint32_t* status,
                         int grid, hipStream_t s) {
  FactorParams P{op, g, omega, n_omega, tiles, flags, ticket, status,
                 (int64_t)n_omega * g.NB * (2 * g.B + 1)};
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
