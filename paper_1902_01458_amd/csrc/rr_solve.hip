// Multi-RHS solves with the band factor of rr_band.hip (Algorithm 1 steps 2,
// 4 and 6; Section 3.1: the one LU serves every solve).
//
//   forward  M X = B:    L y = b (block rows ascending),  U x = y (descending)
//   adjoint  M^H X = B:  U^H z = b (ascending),           L^H x = z (descending)
//
// Block row s of either sweep needs the B neighbouring blocks of the sweep's
// own output, x_s = D_s^-1 (b_s - sum_t T_st x_t), where D_s^-1 is the stored
// inverse of the diagonal triangle, so every step is a complex GEMM on MFMA.
//
// One persistent launch per solve; tasks (shift, sweep, block row) are handed
// out by a ticket counter in dependency order (a task only waits on smaller
// tickets), dependencies are per-block flags.  Each wave owns one 16 x 16 block
// of the T x NP output and reads its MFMA operands straight from memory, so
// the off-diagonal products need no LDS and no barriers: the blocks t far from
// s (published long ago) are consumed first and only the product with the
// immediate predecessor waits on the critical path.  The sweep's intermediate
// blocks live in a row-major workspace (T rows x NP columns per block) so the
// operand loads of all waves are coalesced.  Block s of the workspace holds
// y_s in the first sweep and x_s in the second, so it is written with
// device-coherent stores (st_coherent).
#include "rr_mfma.h"

namespace rr {

enum { OPM_NONE = 0, OPM_UNIT_LOWER = 1, OPM_UPPER = 2 };

// MFMA operand fragments of one wave for a full K = T product: k-step q
// holds op(X)[16rb + l%16][4q + l/16] (A role) or V[4q + l/16][16cb + l%16]
// (B role).  All loads are issued before any value is used (masks are applied
// in a second pass, conjugation inside the MFMA sequence), so the memory
// system overlaps them instead of paying one latency per k-step.
template <typename R, int T>
struct Frag {
  cplx<R> v[T / 4];
};

// A-role fragment of X (CT: X^H instead of X) for row block rb, masked with
// a triangular mask of X's own indices (the diagonal inverse tile).  X is
// stored column-major, or row-major when xt (the factor's U tiles).
template <typename R, int T, bool CT>
__device__ __forceinline__ void load_a(Frag<R, T>& f, const cplx<R>* X, int mask, int rb,
                                       bool xt = false) {
  const int l = threadIdx.x & 63;
  const int i = 16 * rb + (l & 15);
#pragma unroll
  for (int q = 0; q < T / 4; q++) {
    const int k = 4 * q + (l >> 4);
    const int a = CT ? k : i, b = CT ? i : k;
    f.v[q] = X[xt ? a * T + b : b * T + a];
  }
  if (mask != OPM_NONE) {
#pragma unroll
    for (int q = 0; q < T / 4; q++) {
      const int k = 4 * q + (l >> 4);
      const int a = CT ? k : i, b = CT ? i : k;
      if (mask == OPM_UNIT_LOWER && a <= b) f.v[q] = cplx<R>{a == b ? (R)1 : (R)0, (R)0};
      if (mask == OPM_UPPER && a > b) f.v[q] = cplx<R>{(R)0, (R)0};
    }
  }
}

template <typename R, int T, int NP>
__device__ __forceinline__ void load_b(Frag<R, T>& f, const cplx<R>* V, int cb) {
  const int l = threadIdx.x & 63;
  const int j = 16 * cb + (l & 15);
#pragma unroll
  for (int q = 0; q < T / 4; q++) f.v[q] = V[(4 * q + (l >> 4)) * NP + j];
}

// acc (+/-)= op(A) * B over the T k-steps (complex product = 4 real MFMAs);
// CA conjugates the A fragment (the conjugate-transposed factor of the adjoint).
template <typename R, int T, bool CA, bool SUB>
__device__ __forceinline__ void mma_frag(typename Mf<R>::v4& are, typename Mf<R>::v4& aim,
                                         const Frag<R, T>& A, const Frag<R, T>& Bf) {
#pragma unroll
  for (int q = 0; q < T / 4; q++) cmfma<R, CA, SUB>(are, aim, A.v[q], Bf.v[q]);
}

struct Solve2Params {
  BandGeom g;
  int64_t n;
  int n_omega, k;
  int adjoint;
  const void* tiles;
  const double2* Bm;
  int64_t bstride;   // complex elements between the shifts' right-hand sides
  double2* X;        // (n_omega, k, n) result
  void* xs;          // workspace: n_omega * ngroups * NB * T * NP complex R, row-major blocks
  int* flags;        // n_omega * ngroups * NB: 1 = first sweep done, 2 = final
  uint32_t* ticket;
  uint32_t* status;
  int64_t total;     // n_omega * ngroups * 2 * NB
  const uint32_t* skip;  // optional: non-zero at run time = nothing to do
  int ngroups;       // column groups of NP right-hand sides, solved independently
};

// Thread 0 polls flags [t0, t1] of one shift until each reaches `want`, then
// issues one acquire fence; the barrier hands the result to every wave.
__device__ __forceinline__ void wg_wait_range(int* fl, int t0, int t1, int want, uint32_t* status) {
  if (threadIdx.x == 0) {
    bool live = !(__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_TIMEOUT);
    uint64_t t_start = wall_clock64();
    uint32_t polls = 0;
    for (int t = t0; live && t <= t1; t++) {
      while (__hip_atomic_fetch_add(fl + t, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
        __builtin_amdgcn_s_sleep(1);
        if (++polls > kWaitPolls || wall_clock64() - t_start > kWaitTicks) {
          latch(status, ST_TIMEOUT);
          live = false;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Every thread's stores have left the CU (s_waitcnt), then thread 0 writes back
// the L2 (agent release) and sets the flag.  Barriers close the interval on
// both sides (see wg_publish).
__device__ __forceinline__ void wg_publish_one(int* flag, int value) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// Chain tiles a solve task stages in LDS: all three in FP32 (16 + 3 x 32 KiB
// at T = 64), two in FP64 (16 + 2 x 64 KiB of the CU's 160 KiB).  Either way
// one workgroup fills a CU, so no other workgroup's products compete for the
// matrix cores with the product on the dependency chain: measured at n =
// 262144, 16 shifts, k = 20, an FP32 forward / adjoint solve takes 53 / 57 ms
// against 58 / 72 ms with two workgroups per CU (two tiles staged), and an
// FP64 solve 63 against 71 ms with one tile staged.
template <typename R>
constexpr int kChainLds() {
  return sizeof(R) == 4 ? 3 : 2;
}

template <typename R, int T, int NP, bool ADJ>
__global__ __launch_bounds__(64 * (T / 16) * (NP / 16), 2) void k_solve2(Solve2Params P) {
  if (P.skip && __hip_atomic_load(P.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  constexpr int NCB = NP / 16;
  constexpr int NT = 64 * (T / 16) * (NP / 16);
  extern __shared__ __align__(16) char solve_smem[];
  cplx<R>* blk = reinterpret_cast<cplx<R>*>(solve_smem);  // pre-diagonal block, row-major
  cplx<R>* gl = blk + T * NP;  // copies of the chain tiles d = 1 .. kChainLds (T*T each)
  // The ticket broadcast word has LDS of its own.  It must not share the
  // staging block: a task with no far blocks reaches the store into blk[0]
  // with no barrier after the ticket read, so a wave still reading the
  // ticket could see the stored value instead, skip its task and leave the
  // task's flag unpublished.
  __shared__ uint32_t s_ticket;
  typedef typename Mf<R>::v4 v4;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int rb = wave / NCB, cb = wave % NCB;
  const int B = P.g.B, NB = P.g.NB, RT = P.g.row_tiles();
  for (;;) {
    const int64_t ticket = wg_ticket(P.ticket, &s_ticket);
    if (ticket >= P.total) break;
    // (shift, column group) pairs are independent chains of the same factor
    const int nv = P.n_omega * P.ngroups;
    const int wv = (int)(ticket % nv);
    const int w = wv / P.ngroups, grp = wv % P.ngroups;
    const int64_t task = ticket / nv;
    const bool second = task >= NB;
    const int s = second ? (int)(2 * NB - 1 - task) : (int)task;
    int* fl = P.flags + (int64_t)wv * NB;
    const cplx<R>* tw =
        reinterpret_cast<const cplx<R>*>(P.tiles) + (int64_t)w * NB * RT * (T * T);
    auto tile = [&](int r, int t) { return tw + ((int64_t)r * RT + (t - r + B)) * (T * T); };
    auto chain = [&](int r, int c) { return tw + ((int64_t)r * RT + 2 * B + 1 + c) * (T * T); };
    cplx<R>* xw = reinterpret_cast<cplx<R>*>(P.xs) + (int64_t)wv * NB * T * NP;
    const int j = 16 * cb + (l & 15);  // this lane's column in the block
    const int jg = grp * NP + j;       // and among the right-hand sides
    v4 are, aim;
    // right-hand side: b_s (first sweep) or the first sweep's y_s (second)
    if (second) {
      wg_wait_range(fl, s, s, 1, P.status);
      const cplx<R>* ys = xw + (int64_t)s * T * NP;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        cplx<R> v = ys[(16 * rb + Mf<R>::row(l, e)) * NP + j];
        are[e] = v.re;
        aim[e] = v.im;
      }
    } else {
      const double2* Bw = P.Bm + (int64_t)w * P.bstride;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        int64_t r = (int64_t)s * T + 16 * rb + Mf<R>::row(l, e);
        double2 v = make_double2(0.0, 0.0);
        if (jg < P.k && r < P.n) v = Bw[(int64_t)jg * P.n + r];
        are[e] = (R)v.x;
        aim[e] = (R)v.y;
      }
    }
    // x_s = D_s^-1 (b_s - sum_{|t-s|>C} T_st x_t) - sum_{d<=C} G_s,d x_s-+d with
    // C = min(B, kChainD) (G: the chain tiles of rr_band.hip).  Far blocks
    // were published long ago; D_s^-1 goes through LDS (every wave needs the
    // whole column block); then the neighbours, nearest last, each one
    // register MFMA product after its own wait.
    //   forward first: L_st (t < s), D = L^-1, G = CH_FWD_L
    //   forward second: U_st (t > s), D = U^-1, G = CH_FWD_U
    //   adjoint first: U_ts^H (t < s), D = (U^-1)^H, G = CH_ADJ_U^H
    //   adjoint second: L_ts^H (t > s), D = (L^-1)^H, G = CH_ADJ_L^H
    const int want = second ? 2 : 1;
    const int dir = second ? 1 : -1;
    const int mask = (ADJ ? second : !second) ? OPM_UNIT_LOWER : OPM_UPPER;
    const bool ut = ADJ != second;  // off-diagonal tiles of this sweep are U tiles (row-major)
    const int kind = ADJ ? (second ? CH_ADJ_L : CH_ADJ_U) : (second ? CH_FWD_U : CH_FWD_L);
    const int C = min(B, (int)BandGeom::kChainD);
    // the nearest chain tiles go to LDS now, off the dependency chain, so that
    // the products near the chain read their operand at LDS latency
    const int CL = min(C, kChainLds<R>());
    for (int d = 1; d <= CL; d++) {
      if (s + d * dir < 0 || s + d * dir >= NB) break;
      const cplx<R>* g = chain(s, chain_index(kind, d));
      cplx<R>* gd = gl + (d - 1) * T * T;
#pragma unroll 2
      for (int idx = threadIdx.x; idx < T * T; idx += NT) gd[idx] = g[idx];
      __builtin_amdgcn_sched_barrier(0);
    }
    Frag<R, T> fb;
    int f0, f1;
    if (second) { f0 = s + C + 1; f1 = min(NB - 1, s + B); } else { f0 = max(0, s - B); f1 = s - C - 1; }
    if (f0 <= f1) {
      // the older far blocks were published at least a step before the
      // nearest far one: take them first, then wait for that one alone
      const int fn = second ? f0 : f1;
      const int g0 = second ? f0 + 1 : f0, g1 = second ? f1 : f1 - 1;
      if (g0 <= g1) {
        wg_wait_range(fl, g0, g1, want, P.status);
        for (int t = g0; t <= g1; t++) {
          Frag<R, T> fa;
          load_a<R, T, ADJ>(fa, ADJ ? tile(t, s) : tile(s, t), OPM_NONE, rb, ut);
          load_b<R, T, NP>(fb, xw + (int64_t)t * T * NP, cb);
          mma_frag<R, T, ADJ, true>(are, aim, fa, fb);
        }
      }
      Frag<R, T> fa;
      load_a<R, T, ADJ>(fa, ADJ ? tile(fn, s) : tile(s, fn), OPM_NONE, rb, ut);
      wg_wait_range(fl, fn, fn, want, P.status);
      load_b<R, T, NP>(fb, xw + (int64_t)fn * T * NP, cb);
      mma_frag<R, T, ADJ, true>(are, aim, fa, fb);
    }
#pragma unroll
    for (int e = 0; e < 4; e++) blk[(16 * rb + Mf<R>::row(l, e)) * NP + j] = cplx<R>{are[e], aim[e]};
    __syncthreads();
    for (int e = 0; e < 4; e++) { are[e] = 0; aim[e] = 0; }
    {
      Frag<R, T> a_diag;
      load_a<R, T, ADJ>(a_diag, tile(s, s), mask, rb);
      load_b<R, T, NP>(fb, blk, cb);
      mma_frag<R, T, ADJ, false>(are, aim, a_diag, fb);
    }
    // the neighbours, farthest first.  Chain tiles are factor data, final
    // before the launch, so each one's load is issued before the wait for its
    // neighbour (a task is normally taken well before its neighbours are
    // published).
#pragma unroll 1
    for (int d = C; d > CL; d--) {  // chain tiles not staged in LDS
      const int nb = s + d * dir;
      if (nb < 0 || nb >= NB) continue;
      Frag<R, T> ag;
      load_a<R, T, ADJ>(ag, chain(s, chain_index(kind, d)), OPM_NONE, rb, ADJ);
      wg_wait_range(fl, nb, nb, want, P.status);
      load_b<R, T, NP>(fb, xw + (int64_t)nb * T * NP, cb);
      mma_frag<R, T, ADJ, true>(are, aim, ag, fb);
    }
#pragma unroll 1
    for (int d = CL; d >= 1; d--) {  // staged in LDS; d = 1 is the chain itself
      const int nb = s + d * dir;
      if (nb < 0 || nb >= NB) continue;
      wg_wait_range(fl, nb, nb, want, P.status);
      load_b<R, T, NP>(fb, xw + (int64_t)nb * T * NP, cb);
      Frag<R, T> ag;
      load_a<R, T, ADJ>(ag, gl + (d - 1) * T * T, OPM_NONE, rb, ADJ);
      mma_frag<R, T, ADJ, true>(are, aim, ag, fb);
    }
    cplx<R>* xs = xw + (int64_t)s * T * NP;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      st_coherent(xs + (16 * rb + Mf<R>::row(l, e)) * NP + j, cplx<R>{are[e], aim[e]});
    }
    if (second) {
      double2* Xw = P.X + (int64_t)w * P.k * P.n;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        int64_t r = (int64_t)s * T + 16 * rb + Mf<R>::row(l, e);
        if (jg < P.k && r < P.n)
          Xw[(int64_t)jg * P.n + r] = make_double2((double)are[e], (double)aim[e]);
      }
    }
    wg_publish_one(fl + s, want);
  }
}

// LDS of a solve workgroup: the T x NP staging block and kChainLds() T x T
// chain tiles.
template <typename R, int T, int NP>
constexpr size_t solve_lds() {
  return sizeof(cplx<R>) * ((size_t)T * NP + (size_t)kChainLds<R>() * T * T);
}

template <typename R, int T, int NP, bool ADJ>
static hipError_t launch_a(const Solve2Params& P, int grid, hipStream_t s) {
  const size_t lds = solve_lds<R, T, NP>();
  hipLaunchKernelGGL((k_solve2<R, T, NP, ADJ>), dim3(grid), dim3(64 * (T / 16) * (NP / 16)), lds,
                     s, P);
  return hipGetLastError();
}

template <typename R, int T>
static hipError_t prepare_t() {
  hipError_t e = hipSuccess;
  auto set = [&](const void* fn, int np) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(np == 16 ? solve_lds<R, T, 16>() : solve_lds<R, T, 32>()));
  };
  set((const void*)k_solve2<R, T, 16, false>, 16);
  set((const void*)k_solve2<R, T, 16, true>, 16);
  return e;
}

// Dynamic-LDS limits of the solve kernels of one tile / precision (host
// calls, kept out of the launch path so that launches can be captured).
hipError_t prepare_solve(int T, bool fp32) {
  hipError_t e = fp32 ? (T == 64 ? prepare_t<float, 64>() : prepare_t<float, 32>())
                      : (T == 64 ? prepare_t<double, 64>() : prepare_t<double, 32>());
  return e == hipSuccess ? prepare_ssolve(T, fp32) : e;
}

template <typename R, int T, int NP>
static hipError_t launch_t(const Solve2Params& P, int grid, hipStream_t s) {
  return P.adjoint ? launch_a<R, T, NP, true>(P, grid, s) : launch_a<R, T, NP, false>(P, grid, s);
}

template <typename R, int T>
static hipError_t launch_np(const Solve2Params& P, int NP, int grid, hipStream_t s) {
  if (NP == 16) return launch_t<R, T, 16>(P, grid, s);
  return hipErrorInvalidValue;
}

int solve_np(int k) { return ((k + 15) / 16) * 16; }

hipError_t launch_solve(const BandGeom& g, int n, int n_omega, int k, bool fp32,
                        const void* tiles, int adjoint, const double* Bm, int64_t bstride,
                        double* X, void* xs, void* cbuf, int* flags, uint32_t* ticket,
                        uint32_t* status, int grid, hipStream_t s, const uint32_t* skip) {
  if (g.P > 0)
    return launch_ssolve(g, n, n_omega, k, fp32, tiles, adjoint, Bm, bstride, X, xs, cbuf, flags,
                         ticket, status, grid, s, skip);
  // The right-hand sides are split into groups of 16 columns, each an
  // independent chain: half the MFMA work per block step on the chain for
  // k in (16, 32], and twice the chains in flight.
  const int NP = 16, ngroups = solve_np(k) / 16;
  if (ngroups > 2) return hipErrorInvalidValue;  // k <= 32 (rr_factor's k_max bound)
  Solve2Params P{g, n, n_omega, k, adjoint, tiles, (const double2*)Bm, bstride, (double2*)X,
                 xs, flags, ticket, status, (int64_t)n_omega * ngroups * 2 * g.NB, skip,
                 ngroups};
  hipError_t e = launch_fill_u32((uint32_t*)flags, 0u, (int64_t)n_omega * ngroups * g.NB, s);
  if (e == hipSuccess) e = launch_fill_u32(ticket, 0u, 1, s);
  if (e != hipSuccess) return e;
  if (grid > P.total) grid = (int)P.total;
  if (fp32) {
    if (g.T == 64) return launch_np<float, 64>(P, NP, grid, s);
    if (g.T == 32) return launch_np<float, 32>(P, NP, grid, s);
  } else {
    if (g.T == 64) return launch_np<double, 64>(P, NP, grid, s);
    if (g.T == 32) return launch_np<double, 32>(P, NP, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace rr
