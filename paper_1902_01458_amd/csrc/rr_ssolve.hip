// Superblock solves with the band factor (Algorithm 1 steps 2, 4 and 6;
// Section 3.1: the one LU of M(omega) serves every solve).
//
//   forward  M X = B:    L y = b (ascending),    U x = y (descending)
//   adjoint  M^H X = B:  U^H z = b (ascending),  L^H x = z (descending)
//
// A sweep walks superblocks of P consecutive block rows (P T rows) instead of
// single block rows.  With D-hat_S the diagonal block of superblock S in the
// sweep's triangle (block-triangular, P x P tiles) and its inverse stored by
// the factorisation (k_sbinv), one step is two dense products:
//   phase A:  c_S = b_S - sum_t T_st x_t    (t: the tiles of the band outside
//                                            the superblock, already solved)
//   phase B:  x_S = D-hat_S^-1 c_S
// so a sweep takes NB / P dependent steps where the tile-by-tile recurrence
// takes NB, and each step's products are spread over P T / 16 workgroups
// ("pieces": 16 rows x NP columns each; the waves of a workgroup split the
// tiles of the inner dimension and sum their parts in LDS).
//
// One persistent launch per solve.  The shifts are dealt to teams, one team
// per XCD (shift w to team w mod 8): a workgroup serves the team of the XCD
// it runs on, so the pieces of one step, which all read the same solved
// blocks, share that XCD's L2.  Within a team, tickets hand out pieces in
// dependency order -- (sweep, superblock, phase, shift, piece) -- so a piece
// waits only on smaller tickets of its team; a workgroup whose team has no
// tickets left serves the other teams in turn, so the launch cannot deadlock
// and finishes whatever the residency or the spread over XCDs.
// A phase's pieces count themselves done on a per-(shift, sweep, superblock,
// phase) counter; phase A waits for the previous superblock's phase B (which
// implies every earlier step), phase B for its own phase A.  In its home team
// a workgroup takes its next ticket while it waits for the current piece and
// loads that piece's factor tile during the current products, so that a step
// finds the operands of its pieces in registers.  Data handed between
// workgroups (c and the sweep's blocks) is stored device-coherent
// (st_coherent, written through), or, when every team is one XCD serving
// only itself (eight shifts or more), with plain stores into that XCD's L2;
// the counter is incremented once those stores have completed, and readers
// poll it (four polls in flight), then acquire.
#include "rr_mfma.h"

namespace rr {

namespace {

enum { SM_NONE = 0, SM_UNIT_LOWER = 1, SM_UPPER = 2 };

// A long piece (more inner tiles than waves, e.g. a half-band of many tiles)
// walks its tiles in chunks of QC k-steps (4 QC columns of the inner
// dimension of one tile, a quarter of a tile): the A-role fragment of the
// stored tile and the B-role fragments of the solved block for each of the
// NCB column blocks, the next chunk loaded one ahead of the current one's
// MFMAs (two buffers).  Short pieces (below) hold a whole tile instead.
template <typename R, int T, int NCB>
constexpr int ss_qc() { return T / 16; }

template <typename R, int T, int NCB>
struct SChunk {
  cplx<R> a[ss_qc<R, T, NCB>()];
  cplx<R> b[NCB][ss_qc<R, T, NCB>()];
};

// a[q] = op(X)[16 rb + l%16][4 (q0 + q) + l/16] (CT: X^H); X column-major, or
// row-major when xt; the mask applies to X's own indices.
template <typename R, int T, bool CT, int NCB>
__device__ __forceinline__ void sc_load_a(SChunk<R, T, NCB>& c, const cplx<R>* X, int mask,
                                          int rb, bool xt, int q0) {
  constexpr int QC = ss_qc<R, T, NCB>();
  const int l = threadIdx.x & 63;
  const int i = 16 * rb + (l & 15);
#pragma unroll
  for (int q = 0; q < QC; q++) {
    const int k = 4 * (q0 + q) + (l >> 4);
    const int a = CT ? k : i, b = CT ? i : k;
    c.a[q] = X[xt ? a * T + b : b * T + a];
  }
  if (mask != SM_NONE) {
#pragma unroll
    for (int q = 0; q < QC; q++) {
      const int k = 4 * (q0 + q) + (l >> 4);
      const int a = CT ? k : i, b = CT ? i : k;
      if (mask == SM_UNIT_LOWER && a <= b) c.a[q] = cplx<R>{a == b ? (R)1 : (R)0, (R)0};
      if (mask == SM_UPPER && a > b) c.a[q] = cplx<R>{(R)0, (R)0};
    }
  }
}

// b[cb][q] = V[4 (q0 + q) + l/16][16 cb + l%16] of the row-major T x NP block V.
template <typename R, int T, int NP, int NCB>
__device__ __forceinline__ void sc_load_b(SChunk<R, T, NCB>& c, const cplx<R>* V, int q0) {
  constexpr int QC = ss_qc<R, T, NCB>();
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int cb = 0; cb < NCB; cb++)
#pragma unroll
    for (int q = 0; q < QC; q++) c.b[cb][q] = V[(4 * (q0 + q) + (l >> 4)) * NP + 16 * cb + (l & 15)];
}

// Complex products with three real MFMAs instead of four (Gauss): with
// a = ar + i ai (ai negated when CA conjugates a) and b = br + i bi,
//   p1 += ar br,  p2 += ai bi,  p3 += (ar + ai)(br + bi)
// and at the end re = p1 - p2, im = p3 - p1 - p2 (sc_finish).  The sums cost
// one add per operand element; the error of the imaginary part is bounded by
// a small multiple of eps (|ar| + |ai|)(|br| + |bi|), like the four-product
// form's up to a constant.  Flops are still counted as 8 per complex FMA.
//
// A last column block holding at most 8 of the caller's columns (k = 20: 16
// plus 4) takes the real form instead, two MFMAs where Gauss takes three:
//   [Re C | Im C] = [ar ai] [[br, bi], [-bi, br]],
// lanes l%16 < 8 of the 16 output columns holding Re of column l%8 and the
// others its Im (ss_mma, ss_load_b and the reduction's TR case).
template <typename R, int NCB>
struct SAcc {
  typename Mf<R>::v4 p1[NCB], p2[NCB], p3[NCB];
  typename Mf<R>::v4 t;  // the last column block in real form (ss_mma's TR)
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < NCB; c++)
#pragma unroll
      for (int e = 0; e < 4; e++) { p1[c][e] = 0; p2[c][e] = 0; p3[c][e] = 0; }
#pragma unroll
    for (int e = 0; e < 4; e++) t[e] = 0;
  }
};

template <typename R, int T, int NCB, bool CA>
__device__ __forceinline__ void sc_mma(SAcc<R, NCB>& acc, const SChunk<R, T, NCB>& c) {
#pragma unroll
  for (int q = 0; q < ss_qc<R, T, NCB>(); q++) {
    const R ar = c.a[q].re, ai = CA ? -c.a[q].im : c.a[q].im;
    const R sa = ar + ai;
#pragma unroll
    for (int cb = 0; cb < NCB; cb++) {
      const R br = c.b[cb][q].re, bi = c.b[cb][q].im;
      acc.p1[cb] = Mf<R>::op(ar, br, acc.p1[cb]);
      acc.p2[cb] = Mf<R>::op(ai, bi, acc.p2[cb]);
      acc.p3[cb] = Mf<R>::op(sa, br + bi, acc.p3[cb]);
    }
  }
}

// Element e of column block cb: (re, im) of the accumulated product,
// negated when SUB.
template <typename R, int NCB>
__device__ __forceinline__ cplx<R> sc_finish(const SAcc<R, NCB>& acc, int cb, int e, bool sub) {
  const R re = acc.p1[cb][e] - acc.p2[cb][e];
  const R im = acc.p3[cb][e] - acc.p1[cb][e] - acc.p2[cb][e];
  return sub ? cplx<R>{-re, -im} : cplx<R>{re, im};
}

}  // namespace

struct SSolveParams {
  BandGeom g;
  int64_t n;
  int n_omega, k;
  const void* tiles;
  const double2* Bm;
  int64_t bstride;   // complex elements between the shifts' right-hand sides
  double2* X;        // (n_omega, k, n) result
  void* xs;          // n_omega * NB * T * NP complex R: row-major T x NP blocks
  void* cb;          // n_omega * P * T * NP complex R: c of the current superblock
  int* cnt;          // n_omega * 2 sweeps * NS * 2 phases: finished pieces
  uint32_t* tickets;  // one ticket counter per team
  uint32_t* status;
  int teams;         // min(kTeams, n_omega)
  const uint32_t* skip;  // optional: non-zero at run time = nothing to do
  int ahead;         // hold a second ticket in the home team (see k_ssolve)
  int local;         // every team is one XCD and serves only itself (see k_ssolve)
};

constexpr int kTeams = 8;  // XCDs of gfx950

// The XCD this wave runs on (hardware register XCC_ID).
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg((15 << 11) | 20) & 0xF);
}

// Thread 0 optionally takes the next ticket of counter `tk` (its atomic in
// flight while it polls) and polls *c until it reaches `want`, with four
// polls in flight so that a completed step is seen about a quarter of a
// round trip sooner than with one; then one acquire fence.  The barrier hands
// both to every wave.  Bounded like every dataflow wait of the library
// (ST_TIMEOUT).  Returns the ticket, or -1 when `tk` is null.
__device__ __forceinline__ int64_t ss_wait(int* c, int want, uint32_t* status, uint32_t* tk,
                                           uint32_t* slot) {
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    if (tk) t = atomicAdd(tk, 1u);
    if (c) {
      if (!(__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_TIMEOUT)) {
        auto poll = [&]() { return __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
        int v0 = poll(), v1 = poll(), v2 = poll(), v3 = poll();
        const uint64_t t0 = wall_clock64();
        for (uint32_t rounds = 0;; rounds++) {
          if (v0 >= want) break;
          v0 = poll();
          if (v1 >= want) break;
          v1 = poll();
          if (v2 >= want) break;
          v2 = poll();
          if (v3 >= want) break;
          v3 = poll();
          if (rounds > kWaitPolls || wall_clock64() - t0 > kWaitTicks) {
            latch(status, ST_TIMEOUT);
            break;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    if (tk) *slot = t;
  }
  __syncthreads();
  return tk ? (int64_t)__builtin_amdgcn_readfirstlane(*slot) : -1;
}

// Every thread's stores are complete, then thread 0 counts the piece done.
// Everything a piece hands over is stored device-coherent (st_coherent,
// written through) or, in a team confined to one XCD, into the L2 its
// readers share, so waiting for the stores is the whole release: no L2
// write-back is needed before the count.  Barriers close the interval on
// both sides.
__device__ __forceinline__ void ss_done(int* c) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

constexpr int kSsWaves = 8;  // waves per workgroup: they split a piece's inner dimension

template <typename R, int T, int NP>
constexpr size_t ssolve_lds() {  // the waves' partial sums of a piece
  return sizeof(cplx<R>) * (size_t)16 * NP * kSsWaves;
}

// Every piece is short (at most kSsWaves tiles of inner dimension): phase A
// spans at most the half-band's B tiles, phase B at most the superblock's P.
__host__ __device__ inline bool ss_all_short(const BandGeom& g) {
  return g.B <= kSsWaves && g.P <= kSsWaves;
}

// One piece: 16 rows (row block rb of tile row i of superblock S) of one
// phase of one sweep of shift w, and the tiles lo .. hi of its inner
// dimension (band tiles outside the superblock in phase A, the superblock's
// inverse in phase B).
struct SPiece {
  int w, phase, second, S, i, rb, s0, s, lo, hi;
};

__device__ __forceinline__ SPiece ss_decode(int64_t t, int team, int teams, int nw, int npc,
                                            int rpt, const BandGeom& g) {
  SPiece p;
  const int NS = g.NS(), PS = g.P, NB = g.NB, B = g.B;
  const int pc = (int)(t % npc);
  t /= npc;
  p.w = team + teams * (int)(t % nw);
  t /= nw;
  p.phase = (int)(t % 2);
  t /= 2;
  const int si = (int)(t % NS);
  p.second = (int)(t / NS);
  p.S = p.second ? NS - 1 - si : si;
  p.i = pc / rpt;
  p.rb = pc % rpt;
  p.s0 = p.S * PS;
  p.s = p.s0 + p.i;
  p.lo = 0;
  p.hi = -1;
  if (p.s < NB) {
    if (p.phase == 0) {
      if (!p.second) { p.lo = max(0, p.s - B); p.hi = p.s0 - 1; }
      else { p.lo = p.s0 + PS; p.hi = min(NB - 1, p.s + B); }
    } else {
      if (!p.second) { p.lo = 0; p.hi = p.i; }
      else { p.lo = p.i; p.hi = min(PS - 1, NB - 1 - p.s0); }
    }
  }
  return p;
}

// The stored tile that is the A-role operand of inner index x of piece p, its
// mask and whether it is stored row-major.
template <typename R, int T, bool ADJ>
__device__ __forceinline__ const cplx<R>* ss_operand(const SSolveParams& P, const SPiece& p, int x,
                                                     int& mask, bool& xt) {
  const int B = P.g.B, NB = P.g.NB, RT = P.g.row_tiles();
  const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(P.tiles) + (int64_t)p.w * NB * RT * (T * T);
  auto tile = [&](int r, int c) { return tw + ((int64_t)r * RT + (c - r + B)) * (T * T); };
  auto sbt = [&](int r, int slot) { return tw + ((int64_t)r * RT + P.g.sb_index(slot)) * (T * T); };
  if (p.phase == 0) {
    mask = SM_NONE;
    xt = ADJ != (bool)p.second;  // U tiles (row-major) in this sweep
    return ADJ ? tile(x, p.s) : tile(p.s, x);
  }
  const int j = x, i = p.i;
  if (!ADJ) {
    mask = j == i ? (p.second ? SM_UPPER : SM_UNIT_LOWER) : SM_NONE;
    xt = p.second && j != i;  // (U-hat^-1)_ij row-major, (L-hat^-1)_ij column-major
    return j == i ? tile(p.s, p.s) : sbt(p.s, sb_slot(i, j));
  }
  mask = j == i ? (p.second ? SM_UNIT_LOWER : SM_UPPER) : SM_NONE;
  xt = !p.second && j != i;   // ((U-hat^-1)_ji)^H or ((L-hat^-1)_ji)^H
  return j == i ? tile(p.s, p.s) : sbt(p.s0 + j, sb_slot(j, i));
}

// A piece is "short" when its inner dimension has at most one tile per wave
// (every piece of the benchmark's band with T = 64).  A short piece's wave
// loads the A-role values of its tile before the piece's wait, PQ of the T/4
// k-steps (all of them in FP32, a quarter in FP64, where the rest follows in
// chunks of PQ k-steps loaded one ahead), raw: masks are applied after the
// wait so that no load is awaited before it.
template <typename R, int T>
constexpr int ss_pq() { return sizeof(R) == 8 ? T / 16 : T / 4; }

template <typename R, int T>
struct SPre {
  cplx<R> a[ss_pq<R, T>()];
};

template <typename R, int T, bool CT, int N>
__device__ __forceinline__ void ss_load_a(cplx<R>* a, const cplx<R>* X, int rb, bool xt, int q0) {
  const int l = threadIdx.x & 63;
  const int i = 16 * rb + (l & 15);
#pragma unroll
  for (int q = 0; q < N; q++) {
    const int k = 4 * (q0 + q) + (l >> 4);
    const int r = CT ? k : i, c = CT ? i : k;
    a[q] = X[xt ? r * T + c : c * T + r];
  }
}

template <typename R, bool CT, int N>
__device__ __forceinline__ void ss_mask_a(cplx<R>* a, int mask, int rb, int q0) {
  if (mask == SM_NONE) return;
  const int l = threadIdx.x & 63;
  const int i = 16 * rb + (l & 15);
#pragma unroll
  for (int q = 0; q < N; q++) {
    const int k = 4 * (q0 + q) + (l >> 4);
    const int r = CT ? k : i, c = CT ? i : k;
    if (mask == SM_UNIT_LOWER && r <= c) a[q] = cplx<R>{r == c ? (R)1 : (R)0, (R)0};
    if (mask == SM_UPPER && r > c) a[q] = cplx<R>{(R)0, (R)0};
  }
}

template <typename R, int NP, int NCB, int N, bool TR>
__device__ __forceinline__ void ss_load_b(cplx<R> (*b)[N], const cplx<R>* V, int q0) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int cb = 0; cb < NCB; cb++) {
    const int col = 16 * cb + ((TR && cb == NCB - 1) ? (l & 7) : (l & 15));
#pragma unroll
    for (int q = 0; q < N; q++) b[cb][q] = V[(4 * (q0 + q) + (l >> 4)) * NP + col];
  }
}

template <typename R, int NCB, int N, bool CA, bool TR>
__device__ __forceinline__ void ss_mma(SAcc<R, NCB>& acc, const cplx<R>* a, const cplx<R> (*b)[N]) {
  const bool im_lane = (threadIdx.x & 8) != 0;  // lanes 8 .. 15 of each 16
#pragma unroll
  for (int q = 0; q < N; q++) {
    const R ar = a[q].re, ai = CA ? -a[q].im : a[q].im;
    const R sa = ar + ai;
#pragma unroll
    for (int cb = 0; cb < NCB; cb++) {
      const R br = b[cb][q].re, bi = b[cb][q].im;
      if (TR && cb == NCB - 1) {
        // [re | im] = [ar ai] [[br, bi], [-bi, br]]: two real MFMAs
        acc.t = Mf<R>::op(ar, im_lane ? bi : br, acc.t);
        acc.t = Mf<R>::op(ai, im_lane ? br : -bi, acc.t);
      } else {
        acc.p1[cb] = Mf<R>::op(ar, br, acc.p1[cb]);
        acc.p2[cb] = Mf<R>::op(ai, bi, acc.p2[cb]);
        acc.p3[cb] = Mf<R>::op(sa, br + bi, acc.p3[cb]);
      }
    }
  }
}

// The products of a short piece's wave: its tile X (A role, chunk 0 already
// in pre) against the solved block V.  `later` issues the loads the products
// do not need; it runs once the first operands' loads are issued, since
// loads complete in order and the MFMAs would otherwise wait on them too.
template <typename R, int T, int NP, bool CA, bool TR, typename F>
__device__ __forceinline__ void ss_short(SAcc<R, NP / 16>& acc, SPre<R, T>& pre,
                                         const cplx<R>* X, const cplx<R>* V, int mask, int rb,
                                         bool xt, F&& later) {
  constexpr int NCB = NP / 16, PQ = ss_pq<R, T>(), NCK = (T / 4) / PQ;
  cplx<R> ba[NCB][PQ];
  ss_load_b<R, NP, NCB, PQ, TR>(ba, V, 0);
  if constexpr (NCK == 1) {
    later();
    ss_mask_a<R, CA, PQ>(pre.a, mask, rb, 0);
    ss_mma<R, NCB, PQ, CA, TR>(acc, pre.a, ba);
  } else {
    cplx<R> aa[PQ], ab[PQ], bb[NCB][PQ];
    ss_load_a<R, T, CA, PQ>(ab, X, rb, xt, PQ);
    ss_load_b<R, NP, NCB, PQ, TR>(bb, V, PQ);
    later();
    ss_mask_a<R, CA, PQ>(pre.a, mask, rb, 0);
    ss_mma<R, NCB, PQ, CA, TR>(acc, pre.a, ba);
#pragma unroll
    for (int c = 1; c < NCK; c++) {
      if (c % 2 == 1) {
        if (c + 1 < NCK) {
          ss_load_a<R, T, CA, PQ>(aa, X, rb, xt, (c + 1) * PQ);
          ss_load_b<R, NP, NCB, PQ, TR>(ba, V, (c + 1) * PQ);
        }
        ss_mask_a<R, CA, PQ>(ab, mask, rb, c * PQ);
        ss_mma<R, NCB, PQ, CA, TR>(acc, ab, bb);
      } else {
        if (c + 1 < NCK) {
          ss_load_a<R, T, CA, PQ>(ab, X, rb, xt, (c + 1) * PQ);
          ss_load_b<R, NP, NCB, PQ, TR>(bb, V, (c + 1) * PQ);
        }
        ss_mask_a<R, CA, PQ>(aa, mask, rb, c * PQ);
        ss_mma<R, NCB, PQ, CA, TR>(acc, aa, ba);
      }
    }
  }
}

// Loads the first chunk of a short piece's tile for this wave.  The loads
// are issued whatever the piece (from the first stored tile when the wave
// has nothing to load), so that the code around them has no branch: with
// loads on one side of a branch only, the compiler's wait counts after it
// are taken for the worst path, and the products would wait for this
// prefetch as well.
template <typename R, int T, bool ADJ>
__device__ __forceinline__ void ss_prefetch(SPre<R, T>& pre, const SSolveParams& P, const SPiece& p,
                                            int wave, bool want) {
  const int x = p.lo + wave;
  const bool ok = want && p.hi - p.lo + 1 <= kSsWaves && x <= p.hi;
  int mask;
  bool xt = false;
  const cplx<R>* X = reinterpret_cast<const cplx<R>*>(P.tiles);
  if (ok) X = ss_operand<R, T, ADJ>(P, p, x, mask, xt);
  ss_load_a<R, T, ADJ, ss_pq<R, T>()>(pre.a, X, ok ? p.rb : 0, xt, 0);
}

// SHORT: every piece is short (the band and the superblock span at most
// kSsWaves tiles), so the long-piece path is compiled out; its chunk buffers
// would otherwise set the register count (in FP64 with spills).  TR (short
// pieces only): the last column block holds at most 8 of the caller's
// columns and is formed in real form (SAcc).
template <typename R, int T, int NP, bool ADJ, bool SHORT, bool TR>
__global__ __launch_bounds__(64 * kSsWaves) void k_ssolve(SSolveParams P) {
  if (P.skip && __hip_atomic_load(P.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  constexpr int NCB = NP / 16;
  constexpr int RPT = T / 16;  // 16-row blocks per tile
  constexpr int QA = T / 4;    // k-steps per tile
  static_assert(16 * NP <= 64 * kSsWaves, "one element of a piece per thread");
  extern __shared__ __align__(16) char ss_smem[];
  cplx<R>* red = reinterpret_cast<cplx<R>*>(ss_smem);  // [kSsWaves][16][NP]
  __shared__ uint32_t s_ticket, s_next;
  // wave-uniform, so that the tile and block pointers live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NB = P.g.NB, NS = P.g.NS();
  const int npc = P.g.P * RPT;  // pieces per superblock phase
  const int home = xcc_id() % P.teams;
  // With P.local (a team per XCD, launch_ssolve) a workgroup serves its own
  // team only: every piece of a shift then runs on one XCD, whose L2 holds
  // what one piece hands to the next, so the hand-over is stored plainly
  // (the count that announces it is still a device-coherent atomic, and the
  // reader's acquire drops its stale L1 lines).
  const int nserve = P.local ? 1 : P.teams;
  for (int tt = 0; tt < nserve; tt++) {
    const int team = (home + tt) % P.teams;
    const int nw = (P.n_omega - team + P.teams - 1) / P.teams;  // this team's shifts
    const int64_t total = (int64_t)2 * NS * 2 * nw * npc;
    uint32_t* tick = P.tickets + team;
    // In its home team a workgroup holds two tickets: the piece it works on
    // and the next, whose wait it will meet with the operand already loaded.
    // It still finishes its tickets in order, so the smallest unfinished
    // ticket of a team is always a workgroup's current piece, whose inputs
    // are smaller tickets, all finished.  Serving another team (after its
    // own ran out) it takes one ticket at a time, as a piece of that team
    // then never waits on a ticket held back behind a piece of another team.
    // Where the pieces of a phase of all a team's shifts fit one round of
    // the team's workgroups (P.ahead = 0; launch_ssolve sets it), every
    // workgroup takes one ticket at a time: a second ticket would bind a
    // piece of the next phase to a workgroup still busy with another shift's
    // piece, while others are free.
    const bool ahead = tt == 0 && P.ahead;
    int64_t cur = wg_ticket(tick, &s_ticket);
    SPiece pc = ss_decode(cur, team, P.teams, nw, npc, RPT, P.g);
    SPre<R, T> pre;
    ss_prefetch<R, T, ADJ>(pre, P, pc, wave, cur < total);
    while (cur < total) {
      int* cnt_w = P.cnt + (int64_t)pc.w * 2 * NS * 2;
      auto counter = [&](int sw, int sup, int ph) { return cnt_w + ((int64_t)sw * NS + sup) * 2 + ph; };
      cplx<R>* xw = reinterpret_cast<cplx<R>*>(P.xs) + (int64_t)pc.w * NB * T * NP;
      cplx<R>* cw = reinterpret_cast<cplx<R>*>(P.cb) + (int64_t)pc.w * P.g.P * T * NP;
      const int lo = pc.lo, hi = pc.hi, rb = pc.rb, s = pc.s;
      const bool live = s < NB;
      const bool fast = SHORT || hi - lo + 1 <= kSsWaves;
      const int idx = threadIdx.x, er = idx / NP, ec = idx % NP;  // this thread's element
      const bool mine = idx < 16 * NP;
      // the caller's right-hand side of the first sweep (does not depend on the wait)
      double2 rhs = make_double2(0.0, 0.0);
      if (live && pc.phase == 0 && !pc.second && mine) {
        const int64_t r = (int64_t)s * T + 16 * rb + er;
        if (ec < P.k && r < P.n) rhs = P.Bm[(int64_t)pc.w * P.bstride + (int64_t)ec * P.n + r];
      }
      // a long piece (more tiles than waves) walks its tiles in chunks of QC
      // k-steps, two buffers, a chunk ahead; chunk 0's factor data is
      // loaded before the wait
      constexpr int QC = ss_qc<R, T, NCB>(), NCH = QA / QC;
      const int nch = !fast && lo + wave <= hi ? ((hi - lo - wave) / kSsWaves + 1) * NCH : 0;
      auto load = [&](SChunk<R, T, NCB>& c, int q, bool with_a, bool with_b) {
        const int x = lo + wave + (q / NCH) * kSsWaves, q0 = (q % NCH) * QC;
        if (with_a) {
          int mask;
          bool xt;
          const cplx<R>* a = ss_operand<R, T, ADJ>(P, pc, x, mask, xt);
          sc_load_a<R, T, ADJ, NCB>(c, a, mask, rb, xt, q0);
        }
        if (with_b)
          sc_load_b<R, T, NP, NCB>(c, pc.phase == 0 ? xw + (int64_t)x * T * NP
                                                    : cw + (int64_t)x * T * NP, q0);
      };
      SChunk<R, T, NCB> c0;
      if (nch > 0) load(c0, 0, true, false);
      // the step this piece waits for (and, in the home team, the next ticket)
      int* dep = nullptr;
      if (pc.phase == 1) dep = counter(pc.second, pc.S, 0);
      else if (!pc.second) dep = pc.S > 0 ? counter(0, pc.S - 1, 1) : nullptr;
      else dep = pc.S == NS - 1 ? counter(0, NS - 1, 1) : counter(1, pc.S + 1, 1);
      int64_t nxt = ss_wait(dep, npc, P.status, ahead ? tick : nullptr, &s_next);
      SPiece pn = pc;
      SPre<R, T> pren;
      if (ahead) pn = ss_decode(nxt, team, P.teams, nw, npc, RPT, P.g);
      // loads this piece's products do not wait for: the next piece's
      // operand (in flight during this piece's products; for a long piece
      // after them, whose chunk buffers would otherwise hold registers beside
      // it) and the second sweep's right-hand side y_s
      const bool pf = ahead && nxt < total;
      const bool want_ys = live && pc.phase == 0 && pc.second && mine;
      cplx<R> ys;  // (both loads unconditional: see ss_prefetch)
      auto later = [&]() {
        ys = xw[want_ys ? ((int64_t)s * T + 16 * rb + er) * NP + ec : 0];
        ss_prefetch<R, T, ADJ>(pren, P, pn, wave, pf);
      };
      if (!live) later();
      if (live) {
        //   phase A:  -sum_t T_st x_t       (the waves take the tiles in turn)
        //   phase B:  sum_j (D-hat^-1)_ij c_j
        SAcc<R, NCB> acc;
        acc.zero();
        if (fast) {
          const int x = lo + wave;
          if (x <= hi) {
            int mask;
            bool xt;
            const cplx<R>* X = ss_operand<R, T, ADJ>(P, pc, x, mask, xt);
            const cplx<R>* V = (pc.phase == 0 ? xw : cw) + (int64_t)x * T * NP;
            ss_short<R, T, NP, ADJ, TR>(acc, pre, X, V, mask, rb, xt, later);
          } else {
            later();
          }
        } else if (nch > 0) {
          load(c0, 0, false, true);
          SChunk<R, T, NCB> c1;
          for (int q = 0; q < nch; q += 2) {
            if (q + 1 < nch) load(c1, q + 1, true, true);
            sc_mma<R, T, NCB, ADJ>(acc, c0);
            if (q + 1 < nch) {
              if (q + 2 < nch) load(c0, q + 2, true, true);
              sc_mma<R, T, NCB, ADJ>(acc, c1);
            }
          }
        }
        if (!fast) later();
        // the waves' parts into LDS, summed in a fixed order
        const int l = threadIdx.x & 63;
#pragma unroll
        for (int c = 0; c < NCB; c++)
#pragma unroll
          for (int e = 0; e < 4; e++) {
            const int rw = (wave * 16 + Mf<R>::row(l, e)) * NP;
            if (TR && c == NCB - 1) {  // lane l%16 < 8: re of column l%8, else its im
              R* rr = reinterpret_cast<R*>(red);
              const int half = (l >> 3) & 1, col = 16 * c + (l & 7);
              rr[2 * (rw + col) + half] = pc.phase == 0 ? -acc.t[e] : acc.t[e];
              rr[2 * (rw + col + 8) + half] = (R)0;  // columns 8 .. 15 of the block
            } else {
              red[rw + 16 * c + (l & 15)] = sc_finish<R, NCB>(acc, c, e, pc.phase == 0);
            }
          }
        __syncthreads();
        if (want_ys) rhs = make_double2((double)ys.re, (double)ys.im);
        if (mine) {
          R sr = (R)rhs.x, sm = (R)rhs.y;  // zero in phase B
#pragma unroll
          for (int v = 0; v < kSsWaves; v++) {
            const cplx<R> p = red[v * 16 * NP + idx];
            sr += p.re;
            sm += p.im;
          }
          cplx<R>* dst = pc.phase == 0 ? cw + (int64_t)pc.i * T * NP : xw + (int64_t)s * T * NP;
          if (P.local)
            dst[(16 * rb + er) * NP + ec] = cplx<R>{sr, sm};
          else
            st_coherent(dst + (16 * rb + er) * NP + ec, cplx<R>{sr, sm});
          if (pc.phase == 1 && pc.second) {  // the solution into the caller's block
            const int64_t r = (int64_t)s * T + 16 * rb + er;
            if (ec < P.k && r < P.n)
              P.X[((int64_t)pc.w * P.k + ec) * P.n + r] = make_double2((double)sr, (double)sm);
          }
        }
      }
      ss_done(counter(pc.second, pc.S, pc.phase));
      if (!ahead) {
        nxt = wg_ticket(tick, &s_ticket);
        pn = ss_decode(nxt, team, P.teams, nw, npc, RPT, P.g);
        ss_prefetch<R, T, ADJ>(pren, P, pn, wave, nxt < total);
      }
      cur = nxt;
      pc = pn;
      pre = pren;
    }
  }
}

template <typename R, int T, int NP, bool ADJ>
static hipError_t ss_launch(const SSolveParams& P, int grid, hipStream_t s) {
  if (ss_all_short(P.g) && P.k - (NP - 16) <= 8)  // the last block's columns: at most 8
    hipLaunchKernelGGL((k_ssolve<R, T, NP, ADJ, true, true>), dim3(grid), dim3(64 * kSsWaves),
                       (ssolve_lds<R, T, NP>()), s, P);
  else if (ss_all_short(P.g))
    hipLaunchKernelGGL((k_ssolve<R, T, NP, ADJ, true, false>), dim3(grid), dim3(64 * kSsWaves),
                       (ssolve_lds<R, T, NP>()), s, P);
  else
    hipLaunchKernelGGL((k_ssolve<R, T, NP, ADJ, false, false>), dim3(grid), dim3(64 * kSsWaves),
                       (ssolve_lds<R, T, NP>()), s, P);
  return hipGetLastError();
}

template <typename R, int T>
static hipError_t ss_prepare_t() {
  hipError_t e = hipSuccess;
  auto set = [&](const void* fn, size_t lds) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  };
  set((const void*)k_ssolve<R, T, 16, false, false, false>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 16, true, false, false>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 32, false, false, false>, ssolve_lds<R, T, 32>());
  set((const void*)k_ssolve<R, T, 32, true, false, false>, ssolve_lds<R, T, 32>());
  set((const void*)k_ssolve<R, T, 16, false, true, false>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 16, true, true, false>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 32, false, true, false>, ssolve_lds<R, T, 32>());
  set((const void*)k_ssolve<R, T, 32, true, true, false>, ssolve_lds<R, T, 32>());
  set((const void*)k_ssolve<R, T, 16, false, true, true>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 16, true, true, true>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 32, false, true, true>, ssolve_lds<R, T, 32>());
  set((const void*)k_ssolve<R, T, 32, true, true, true>, ssolve_lds<R, T, 32>());
  return e;
}

hipError_t prepare_ssolve(int T, bool fp32) {
  if (fp32) return T == 64 ? ss_prepare_t<float, 64>() : ss_prepare_t<float, 32>();
  return T == 64 ? ss_prepare_t<double, 64>() : ss_prepare_t<double, 32>();
}

template <typename R, int T>
static hipError_t ss_dispatch(const SSolveParams& P, int NP, int adjoint, int grid,
                              hipStream_t s) {
  if (NP == 16)
    return adjoint ? ss_launch<R, T, 16, true>(P, grid, s) : ss_launch<R, T, 16, false>(P, grid, s);
  if (NP == 32)
    return adjoint ? ss_launch<R, T, 32, true>(P, grid, s) : ss_launch<R, T, 32, false>(P, grid, s);
  return hipErrorInvalidValue;
}

// piece counters, then the teams' ticket counters
int64_t ssolve_counters(const BandGeom& g, int n_omega) {
  return (int64_t)n_omega * 2 * g.NS() * 2 + kTeams;
}

hipError_t launch_ssolve(const BandGeom& g, int n, int n_omega, int k, bool fp32,
                         const void* tiles, int adjoint, const double* Bm, int64_t bstride,
                         double* X, void* xs, void* cbuf, int* cnt, uint32_t* ticket,
                         uint32_t* status, int grid, hipStream_t s, const uint32_t* skip) {
  const int NP = solve_np(k);
  if (NP > 32 || g.P < 1) return hipErrorInvalidValue;
  (void)ticket;  // the teams' counters follow the piece counters in cnt
  const int npc = g.P * (g.T / 16);
  const int64_t npiece = (int64_t)n_omega * 2 * g.NS() * 2;
  SSolveParams P{g, n, n_omega, k, tiles, (const double2*)Bm, bstride, (double2*)X, xs, cbuf,
                 cnt, (uint32_t*)(cnt + npiece), status, n_omega < kTeams ? n_omega : kTeams,
                 skip};
  {  // a second ticket where a phase's pieces outnumber a team's CUs, and in
     // FP32 also where they just fill them: without slack the second ticket
     // is the only lead for FP32's whole-tile prefetch of the next piece
     // (FP32, 16 shifts, 4 block rows: forward / adjoint 32.1 / 33.4 ms with
     // it, 34.0 / 42.0 without; FP64, which prefetches a quarter tile: 42.4
     // with, 38.9 without).  With slack (one shift: 32 pieces for 256 CUs)
     // one ticket each already reaches phases ahead.
    static int cus = 0;
    if (cus == 0) {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
          cus <= 0)
        cus = 256;
    }
    const int per_team = (n_omega + P.teams - 1) / P.teams;
    const int64_t pieces = (int64_t)npc * per_team, team_cus = cus / P.teams;
    P.ahead = (fp32 ? pieces >= team_cus : pieces > team_cus) ? 1 : 0;
  }
  hipError_t e = launch_fill_u32((uint32_t*)cnt, 0u, ssolve_counters(g, n_omega), s);
  if (e != hipSuccess) return e;
  const int64_t total = npiece * npc;
  if (grid > total) grid = (int)total;
  // a team per XCD, each with workgroups of its own (the launch deals them
  // to the XCDs in turn): handoffs within one L2
  P.local = P.teams == kTeams && grid >= 8 * kTeams ? 1 : 0;
  if (fp32) {
    if (g.T == 64) return ss_dispatch<float, 64>(P, NP, adjoint, grid, s);
    if (g.T == 32) return ss_dispatch<float, 32>(P, NP, adjoint, grid, s);
  } else {
    if (g.T == 64) return ss_dispatch<double, 64>(P, NP, adjoint, grid, s);
    if (g.T == 32) return ss_dispatch<double, 32>(P, NP, adjoint, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace rr
