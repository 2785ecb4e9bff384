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
// implies every earlier step), phase B for its own phase A.  Data handed
// between workgroups (c and the sweep's blocks) is stored device-coherent
// (st_coherent) before the release and the counter increment; readers poll
// with atomics, then acquire.
#include "rr_mfma.h"

namespace rr {

namespace {

enum { SM_NONE = 0, SM_UNIT_LOWER = 1, SM_UPPER = 2 };

// A piece's products are walked in chunks of QC k-steps (4 QC columns of the
// inner dimension of one tile): the A-role fragment of the stored tile and
// the B-role fragments of the solved block for each of the NCB column
// blocks.  With one column block in FP32 a chunk is a whole tile, so that
// every load of a wave's tile is in flight before its first MFMA; otherwise
// (more registers per chunk) a chunk is a half (FP32) or a quarter (FP64) of
// a tile and the next chunk is loaded one ahead of the current one's MFMAs
// (two buffers).
template <typename R, int T, int NCB>
constexpr int ss_qc() { return sizeof(R) == 8 ? T / 16 : (NCB == 1 ? T / 4 : T / 8); }

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
template <typename R, int NCB>
struct SAcc {
  typename Mf<R>::v4 p1[NCB], p2[NCB], p3[NCB];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < NCB; c++)
#pragma unroll
      for (int e = 0; e < 4; e++) { p1[c][e] = 0; p2[c][e] = 0; p3[c][e] = 0; }
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
};

constexpr int kTeams = 8;  // XCDs of gfx950

// The XCD this wave runs on (hardware register XCC_ID).
__device__ __forceinline__ int xcc_id() {
  return (int)(__builtin_amdgcn_s_getreg((15 << 11) | 20) & 0xF);
}

// Thread 0 polls *c until it reaches `want`, then issues one acquire fence;
// the barrier hands the result to every wave.  Bounded like every dataflow
// wait of the library (ST_TIMEOUT).
__device__ __forceinline__ void ss_wait(int* c, int want, uint32_t* status) {
  if (threadIdx.x == 0) {
    bool live =
        !(__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_TIMEOUT);
    const uint64_t t0 = wall_clock64();
    uint32_t polls = 0;
    while (live &&
           __hip_atomic_fetch_add(c, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
      __builtin_amdgcn_s_sleep(1);
      if (++polls > kWaitPolls || wall_clock64() - t0 > kWaitTicks) {
        latch(status, ST_TIMEOUT);
        live = false;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Every thread's stores are complete, then thread 0 releases and counts the
// piece done; barriers close the interval on both sides.
__device__ __forceinline__ void ss_done(int* c) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

constexpr int kSsWaves = 8;  // waves per workgroup: they split a piece's inner dimension

template <typename R, int T, int NP>
constexpr size_t ssolve_lds() {  // per-wave partial sums, the summed piece, its b
  return sizeof(cplx<R>) * (size_t)16 * NP * (kSsWaves + 1) + sizeof(double2) * 16 * NP;
}

template <typename R, int T, int NP, bool ADJ>
__global__ __launch_bounds__(64 * kSsWaves) void k_ssolve(SSolveParams P) {
  if (P.skip && __hip_atomic_load(P.skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  constexpr int NCB = NP / 16;
  constexpr int NT = 64 * kSsWaves;
  constexpr int RPT = T / 16;  // 16-row blocks per tile
  extern __shared__ __align__(16) char ss_smem[];
  cplx<R>* red = reinterpret_cast<cplx<R>*>(ss_smem);   // [kSsWaves][16][NP]
  cplx<R>* outb = red + kSsWaves * 16 * NP;              // [16][NP]
  double2* bin = reinterpret_cast<double2*>(outb + 16 * NP);  // [16][NP] right-hand side
  __shared__ uint32_t s_ticket;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int B = P.g.B, NB = P.g.NB, RT = P.g.row_tiles(), PS = P.g.P, NS = P.g.NS();
  const int npc = PS * RPT;  // pieces per superblock phase
  const int home = xcc_id() % P.teams;
  for (int tt = 0; tt < P.teams; tt++) {
   const int team = (home + tt) % P.teams;
   const int nw = (P.n_omega - team + P.teams - 1) / P.teams;  // this team's shifts
   const int64_t total = (int64_t)2 * NS * 2 * nw * npc;
   for (;;) {
    const int64_t ticket = wg_ticket(P.tickets + team, &s_ticket);
    if (ticket >= total) break;
    int64_t t = ticket;
    const int pc = (int)(t % npc);
    t /= npc;
    const int w = team + P.teams * (int)(t % nw);
    t /= nw;
    const int phase = (int)(t % 2);
    t /= 2;
    const int si = (int)(t % NS);
    const int second = (int)(t / NS);
    const int S = second ? NS - 1 - si : si;
    const int i = pc / RPT, rb = pc % RPT;
    const int s0 = S * PS, s = s0 + i;
    int* cnt_w = P.cnt + (int64_t)w * 2 * NS * 2;
    auto counter = [&](int sw, int sup, int ph) { return cnt_w + ((int64_t)sw * NS + sup) * 2 + ph; };
    const cplx<R>* tw = reinterpret_cast<const cplx<R>*>(P.tiles) + (int64_t)w * NB * RT * (T * T);
    auto tile = [&](int r, int c) { return tw + ((int64_t)r * RT + (c - r + B)) * (T * T); };
    auto sbt = [&](int r, int slot) {
      return tw + ((int64_t)r * RT + P.g.sb_index(slot)) * (T * T);
    };
    cplx<R>* xw = reinterpret_cast<cplx<R>*>(P.xs) + (int64_t)w * NB * T * NP;
    cplx<R>* cw = reinterpret_cast<cplx<R>*>(P.cb) + (int64_t)w * PS * T * NP;
    // this piece's inner dimension: tiles t0 .. t1 of the band outside the
    // superblock (phase A), or j0 .. j1 of the superblock's inverse (phase B)
    int lo = 0, hi = -1;
    if (s < NB) {
      if (phase == 0) {
        if (!second) { lo = max(0, s - B); hi = s0 - 1; }
        else { lo = s0 + PS; hi = min(NB - 1, s + B); }
      } else {
        if (!second) { lo = 0; hi = i; }
        else { lo = i; hi = min(PS - 1, NB - 1 - s0); }
      }
    }
    // A-role operand of inner index x: pointer, mask, row-major storage
    auto operand = [&](int x, int& mask, bool& xt) -> const cplx<R>* {
      if (phase == 0) {
        mask = SM_NONE;
        xt = ADJ != (bool)second;  // U tiles (row-major) in this sweep
        return ADJ ? tile(x, s) : tile(s, x);
      }
      const int j = x;
      if (!ADJ) {
        mask = j == i ? (second ? SM_UPPER : SM_UNIT_LOWER) : SM_NONE;
        xt = second && j != i;       // (U-hat^-1)_ij row-major, (L-hat^-1)_ij column-major
        return j == i ? tile(s, s) : sbt(s, sb_slot(i, j));
      }
      mask = j == i ? (second ? SM_UNIT_LOWER : SM_UPPER) : SM_NONE;
      xt = !second && j != i;        // ((U-hat^-1)_ji)^H or ((L-hat^-1)_ji)^H
      return j == i ? tile(s, s) : sbt(s0 + j, sb_slot(j, i));
    };
    // this wave's chunks: tiles x = lo + wave, lo + wave + kSsWaves, ... (NCH
    // chunks each); chunk 0's factor data does not depend on the wait and
    // is loaded before it
    constexpr int QC = ss_qc<R, T, NCB>(), NCH = (T / 4) / QC;
    const int nch = lo + wave <= hi ? ((hi - lo - wave) / kSsWaves + 1) * NCH : 0;
    auto load = [&](SChunk<R, T, NCB>& c, int idx, bool with_a, bool with_b) {
      const int x = lo + wave + (idx / NCH) * kSsWaves, q0 = (idx % NCH) * QC;
      if (with_a) {
        int mask;
        bool xt;
        const cplx<R>* a = operand(x, mask, xt);
        sc_load_a<R, T, ADJ, NCB>(c, a, mask, rb, xt, q0);
      }
      if (with_b)
        sc_load_b<R, T, NP, NCB>(c, phase == 0 ? xw + (int64_t)x * T * NP
                                               : cw + (int64_t)x * T * NP, q0);
    };
    SChunk<R, T, NCB> c0;
    if (nch > 0) load(c0, 0, true, false);
    if (s < NB && phase == 0 && !second) {  // the caller's right-hand side (row-fastest)
      const double2* Bw = P.Bm + (int64_t)w * P.bstride;
      for (int idx = threadIdx.x; idx < 16 * NP; idx += NT) {
        const int rr = idx % 16, c = idx / 16;
        const int64_t r = (int64_t)s * T + 16 * rb + rr;
        double2 v = make_double2(0.0, 0.0);
        if (c < P.k && r < P.n) v = Bw[(int64_t)c * P.n + r];
        bin[rr * NP + c] = v;
      }
    }
    // the step this piece waits for
    if (phase == 1) {
      ss_wait(counter(second, S, 0), npc, P.status);
    } else if (!second) {
      if (S > 0) ss_wait(counter(0, S - 1, 1), npc, P.status);
    } else {
      if (S == NS - 1) ss_wait(counter(0, NS - 1, 1), npc, P.status);
      else ss_wait(counter(1, S + 1, 1), npc, P.status);
    }
    if (s < NB) {
      SAcc<R, NCB> acc;
      acc.zero();
      if (phase == 0 && second) {  // the first sweep's y_s
        const cplx<R>* ys = xw + (int64_t)s * T * NP;
        for (int idx = threadIdx.x; idx < 16 * NP; idx += NT) {
          const int rr = idx / NP, c = idx % NP;
          cplx<R> v = ys[(16 * rb + rr) * NP + c];
          bin[idx] = make_double2((double)v.re, (double)v.im);
        }
      }
      //   phase A:  -sum_t T_st x_t       (the waves take the tiles in turn)
      //   phase B:  sum_j (D-hat^-1)_ij c_j
      if (nch > 0) load(c0, 0, false, true);
      if constexpr (NCH == 1) {  // one buffer: a chunk is a whole tile
        for (int idx = 0; idx < nch; idx++) {
          if (idx > 0) load(c0, idx, true, true);
          sc_mma<R, T, NCB, ADJ>(acc, c0);
        }
      } else {                         // two buffers, one chunk ahead
        SChunk<R, T, NCB> c1;
        for (int idx = 0; idx < nch; idx += 2) {
          if (idx + 1 < nch) load(c1, idx + 1, true, true);
          sc_mma<R, T, NCB, ADJ>(acc, c0);
          if (idx + 1 < nch) {
            if (idx + 2 < nch) load(c0, idx + 2, true, true);
            sc_mma<R, T, NCB, ADJ>(acc, c1);
          }
        }
      }
      // the waves' parts into LDS, summed in a fixed order
#pragma unroll
      for (int c = 0; c < NCB; c++)
#pragma unroll
        for (int e = 0; e < 4; e++)
          red[(wave * 16 + Mf<R>::row(l, e)) * NP + 16 * c + (l & 15)] =
              sc_finish<R, NCB>(acc, c, e, phase == 0);
      __syncthreads();
      for (int idx = threadIdx.x; idx < 16 * NP; idx += NT) {
        R sr = 0, sm = 0;
        if (phase == 0) {
          const double2 b = bin[idx];
          sr = (R)b.x;
          sm = (R)b.y;
        }
#pragma unroll
        for (int v = 0; v < kSsWaves; v++) {
          const cplx<R> p = red[v * 16 * NP + idx];
          sr += p.re;
          sm += p.im;
        }
        const int rr = idx / NP, c = idx % NP;
        cplx<R>* dst = phase == 0 ? cw + (int64_t)i * T * NP : xw + (int64_t)s * T * NP;
        st_coherent(dst + (16 * rb + rr) * NP + c, cplx<R>{sr, sm});
        outb[idx] = cplx<R>{sr, sm};
      }
      if (phase == 1 && second) {  // the solution into the caller's block (row-fastest)
        __syncthreads();
        double2* Xw = P.X + (int64_t)w * P.k * P.n;
        for (int idx = threadIdx.x; idx < 16 * NP; idx += NT) {
          const int rr = idx % 16, c = idx / 16;
          const int64_t r = (int64_t)s * T + 16 * rb + rr;
          if (c < P.k && r < P.n) {
            const cplx<R> v = outb[rr * NP + c];
            Xw[(int64_t)c * P.n + r] = make_double2((double)v.re, (double)v.im);
          }
        }
      }
    }
    ss_done(counter(second, S, phase));
   }
  }
}

template <typename R, int T, int NP, bool ADJ>
static hipError_t ss_launch(const SSolveParams& P, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_ssolve<R, T, NP, ADJ>), dim3(grid), dim3(64 * kSsWaves),
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
  set((const void*)k_ssolve<R, T, 16, false>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 16, true>, ssolve_lds<R, T, 16>());
  set((const void*)k_ssolve<R, T, 32, false>, ssolve_lds<R, T, 32>());
  set((const void*)k_ssolve<R, T, 32, true>, ssolve_lds<R, T, 32>());
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
  hipError_t e = launch_fill_u32((uint32_t*)cnt, 0u, ssolve_counters(g, n_omega), s);
  if (e != hipSuccess) return e;
  const int64_t total = npiece * npc;
  if (grid > total) grid = (int)total;
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
