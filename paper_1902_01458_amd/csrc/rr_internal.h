// Internal declarations shared by the HIP sources of librr.so (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rr.h"

namespace rr {

// ---------------------------------------------------------------------------
// Device status word (latched per handle, read by rr_check)
// ---------------------------------------------------------------------------
enum : uint32_t {
  ST_SINGULAR = 1u << 0,
  ST_NOT_CONVERGED = 1u << 1,
  ST_BREAKDOWN = 1u << 2,
  ST_NONFINITE = 1u << 3,
  ST_TIMEOUT = 1u << 4,
  ST_SVD_NOT_CONVERGED = 1u << 5,  // the k x k Jacobi SVD still rotated at its sweep cap
};

// Wall-clock bound of any dataflow wait (constant 100 MHz counter ticks).
// A legitimate wait is shorter than one full factorisation; 20 s means a bug.
constexpr uint64_t kWaitTicks = 20ull * 100000000ull;

template <typename R>
struct cplx {
  R re, im;
};

__device__ __forceinline__ void latch(uint32_t* status, uint32_t bit) {
  atomicOr(status, bit);
}

// Store of data that another workgroup of the same launch reads after a flag
// handshake (tiles of the factorisation, blocks of the solves).  gfx950 has
// one L2 per XCD.  With ordinary write-back stores, an agent-scope release
// before the flag and an acquire after it did not reliably hand a band tile
// to readers on other XCDs (nor did system-scope fences): at n = 262144 with
// 16 shifts about half of the refactorisations gave a wrong LU.  A relaxed
// agent-scope atomic store is device-coherent (sc1, written through), and the
// s_waitcnt before the release covers its completion; with every handed-over
// tile stored this way none of 48 factorisations was wrong.  Readers keep
// ordinary loads after their acquire.  As every handed-over value is written
// through, a writer's release needs no L2 write-back: the factorisation and
// the solves wait for their stores' completion and release at workgroup
// scope before the flag or count.  (The superblock solve stores plainly where
// its writer and readers share one XCD, and so its L2: a team per XCD.)
__device__ __forceinline__ void st_coherent(cplx<float>* p, cplx<float> v) {
  uint64_t bits = (uint64_t)__float_as_uint(v.re) | ((uint64_t)__float_as_uint(v.im) << 32);
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), bits, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(cplx<double>* p, cplx<double> v) {
  __hip_atomic_store(&p->re, v.re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->im, v.im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Hard bound on polls of one wait, independent of the clock (a poll is one
// device-coherent atomic plus a short sleep, i.e. at least ~1 us).
constexpr uint32_t kWaitPolls = 1u << 25;

// Next ticket of a persistent launch, the same value in every thread.  The
// leading barrier closes the previous task (its readers of *slot are done).
// Every flag publish before it ends with a barrier too: with the flag store
// and the ticket fetch both guarded by "thread 0" and nothing convergent in
// between, the compiler may otherwise send the other threads straight to the
// ticket barrier, splitting the persistent loop so that only thread 0 ever
// leaves it to take a new ticket.
__device__ __forceinline__ int64_t wg_ticket(uint32_t* counter, uint32_t* slot) {
  __syncthreads();
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1u);
  __syncthreads();
  return (int64_t)__builtin_amdgcn_readfirstlane(*slot);
}

// ---------------------------------------------------------------------------
// Launch helpers implemented in the .hip files
// ---------------------------------------------------------------------------
struct OpDesc {  // the operator on the device
  int nx, ny, n;
  const double* coef;
};

struct BandGeom {  // tile geometry of the band factor
  int T;     // tile edge
  int B;     // tiles per half-band: ceil(b / T)
  int NB;    // block rows: ceil(n / T)
  int P = 0; // superblock: P consecutive block rows solved as one step
             // (rr_ssolve.hip); 0 = the tile-by-tile solve (rr_solve.hip)
  // Block row s stores its 2B+1 band tiles (s, s-B) .. (s, s+B), then, for
  // the tile-by-tile solve only (P = 0), the kChain chain tiles of its
  // recurrences, then the diagonal tile's LU with inverted 16 x 16 diagonal
  // blocks, read only by the factorisation itself (rr_band.hip), then
  // (P > 1) P - 1 tiles of the inverses of its superblock's diagonal block
  // (sb_slot below).
  static constexpr int kChainD = 3;            // neighbour distances with chain tiles
  static constexpr int kChain = 4 * kChainD;   // chain_index() below
  __host__ __device__ int chain_tiles() const { return P > 0 ? 0 : kChain; }
  __host__ __device__ int sb_slots() const { return P > 1 ? P - 1 : 0; }
  __host__ __device__ int lub_index() const { return 2 * B + 1 + chain_tiles(); }
  __host__ __device__ int sb_index(int slot) const { return lub_index() + 1 + slot; }
  __host__ __device__ int row_tiles() const { return lub_index() + 1 + sb_slots(); }
  __host__ __device__ int64_t tiles_per_omega() const { return (int64_t)NB * row_tiles(); }
  __host__ __device__ int NS() const { return P > 0 ? (NB + P - 1) / P : 0; }  // superblocks
};

// Superblock S holds block rows s0 = S P .. s0 + P - 1.  Its diagonal block
// is block-lower L-hat (tiles L_ij, j <= i) times block-upper U-hat; the
// factorisation's last pass stores the off-diagonal tiles of their inverses:
// (L-hat^-1)_ij, j < i, column-major like L tiles, and (U-hat^-1)_ij, j > i,
// row-major like U tiles, in block row s0 + i, at aux slot j (L) or j - 1
// (U); the diagonal tiles of both inverses are the diagonal tile's own
// [U^-1 | L^-1].
__host__ __device__ inline int sb_slot(int i, int j) { return j < i ? j : j - 1; }

// Chain tiles of block row s (formed by the factorisation, read by the
// solves): one kind per sweep, for the neighbours at distance d = 1 .. kChainD.
enum { CH_FWD_L = 0, CH_FWD_U = 1, CH_ADJ_U = 2, CH_ADJ_L = 3 };
__host__ __device__ inline int chain_index(int kind, int d) {
  return BandGeom::kChainD * kind + d - 1;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s);
hipError_t launch_burgers_coeffs(int nx, int ny, const double* U, double hx, double hy,
                                 double nu, double* coef, double* phi, hipStream_t s);
// Y = b - M X (residual) or Y = M X; adjoint applies M^H.  k columns per shift.
// Bm's blocks are bstride elements apart (0: one block shared by every shift).
// skip: optional device word; when non-zero at run time the kernel does nothing.
hipError_t launch_apply(const OpDesc& op, const double* omega /*dev 2*n_omega*/, int n_omega,
                        int k, int adjoint, const double* X, const double* Bm, int64_t bstride,
                        double* Y, hipStream_t s, const uint32_t* skip = nullptr);
// Theta (k, n) of step 1 for an elementwise kind (RR_TM_ORTHONORMAL: the
// unweighted Gaussian matrix, to be orthonormalised and weighted by the
// caller); zeta: nonzeros per row of RR_TM_SPARSE, already in [1, k].
hipError_t launch_sketch(const OpDesc& op, const double* phi, int k, uint64_t seed, int kind,
                         int zeta, double* Theta, hipStream_t s);
// Theta[j][r] *= phi[r / 2]
hipError_t launch_weight_rows(int64_t n, int k, const double* phi, double* Theta, hipStream_t s);

// Band LU: tiles = n_omega * tiles_per_omega() tiles of T*T complex (R = float|double).
// counters: two device words (task tickets, diagonal-worker roles); the launch
// has grid + n_omega workgroups.
// ev (optional, two events): recorded right before and after the first
// factor kernel launch (timing of that kernel alone).
hipError_t launch_factor(const OpDesc& op, const BandGeom& g, const double* omega,
                         int n_omega, bool fp32, void* tiles, int* flags, uint32_t* counters,
                         uint32_t* status, int grid, hipStream_t s,
                         const hipEvent_t* ev = nullptr);
// Dynamic-LDS attributes of the factor / solve kernels for one tile and
// precision; called when a handle is created, never on the launch path.
hipError_t prepare_factor(int T, bool fp32);
hipError_t prepare_solve(int T, bool fp32);
// Multi-RHS solve with the band factor: X = M^-1 Bm (adjoint: M^-H Bm).
// Bm's blocks are bstride complex elements apart (0: shared); Bm may alias X.
// xs: workspace of n_omega * NB * T * solve_np(k) complex (FP64 size).
// With g.P > 0 the superblock solve runs (rr_ssolve.hip; cbuf: n_omega * P *
// T * solve_np(k) complex, FP64 size; flags: ssolve_counters() words), else
// the tile-by-tile solve (rr_solve.hip).
int solve_np(int k);
hipError_t launch_solve(const BandGeom& g, int n, int n_omega, int k, bool fp32,
                        const void* tiles, int adjoint, const double* Bm, int64_t bstride,
                        double* X, void* xs, void* cbuf, int* flags, uint32_t* ticket,
                        uint32_t* status, int grid, hipStream_t s,
                        const uint32_t* skip = nullptr);
hipError_t launch_ssolve(const BandGeom& g, int n, int n_omega, int k, bool fp32,
                         const void* tiles, int adjoint, const double* Bm, int64_t bstride,
                         double* X, void* xs, void* cbuf, int* cnt, uint32_t* ticket,
                         uint32_t* status, int grid, hipStream_t s, const uint32_t* skip);
int64_t ssolve_counters(const BandGeom& g, int n_omega);
hipError_t prepare_ssolve(int T, bool fp32);

// Small dense / tall-skinny kernels (rr_small.hip)
constexpr int kJacobiSweeps = 40;  // one-sided Jacobi: sweeps before non-convergence
struct SmallWs {   // workspace for tall-skinny reductions
  double* partial;     // n_omega * nchunk * kmax*kmax complex
  double* G;           // n_omega * kmax*kmax complex
  double* R;           // n_omega * kmax*kmax complex (upper triangular factor)
  double* Rinv;        // n_omega * kmax*kmax complex (applied matrix)
  double* W;           // n_omega * kmax*kmax complex (SVD right vectors)
  double* Ut;          // n_omega * kmax*kmax complex (SVD left vectors)
  double* rho;         // n_omega * kRhoStride: each column's last relative correction
                       // (refinement), then the measured contraction per direction
  uint32_t* shifted;   // n_omega: 1 where the first Cholesky QR pass needed the shift
  int nchunk;
  int kmax;
  int jacobi_sweeps = kJacobiSweeps;  // sweep cap of the k x k Jacobi SVD
  double* big1 = nullptr;  // wide sketches (k > 32): n_omega * (kmax+1)^2 complex each
  double* big2 = nullptr;
};
// CholQR2 in place: Y <- Q = Y R^-1 with R upper, real positive diagonal.
// A shift whose Gram matrix is not numerically positive definite takes
// shifted CholeskyQR3 instead (three passes, the first with a diagonal shift).
hipError_t launch_cholqr2(int n, int n_omega, int k, double* Y, SmallWs& ws, uint32_t* status,
                          hipStream_t s);
// Z = Qz R (CholQR2, or shifted CholQR3 as above); SVD of R^H = Ut S W^H; sigma = S; V = Z R^-1 W;
// if Uqu != NULL also Uqu = Q Ut.
hipError_t launch_small_svd(int n, int n_omega, int k, const double* Z, const double* Q,
                            double* sigma, double* V, double* Uqu, SmallWs& ws,
                            uint32_t* status, hipStream_t s);
// U_j = scale_j W_j for every shift (W may alias U)
hipError_t launch_scale_cols(int n, int n_omega, int k, const double* W, const double* scale,
                             double* U, hipStream_t s);
// sigma_j = ||W_j||, U_j = W_j / sigma_j  (W may alias U)
hipError_t launch_colnorm_scale(int n, int n_omega, int k, const double* W, double* sigma,
                                double* U, SmallWs& ws, uint32_t* status, hipStream_t s);
// GMRES-IR workspace (rr_gmres.hip): m + 1 Krylov blocks V of n_omega*k_max*n
// complex, the product block t, and per column (w*k + c) the Hessenberg
// matrix H ((m+1) x m), the projections h (m+1), beta, y (m) and the chunk
// partial sums of the projections.
constexpr int kGmresMaxRestart = 16;
struct GmresWs {
  double* V = nullptr;
  double* t = nullptr;
  double* H = nullptr;
  double* h = nullptr;
  double* beta = nullptr;
  double* y = nullptr;
  double* partial = nullptr;
  int m = 0;  // restart length; 0: plain refinement
};
int gmres_nchunk(int64_t n);
// x -= V_{0..j} (V_{0..j}^H x) per column, the projections added to column j of H
hipError_t launch_gs_project(int64_t n, int n_omega, int k, int j, const GmresWs& g, double* x,
                             const uint32_t* skip, hipStream_t s);
// H[j+1][j] = norm per column
hipError_t launch_store_subdiag(int n_omega, int k, int j, const GmresWs& g, const double* norm,
                                const uint32_t* skip, hipStream_t s);
// y = argmin || beta e_1 - H y || per column, out = V_{0..m-1} y
hipError_t launch_gmres_finish(int64_t n, int n_omega, int k, const GmresWs& g, double* out,
                               const uint32_t* skip, hipStream_t s);
// X += D after correction `it` (0-based) and the per-column convergence test
// on e_j = ||D_j|| / ||X_j||: converged when e_j <= tol or when the error left,
// estimated as e_j times the measured contraction of this shift and
// direction (the ratio of successive corrections; rr_small.hip), is below
// tol / 2.
constexpr int kRhoStride = 64;  // doubles per shift in SmallWs::rho
constexpr int kRhoSlot = 62;    // [62]: measured contraction (both directions)
constexpr int kProbeSlot = 32;  // [32, 32 + p): the probe columns' errors before correcting
// X += D over the first kk columns (default k), the converged test on the
// first k; with probes (p > 0: columns k .. k+p-1 solve M x = M z for the
// known z of Z, p blocks of n per shift) the first correction (it = 0) also
// measures the contraction on them.
hipError_t launch_refine_update(int n, int n_omega, int k, double* X, const double* D,
                                double tol, int it, int adjoint, SmallWs& ws, uint32_t* status,
                                uint32_t* fail_count, hipStream_t s,
                                const uint32_t* skip = nullptr, int kk = 0, int p = 0,
                                const double* Z = nullptr);
// The probe columns' errors ||X_{k0+q} - Z_q|| (q < p) after the first solve,
// kept in the contraction rows for the first correction.
hipError_t launch_probe_errors(int n, int n_omega, int kk, int k0, int p, const double* X,
                               const double* Z, SmallWs& ws, uint32_t* status, hipStream_t s);
// ncols columns from src (shift stride sws complex, 0 = shared; first column
// sc0) to dst (shift stride dws, first column dc0); columns are n long
hipError_t launch_cols_place(int64_t n, int n_omega, int ncols, const double* src, int64_t sws,
                             int sc0, double* dst, int64_t dws, int dc0, hipStream_t s);
// Zero the measured contractions of every shift (after a refactorisation).
hipError_t launch_refine_reset(int n_omega, double* rho, hipStream_t s);
// Wide sketches, 32 < k <= kMaxWideK (rr_bigk.hip), FP64 only
constexpr int kMaxWideK = 512;
int gramb_chunks(int64_t n);
hipError_t launch_cholqr2_big(int64_t n, int n_omega, int k, double* Y, double* tmp, SmallWs& ws,
                              uint32_t* status, hipStream_t s);
hipError_t launch_small_svd_big(int64_t n, int n_omega, int k, const double* Z, const double* Q,
                                double* sigma, double* V, double* Uqu, double* tmp,
                                SmallWs& ws, uint32_t* status, hipStream_t s);
hipError_t launch_colnorm_big(int64_t n, int n_omega, int k, const double* X, double* sigma,
                              double* U, uint32_t* status, hipStream_t s);
// columns [c0, c0 + kg) of a block with k columns per shift (shift stride
// wstride complex, 0 = shared) to / from a block of kg columns per shift
hipError_t launch_cols_copy(int64_t n, int n_omega, int k, int64_t wstride, int c0, int kg,
                            const double* src, double* dst, bool gather, hipStream_t s);

// LU-free Krylov solves (rr_krylov.hip)
int krylov_nchunk(int64_t n);
size_t ilu0_lds(int ny);
size_t pc_bytes(int precond, int nx, int ny, int n_omega);
hipError_t prepare_krylov(int ny);
// Dinv[w][p] (4 complex): the inverted node blocks of the preconditioner
hipError_t launch_pc_setup(const OpDesc& op, int precond, const double* omega, int n_omega,
                           double* Dinv, uint32_t* status, hipStream_t s);
// Y = K^-1 X (or K^-H X) for k columns of every shift; systems with
// active[q] == 0 are left alone (active may be NULL)
hipError_t launch_pc_apply(const OpDesc& op, int precond, int n_omega, int k, int adjoint,
                           const double* Dinv, const double* X, double* Y,
                           const uint32_t* active, const uint32_t* skip, hipStream_t s);
// partial sums of <A_e, B_e> per system (npair 1 or 2)
hipError_t launch_kdot(int64_t n, int n_omega, int k, int npair, const double* A0,
                       const double* B0, const double* A1, const double* B1, double* partial,
                       const uint32_t* active, const uint32_t* skip, hipStream_t s);
// the scalar steps of BiCGStab (mode 0 start, 1 rho / beta, 2 alpha, 3 omega,
// 4 convergence check), ks: 4 complex per system
hipError_t launch_bicg_scalars(int N, int64_t n, int mode, int it, double tol,
                               const double* partial, double* ks, double* bnorm2,
                               uint32_t* active, uint32_t* conv, uint32_t* status,
                               const uint32_t* skip, hipStream_t s);
// vector steps: 0 p = r + beta (p - omega v); 1 r -= alpha v;
// 2 x += alpha y + omega z, r -= omega t; 3 x += d
hipError_t launch_bicg_vec(int which, int64_t n, int n_omega, int k, const double* ks,
                           const double* a, const double* b, const double* c, double* x,
                           double* y, const uint32_t* active, const uint32_t* skip,
                           hipStream_t s);
hipError_t launch_kcopy(int64_t count, const double* a, double* b, hipStream_t s);
hipError_t launch_latch_live(int N, const uint32_t* active, uint32_t* status, uint32_t bit,
                             hipStream_t s);
// gradient kernel (rr_grad.hip)
hipError_t launch_grad(int nx, int ny, double hx, double hy, int n_omega,
                       const double* omega, const double* sigma1, const double* u1,
                       const double* v1, int64_t stride, double* dU, double* dnu,
                       double* domega, double* partial, int nchunk, hipStream_t s);

}  // namespace rr

// ---------------------------------------------------------------------------
// The handle
// ---------------------------------------------------------------------------
struct rr_factors {
  int nx, ny, n, n_omega, k_max;
  rr_precision prec;
  rr::BandGeom geom;
  int grid;        // persistent workgroups of the factorisation
  int solve_grid;  // persistent workgroups of a solve
  int refine_iters;
  double refine_tol;         // projection / recovery solves
  double refine_tol_sketch;  // sketch and subspace-iteration solves
  rr::GmresWs gm;                           // GMRES-IR (mixed) or the Krylov GMRES
  // LU-free solves (rr_tuning.solver != RR_SOLVER_BAND_LU)
  int solver = RR_SOLVER_BAND_LU;
  int precond = RR_PRECOND_JACOBI;
  int krylov_maxit = 1000;
  double krylov_tol = 1e-10;
  double* pc_dinv = nullptr;     // n_omega * nx*ny * 4 complex
  double* kv[7] = {};            // BiCGStab blocks r, rhat, p, v, y, z, t (GMRES: kv[0])
  double* kpart = nullptr;       // dot-product partial sums
  double* wide_tmp = nullptr;    // k_max > 32: n_omega * max(k_max, 64) * n complex
  double* kscal = nullptr;       // per-system BiCGStab scalars
  double* kbnorm = nullptr;      // per-system ||b||^2
  uint32_t* kactive = nullptr;   // per-system: 1 while not converged
  rr_test_matrix tm_kind = RR_TM_GAUSSIAN;  // step 1's test matrix
  int tm_zeta = 0;
  // private copies of the problem
  double* coef = nullptr;
  double* phi = nullptr;
  double* U = nullptr;
  double hx = 0, hy = 0, nu = 0;
  bool has_burgers = false;
  double* omega = nullptr;            // device, 2*n_omega (re, im)
  std::vector<double> omega_host;     // 2*n_omega
  // factors and dataflow state
  void* tiles = nullptr;
  size_t tile_bytes = 0;
  int* flags = nullptr;               // max(factor flags, solve flags)
  size_t flag_count = 0;
  uint32_t* ctrl = nullptr;           // [0] status, [1] ticket, [2] refine fails
  void* xs = nullptr;                 // solve sweep workspace (row-major blocks)
  void* cbuf = nullptr;               // superblock solve: c of the current superblock
  // vector workspaces (n_omega*k_max*n complex each unless noted)
  double* theta = nullptr;            // k_max*n (shared by all shifts)
  double* work1 = nullptr;
  double* work2 = nullptr;
  double* work3 = nullptr;
  // refinement probes (mixed, plain refinement): probe_np columns per shift
  // in the blocks b, x, r (right-hand sides, solutions, residuals) and
  // probe_p known solutions z per shift
  double* probe_b = nullptr;
  double* probe_x = nullptr;
  double* probe_r = nullptr;
  double* probe_z = nullptr;
  int probe_np = 0, probe_p = 0;
  bool rho_fresh = false;             // no solve has measured the contraction since the factor
  rr::SmallWs small{};
  double* grad_partial = nullptr;
  int grad_nchunk = 0;
  size_t bytes = 0;
  // allocator the handle was created with (NULL: hipMalloc / hipFree)
  rr_alloc_fn alloc = nullptr;
  rr_free_fn dealloc = nullptr;
  void* alloc_ctx = nullptr;
  void* alloc_stream = nullptr;
  int refine_used = 0;
  bool sticky_hip_error = false;
  // optional timing events (rr_set_timing_events): [0, 1] around the factor
  // kernel, [2, 3] around the main solve launch of each solve call
  hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};
};
