/*
 * rr.h -- C ABI of the MI355X randomized resolvent library (librr.so).
 *
 * Randomized resolvent analysis (Ribeiro, Yeh & Taira, arXiv:1902.01458):
 * for a real linear operator L (eq. 1) and a frequency omega, the leading
 * singular values sigma_j (gains) and singular vectors (forcing modes v_j,
 * response modes u_j) of the resolvent H(omega) = (i omega I - L)^-1
 * (eq. 4-5) are found from a thin random sketch (Algorithm 1).
 *
 * Sign convention: the paper writes the resolvent as (-i omega I - L)^-1 for
 * an e^{-i omega t} transform; this library uses M(omega) = i omega I - L.
 * For real L and real omega the gains agree and the modes are conjugated.
 * Complex shifts: the paper's discounted resolvent (Section 2.1) takes
 * omega = omega_r + i beta in its convention, i.e. [-i omega_r I - (L - beta
 * I)]^-1, the growth rates of L lowered by beta.  Here that operator is
 * M = i omega_r I - (L - beta I), reached with omega = omega_r - i beta
 * (omega_im = -beta); for real L its gains are the paper's and its modes the
 * complex conjugates.
 *
 * Call sequence (Algorithm 1):
 *   rr_factor        one LU of M(omega) per shift, reused by every solve
 *                    (Section 3.1: the factorisation is computed once and
 *                    passed to the three linear solves)
 *   rr_sketch_solve  steps 1-3 plus the power/subspace iteration of
 *                    Section 2.2.1: Theta = diag(Phi) Omega (eq. 10),
 *                    Y = M^-1 Theta, Q = orth(Y)
 *   rr_adjoint_solve step 4: Z = M^-H Q, so that B = Q^H H = Z^H
 *   rr_gains         step 5 (SVD of B), eq. 8 (Halko response modes Q Ut) and
 *                    steps 6-9 (eq. 9: H v_j = sigma_j u_j, the paper's
 *                    recovery of sigma_j and u_j)
 *   rr_resvd         optional steps 10-11: SVD of U^Sigma, improved V
 *   rr_grad          d sigma_1 / d(U, nu, omega) by first-order perturbation
 *                    of eq. 5 (not in the paper; see rr_grad below)
 *
 * Conventions for every entry point
 *   - Complex arrays are interleaved (re, im) doubles (torch.complex128).
 *   - Blocks of vectors are (n_omega, k, n): column j of shift w starts at
 *     element (w*k + j)*n, each column contiguous.
 *   - Pointers documented as "device" must be device memory of the current
 *     HIP device; "host" pointers are read before the call returns.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). All work
 *     is ordered on it; entry points return before the GPU work completes,
 *     except rr_check, rr_autotune and rr_factors_free (which synchronise).
 *   - The caller owns all input and output buffers; the library owns the
 *     rr_factors handle and everything it allocated for it.
 *   - Errors visible on the host (bad sizes, NULL pointers, allocation
 *     failure) are returned before anything is launched. Errors found on the
 *     device (zero pivot, non-finite values, Cholesky breakdown, refinement
 *     not converged) are latched in the handle and returned by rr_check.
 *     After an error the contents of the outputs are unspecified.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - No call allocates device memory except rr_factor (which sizes every
 *     workspace for k <= k_max, through rr_set_allocator's allocator if one
 *     is registered), rr_autotune (trial handles) and the test helper
 *     rr_apply (a shift buffer; it synchronises), and no
 *     launch path makes a host-side runtime call, so the sequence refactor /
 *     sketch_solve / adjoint_solve / gains / grad can be captured into a HIP
 *     graph (rr_graph_capture does so for one pass of Algorithm 1).
 */
#ifndef RR_H
#define RR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RR_OK = 0,
  RR_ERR_INVALID = 1,        /* bad argument (size, pointer, option)          */
  RR_ERR_SINGULAR = 2,       /* zero or non-finite pivot in the band LU       */
  RR_ERR_NOT_CONVERGED = 3,  /* mixed-precision refinement missed tolerance   */
  RR_ERR_BREAKDOWN = 4,      /* Gram matrix not positive definite (CholQR)    */
  RR_ERR_NONFINITE = 5,      /* NaN/Inf in inputs or results                  */
  RR_ERR_NOMEM = 6,          /* device allocation failed                      */
  RR_ERR_HIP = 7,            /* HIP runtime error (sticky for the handle)     */
  RR_ERR_TIMEOUT = 8         /* a dataflow wait exceeded its bound (bug)      */
} rr_status;

typedef enum {
  RR_FP64 = 0,   /* complex FP64 factor and solves (FP64 MFMA)                */
  RR_MIXED = 1   /* complex FP32 factor and solves (FP32 MFMA, FP32
                    accumulation) + iterative refinement whose residual
                    M x - b is computed in FP64 from the stencil              */
} rr_precision;

typedef enum {
  RR_RESP_AV = 0,   /* u_j = M^-1 v_j / ||M^-1 v_j||  (eq. 9, Alg. 1 steps 6-9) */
  RR_RESP_QU = 1,   /* u_j = Q Ut_j                    (eq. 8, Halko et al.)    */
  RR_RESP_NONE = 2  /* gains and forcing modes only                             */
} rr_response;

/* The operator L: 12 real stencil coefficients per interior node of an
 * nx x ny grid.  Node p = j + ny*i (y fastest); unknown 2p is the u-component
 * and 2p+1 the v-component at node p, so the half-bandwidth is 2*ny.
 *   coef[12*p + 0..5]  u-row: C (u_p), E (u at i+1), W (i-1), N (j+1), S (j-1),
 *                      Cpl (v_p)
 *   coef[12*p + 6..11] v-row: C (v_p), E, W, N, S, Cpl (u_p)
 * Neighbours outside the grid contribute nothing (homogeneous Dirichlet).
 * Any operator of this shape is accepted (the tests feed normal operators
 * with closed-form gains through it); rr_burgers_coeffs fills it for the
 * linearised viscous Burgers operator. */
typedef struct {
  int32_t nx, ny;
  const double* coef;  /* device, nx*ny*12                                       */
  const double* phi;   /* device, nx*ny sketch row weights (eq. 10), or NULL
                          for the unweighted Gaussian test matrix of Alg. 1 l.1  */
  /* Optional Burgers description, needed only by rr_grad:                       */
  const double* U;     /* device, (nx+2)*(ny+2) base flow incl. the boundary
                          ring, index i*(ny+2)+j; NULL if rr_grad is not used    */
  double x0, x1, y0, y1, nu;  /* domain and viscosity (grid spacing
                          h = (x1-x0)/(nx+1), (y1-y0)/(ny+1))                     */
} rr_problem;

/* Tuning knobs; pass NULL to rr_factor for defaults (or the autotuner's pick). */
typedef struct {
  int32_t tile;          /* band tile edge T: 32 or 64 (default 64)             */
  int32_t grid;          /* persistent workgroups of the factorisation; 0 = 2
                            per CU (the solves use at least 2 per CU)          */
  int32_t refine_iters;  /* mixed only: most corrections per solve (default 6,
                            at most 16).  The launches are fixed (graph-safe)
                            but skip their work on the device once every
                            column of every shift has converged               */
  double  refine_tol;    /* mixed only: a column has converged when its last
                            correction d_j has e_j = ||d_j|| / ||x_j|| <= tol,
                            or when the error it leaves, estimated as e_j
                            times the contraction per correction, is at most
                            tol / 2.  The contraction is measured, never
                            assumed: on the first refined solve after a
                            factorisation by probe systems M x = M z with
                            known z solved in the solve's spare columns (a
                            forward solve with 4 or more spare, e.g. k = 20
                            of 32) or else by the ratio of two successive
                            corrections; the largest value since the
                            factorisation is kept per shift and shared by
                            forward and adjoint solves, whose iteration
                            matrices are similar.  For the
                            projection (step 4) and recovery (step 6) solves
                            (default 1e-10)                                     */
  double  refine_tol_sketch; /* mixed only: the same test for the sketch and
                            subspace-iteration solves, which only fix the
                            basis Q (default 1e-8).  For either tolerance a
                            value of 1 or more means no correction at all      */
  int32_t refine_method; /* mixed only: RR_REFINE_PLAIN (default; correction
                            d = M32^-1 r) or RR_REFINE_GMRES (GMRES-IR: d from
                            gmres_restart steps of GMRES on M32^-1 M d =
                            M32^-1 r with M applied in FP64, for shifts where
                            kappa(M) eps_32 is near or above one and plain
                            refinement stalls; Carson & Higham, SISC 2017).
                            Each GMRES-IR correction costs gmres_restart + 1
                            FP32 solves and holds gmres_restart + 2 more
                            blocks of n_omega*k_max*n complex FP64 (not
                            counted by rr_factor_bytes)                        */
  int32_t gmres_restart; /* steps per GMRES-IR correction, 1 .. 16 (default 8) */
  int32_t superblock;    /* block rows (tiles) a solve step takes at once: the
                            sweeps of every solve walk superblocks of this many
                            block rows, x_S = D_S^-1 (b_S - sum T x), with the
                            inverses D_S^-1 of the superblocks' diagonal blocks
                            formed after each factorisation.  1 .. 8; 0 = the
                            default (256 rows per step, at most the half-band's
                            tiles); negative = one block row per step (the
                            tile-by-tile recurrence with chain tiles)          */
  int32_t solver;        /* RR_SOLVER_BAND_LU (default): the band LU of
                            M(omega) serves every solve (Section 3.1).
                            RR_SOLVER_BICGSTAB / RR_SOLVER_GMRES: no LU at
                            all; every solve of Algorithm 1 is a Krylov
                            iteration with M applied from the stencil and the
                            preconditioner `precond` (the option the paper
                            names at the end of Section 3.2, for operators
                            whose band LU does not fit in memory).  FP64 only
                            (prec must be RR_FP64); tile, grid, superblock
                            and the refinement fields are then unused, and
                            GMRES restarts every gmres_restart steps          */
  int32_t precond;       /* Krylov only: RR_PRECOND_JACOBI (default; the 2 x 2
                            node blocks of M inverted) or RR_PRECOND_ILU0
                            (block ILU(0) in the natural node order)          */
  int32_t krylov_maxit;  /* Krylov only: most iterations per solve (GMRES:
                            inner steps, rounded up to whole restarts);
                            default 1000, at most 100000.  The launches are
                            fixed (graph-safe) and skip their work once every
                            system has converged; a system still above
                            tolerance at the end latches RR_ERR_NOT_CONVERGED */
  double  krylov_tol;    /* Krylov only: a system has converged when
                            ||b - M x|| <= tol ||b|| (default 1e-10)          */
} rr_tuning;

enum { RR_REFINE_PLAIN = 0, RR_REFINE_GMRES = 1 };
enum { RR_SOLVER_BAND_LU = 0, RR_SOLVER_BICGSTAB = 1, RR_SOLVER_GMRES = 2 };
enum { RR_PRECOND_JACOBI = 0, RR_PRECOND_ILU0 = 1 };

/* Test matrices Omega of Algorithm 1 step 1 (Section 2.2.2), each weighted by
 * the problem's Phi (eq. 10) when it has one.  RR_TM_RADEMACHER: real +-1
 * entries.  RR_TM_SPARSE: ultrasparse Rademacher, zeta entries +-1 per row in
 * random columns, the rest 0.  RR_TM_ORTHONORMAL: the Gaussian matrix with
 * its columns orthonormalised (Cholesky QR) before the weighting. */
typedef enum {
  RR_TM_GAUSSIAN = 0,
  RR_TM_RADEMACHER = 1,
  RR_TM_SPARSE = 2,
  RR_TM_ORTHONORMAL = 3
} rr_test_matrix;

typedef struct rr_factors rr_factors;

/* Fill coef (and phi) for the 2-D linearised viscous Burgers operator about
 * the base flow (U(x,y), V = 0) with second-order central differences:
 *   u-row: nu Lap u - U u_x - U_x u - U_y v;   v-row: nu Lap v - U v_x
 * U_x, U_y are central differences of the nodal U (ring values included);
 * phi = sqrt(U_x^2 + U_y^2) + 0.1, the base-flow gradient weighting of the
 * physics-informed test matrix (eq. 10).  U: device (nx+2)*(ny+2); coef_out:
 * device nx*ny*12; phi_out: device nx*ny or NULL. */
rr_status rr_burgers_coeffs(int32_t nx, int32_t ny, const double* U, double x0, double x1,
                            double y0, double y1, double nu, double* coef_out,
                            double* phi_out, void* stream);

/* Apply the shifted operator: Y = M(omega_w) X for every shift w (FP64, from
 * the stencil; used for residuals and tests).  X, Y: device (n_omega, k, n)
 * complex.  omega_re/omega_im: host, n_omega each (omega_im may be NULL).
 * adjoint != 0 applies M^H instead.  Allocates a small shift buffer and
 * synchronises `stream` before returning. */
rr_status rr_apply(const rr_problem* p, const double* omega_re, const double* omega_im,
                   int32_t n_omega, int32_t k, int32_t adjoint, const double* X, double* Y,
                   void* stream);

/* Factor M(omega_w) = L_w U_w (no pivoting, band kl = ku = 2*ny) for each of
 * the n_omega shifts; the factors live in the returned handle, which also
 * takes private copies of coef, phi and U.  k_max bounds the sketch width of
 * later calls (workspaces are sized for it): 1 .. 32 in mixed precision,
 * 1 .. 512 in FP64, where widths above 32 (the k study of Section 3.2,
 * Fig. 7) take global-memory k x k kernels and band solves of 32 columns at
 * a time, and a Gram matrix that is not numerically positive definite is
 * reported as RR_ERR_BREAKDOWN instead of taking shifted CholeskyQR3.
 * rr_resvd takes the same widths.  omega_re / omega_im: host arrays
 * of n_omega doubles (omega_im may be NULL: real shifts).  On success *out is
 * a new handle; the factorisation itself is enqueued on `stream` and its
 * device-side status is reported by rr_check. */
rr_status rr_factor(const rr_problem* p, const double* omega_re, const double* omega_im,
                    int32_t n_omega, int32_t k_max, rr_precision prec,
                    const rr_tuning* tune, void* stream, rr_factors** out);

/* Re-run the factorisation in place for the same shifts (e.g. inside a graph
 * or to time it).  Same semantics as the factorisation part of rr_factor. */
rr_status rr_refactor(rr_factors* f, void* stream);

/* Steps 1-3 of Algorithm 1 with q rounds of subspace iteration (Section
 * 2.2.1): Theta[r, j] = phi[r/2] * w(r, j) with w a standard complex normal
 * drawn by Box-Muller from Philox4x32-10 at counter (r, j, 0, 0) under key
 * (seed & 0xffffffff, seed >> 32), or another test matrix chosen with
 * rr_set_test_matrix; one Theta shared by every shift.  Then
 * Y = M^-1 Theta, Q = orth(Y); q times: Q = orth(M^-1 orth(M^-H Q)).
 * orth() is Cholesky QR applied twice (Gram and Cholesky in FP64), whose R
 * has a real positive diagonal; for a shift whose Gram matrix is not
 * numerically positive definite (cond(Y) above about 1e8) it is shifted
 * Cholesky QR3 (Fukaya et al., SISC 2020), and RR_ERR_BREAKDOWN is latched
 * only if that fails too.  The same holds for the QR of Z in rr_gains and of
 * U^Sigma in rr_resvd.  Q: device (n_omega, k, n) complex output. */
rr_status rr_sketch_solve(rr_factors* f, int32_t k, uint64_t seed, int32_t power_iters,
                          double* Q, void* stream);

/* Test matrix of the handle's later rr_sketch_solve calls and graph
 * captures (the default is RR_TM_GAUSSIAN).  zeta: nonzeros per row for
 * RR_TM_SPARSE (0: min(k, 8); values above k act as k), ignored otherwise.
 * Host only: no device call.  RR_ERR_INVALID for a NULL handle, an unknown
 * kind or a negative zeta (the setting is then unchanged). */
rr_status rr_set_test_matrix(rr_factors* f, rr_test_matrix kind, int32_t zeta);

/* Step 4: Z = M^-H Q for every shift (B = Z^H).  Q, Z: device (n_omega, k, n). */
rr_status rr_adjoint_solve(rr_factors* f, int32_t k, const double* Q, double* Z, void* stream);

/* Plain forward solve X = M^-1 Bm for every shift (with refinement in the
 * mixed path).  Bm, X: device (n_omega, k, n).  X may not alias Bm. */
rr_status rr_solve(rr_factors* f, int32_t k, const double* Bm, double* X, void* stream);

/* Steps 5-9: SVD of B = Z^H (via Z = Qz R, SVD of the k x k R^H = Ut S W^H)
 * gives sigma_B (descending) and the forcing modes V = Qz W.  Then
 *   RR_RESP_AV: Us = M^-1 V, sigma_AV_j = ||Us_j||, Uresp_j = Us_j/sigma_AV_j
 *   RR_RESP_QU: Uresp = Q Ut (sigma_AV untouched)
 * sigma_B, sigma_AV: device n_omega*k doubles (sigma_AV may be NULL unless
 * mode is RR_RESP_AV); V, Uresp: device (n_omega, k, n) complex (Uresp may be
 * NULL for RR_RESP_NONE).  Q is needed only for RR_RESP_QU. */
rr_status rr_gains(rr_factors* f, int32_t k, const double* Q, const double* Z,
                   rr_response mode, double* sigma_B, double* sigma_AV, double* V,
                   double* Uresp, void* stream);

/* Optional steps 10-11 of Algorithm 1: the SVD of U^Sigma = M^-1 V (the
 * recovered, unnormalised response modes of step 6) gives orthonormal
 * response modes U and gains sigma, and its right singular vectors W refine
 * the forcing modes, V <- V W.  U^Sigma is Us (device (n_omega, k, n)
 * complex) when scale is NULL, else Us with column j of shift w multiplied
 * by scale[w*k + j] (device, n_omega*k doubles), so that the unit modes and
 * sigma_AV of rr_gains can be passed as they are.  V: device (n_omega, k, n),
 * the forcing modes of rr_gains.  Outputs: sigma (device n_omega*k,
 * descending), U and Vnew (device (n_omega, k, n)); they may not alias the
 * inputs or each other.  Everything runs in FP64, on the handle's
 * workspaces (no allocation).  RR_ERR_INVALID for a NULL handle or pointer,
 * k outside [1, k_max] or aliased outputs, before anything is launched;
 * device-side failures (a non-finite Gram matrix) are latched as for the
 * other calls (rr_check). */
rr_status rr_resvd(rr_factors* f, int32_t k, const double* Us, const double* scale,
                   const double* V, double* sigma, double* U, double* Vnew, void* stream);

/* Gradient of the leading gain (not part of the paper's method): for a
 * simple sigma with H v = sigma u and u^H H = sigma v^H, a perturbation gives
 *   d sigma / dp     = sigma^2 Re(v^H (dL/dp) u)   for p = U at a node, nu
 *   d sigma / domega = sigma^2 Im(v^H u)
 * evaluated as a stencil reduction.  Needs the Burgers description in the
 * problem (U != NULL).  sigma1: device n_omega; u1, v1: device n_omega vectors
 * of n complex (response, forcing), at stride `vec_stride` complex elements
 * between shifts (k*n for the first column of a (n_omega, k, n) block);
 * dU: device n_omega*(nx+2)*(ny+2), the derivative with respect to every
 * value of the base-flow array U in U's own layout (index i*(ny+2)+j), ring
 * included: a ring value enters L through the central difference U_x or U_y
 * of its one interior neighbour (corners: zero); dnu, domega: device n_omega
 * each. */
rr_status rr_grad(rr_factors* f, const double* sigma1, const double* u1, const double* v1,
                  int64_t vec_stride, double* dU, double* dnu, double* domega, void* stream);

/* rr_grad for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same gradient, by the same kernels, without a handle.  The problem gives
 * the grid and domain (p->nx, p->ny, p->x0..y1; coef, phi, U and nu are not
 * read); sigma1, u1, v1, vec_stride, dU, dnu, domega are as for rr_grad, for
 * n_omega shifts.  The kernels' partial sums live in a file-scope device
 * array of 2^18 doubles (2 MiB) per GPU, held until the process ends, so
 * 2 * n_omega * ceil((nx+2)(ny+2) / 256) may not exceed 2^18 (RR_ERR_INVALID
 * otherwise, before anything is launched; e.g. 63 shifts at 1024 x 512).
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from several threads) race and must be ordered
 * by the caller.  The first call on a device looks the array up
 * (hipGetSymbolAddress, no allocation); every call then only reads the
 * current device and launches the two kernels. */
rr_status rr_grad_noalloc(const rr_problem* p, int32_t n_omega, const double* sigma1,
                          const double* u1, const double* v1, int64_t vec_stride, double* dU,
                          double* dnu, double* domega, void* stream);

/* Synchronise `stream` and return (then clear) the first device-side error
 * latched in the handle since the last check; RR_OK if none. */
rr_status rr_check(rr_factors* f, void* stream);

/* Largest number of correction steps any mixed-precision solve needed since
 * the previous rr_check (0 for FP64); valid after rr_check. */
int32_t rr_refine_count(rr_factors* f);

/* Timing hook: HIP events (hipEvent_t, or NULL for none) that later calls on
 * this handle record on their stream right before and right after the band
 * factorisation kernel (rr_factor's and rr_refactor's launch of the first 64
 * shifts; not the flag fill or the superblock inverses) and the main solve
 * launch of every solve call (the first FP32 or FP64 solve of a logical
 * solve, with its two small counter fills, not the refinement corrections),
 * so that one kernel's duration can be measured inside a timed pass.  The
 * caller keeps the events alive while they are set; passing NULLs clears
 * them.  Host only; RR_ERR_INVALID for a NULL handle. */
rr_status rr_set_timing_events(rr_factors* f, void* factor_begin, void* factor_end,
                               void* solve_begin, void* solve_end);

/* Sweep cap of the one-sided Jacobi SVD of the k x k factor (Algorithm 1
 * step 5, and step 10 in rr_resvd); default 40, in [1, 64].  A sweep that
 * still rotates a pair at the cap latches RR_ERR_NOT_CONVERGED (reported by
 * rr_check; the gains and modes are then those of the last sweep).  Host
 * only; RR_ERR_INVALID for a NULL handle or a value out of range (the
 * setting is then unchanged).  Lowering it is how the non-convergence
 * report is tested. */
rr_status rr_set_jacobi_sweeps(rr_factors* f, int32_t sweeps);

/* Device bytes held by the handle. */
size_t rr_bytes(const rr_factors* f);

/* Free a handle (NULL-safe). Synchronises the device first. */
void rr_factors_free(rr_factors* f);

/* Device allocator for the handles created after this call (process-wide):
 * alloc(bytes, stream, ctx) returns device memory or NULL, dealloc(ptr, ctx)
 * returns it; NULL, NULL restores hipMalloc / hipFree.  This lets a
 * framework's caching allocator (PyTorch's) own the factors and workspaces.
 * `stream` is the one given to rr_factor; a handle frees through the
 * allocator that created it, after synchronising the device.  Returns
 * RR_ERR_INVALID if exactly one of the two is NULL. */
typedef void* (*rr_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*rr_free_fn)(void* ptr, void* ctx);
rr_status rr_set_allocator(rr_alloc_fn alloc, rr_free_fn dealloc, void* ctx);

/* Device bytes rr_factor would allocate for these sizes (with phi and U),
 * 0 for invalid sizes; tile 0 means the default.  A sweep too large for the
 * device is split into chunks of shifts sized with it. */
size_t rr_factor_bytes(int32_t nx, int32_t ny, int32_t n_omega, int32_t k_max, rr_precision prec,
                       int32_t tile);

/* Captured sweep: one pass of Algorithm 1 for every shift of the handle --
 * optionally the refactorisation (refactor != 0, e.g. after the caller changed
 * nothing but wants the factor re-timed, or to keep the whole pass in one
 * graph), then rr_sketch_solve, rr_adjoint_solve and rr_gains with the
 * arguments given here -- recorded once into a HIP graph and replayed with a
 * single launch.  The buffers named at capture are the ones every replay
 * reads and writes; the caller keeps them alive while the graph exists.
 * Capture runs on a private stream, so no stream argument is taken; replays
 * are ordered on the stream passed to rr_graph_launch, and their device-side
 * status is latched in the handle as for the eager calls (rr_check).  The
 * handle must outlive the graph.  Nothing is launched by rr_graph_capture. */
typedef struct rr_graph rr_graph;
rr_status rr_graph_capture(rr_factors* f, int32_t refactor, int32_t k, uint64_t seed, int32_t q,
                           rr_response mode, double* Q, double* Z, double* sigma_B,
                           double* sigma_AV, double* V, double* Uresp, rr_graph** out);
rr_status rr_graph_launch(rr_graph* g, void* stream);
void rr_graph_free(rr_graph* g);

/* Autotuner for the band tile, the persistent grid and the solve's
 * superblock: it first tries tile 64 and 32 with one and two workgroups per
 * CU (default superblock), then, for the best of those, superblocks of 2, 4
 * and 8 block rows and the tile-by-tile solve; each candidate builds a trial
 * handle for this operator and the first max_shifts shifts (all when
 * max_shifts <= 0), runs one warm-up pass and one timed pass of
 * refactorisation, sketch solve and adjoint solve, and is scored factor +
 * 2.5 * (sketch + adjoint), the cost of one pass of Algorithm 1 with a
 * subspace iteration.  The fastest candidate is written to *out (refinement
 * fields zero: defaults) and its score in ms to *out_ms (may be NULL).
 * Candidates that do not fit in device memory are skipped.  When the
 * environment variable RR_AUTOTUNE_CACHE names a file, picks are kept there
 * (a JSON object keyed by GPU architecture, grid, shift count, k and
 * precision): a key already in it is returned with its stored score and no
 * trial runs; a new pick is added.  Synchronises `stream`; allocates and
 * frees its own trial handles and blocks; the caller's handles are
 * untouched. */
rr_status rr_autotune(const rr_problem* p, const double* omega_re, const double* omega_im,
                      int32_t n_omega, int32_t k, rr_precision prec, int32_t max_shifts,
                      void* stream, rr_tuning* out, double* out_ms);

/* Message for the last error returned on this thread (never NULL). */
const char* rr_last_error(void);

/* Test hooks for the device random-number generator.
 * rr_philox_raw: out_dev[4*i .. 4*i+3] = Philox4x32-10 output words of counter
 * (i, c1, c2, 0) under key (k0, k1), for i < count (device, 4*count words).
 * rr_sketch: the test matrix of rr_sketch_solve, Theta (k, n) complex
 * (device), row weights p->phi (NULL = unweighted); p->coef is not read.
 * kind: an elementwise kind (RR_TM_ORTHONORMAL needs a handle and is
 * rejected); zeta as for rr_set_test_matrix. */
rr_status rr_philox_raw(uint32_t* out_dev, int64_t count, uint32_t c1, uint32_t c2, uint32_t k0,
                        uint32_t k1, void* stream);
rr_status rr_sketch(const rr_problem* p, int32_t k, uint64_t seed, rr_test_matrix kind,
                    int32_t zeta, double* theta, void* stream);

/* Test hook: Y = K^-1 X (adjoint: K^-H X) with the preconditioner K of a
 * Krylov handle (rr_tuning.solver), for k columns of every shift; X and Y
 * are device blocks of n_omega * k * n complex (k-column blocks per shift,
 * the layout of every block), and Y may be X.  RR_ERR_INVALID for a band-LU
 * handle or k outside [1, k_max]. */
rr_status rr_precond_apply(rr_factors* f, int32_t k, int32_t adjoint, const double* X, double* Y,
                           void* stream);

/* Test hook for the factorisation's task order (host only, no device call).
 * Writes the ticket tasks of one shift of a band of B tiles each side and NB
 * block rows, in the order the factor launch hands them out, as (kind, r, t)
 * int32 triples into out[3*i .. 3*i+2] for i < cap (host memory): kind 0 =
 * finalisation of tile (r, t) (its last update, then the triangular solve
 * with the LU of diagonal tile min(r, t)), 1 = its early updates written as a
 * partial tile, 2 / 3 = the chain tiles of diagonal tile r (column / row
 * side).  Diagonal tiles are factored outside this order, one worker per
 * shift.  Returns the number of tasks (which may exceed cap), or -1 if B or
 * NB is not positive. */
int64_t rr_factor_schedule(int32_t B, int32_t NB, int32_t* out, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* RR_H */
