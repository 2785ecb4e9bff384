// Host side of the C ABI: argument checks, workspace ownership and the order
// of launches for each call of Algorithm 1.  Every numerical step runs in the
// kernels of rr_operator.hip, rr_band.hip, rr_small.hip and rr_grad.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "rr_internal.h"

using namespace rr;

namespace {

thread_local std::string g_err = "no error";

rr_status fail(rr_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define RR_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(RR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return cus > 0 ? cus : 256;
}

bool is_dev_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Process-wide device allocator for new handles (rr_set_allocator); each
// handle keeps the one it was created with.
rr_alloc_fn g_alloc = nullptr;
rr_free_fn g_dealloc = nullptr;
void* g_alloc_ctx = nullptr;

template <typename T>
rr_status dalloc(rr_factors* f, T** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (f->alloc) {
    *p = (T*)f->alloc(bytes, f->alloc_stream, f->alloc_ctx);
    if (!*p) return fail(RR_ERR_NOMEM, "allocator returned NULL for " + std::to_string(bytes));
  } else {
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return fail(RR_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  f->bytes += bytes;
  return RR_OK;
}

void free_all(rr_factors* f) {
  void* ps[] = {f->coef, f->phi, f->U, f->omega, f->tiles, f->xs, f->cbuf, f->flags, f->ctrl,
                f->theta,
                f->work1, f->work2, f->work3, f->small.partial, f->small.G, f->small.R,
                f->small.Rinv, f->small.W, f->small.Ut, f->small.rho, f->small.shifted, f->grad_partial,
                f->gm.V, f->gm.t, f->gm.H, f->gm.h, f->gm.beta, f->gm.y, f->gm.partial,
                f->pc_dinv, f->kv[0], f->kv[1], f->kv[2], f->kv[3], f->kv[4], f->kv[5],
                f->kv[6], f->kpart, f->kscal, f->kbnorm, f->kactive, f->small.big1,
                f->small.big2, f->wide_tmp, f->probe_b, f->probe_x, f->probe_r, f->probe_z};
  for (void* p : ps) {
    if (!p) continue;
    if (f->dealloc) f->dealloc(p, f->alloc_ctx);
    else (void)hipFree(p);
  }
}

OpDesc opdesc(const rr_factors* f) { return OpDesc{f->nx, f->ny, f->n, f->coef}; }

uint32_t* st_word(rr_factors* f) { return f->ctrl; }
uint32_t* ticket_word(rr_factors* f) { return f->ctrl + 1; }
uint32_t* fail_word(rr_factors* f) { return f->ctrl + 2; }
uint32_t* conv_word(rr_factors* f) { return f->ctrl + 3; }
// ctrl[20], ctrl[21]: the factorisation's task tickets and diagonal-worker roles
uint32_t* factor_counters(rr_factors* f) { return f->ctrl + 20; }
// ctrl[4 + it]: unconverged columns after correction it (mixed solves)
constexpr int kMaxRefine = 16;
// Sketch widths above this take the wide k x k kernels (rr_bigk.hip) and
// band solves in groups of this many columns (FP64 only).
constexpr int kNarrowK = 32;

// Refinement probes: the columns a solve of k columns has spare (the solve
// runs solve_np(k) of them), at most kMaxProbes; fewer than kMinProbes are
// not used.
constexpr int kMinProbes = 4, kMaxProbes = 12;
constexpr uint64_t kProbeSeed = 0x70726f6265ull;  // the probes' Philox key
int probe_cols(int k, int np_max) {
  const int p = std::min(solve_np(k), np_max) - k;
  return p >= kMinProbes ? std::min(p, kMaxProbes) : 0;
}

// The k x k steps for narrow (k <= 32: LDS-resident) or wide sketches.
hipError_t cholqr(rr_factors* f, int n_omega, int k, double* Y, hipStream_t s) {
  if (k <= kNarrowK) return launch_cholqr2(f->n, n_omega, k, Y, f->small, st_word(f), s);
  return launch_cholqr2_big(f->n, n_omega, k, Y, f->wide_tmp, f->small, st_word(f), s);
}
hipError_t small_svd(rr_factors* f, int k, const double* Z, const double* Q, double* sigma,
                     double* V, double* Uqu, hipStream_t s) {
  if (k <= kNarrowK)
    return launch_small_svd(f->n, f->n_omega, k, Z, Q, sigma, V, Uqu, f->small, st_word(f), s);
  return launch_small_svd_big(f->n, f->n_omega, k, Z, Q, sigma, V, Uqu, f->wide_tmp, f->small,
                              st_word(f), s);
}
hipError_t colnorm_scale(rr_factors* f, int k, const double* W, double* sigma, double* U,
                         hipStream_t s) {
  if (k <= kNarrowK)
    return launch_colnorm_scale(f->n, f->n_omega, k, W, sigma, U, f->small, st_word(f), s);
  return launch_colnorm_big(f->n, f->n_omega, k, W, sigma, U, st_word(f), s);
}

// After correction `it`: record the unconverged-column count and mark the
// solve converged when it is zero (later corrections then skip their work).
__global__ void k_refine_step(const uint32_t* fail, uint32_t* slot, uint32_t* conv) {
  if (threadIdx.x == 0) {
    uint32_t nf = *fail;
    atomicMax(slot, nf);
    if (nf == 0) *conv = 1u;
  }
}
__global__ void k_latch_unless(const uint32_t* conv, uint32_t* status, uint32_t bit) {
  if (threadIdx.x == 0 && !*conv) atomicOr(status, bit);
}

// GMRES-IR correction: r <- m steps of GMRES on M32^-1 M d = M32^-1 r (left
// preconditioned, zero initial guess), every (shift, column) on its own
// Krylov space, classical Gram-Schmidt applied twice.  Fixed launches; all of
// them skip their work once every column has converged.
hipError_t gmres_correction(rr_factors* f, int k, int adjoint, double* r, hipStream_t s) {
  GmresWs& g = f->gm;
  const int m = g.m, n_omega = f->n_omega;
  const int64_t blk = (int64_t)k * f->n, vstride = (int64_t)n_omega * blk;
  const uint32_t* skip = conv_word(f);
  auto V = [&](int i) { return g.V + 2 * i * vstride; };
  hipError_t e = launch_fill_u32((uint32_t*)g.H, 0u, (int64_t)n_omega * k * (m + 1) * m * 4, s);
  // the preconditioner: the FP32 band LU (GMRES-IR), or the Krylov handle's K
  auto solve32 = [&](const double* in, double* out) {
    if (f->solver != RR_SOLVER_BAND_LU)
      return launch_pc_apply(opdesc(f), f->precond, n_omega, k, adjoint, f->pc_dinv, in, out,
                             nullptr, skip, s);
    return launch_solve(f->geom, f->n, n_omega, k, true, f->tiles, adjoint, in, blk, out, f->xs,
                        f->cbuf, f->flags, ticket_word(f), st_word(f), f->solve_grid, s, skip);
  };
  if (e == hipSuccess) e = solve32(r, V(0));
  if (e == hipSuccess)
    e = colnorm_scale(f, k, V(0), g.beta, V(0), s);
  for (int j = 0; e == hipSuccess && j < m; j++) {
    e = launch_apply(opdesc(f), f->omega, n_omega, k, adjoint, V(j), nullptr, blk, g.t, s, skip);
    if (e == hipSuccess) e = solve32(g.t, V(j + 1));
    for (int pass = 0; e == hipSuccess && pass < 2; pass++)
      e = launch_gs_project(f->n, n_omega, k, j, g, V(j + 1), skip, s);
    double* nrm = g.h;  // free until the next projection
    if (e == hipSuccess)
      e = colnorm_scale(f, k, V(j + 1), nrm, V(j + 1), s);
    if (e == hipSuccess) e = launch_store_subdiag(n_omega, k, j, g, nrm, skip, s);
  }
  if (e == hipSuccess) e = launch_gmres_finish(f->n, n_omega, k, g, r, skip, s);
  return e;
}

// X = M^-1 Bm (or M^-H Bm) without the LU: preconditioned BiCGStab or
// restarted GMRES (left-preconditioned, the GMRES-IR cycle with K in place
// of the FP32 LU), one system per (shift, column), from x = 0 until
// ||b - M x|| <= krylov_tol ||b||.  A fixed number of launches; all of them
// skip their work once every system has converged.
rr_status krylov_solve(rr_factors* f, int k, int adjoint, const double* Bm, int64_t bstride,
                       double* X, hipStream_t s) {
  const OpDesc op = opdesc(f);
  const int nw = f->n_omega, N = nw * k;
  const int64_t n = f->n, total = (int64_t)nw * k * n;
  const double tol = f->krylov_tol;
  uint32_t* conv = conv_word(f);
  uint32_t* act = f->kactive;
  uint32_t* st = st_word(f);
  double* r = f->kv[0];
  RR_HIP(launch_fill_u32(conv, 0u, 1, s));
  RR_HIP(launch_fill_u32((uint32_t*)X, 0u, total * 4, s));  // x = 0
  // r = b - M 0 = b (the apply also spreads a right-hand side shared by the shifts)
  RR_HIP(launch_apply(op, f->omega, nw, k, adjoint, X, Bm, bstride, r, s));
  RR_HIP(launch_kdot(n, nw, k, 1, r, r, nullptr, nullptr, f->kpart, nullptr, nullptr, s));
  RR_HIP(launch_bicg_scalars(N, n, 0, 0, tol, f->kpart, f->kscal, f->kbnorm, act, conv, st,
                             nullptr, s));
  if (f->solver == RR_SOLVER_BICGSTAB) {
    double *rh = f->kv[1], *p = f->kv[2], *v = f->kv[3], *y = f->kv[4], *z = f->kv[5],
           *t = f->kv[6];
    RR_HIP(launch_kcopy(total, r, rh, s));
    RR_HIP(launch_fill_u32((uint32_t*)p, 0u, total * 4, s));
    RR_HIP(launch_fill_u32((uint32_t*)v, 0u, total * 4, s));
    for (int it = 0; it < f->krylov_maxit; it++) {
      // rho = <rhat, r>, beta; p = r + beta (p - omega v); y = K^-1 p; v = M y
      RR_HIP(launch_kdot(n, nw, k, 1, rh, r, nullptr, nullptr, f->kpart, act, conv, s));
      RR_HIP(launch_bicg_scalars(N, n, 1, it, tol, f->kpart, f->kscal, f->kbnorm, act, conv, st,
                                 conv, s));
      RR_HIP(launch_bicg_vec(0, n, nw, k, f->kscal, r, v, nullptr, nullptr, p, act, conv, s));
      RR_HIP(launch_pc_apply(op, f->precond, nw, k, adjoint, f->pc_dinv, p, y, act, conv, s));
      RR_HIP(launch_apply(op, f->omega, nw, k, adjoint, y, nullptr, 0, v, s, conv));
      // alpha = rho / <rhat, v>; s = r - alpha v (kept in r)
      RR_HIP(launch_kdot(n, nw, k, 1, rh, v, nullptr, nullptr, f->kpart, act, conv, s));
      RR_HIP(launch_bicg_scalars(N, n, 2, it, tol, f->kpart, f->kscal, f->kbnorm, act, conv, st,
                                 conv, s));
      RR_HIP(launch_bicg_vec(1, n, nw, k, f->kscal, nullptr, v, nullptr, nullptr, r, act, conv, s));
      // z = K^-1 s; t = M z; omega = <t, s> / <t, t>
      RR_HIP(launch_pc_apply(op, f->precond, nw, k, adjoint, f->pc_dinv, r, z, act, conv, s));
      RR_HIP(launch_apply(op, f->omega, nw, k, adjoint, z, nullptr, 0, t, s, conv));
      RR_HIP(launch_kdot(n, nw, k, 2, t, r, t, t, f->kpart, act, conv, s));
      RR_HIP(launch_bicg_scalars(N, n, 3, it, tol, f->kpart, f->kscal, f->kbnorm, act, conv, st,
                                 conv, s));
      // x += alpha y + omega z; r = s - omega t; then the convergence test
      RR_HIP(launch_bicg_vec(2, n, nw, k, f->kscal, y, z, t, X, r, act, conv, s));
      RR_HIP(launch_kdot(n, nw, k, 1, r, r, nullptr, nullptr, f->kpart, act, conv, s));
      RR_HIP(launch_bicg_scalars(N, n, 4, it, tol, f->kpart, f->kscal, f->kbnorm, act, conv, st,
                                 conv, s));
    }
  } else {
    const int m = f->gm.m;
    const int cycles = (f->krylov_maxit + m - 1) / m;
    for (int c = 0; c <= cycles; c++) {
      if (c > 0) {  // r = b - M x and the convergence test
        RR_HIP(launch_apply(op, f->omega, nw, k, adjoint, X, Bm, bstride, r, s, conv));
        RR_HIP(launch_kdot(n, nw, k, 1, r, r, nullptr, nullptr, f->kpart, act, conv, s));
        RR_HIP(launch_bicg_scalars(N, n, 4, c, tol, f->kpart, f->kscal, f->kbnorm, act, conv, st,
                                   conv, s));
      }
      if (c == cycles) break;
      RR_HIP(gmres_correction(f, k, adjoint, r, s));  // r <- m steps of GMRES on K^-1 M d = K^-1 r
      RR_HIP(launch_bicg_vec(3, n, nw, k, nullptr, r, nullptr, nullptr, X, nullptr, act, conv, s));
    }
  }
  RR_HIP(launch_latch_live(N, act, st, ST_NOT_CONVERGED, s));
  return RR_OK;
}

// X = M^-1 Bm (or M^-H): one FP64 band solve, or FP32 solves with FP64
// residual refinement to `tol`.  Bm's blocks are bstride apart (0 = shared by
// all shifts).  The mixed loop has a fixed number of launches; once every
// column of every shift has converged the remaining ones return at once.
rr_status solve_any(rr_factors* f, int k, int adjoint, const double* Bm, int64_t bstride,
                    double* X, double tol, hipStream_t s) {
  if (f->solver != RR_SOLVER_BAND_LU) {
    if (f->tev[2]) RR_HIP(hipEventRecord(f->tev[2], s));
    rr_status st = krylov_solve(f, k, adjoint, Bm, bstride, X, s);
    if (f->tev[3]) RR_HIP(hipEventRecord(f->tev[3], s));
    return st;
  }
  if (k > kNarrowK) {
    // a wide block (FP64 only): the band solve takes 32 columns at a time,
    // gathered into and scattered from two narrow blocks
    double* nb = f->wide_tmp;
    double* nx = f->wide_tmp + 2 * (size_t)f->n_omega * kNarrowK * f->n;
    for (int c0 = 0; c0 < k; c0 += kNarrowK) {
      const int kg = std::min(kNarrowK, k - c0);
      RR_HIP(launch_cols_copy(f->n, f->n_omega, k, bstride, c0, kg, Bm, nb, true, s));
      RR_HIP(launch_solve(f->geom, f->n, f->n_omega, kg, false, f->tiles, adjoint, nb,
                          (int64_t)kg * f->n, nx, f->xs, f->cbuf, f->flags, ticket_word(f),
                          st_word(f), f->solve_grid, s));
      RR_HIP(launch_cols_copy(f->n, f->n_omega, k, (int64_t)k * f->n, c0, kg, nx, X, false, s));
    }
    return RR_OK;
  }
  const bool mixed = f->prec == RR_MIXED;
  const bool refine = mixed && tol < 1.0;  // a tolerance of 1 or more asks for no correction
  // The first refined solve after a factorisation measures the contraction.
  // Where a forward solve has spare columns (it runs solve_np(k)), p probe
  // systems M x = M z with known z ride along in them: their exact errors
  // before and after the first correction give it, so no second correction
  // is needed for the measurement.
  const int p = refine && f->rho_fresh && !adjoint && f->gm.m == 0 && f->probe_z
                    ? std::min(probe_cols(k, f->probe_np), f->probe_p)
                    : 0;
  if (refine) f->rho_fresh = false;
  const int kk = k + p;
  const int64_t n = f->n, pblk = (int64_t)kk * n;
  const double* B1 = Bm;
  int64_t bs1 = bstride;
  double* X1 = X;
  double* res = f->work3;
  if (p > 0) {  // [Bm | M z] into the probe block
    RR_HIP(launch_cols_place(n, f->n_omega, k, Bm, bstride, 0, f->probe_b, pblk, 0, s));
    RR_HIP(launch_apply(opdesc(f), f->omega, f->n_omega, p, adjoint, f->probe_z, nullptr, 0,
                        f->probe_r, s));
    RR_HIP(launch_cols_place(n, f->n_omega, p, f->probe_r, (int64_t)p * n, 0, f->probe_b, pblk,
                             k, s));
    B1 = f->probe_b;
    bs1 = pblk;
    X1 = f->probe_x;
    res = f->probe_r;
  }
  if (f->tev[2]) RR_HIP(hipEventRecord(f->tev[2], s));
  RR_HIP(launch_solve(f->geom, f->n, f->n_omega, kk, mixed, f->tiles, adjoint, B1, bs1, X1,
                      f->xs, f->cbuf, f->flags, ticket_word(f), st_word(f), f->solve_grid, s));
  if (f->tev[3]) RR_HIP(hipEventRecord(f->tev[3], s));
  if (!refine) return RR_OK;
  if (p > 0)
    RR_HIP(launch_probe_errors(f->n, f->n_omega, kk, k, p, X1, f->probe_z, f->small, st_word(f),
                               s));
  RR_HIP(launch_fill_u32(conv_word(f), 0u, 1, s));
  for (int it = 0; it < f->refine_iters; it++) {
    // res = Bm - M X in FP64 from the stencil, then res <- M32^-1 res (or the
    // GMRES-IR correction), X += res
    RR_HIP(launch_apply(opdesc(f), f->omega, f->n_omega, kk, adjoint, X1, B1, bs1, res, s,
                        conv_word(f)));
    if (f->gm.m > 0) {
      RR_HIP(gmres_correction(f, k, adjoint, res, s));
    } else {
      RR_HIP(launch_solve(f->geom, f->n, f->n_omega, kk, true, f->tiles, adjoint, res, pblk, res,
                          f->xs, f->cbuf, f->flags, ticket_word(f), st_word(f), f->solve_grid, s,
                          conv_word(f)));
    }
    RR_HIP(launch_fill_u32(fail_word(f), 0u, 1, s));
    RR_HIP(launch_refine_update(f->n, f->n_omega, k, X1, res, tol, it, adjoint, f->small,
                                st_word(f), fail_word(f), s, conv_word(f), kk, p, f->probe_z));
    hipLaunchKernelGGL(k_refine_step, dim3(1), dim3(64), 0, s, (const uint32_t*)fail_word(f),
                       f->ctrl + 4 + it, conv_word(f));
  }
  hipLaunchKernelGGL(k_latch_unless, dim3(1), dim3(64), 0, s, (const uint32_t*)conv_word(f),
                     st_word(f), (uint32_t)ST_NOT_CONVERGED);
  RR_HIP(hipGetLastError());
  if (p > 0)  // the caller's columns back
    RR_HIP(launch_cols_place(n, f->n_omega, k, X1, pblk, 0, X, (int64_t)k * n, 0, s));
  return RR_OK;
}

// Device allocations of a handle, in one place for rr_factor and rr_factor_bytes.
struct Plan {
  BandGeom geom;
  size_t coef, phi, U, omega, tiles, xs, cbuf, flags, ctrl, theta, vec, work3, partial, kk2, rho,
      shifted, grad, big = 0, wide = 0, probe_blk = 0, probe_z = 0;
  int nchunk, grad_nchunk, probe_np = 0, probe_p = 0;
  size_t nflags;
  size_t total() const {
    return coef + phi + U + omega + tiles + xs + cbuf + flags + ctrl + theta + 2 * vec + work3 +
           partial + 5 * kk2 + rho + shifted + grad + 2 * big + wide + 3 * probe_blk + probe_z;
  }
};

// Block rows per superblock solve step: `want` > 0 as asked (at most 8), 0
// the default (256 rows: 4 tiles of 64, 8 of 32, at most the half-band's
// tiles), < 0 the tile-by-tile solve (0 returned).
int superblock_tiles(int want, int T, int B) {
  if (want < 0) return 0;
  if (want > 0) return std::min(want, 8);
  return std::max(1, std::min(B, 256 / T));
}

Plan make_plan(int nx, int ny, int n_omega, int k_max, rr_precision prec, int T, bool has_phi,
               bool has_U, int sb, bool probes) {
  Plan pl{};
  const int64_t n = 2 * (int64_t)nx * ny;
  const size_t nn = (size_t)nx * ny;
  pl.geom.T = T;
  pl.geom.B = (2 * ny + T - 1) / T;
  pl.geom.NB = (int)((n + T - 1) / T);
  pl.geom.P = superblock_tiles(sb, T, pl.geom.B);
  const size_t elem = prec == RR_MIXED ? 2 * sizeof(float) : 2 * sizeof(double);
  pl.coef = nn * 12 * sizeof(double);
  pl.phi = has_phi ? nn * sizeof(double) : 0;
  pl.U = has_U ? (size_t)(nx + 2) * (ny + 2) * sizeof(double) : 0;
  pl.omega = 2 * (size_t)n_omega * sizeof(double);
  pl.tiles = (size_t)n_omega * pl.geom.tiles_per_omega() * T * T * elem;
  const int kn = std::min(k_max, kNarrowK);  // widest solve launch
  pl.xs = (size_t)n_omega * pl.geom.NB * T * solve_np(kn) * 2 * sizeof(double);
  pl.cbuf = (size_t)n_omega * std::max(pl.geom.P, 1) * T * solve_np(kn) * 2 * sizeof(double);
  pl.nflags = std::max({(size_t)n_omega * pl.geom.tiles_per_omega(), (size_t)n_omega * pl.geom.NB,
                        (size_t)ssolve_counters(pl.geom, n_omega)});
  pl.flags = pl.nflags * sizeof(int);
  pl.ctrl = 64 * sizeof(uint32_t);
  pl.theta = (size_t)k_max * n * 2 * sizeof(double);
  pl.vec = (size_t)n_omega * k_max * n * 2 * sizeof(double);
  pl.work3 = prec == RR_MIXED ? pl.vec : 0;
  pl.nchunk = (int)((n + 2047) / 2048);
  const size_t kk = (size_t)std::max(k_max * k_max, 64);
  const size_t kkn = (size_t)std::max(kn * kn, 64);
  // (at least 96 complex per chunk: the refinement's three partial rows of 64)
  pl.partial = (size_t)n_omega * std::max<size_t>(pl.nchunk * std::max<size_t>(kkn, 96),
                                                  k_max > kNarrowK ? gramb_chunks(n) * kk : 0) *
               2 * sizeof(double);
  if (k_max > kNarrowK) {  // the wide k x k steps' scratch and one wide block
    pl.big = (size_t)n_omega * (k_max + 1) * (k_max + 1) * 2 * sizeof(double);
    pl.wide = (size_t)n_omega * std::max(k_max, 2 * kNarrowK) * n * 2 * sizeof(double);
  }
  pl.kk2 = (size_t)n_omega * kk * 2 * sizeof(double);
  pl.rho = prec == RR_MIXED ? (size_t)n_omega * kRhoStride * sizeof(double) : 0;
  if (prec == RR_MIXED && probes && probe_cols(kn, solve_np(kn)) > 0) {
    pl.probe_np = solve_np(kn);
    pl.probe_p = probe_cols(kn, pl.probe_np);
    pl.probe_blk = (size_t)n_omega * pl.probe_np * n * 2 * sizeof(double);
    pl.probe_z = (size_t)n_omega * pl.probe_p * n * 2 * sizeof(double);
  }
  pl.shifted = (size_t)n_omega * sizeof(uint32_t);
  pl.grad_nchunk = (int)(((size_t)(nx + 2) * (ny + 2) + 255) / 256);  // k_grad's blocks
  pl.grad = (size_t)n_omega * pl.grad_nchunk * 2 * sizeof(double);
  return pl;
}

rr_status check_k(const rr_factors* f, int k) {
  if (!f) return fail(RR_ERR_INVALID, "NULL handle");
  if (f->sticky_hip_error) return fail(RR_ERR_HIP, "handle is unusable after a HIP error");
  if (k < 1 || k > f->k_max) return fail(RR_ERR_INVALID, "k must be in [1, k_max]");
  return RR_OK;
}



}  // namespace

extern "C" {

const char* rr_last_error(void) { return g_err.c_str(); }

rr_status rr_burgers_coeffs(int32_t nx, int32_t ny, const double* U, double x0, double x1,
                            double y0, double y1, double nu, double* coef_out, double* phi_out,
                            void* stream) {
  if (nx < 1 || ny < 1) return fail(RR_ERR_INVALID, "nx, ny must be >= 1");
  if (!U || !coef_out) return fail(RR_ERR_INVALID, "NULL pointer");
  if (!(x1 > x0) || !(y1 > y0)) return fail(RR_ERR_INVALID, "empty domain");
  double hx = (x1 - x0) / (nx + 1), hy = (y1 - y0) / (ny + 1);
  RR_HIP(launch_burgers_coeffs(nx, ny, U, hx, hy, nu, coef_out, phi_out, (hipStream_t)stream));
  return RR_OK;
}

rr_status rr_apply(const rr_problem* p, const double* omega_re, const double* omega_im,
                   int32_t n_omega, int32_t k, int32_t adjoint, const double* X, double* Y,
                   void* stream) {
  if (!p || !p->coef || !X || !Y || !omega_re) return fail(RR_ERR_INVALID, "NULL pointer");
  if (p->nx < 1 || p->ny < 1 || n_omega < 1 || k < 1 || n_omega > 65535 || k > 65535)
    return fail(RR_ERR_INVALID, "bad sizes");
  hipStream_t s = (hipStream_t)stream;
  std::vector<double> om(2 * n_omega);
  for (int i = 0; i < n_omega; i++) {
    om[2 * i] = omega_re[i];
    om[2 * i + 1] = omega_im ? omega_im[i] : 0.0;
  }
  double* dom = nullptr;
  RR_HIP(hipMalloc((void**)&dom, om.size() * sizeof(double)));
  RR_HIP(hipMemcpyAsync(dom, om.data(), om.size() * sizeof(double), hipMemcpyHostToDevice, s));
  OpDesc op{p->nx, p->ny, 2 * p->nx * p->ny, p->coef};
  hipError_t e = launch_apply(op, dom, n_omega, k, adjoint, X, nullptr, 0, Y, s);
  (void)hipStreamSynchronize(s);
  (void)hipFree(dom);
  if (e != hipSuccess) return fail(RR_ERR_HIP, hipGetErrorString(e));
  return RR_OK;
}

rr_status rr_factor(const rr_problem* p, const double* omega_re, const double* omega_im,
                    int32_t n_omega, int32_t k_max, rr_precision prec, const rr_tuning* tune,
                    void* stream, rr_factors** out) {
  if (!out) return fail(RR_ERR_INVALID, "NULL output handle pointer");
  *out = nullptr;
  if (!p || !p->coef || !omega_re) return fail(RR_ERR_INVALID, "NULL pointer");
  if (p->nx < 1 || p->ny < 1) return fail(RR_ERR_INVALID, "nx, ny must be >= 1");
  if (n_omega < 1) return fail(RR_ERR_INVALID, "n_omega must be >= 1");
  if (prec != RR_FP64 && prec != RR_MIXED) return fail(RR_ERR_INVALID, "unknown precision");
  if (k_max < 1 || k_max > (prec == RR_FP64 ? kMaxWideK : kNarrowK))
    return fail(RR_ERR_INVALID, prec == RR_FP64 ? "k_max must be in [1, 512]"
                                                : "k_max must be in [1, 32] in mixed precision");
  int64_t n64 = 2 * (int64_t)p->nx * p->ny;
  if (n64 > (1ll << 30)) return fail(RR_ERR_INVALID, "operator too large");
  if (k_max > n64) return fail(RR_ERR_INVALID, "k_max exceeds n");
  for (int i = 0; i < n_omega; i++)
    if (!std::isfinite(omega_re[i]) || (omega_im && !std::isfinite(omega_im[i])))
      return fail(RR_ERR_INVALID, "non-finite omega");
  int T = tune && tune->tile ? tune->tile : 64;
  if (T != 32 && T != 64) return fail(RR_ERR_INVALID, "tile must be 32 or 64");
  if (tune && (tune->refine_iters < 0 || tune->refine_iters > kMaxRefine))
    return fail(RR_ERR_INVALID, "refine_iters out of range");
  if (tune && tune->refine_method != RR_REFINE_PLAIN && tune->refine_method != RR_REFINE_GMRES)
    return fail(RR_ERR_INVALID, "unknown refine_method");
  if (tune && tune->refine_method == RR_REFINE_GMRES &&
      (tune->gmres_restart < 0 || tune->gmres_restart > kGmresMaxRestart))
    return fail(RR_ERR_INVALID, "gmres_restart out of range");
  if (tune && tune->superblock > 8) return fail(RR_ERR_INVALID, "superblock must be <= 8");
  const int solver = tune ? tune->solver : RR_SOLVER_BAND_LU;
  if (solver != RR_SOLVER_BAND_LU && solver != RR_SOLVER_BICGSTAB && solver != RR_SOLVER_GMRES)
    return fail(RR_ERR_INVALID, "unknown solver");
  const bool krylov = solver != RR_SOLVER_BAND_LU;
  if (krylov) {
    if (prec != RR_FP64) return fail(RR_ERR_INVALID, "the Krylov solvers run in FP64 only");
    if (tune->precond != RR_PRECOND_JACOBI && tune->precond != RR_PRECOND_ILU0)
      return fail(RR_ERR_INVALID, "unknown preconditioner");
    if (tune->krylov_maxit < 0 || tune->krylov_maxit > 100000)
      return fail(RR_ERR_INVALID, "krylov_maxit out of range");
    if (!(tune->krylov_tol >= 0.0) || tune->krylov_tol >= 1.0)
      return fail(RR_ERR_INVALID, "krylov_tol must be in [0, 1)");
    if (tune->gmres_restart < 0 || tune->gmres_restart > kGmresMaxRestart)
      return fail(RR_ERR_INVALID, "gmres_restart out of range");
    if (tune->precond == RR_PRECOND_ILU0 && ilu0_lds(p->ny) > 160 * 1024)
      return fail(RR_ERR_INVALID, "ILU(0) holds two anti-diagonals of ny nodes in LDS: ny too large");
  }
  if (!is_dev_ptr(p->coef) || (p->phi && !is_dev_ptr(p->phi)) || (p->U && !is_dev_ptr(p->U)))
    return fail(RR_ERR_INVALID, "coef/phi/U must be device pointers");

  rr_factors* f = new rr_factors();
  f->alloc = g_alloc;
  f->dealloc = g_dealloc;
  f->alloc_ctx = g_alloc_ctx;
  f->alloc_stream = stream;
  f->nx = p->nx;
  f->ny = p->ny;
  f->n = (int)n64;
  f->n_omega = n_omega;
  f->k_max = k_max;
  f->prec = prec;
  const int b = 2 * p->ny;
  f->geom.T = T;
  f->geom.B = (b + T - 1) / T;
  f->geom.NB = (f->n + T - 1) / T;
  f->geom.P = superblock_tiles(tune ? tune->superblock : 0, T, f->geom.B);
  f->grid = tune && tune->grid > 0 ? tune->grid : 2 * device_cus();
  // the solves' persistent workgroups queue behind the resident ones, so a
  // grid of two per CU never idles a CU that could hold two
  f->solve_grid = std::max(tune && tune->grid > 0 ? tune->grid : 0, 2 * device_cus());
  f->refine_iters = tune && tune->refine_iters ? tune->refine_iters : 6;
  f->refine_tol = tune && tune->refine_tol > 0 ? tune->refine_tol : 1e-10;
  f->refine_tol_sketch = tune && tune->refine_tol_sketch > 0 ? tune->refine_tol_sketch : 1e-8;
  f->solver = solver;
  if (krylov) {
    f->precond = tune->precond;
    f->krylov_maxit = tune->krylov_maxit ? tune->krylov_maxit : 1000;
    f->krylov_tol = tune->krylov_tol > 0 ? tune->krylov_tol : 1e-10;
  }
  f->omega_host.resize(2 * n_omega);
  for (int i = 0; i < n_omega; i++) {
    f->omega_host[2 * i] = omega_re[i];
    f->omega_host[2 * i + 1] = omega_im ? omega_im[i] : 0.0;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t nn = (size_t)p->nx * p->ny;
  const bool gmres_ir = prec == RR_MIXED && tune && tune->refine_method == RR_REFINE_GMRES;
  const Plan pl = make_plan(p->nx, p->ny, n_omega, k_max, prec, T, p->phi != nullptr,
                            p->U != nullptr, tune ? tune->superblock : 0, !krylov && !gmres_ir);
  f->tile_bytes = pl.tiles;
  rr_status st = RR_OK;
#define ALLOC(ptr, bytes)                      \
  do {                                         \
    st = dalloc(f, &(ptr), (bytes));           \
    if (st != RR_OK) goto fail_free;           \
  } while (0)
  ALLOC(f->coef, pl.coef);
  if (p->phi) ALLOC(f->phi, pl.phi);
  if (p->U) ALLOC(f->U, pl.U);
  ALLOC(f->omega, pl.omega);
  if (!krylov) {  // the band LU and its dataflow state
    ALLOC(f->tiles, pl.tiles);
    ALLOC(f->xs, pl.xs);
    ALLOC(f->cbuf, pl.cbuf);
    ALLOC(f->flags, pl.flags);
    f->flag_count = pl.nflags;
  } else {        // the preconditioner and the Krylov vectors
    const size_t cols = (size_t)n_omega * k_max, cplx = 2 * sizeof(double);
    ALLOC(f->pc_dinv, pc_bytes(f->precond, p->nx, p->ny, n_omega));
    const int nvec = solver == RR_SOLVER_BICGSTAB ? 7 : 1;
    for (int v = 0; v < nvec; v++) ALLOC(f->kv[v], pl.vec);
    ALLOC(f->kpart, cols * krylov_nchunk(n64) * 2 * cplx);
    ALLOC(f->kscal, cols * 4 * cplx);
    ALLOC(f->kbnorm, cols * sizeof(double));
    ALLOC(f->kactive, cols * sizeof(uint32_t));
  }
  ALLOC(f->ctrl, pl.ctrl);
  ALLOC(f->theta, pl.theta);
  ALLOC(f->work1, pl.vec);
  ALLOC(f->work2, pl.vec);
  if (prec == RR_MIXED) ALLOC(f->work3, pl.work3);
  ALLOC(f->small.partial, pl.partial);
  ALLOC(f->small.G, pl.kk2);
  ALLOC(f->small.R, pl.kk2);
  ALLOC(f->small.Rinv, pl.kk2);
  ALLOC(f->small.W, pl.kk2);
  ALLOC(f->small.Ut, pl.kk2);
  if (prec == RR_MIXED) ALLOC(f->small.rho, pl.rho);
  if (pl.probe_blk) {
    ALLOC(f->probe_b, pl.probe_blk);
    ALLOC(f->probe_x, pl.probe_blk);
    ALLOC(f->probe_r, pl.probe_blk);
    ALLOC(f->probe_z, pl.probe_z);
    f->probe_np = pl.probe_np;
    f->probe_p = pl.probe_p;
  }
  ALLOC(f->small.shifted, pl.shifted);
  if (k_max > kNarrowK) {
    ALLOC(f->small.big1, pl.big);
    ALLOC(f->small.big2, pl.big);
    ALLOC(f->wide_tmp, pl.wide);
  }
  f->small.nchunk = pl.nchunk;
  f->small.kmax = k_max;
  f->grad_nchunk = pl.grad_nchunk;
  ALLOC(f->grad_partial, pl.grad);
  if ((prec == RR_MIXED && tune && tune->refine_method == RR_REFINE_GMRES) ||
      solver == RR_SOLVER_GMRES) {
    const int m = tune->gmres_restart ? tune->gmres_restart : (krylov ? kGmresMaxRestart : 8);
    const size_t cols = (size_t)n_omega * k_max, cplx = 2 * sizeof(double);
    f->gm.m = m;
    ALLOC(f->gm.V, (size_t)(m + 1) * pl.vec);
    ALLOC(f->gm.t, pl.vec);
    ALLOC(f->gm.H, cols * (m + 1) * m * cplx);
    ALLOC(f->gm.h, cols * (m + 1) * cplx);
    ALLOC(f->gm.beta, cols * sizeof(double));
    ALLOC(f->gm.y, cols * m * cplx);
    ALLOC(f->gm.partial, cols * gmres_nchunk(n64) * (m + 1) * cplx);
  }
#undef ALLOC
  {
    hipError_t e = hipMemcpyAsync(f->coef, p->coef, nn * 12 * sizeof(double),
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && p->phi)
      e = hipMemcpyAsync(f->phi, p->phi, nn * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && p->U)
      e = hipMemcpyAsync(f->U, p->U, (size_t)(p->nx + 2) * (p->ny + 2) * sizeof(double),
                         hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(f->omega, f->omega_host.data(), 2 * n_omega * sizeof(double),
                         hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill_u32(f->ctrl, 0u, 64, s);
    // the Krylov blocks start finite (their norms are taken on every cycle,
    // also the ones that skip their other work)
    if (e == hipSuccess && f->gm.V)
      e = launch_fill_u32((uint32_t*)f->gm.V, 0u, (int64_t)((f->gm.m + 1) * pl.vec / 4), s);
    if (e != hipSuccess) {
      st = fail(RR_ERR_HIP, hipGetErrorString(e));
      goto fail_free;
    }
  }
  if (p->U) {
    if (!(p->x1 > p->x0) || !(p->y1 > p->y0)) {
      st = fail(RR_ERR_INVALID, "empty domain");
      goto fail_free;
    }
    f->hx = (p->x1 - p->x0) / (p->nx + 1);
    f->hy = (p->y1 - p->y0) / (p->ny + 1);
    f->nu = p->nu;
    f->has_burgers = true;
  }
  {
    hipError_t e = krylov ? prepare_krylov(p->ny) : prepare_factor(T, prec == RR_MIXED);
    if (e == hipSuccess && !krylov) e = prepare_solve(T, prec == RR_MIXED);
    if (e != hipSuccess) {
      st = fail(RR_ERR_HIP, std::string("kernel attributes: ") + hipGetErrorString(e));
      goto fail_free;
    }
  }
  st = rr_refactor(f, stream);
  if (st != RR_OK) goto fail_free;
  if (f->probe_z) {
    // The probes' known solutions: FP32 solves of complex Gaussian forcing,
    // so that they have the make-up of the responses the refinement meets
    // (the contraction measured on white-noise probes came out up to 2x
    // smaller than on the solutions themselves; on such responses within
    // about 10 %).  Any vectors would do: the probes solve M x = M z for z.
    hipError_t e = launch_sketch(opdesc(f), nullptr, f->probe_p, kProbeSeed, RR_TM_GAUSSIAN, 0,
                                 f->probe_r, s);
    if (e == hipSuccess)
      e = launch_solve(f->geom, f->n, n_omega, f->probe_p, true, f->tiles, 0, f->probe_r, 0,
                       f->probe_z, f->xs, f->cbuf, f->flags, ticket_word(f), st_word(f),
                       f->solve_grid, s);
    if (e != hipSuccess) {
      st = fail(RR_ERR_HIP, hipGetErrorString(e));
      goto fail_free;
    }
  }
  // the omega upload reads a host vector owned by the handle: nothing to wait for
  *out = f;
  return RR_OK;
fail_free:
  (void)hipStreamSynchronize(s);
  free_all(f);
  delete f;
  return st;
}

rr_status rr_refactor(rr_factors* f, void* stream) {
  if (!f) return fail(RR_ERR_INVALID, "NULL handle");
  if (f->sticky_hip_error) return fail(RR_ERR_HIP, "handle is unusable after a HIP error");
  if (f->solver != RR_SOLVER_BAND_LU) {  // no LU: the preconditioner of every shift
    if (f->tev[0]) (void)hipEventRecord(f->tev[0], (hipStream_t)stream);
    hipError_t e = launch_pc_setup(opdesc(f), f->precond, f->omega, f->n_omega, f->pc_dinv,
                                   st_word(f), (hipStream_t)stream);
    if (f->tev[1]) (void)hipEventRecord(f->tev[1], (hipStream_t)stream);
    if (e != hipSuccess) {
      f->sticky_hip_error = true;
      return fail(RR_ERR_HIP, std::string("preconditioner launch: ") + hipGetErrorString(e));
    }
    return RR_OK;
  }
  hipError_t e = launch_factor(opdesc(f), f->geom, f->omega, f->n_omega, f->prec == RR_MIXED,
                               f->tiles, f->flags, factor_counters(f), st_word(f), f->grid,
                               (hipStream_t)stream, f->tev);
  // a new factor: the refinement's measured contractions no longer hold
  if (e == hipSuccess && f->small.rho)
    e = launch_refine_reset(f->n_omega, f->small.rho, (hipStream_t)stream);
  f->rho_fresh = f->small.rho != nullptr;
  if (e != hipSuccess) {
    f->sticky_hip_error = true;
    return fail(RR_ERR_HIP, std::string("factor launch: ") + hipGetErrorString(e));
  }
  return RR_OK;
}

rr_status rr_sketch_solve(rr_factors* f, int32_t k, uint64_t seed, int32_t power_iters, double* Q,
                          void* stream) {
  rr_status st = check_k(f, k);
  if (st != RR_OK) return st;
  if (!Q) return fail(RR_ERR_INVALID, "NULL Q");
  if (power_iters < 0 || power_iters > 64) return fail(RR_ERR_INVALID, "bad power_iters");
  hipStream_t s = (hipStream_t)stream;
  const int64_t blk = (int64_t)k * f->n;
  RR_HIP(launch_fill_u32(f->ctrl + 4, 0u, kMaxRefine, s));
  {                                                                                 // step 1
    const int z = f->tm_zeta <= 0 ? std::min(k, 8) : std::min<int>(f->tm_zeta, k);
    RR_HIP(launch_sketch(opdesc(f), f->phi, k, seed, f->tm_kind, z, f->theta, s));
    if (f->tm_kind == RR_TM_ORTHONORMAL) {  // orthonormal columns, then eq. 10's weights
      RR_HIP(cholqr(f, 1, k, f->theta, s));
      if (f->phi) RR_HIP(launch_weight_rows(f->n, k, f->phi, f->theta, s));
    }
  }
  const double ts = f->refine_tol_sketch;
  if ((st = solve_any(f, k, 0, f->theta, 0, Q, ts, s)) != RR_OK) return st;         // step 2
  RR_HIP(cholqr(f, f->n_omega, k, Q, s));                                          // step 3
  for (int it = 0; it < power_iters; it++) {                                        // 2.2.1
    if ((st = solve_any(f, k, 1, Q, blk, f->work1, ts, s)) != RR_OK) return st;
    RR_HIP(cholqr(f, f->n_omega, k, f->work1, s));
    if ((st = solve_any(f, k, 0, f->work1, blk, Q, ts, s)) != RR_OK) return st;
    RR_HIP(cholqr(f, f->n_omega, k, Q, s));
  }
  return RR_OK;
}

rr_status rr_set_test_matrix(rr_factors* f, rr_test_matrix kind, int32_t zeta) {
  if (!f) return fail(RR_ERR_INVALID, "NULL handle");
  if (kind != RR_TM_GAUSSIAN && kind != RR_TM_RADEMACHER && kind != RR_TM_SPARSE &&
      kind != RR_TM_ORTHONORMAL)
    return fail(RR_ERR_INVALID, "unknown test matrix kind");
  if (zeta < 0) return fail(RR_ERR_INVALID, "zeta must be >= 0");
  f->tm_kind = kind;
  f->tm_zeta = zeta;
  return RR_OK;
}

rr_status rr_adjoint_solve(rr_factors* f, int32_t k, const double* Q, double* Z, void* stream) {
  rr_status st = check_k(f, k);
  if (st != RR_OK) return st;
  if (!Q || !Z) return fail(RR_ERR_INVALID, "NULL pointer");
  if (Q == Z && f->prec == RR_MIXED) return fail(RR_ERR_INVALID, "Z may not alias Q (mixed)");
  return solve_any(f, k, 1, Q, (int64_t)k * f->n, Z, f->refine_tol,                // step 4
                   (hipStream_t)stream);
}

rr_status rr_solve(rr_factors* f, int32_t k, const double* Bm, double* X, void* stream) {
  rr_status st = check_k(f, k);
  if (st != RR_OK) return st;
  if (!Bm || !X) return fail(RR_ERR_INVALID, "NULL pointer");
  if (Bm == X) return fail(RR_ERR_INVALID, "X may not alias Bm");
  return solve_any(f, k, 0, Bm, (int64_t)k * f->n, X, f->refine_tol, (hipStream_t)stream);
}

rr_status rr_gains(rr_factors* f, int32_t k, const double* Q, const double* Z, rr_response mode,
                   double* sigma_B, double* sigma_AV, double* V, double* Uresp, void* stream) {
  rr_status st = check_k(f, k);
  if (st != RR_OK) return st;
  if (!Z || !sigma_B || !V) return fail(RR_ERR_INVALID, "NULL pointer");
  if (mode == RR_RESP_AV && !sigma_AV) return fail(RR_ERR_INVALID, "sigma_AV needed for AV");
  if (mode == RR_RESP_QU && (!Q || !Uresp)) return fail(RR_ERR_INVALID, "Q, Uresp needed for QU");
  if (mode != RR_RESP_AV && mode != RR_RESP_QU && mode != RR_RESP_NONE)
    return fail(RR_ERR_INVALID, "unknown response mode");
  if (V == Z || (Uresp && (Uresp == V || Uresp == Z)))
    return fail(RR_ERR_INVALID, "outputs may not alias inputs");
  hipStream_t s = (hipStream_t)stream;
  // step 5 (and eq. 8 when asked)
  RR_HIP(small_svd(f, k, Z, Q, sigma_B, V, mode == RR_RESP_QU ? Uresp : nullptr, s));
  if (mode == RR_RESP_AV) {
    // steps 6-9: W = M^-1 V, sigma_j = ||W_j||, u_j = W_j / sigma_j
    double* W = Uresp ? Uresp : f->work2;
    if ((st = solve_any(f, k, 0, V, (int64_t)k * f->n, W, f->refine_tol, s)) != RR_OK) return st;
    RR_HIP(colnorm_scale(f, k, W, sigma_AV, Uresp, s));
  }
  return RR_OK;
}

rr_status rr_resvd(rr_factors* f, int32_t k, const double* Us, const double* scale,
                   const double* V, double* sigma, double* U, double* Vnew, void* stream) {
  rr_status st = check_k(f, k);
  if (st != RR_OK) return st;
  if (!Us || !V || !sigma || !U || !Vnew) return fail(RR_ERR_INVALID, "NULL pointer");
  if (U == Us || U == V || Vnew == Us || Vnew == V || U == Vnew)
    return fail(RR_ERR_INVALID, "outputs may not alias inputs or each other");
  hipStream_t s = (hipStream_t)stream;
  const double* X = Us;
  if (scale) {  // U^Sigma from the unit response modes and their gains
    RR_HIP(launch_scale_cols(f->n, f->n_omega, k, Us, scale, f->work2, s));
    X = f->work2;
  }
  // step 10: U^Sigma = Qz R, R^H = Ut S W^H, so U^Sigma = (Qz W) S Ut^H: the
  // left singular vectors are Qz W and the right ones Ut; step 11: V <- V Ut
  RR_HIP(small_svd(f, k, X, V, sigma, U, Vnew, s));
  return RR_OK;
}

rr_status rr_grad(rr_factors* f, const double* sigma1, const double* u1, const double* v1,
                  int64_t vec_stride, double* dU, double* dnu, double* domega, void* stream) {
  if (!f) return fail(RR_ERR_INVALID, "NULL handle");
  if (!f->has_burgers) return fail(RR_ERR_INVALID, "rr_grad needs the Burgers description (U)");
  if (!sigma1 || !u1 || !v1 || !dU || !dnu || !domega) return fail(RR_ERR_INVALID, "NULL pointer");
  if (vec_stride < f->n && f->n_omega > 1) return fail(RR_ERR_INVALID, "vec_stride < n");
  RR_HIP(launch_grad(f->nx, f->ny, f->hx, f->hy, f->n_omega, f->omega, sigma1, u1, v1, vec_stride,
                     dU, dnu, domega, f->grad_partial, f->grad_nchunk, (hipStream_t)stream));
  return RR_OK;
}

// ---------------------------------------------------------------------------
// Gradient without allocation: the partial sums of k_grad go to a file-scope
// device array instead of a handle's workspace.  Each GPU the library runs on
// holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (the array's name is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr int64_t kGradScratchDoubles = int64_t(1) << 18;  // 2 MiB per GPU
static __device__ __align__(256) double scratch[kGradScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// This device's copy of `scratch`, looked up once per device (with that
// device current) and kept.
rr_status scratch_for_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(RR_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(RR_ERR_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return RR_OK;
}
}  // namespace

rr_status rr_grad_noalloc(const rr_problem* p, int32_t n_omega, const double* sigma1,
                          const double* u1, const double* v1, int64_t vec_stride, double* dU,
                          double* dnu, double* domega, void* stream) {
  if (!p || !sigma1 || !u1 || !v1 || !dU || !dnu || !domega)
    return fail(RR_ERR_INVALID, "NULL pointer");
  if (p->nx < 1 || p->ny < 1 || n_omega < 1 || n_omega > 65535)
    return fail(RR_ERR_INVALID, "bad sizes");
  if (!(p->x1 > p->x0) || !(p->y1 > p->y0)) return fail(RR_ERR_INVALID, "empty domain");
  const int64_t n = 2 * (int64_t)p->nx * p->ny;
  if (vec_stride < n && n_omega > 1) return fail(RR_ERR_INVALID, "vec_stride < n");
  const int64_t nfull = (int64_t)(p->nx + 2) * (p->ny + 2);
  const int64_t nchunk = (nfull + 255) / 256;  // k_grad's blocks per shift
  const int64_t need = 2 * nchunk * n_omega;
  if (need > kGradScratchDoubles)
    return fail(RR_ERR_INVALID, "rr_grad_noalloc needs " + std::to_string(need) +
                                    " doubles of scratch; the maximum is " +
                                    std::to_string(kGradScratchDoubles));
  double* ws = nullptr;
  rr_status st = scratch_for_current_device(&ws);
  if (st != RR_OK) return st;
  const double hx = (p->x1 - p->x0) / (p->nx + 1), hy = (p->y1 - p->y0) / (p->ny + 1);
  RR_HIP(launch_grad(p->nx, p->ny, hx, hy, n_omega, nullptr, sigma1, u1, v1, vec_stride, dU,
                     dnu, domega, ws, (int)nchunk, (hipStream_t)stream));
  return RR_OK;
}

rr_status rr_check(rr_factors* f, void* stream) {
  if (!f) return fail(RR_ERR_INVALID, "NULL handle");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    f->sticky_hip_error = true;
    return fail(RR_ERR_HIP, std::string("stream: ") + hipGetErrorString(e));
  }
  uint32_t ctrl[4 + kMaxRefine];
  e = hipMemcpy(ctrl, f->ctrl, sizeof(ctrl), hipMemcpyDeviceToHost);
  if (e == hipSuccess) {  // the correction counts restart at every check
    const uint32_t zeros[kMaxRefine] = {};
    e = hipMemcpy(f->ctrl + 4, zeros, sizeof(zeros), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    f->sticky_hip_error = true;
    return fail(RR_ERR_HIP, hipGetErrorString(e));
  }
  f->refine_used = 0;
  if (f->prec == RR_MIXED) {
    f->refine_used = f->refine_iters;
    for (int it = 0; it < f->refine_iters; it++)
      if (ctrl[4 + it] == 0) { f->refine_used = it + 1; break; }
  }
  uint32_t w = ctrl[0];
  if (w) {
    uint32_t zero = 0;
    (void)hipMemcpy(f->ctrl, &zero, sizeof(zero), hipMemcpyHostToDevice);
  }
  if (w & ST_TIMEOUT) return fail(RR_ERR_TIMEOUT, "a dataflow wait timed out");
  if (w & ST_SINGULAR)
    return fail(RR_ERR_SINGULAR, f->solver != RR_SOLVER_BAND_LU
                                     ? "singular node block in the preconditioner"
                                     : "zero or non-finite pivot in the band LU");
  if (w & ST_NONFINITE) return fail(RR_ERR_NONFINITE, "non-finite values in the results");
  if (w & ST_BREAKDOWN)
    return fail(RR_ERR_BREAKDOWN, f->solver == RR_SOLVER_BICGSTAB
                                      ? "BiCGStab breakdown (a vanishing rho or <rhat, v>) or "
                                        "a Gram matrix not positive definite"
                                      : "Gram matrix not positive definite");
  if (w & ST_SVD_NOT_CONVERGED)
    return fail(RR_ERR_NOT_CONVERGED, "the k x k Jacobi SVD did not converge in " +
                                          std::to_string(f->small.jacobi_sweeps) + " sweeps");
  if ((w & ST_NOT_CONVERGED) && f->solver != RR_SOLVER_BAND_LU)
    return fail(RR_ERR_NOT_CONVERGED, "a Krylov solve missed its tolerance in " +
                                          std::to_string(f->krylov_maxit) + " iterations");
  if (w & ST_NOT_CONVERGED) {
    std::string m = "refinement did not converge (most unconverged columns after each correction:";
    for (int it = 0; it < f->refine_iters; it++) m += " " + std::to_string(ctrl[4 + it]);
    return fail(RR_ERR_NOT_CONVERGED, m + ")");
  }
  return RR_OK;
}

int32_t rr_refine_count(rr_factors* f) { return f ? f->refine_used : 0; }

rr_status rr_precond_apply(rr_factors* f, int32_t k, int32_t adjoint, const double* X, double* Y,
                           void* stream) {
  if (!f || !X || !Y) return fail(RR_ERR_INVALID, "NULL pointer");
  if (f->solver == RR_SOLVER_BAND_LU) return fail(RR_ERR_INVALID, "not a Krylov handle");
  if (k < 1 || k > f->k_max) return fail(RR_ERR_INVALID, "k out of range");
  RR_HIP(launch_pc_apply(opdesc(f), f->precond, f->n_omega, k, adjoint ? 1 : 0, f->pc_dinv, X, Y,
                         nullptr, nullptr, (hipStream_t)stream));
  return RR_OK;
}

rr_status rr_set_timing_events(rr_factors* f, void* factor_begin, void* factor_end,
                               void* solve_begin, void* solve_end) {
  if (!f) return fail(RR_ERR_INVALID, "NULL handle");
  f->tev[0] = (hipEvent_t)factor_begin;
  f->tev[1] = (hipEvent_t)factor_end;
  f->tev[2] = (hipEvent_t)solve_begin;
  f->tev[3] = (hipEvent_t)solve_end;
  return RR_OK;
}

rr_status rr_set_jacobi_sweeps(rr_factors* f, int32_t sweeps) {
  if (!f) return fail(RR_ERR_INVALID, "NULL handle");
  if (sweeps < 1 || sweeps > 64) return fail(RR_ERR_INVALID, "sweeps must be in [1, 64]");
  f->small.jacobi_sweeps = sweeps;
  return RR_OK;
}

size_t rr_bytes(const rr_factors* f) { return f ? f->bytes : 0; }

void rr_factors_free(rr_factors* f) {
  if (!f) return;
  (void)hipDeviceSynchronize();
  free_all(f);
  delete f;
}

rr_status rr_set_allocator(rr_alloc_fn alloc, rr_free_fn dealloc, void* ctx) {
  if ((alloc == nullptr) != (dealloc == nullptr))
    return fail(RR_ERR_INVALID, "alloc and dealloc must both be set or both be NULL");
  g_alloc = alloc;
  g_dealloc = dealloc;
  g_alloc_ctx = ctx;
  return RR_OK;
}

size_t rr_factor_bytes(int32_t nx, int32_t ny, int32_t n_omega, int32_t k_max, rr_precision prec,
                       int32_t tile) {
  if (nx < 1 || ny < 1 || n_omega < 1 || k_max < 1) return 0;
  if (k_max > (prec == RR_FP64 ? kMaxWideK : kNarrowK)) return 0;
  const int T = tile ? tile : 64;
  if (T != 32 && T != 64) return 0;
  return make_plan(nx, ny, n_omega, k_max, prec, T, true, true, 0, true).total();
}

// ---------------------------------------------------------------------------
// Captured sweeps
// ---------------------------------------------------------------------------
struct rr_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

void rr_graph_free(rr_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

rr_status rr_graph_capture(rr_factors* f, int32_t refactor, int32_t k, uint64_t seed, int32_t q,
                           rr_response mode, double* Q, double* Z, double* sigma_B,
                           double* sigma_AV, double* V, double* Uresp, rr_graph** out) {
  if (!out) return fail(RR_ERR_INVALID, "NULL output graph pointer");
  *out = nullptr;
  rr_status st = check_k(f, k);
  if (st != RR_OK) return st;
  if (!Q || !Z || !sigma_B || !V) return fail(RR_ERR_INVALID, "NULL pointer");
  if (Q == Z) return fail(RR_ERR_INVALID, "Z may not alias Q");
  // Capture on a private stream (the legacy default stream cannot capture);
  // replays are ordered on whatever stream rr_graph_launch is given.
  hipStream_t cs = nullptr;
  RR_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(RR_ERR_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  if (refactor) st = rr_refactor(f, cs);
  if (st == RR_OK) st = rr_sketch_solve(f, k, seed, q, Q, cs);
  if (st == RR_OK) st = rr_adjoint_solve(f, k, Q, Z, cs);
  if (st == RR_OK) st = rr_gains(f, k, Q, Z, mode, sigma_B, sigma_AV, V, Uresp, cs);
  rr_graph* g = new rr_graph();
  e = hipStreamEndCapture(cs, &g->graph);
  (void)hipStreamDestroy(cs);
  if (st == RR_OK && e != hipSuccess)
    st = fail(RR_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  if (st == RR_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
      st = fail(RR_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  if (st != RR_OK) {
    rr_graph_free(g);
    return st;
  }
  *out = g;
  return RR_OK;
}

rr_status rr_graph_launch(rr_graph* g, void* stream) {
  if (!g || !g->exec) return fail(RR_ERR_INVALID, "NULL graph");
  RR_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return RR_OK;
}

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// Cache of autotuner picks: a JSON object, one entry per line,
//   "gfx950|512x256|w16|k20|mixed": {"tile": 64, "grid": 512, "superblock": 4, "ms": 812.5},
// at the path named by RR_AUTOTUNE_CACHE (no cache when unset).
std::string tune_key(const rr_problem* p, int nw, int k, rr_precision prec) {
  std::string arch = "gpu";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  } else {
    (void)hipGetLastError();
  }
  return arch + "|" + std::to_string(p->nx) + "x" + std::to_string(p->ny) + "|w" +
         std::to_string(nw) + "|k" + std::to_string(k) + "|" + (prec == RR_MIXED ? "mixed" : "fp64");
}

std::vector<std::string> cache_lines(const char* path) {
  std::vector<std::string> out;
  FILE* fh = std::fopen(path, "r");
  if (!fh) return out;
  char buf[1024];
  while (std::fgets(buf, sizeof(buf), fh)) {
    std::string ln(buf);
    if (ln.find("\": {") != std::string::npos) {
      while (!ln.empty() && (ln.back() == '\n' || ln.back() == ',' || ln.back() == '\r'))
        ln.pop_back();
      out.push_back(ln);
    }
  }
  std::fclose(fh);
  return out;
}

bool cache_lookup(const char* path, const std::string& key, rr_tuning* t, double* ms) {
  for (const std::string& ln : cache_lines(path)) {
    if (ln.compare(0, key.size() + 2, "\"" + key + "\"") != 0) continue;
    const size_t o = ln.find('{');
    int tile = 0, grid = 0, sb = 0;
    double v = 0;
    if (std::sscanf(ln.c_str() + o, "{\"tile\": %d, \"grid\": %d, \"superblock\": %d, \"ms\": %lf}",
                    &tile, &grid, &sb, &v) == 4) {
      *t = rr_tuning{};
      t->tile = tile;
      t->grid = grid;
      t->superblock = sb;
      *ms = v;
      return true;
    }
  }
  return false;
}

void cache_store(const char* path, const std::string& key, const rr_tuning& t, double ms) {
  std::vector<std::string> lines;
  for (const std::string& ln : cache_lines(path))
    if (ln.compare(0, key.size() + 2, "\"" + key + "\"") != 0) lines.push_back(ln);
  char buf[512];
  std::snprintf(buf, sizeof(buf), "\"%s\": {\"tile\": %d, \"grid\": %d, \"superblock\": %d, \"ms\": %.17g}",
                key.c_str(), t.tile, t.grid, t.superblock, ms);
  lines.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fh = std::fopen(tmp.c_str(), "w");
  if (!fh) return;
  std::fprintf(fh, "{\n");
  for (size_t i = 0; i < lines.size(); i++)
    std::fprintf(fh, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
  std::fprintf(fh, "}\n");
  std::fclose(fh);
  (void)std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" {

rr_status rr_autotune(const rr_problem* p, const double* omega_re, const double* omega_im,
                      int32_t n_omega, int32_t k, rr_precision prec, int32_t max_shifts,
                      void* stream, rr_tuning* out, double* out_ms) {
  if (!p || !omega_re || !out) return fail(RR_ERR_INVALID, "NULL pointer");
  if (n_omega < 1 || k < 1 || k > 32) return fail(RR_ERR_INVALID, "bad n_omega or k");
  const int nw = (max_shifts > 0 && max_shifts < n_omega) ? max_shifts : n_omega;
  const int64_t n = 2 * (int64_t)p->nx * p->ny;
  hipStream_t s = (hipStream_t)stream;
  const char* cache = std::getenv("RR_AUTOTUNE_CACHE");
  const std::string key = tune_key(p, nw, k, prec);
  if (cache && *cache) {
    double ms = 0;
    if (cache_lookup(cache, key, out, &ms)) {
      if (out_ms) *out_ms = ms;
      return RR_OK;
    }
  }
  const int cus = device_cus();
  double *Q = nullptr, *Z = nullptr;
  const size_t vb = (size_t)nw * k * n * 2 * sizeof(double);
  if (hipMalloc((void**)&Q, vb) != hipSuccess || hipMalloc((void**)&Z, vb) != hipSuccess) {
    (void)hipGetLastError();
    if (Q) (void)hipFree(Q);
    return fail(RR_ERR_NOMEM, "autotune: no room for the trial blocks");
  }
  hipEvent_t ev[4];
  for (auto& x : ev) (void)hipEventCreate(&x);
  // one trial: factor, sketch solve and adjoint solve of the first nw shifts;
  // score = factor + 2.5 (sketch + adjoint), one pass of Algorithm 1 with a
  // subspace iteration; < 0 when the candidate does not fit in memory
  auto trial = [&](const rr_tuning& t, double* score) -> rr_status {
    *score = -1.0;
    rr_factors* h = nullptr;
    rr_status fs = rr_factor(p, omega_re, omega_im, nw, k, prec, &t, stream, &h);
    if (fs == RR_ERR_NOMEM) return RR_OK;
    if (fs != RR_OK) return fs;
    fs = rr_sketch_solve(h, k, 0, 0, Q, stream);  // warm-up pass
    if (fs == RR_OK) fs = rr_adjoint_solve(h, k, Q, Z, stream);
    if (fs == RR_OK) fs = rr_check(h, stream);
    float ms_f = 0, ms_s = 0, ms_a = 0;
    if (fs == RR_OK) {
      (void)hipEventRecord(ev[0], s);
      fs = rr_refactor(h, stream);
      (void)hipEventRecord(ev[1], s);
      if (fs == RR_OK) fs = rr_sketch_solve(h, k, 0, 0, Q, stream);
      (void)hipEventRecord(ev[2], s);
      if (fs == RR_OK) fs = rr_adjoint_solve(h, k, Q, Z, stream);
      (void)hipEventRecord(ev[3], s);
      if (fs == RR_OK) fs = rr_check(h, stream);
      (void)hipEventElapsedTime(&ms_f, ev[0], ev[1]);
      (void)hipEventElapsedTime(&ms_s, ev[1], ev[2]);
      (void)hipEventElapsedTime(&ms_a, ev[2], ev[3]);
    }
    rr_factors_free(h);
    if (fs == RR_OK) *score = ms_f + 2.5 * (ms_s + ms_a);
    return fs;
  };
  rr_status st = RR_OK;
  double best = -1.0;
  rr_tuning pick{};
  // the tile and the persistent grid with the default superblock, then the
  // superblock (and the tile-by-tile solve) for that tile and grid
  const int tiles[2] = {64, 32};
  const int grids[2] = {cus, 2 * cus};
  for (int ti = 0; ti < 2 && st == RR_OK; ti++)
    for (int gi = 0; gi < 2 && st == RR_OK; gi++) {
      rr_tuning t{};
      t.tile = tiles[ti];
      t.grid = grids[gi];
      double sc = 0;
      st = trial(t, &sc);
      if (st == RR_OK && sc >= 0 && (best < 0 || sc < best)) {
        best = sc;
        pick = t;
      }
    }
  if (st == RR_OK && best >= 0) {
    const int B = (2 * p->ny + pick.tile - 1) / pick.tile;
    const int dflt = superblock_tiles(0, pick.tile, B);
    const int sbs[4] = {-1, 2, 4, 8};
    const rr_tuning base = pick;
    for (int i = 0; i < 4 && st == RR_OK; i++) {
      if (sbs[i] == dflt || (sbs[i] > 0 && sbs[i] > 2 * B)) continue;
      rr_tuning t = base;
      t.superblock = sbs[i];
      double sc = 0;
      st = trial(t, &sc);
      if (st == RR_OK && sc >= 0 && sc < best) {
        best = sc;
        pick = t;
      }
    }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  (void)hipFree(Q);
  (void)hipFree(Z);
  if (st != RR_OK) return st;
  if (best < 0) return fail(RR_ERR_NOMEM, "autotune: no candidate fits in device memory");
  *out = pick;
  if (out_ms) *out_ms = best;
  if (cache && *cache) cache_store(cache, key, pick, best);
  return RR_OK;
}

}  // extern "C"
