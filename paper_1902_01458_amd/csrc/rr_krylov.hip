// LU-free solves of the shifted systems M(omega) X = B and M^H X = B: the
// paper notes (Section 3.2, after Fig. 7) that BiCGStab or GMRES with an
// incomplete-LU or Jacobi preconditioner can stand in for the direct solves;
// that is what lets Algorithm 1 run where the band LU no longer fits in
// memory.  Everything here is FP64 and batched: every (shift, column) pair is
// its own linear system, M is applied from the stencil (k_apply).
//
// Preconditioners K ~ M, both built from the 2 x 2 node blocks of M (the two
// velocity components of a grid node couple through the base-flow shear):
//   Jacobi:  K = D = the block diagonal of M.
//   ILU(0):  K = (D + L) D^-1 (D + U) with L, U the strict block triangles of
//            M in natural order (p = j + ny i) and D from the recurrence
//              D_p = M_pp - M_p,p-1 D_p-1^-1 M_p-1,p - M_p,p-ny D_p-ny^-1 M_p-ny,p
//            (block ILU(0): on this stencil the dropped fill is exactly the
//            two cross terms, so L and U keep M's own off-diagonal blocks).
//            Both the recurrence and the triangular sweeps of K^-1 depend on
//            the previous anti-diagonal of the grid only (p - 1 and p - ny lie
//            on i + j - 1), so one workgroup walks the nx + ny - 1
//            anti-diagonals of a system with the previous one in LDS.
// Off-diagonal blocks of M are diagonal 2 x 2 (each component couples to the
// same component of a neighbour), with entries -c from the stencil row.
#include "rr_internal.h"

namespace rr {

namespace {

constexpr int kKChunk = 2048;  // rows per partial sum of the batched dot products
constexpr int kKThreads = 256;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// 2 x 2 complex matrix, row-major: m[0] m[1] / m[2] m[3]
struct C2 {
  double2 m[4];
};

__device__ __forceinline__ bool inv2(const C2& A, C2& X) {
  const double2 det = csub(cmul(A.m[0], A.m[3]), cmul(A.m[1], A.m[2]));
  const double dd = det.x * det.x + det.y * det.y;
  if (!(dd > 0.0) || !isfinite(dd)) return false;
  const double2 id = make_double2(det.x / dd, -det.y / dd);
  X.m[0] = cmul(A.m[3], id);
  X.m[1] = cmul(make_double2(-A.m[1].x, -A.m[1].y), id);
  X.m[2] = cmul(make_double2(-A.m[2].x, -A.m[2].y), id);
  X.m[3] = cmul(A.m[0], id);
  return true;
}

// y = A x (or A^H x) for a 2-vector x = (x0, x1)
__device__ __forceinline__ void mv2(const C2& A, bool herm, double2 x0, double2 x1, double2& y0,
                                    double2& y1) {
  if (!herm) {
    y0 = cadd(cmul(A.m[0], x0), cmul(A.m[1], x1));
    y1 = cadd(cmul(A.m[2], x0), cmul(A.m[3], x1));
  } else {
    y0 = cadd(cmulc(A.m[0], x0), cmulc(A.m[2], x1));
    y1 = cadd(cmulc(A.m[1], x0), cmulc(A.m[3], x1));
  }
}

// The node block M_pp = i omega I - L_pp of shift (om_r, om_i) from the
// stencil row c (12 coefficients: u row c[0..5], v row c[6..11]).
__device__ __forceinline__ C2 node_block(const double* c, double om_r, double om_i) {
  C2 A;
  A.m[0] = make_double2(-om_i - c[0], om_r);
  A.m[1] = make_double2(-c[5], 0.0);
  A.m[2] = make_double2(-c[11], 0.0);
  A.m[3] = make_double2(-om_i - c[6], om_r);
  return A;
}

__device__ __forceinline__ C2 load_c2(const double2* p) {
  C2 A;
#pragma unroll
  for (int e = 0; e < 4; e++) A.m[e] = p[e];
  return A;
}
__device__ __forceinline__ void store_c2(double2* p, const C2& A) {
#pragma unroll
  for (int e = 0; e < 4; e++) p[e] = A.m[e];
}

// Jacobi: Dinv[w][p] = M_pp^-1 for every node and shift.
__global__ void k_pc_jacobi(int nn, const double* __restrict__ coef,
                            const double* __restrict__ omega, double2* __restrict__ Dinv,
                            uint32_t* status) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, w = blockIdx.y;
  if (p >= nn) return;
  C2 A = node_block(coef + 12 * (int64_t)p, omega[2 * w], omega[2 * w + 1]), X;
  if (!inv2(A, X)) {
    latch(status, ST_SINGULAR);
    X.m[0] = X.m[3] = make_double2(1, 0);
    X.m[1] = X.m[2] = make_double2(0, 0);
  }
  store_c2(Dinv + ((int64_t)w * nn + p) * 4, X);
}

// Block ILU(0) data of a shift, stored by anti-diagonal: slot (d, j) = d ny +
// j holds node (i, j) = (d - j, j) (slots with i outside 0 .. nx-1 unused),
// as kIluFields arrays of slots double2 (structure of arrays), so that the
// sweeps, whose threads take consecutive j on one anti-diagonal, read
// consecutive words:
//   0-3   D_p^-1 (row-major 2 x 2)
//   4, 5  forward, K:   (c4, c10) of p, (c2, c8) of p      (blocks to p-1, p-ny)
//   6, 7  forward, K^H: (c3, c9) of p-1, (c1, c7) of p-ny
//   8, 9  backward, K:  (c3, c9) of p, (c1, c7) of p
//   10,11 backward, K^H:(c4, c10) of p+1, (c2, c8) of p+ny
// (the stencil coefficients themselves; the blocks are minus them, and
// neighbours outside the grid hold zeros).  In the natural node order every
// operand load of a sweep step touches one cache line per thread, which
// bounds the sweep (measured: 10 ms per apply at 1024 x 512 against 3.9 ms
// with the operands read coalesced).
constexpr int kIluFields = 12;
__host__ __device__ inline int64_t ilu_slots(int nx, int ny) { return (int64_t)(nx + ny - 1) * ny; }

// Block ILU(0) of one shift per workgroup: D_p by the recurrence in the
// header, anti-diagonal by anti-diagonal (d = i + j), the previous
// anti-diagonal's D^-1 in LDS indexed by j.  Stores D^-1 and the
// coefficient pairs in the anti-diagonal layout above.
__global__ __launch_bounds__(kKThreads) void k_pc_ilu0(int nx, int ny,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ omega,
                                                       double2* __restrict__ Dinv,
                                                       uint32_t* status) {
  extern __shared__ __align__(16) char kl_smem[];
  C2* ring = reinterpret_cast<C2*>(kl_smem);  // [2][ny]
  const int w = blockIdx.x;
  const double om_r = omega[2 * w], om_i = omega[2 * w + 1];
  const int64_t ns = ilu_slots(nx, ny);
  double2* Fw = Dinv + (int64_t)w * kIluFields * ns;
  for (int d = 0; d < nx + ny - 1; d++) {
    C2* cur = ring + (d & 1) * ny;
    const C2* prev = ring + ((d + 1) & 1) * ny;
    const int j0 = max(0, d - nx + 1), j1 = min(ny - 1, d);
    for (int j = j0 + threadIdx.x; j <= j1; j += blockDim.x) {
      const int i = d - j, p = j + ny * i;
      const double* c = coef + 12 * (int64_t)p;
      C2 D = node_block(c, om_r, om_i);
      if (j > 0) {  // - M_p,p-1 D_p-1^-1 M_p-1,p: diag(-c4, -c10) E diag(-c3', -c9')
        const double* cq = coef + 12 * (int64_t)(p - 1);
        const C2& E = prev[j - 1];
        const double a[2] = {-c[4], -c[10]}, b[2] = {-cq[3], -cq[9]};
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
          for (int s = 0; s < 2; s++) D.m[2 * r + s] = csub(D.m[2 * r + s], cscale(a[r] * b[s], E.m[2 * r + s]));
      }
      if (i > 0) {  // - M_p,p-ny D_p-ny^-1 M_p-ny,p: diag(-c2, -c8) E diag(-c1', -c7')
        const double* cq = coef + 12 * (int64_t)(p - ny);
        const C2& E = prev[j];
        const double a[2] = {-c[2], -c[8]}, b[2] = {-cq[1], -cq[7]};
#pragma unroll
        for (int r = 0; r < 2; r++)
#pragma unroll
          for (int s = 0; s < 2; s++) D.m[2 * r + s] = csub(D.m[2 * r + s], cscale(a[r] * b[s], E.m[2 * r + s]));
      }
      C2 X;
      if (!inv2(D, X)) {
        latch(status, ST_SINGULAR);
        X.m[0] = X.m[3] = make_double2(1, 0);
        X.m[1] = X.m[2] = make_double2(0, 0);
      }
      cur[j] = X;
      const int64_t sl = (int64_t)d * ny + j;
#pragma unroll
      for (int e = 0; e < 4; e++) Fw[e * ns + sl] = X.m[e];
      const double* cl = coef + 12 * (int64_t)(j > 0 ? p - 1 : p);
      const double* cu = coef + 12 * (int64_t)(i > 0 ? p - ny : p);
      const double* cr = coef + 12 * (int64_t)(j < ny - 1 ? p + 1 : p);
      const double* cd = coef + 12 * (int64_t)(i < nx - 1 ? p + ny : p);
      const bool hl = j > 0, hu = i > 0, hr = j < ny - 1, hd = i < nx - 1;
      Fw[4 * ns + sl] = make_double2(c[4], c[10]);
      Fw[5 * ns + sl] = make_double2(c[2], c[8]);
      Fw[6 * ns + sl] = hl ? make_double2(cl[3], cl[9]) : make_double2(0, 0);
      Fw[7 * ns + sl] = hu ? make_double2(cu[1], cu[7]) : make_double2(0, 0);
      Fw[8 * ns + sl] = make_double2(c[3], c[9]);
      Fw[9 * ns + sl] = make_double2(c[1], c[7]);
      Fw[10 * ns + sl] = hr ? make_double2(cr[4], cr[10]) : make_double2(0, 0);
      Fw[11 * ns + sl] = hd ? make_double2(cd[2], cd[8]) : make_double2(0, 0);
    }
    __syncthreads();
  }
}

// Y = K^-1 X (or K^-H X) with K = D (Jacobi), for every (shift, column).
__global__ void k_pc_jacobi_apply(int nn, int k, int adjoint, const double2* __restrict__ Dinv,
                                  const double2* X, double2* Y, const uint32_t* active,
                                  const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y, w = blockIdx.z;
  if (p >= nn) return;
  const int64_t q = (int64_t)w * k + c;
  if (active && !active[q]) return;
  const int64_t off = q * 2 * nn + 2 * (int64_t)p;
  const C2 E = load_c2(Dinv + ((int64_t)w * nn + p) * 4);
  double2 y0, y1;
  mv2(E, adjoint != 0, X[off], X[off + 1], y0, y1);
  Y[off] = y0;
  Y[off + 1] = y1;
}

// Y = K^-1 X (or K^-H X) with the block ILU(0) K, one workgroup per
// (column, shift): the block-lower sweep by ascending anti-diagonals, then the
// block-upper one by descending ones, each node reading its two neighbours of
// the previous anti-diagonal from LDS.  Y may alias X.
//   forward  w_p = D_p^-1 (x_p - M_p,p-1 w_p-1 - M_p,p-ny w_p-ny)
//   backward y_p = w_p - D_p^-1 (M_p,p+1 y_p+1 + M_p,p+ny y_p+ny)
// and for K^H = (D + U)^H D^-H (D + L)^H:
//   forward  w_p = D_p^-H (x_p - M_p-1,p w_p-1 - M_p-ny,p w_p-ny)
//   backward y_p = w_p - D_p^-H (M_p+1,p y_p+1 + M_p+ny,p y_p+ny)
// (the off-diagonal blocks are real and diagonal, so ^H leaves them as they are).
__global__ __launch_bounds__(kKThreads) void k_pc_ilu0_apply(int nx, int ny, int k, int adjoint,
                                                             const double* __restrict__ coef,
                                                             const double2* __restrict__ Dinv,
                                                             const double2* X, double2* Y,
                                                             const uint32_t* active,
                                                             const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  extern __shared__ __align__(16) char ka_smem[];
  double2* ring = reinterpret_cast<double2*>(ka_smem);  // [2][ny][2]
  const int c = blockIdx.x, w = blockIdx.y, nn = nx * ny;
  const int64_t q = (int64_t)w * k + c;
  if (active && !active[q]) return;
  const int64_t off = q * 2 * nn;
  const double2* x = X + off;
  double2* y = Y + off;
  const int64_t ns = ilu_slots(nx, ny);
  const double2* Fw = Dinv + (int64_t)w * kIluFields * ns;
  const bool herm = adjoint != 0;
  const int nd = nx + ny - 1;
  auto dblock = [&](int64_t sl) {
    C2 D;
#pragma unroll
    for (int e = 0; e < 4; e++) D.m[e] = Fw[e * ns + sl];
    return D;
  };
  for (int d = 0; d < nd; d++) {
    double2* cur = ring + (d & 1) * 2 * ny;
    const double2* prev = ring + ((d + 1) & 1) * 2 * ny;
    const int j0 = max(0, d - nx + 1), j1 = min(ny - 1, d);
    for (int j = j0 + threadIdx.x; j <= j1; j += blockDim.x) {
      const int i = d - j, p = j + ny * i;
      const int64_t sl = (int64_t)d * ny + j;
      double2 r0 = x[2 * p], r1 = x[2 * p + 1];
      if (j > 0) {
        const double2 a = Fw[(herm ? 6 : 4) * ns + sl];
        r0 = csub(r0, cscale(-a.x, prev[2 * (j - 1)]));
        r1 = csub(r1, cscale(-a.y, prev[2 * (j - 1) + 1]));
      }
      if (i > 0) {
        const double2 a = Fw[(herm ? 7 : 5) * ns + sl];
        r0 = csub(r0, cscale(-a.x, prev[2 * j]));
        r1 = csub(r1, cscale(-a.y, prev[2 * j + 1]));
      }
      double2 w0, w1;
      mv2(dblock(sl), herm, r0, r1, w0, w1);
      cur[2 * j] = w0;
      cur[2 * j + 1] = w1;
      y[2 * p] = w0;
      y[2 * p + 1] = w1;
    }
    __syncthreads();
  }
  for (int d = nd - 1; d >= 0; d--) {
    double2* cur = ring + (d & 1) * 2 * ny;
    const double2* nxt = ring + ((d + 1) & 1) * 2 * ny;
    const int j0 = max(0, d - nx + 1), j1 = min(ny - 1, d);
    for (int j = j0 + threadIdx.x; j <= j1; j += blockDim.x) {
      const int i = d - j, p = j + ny * i;
      const int64_t sl = (int64_t)d * ny + j;
      double2 t0 = make_double2(0, 0), t1 = make_double2(0, 0);
      if (j < ny - 1) {
        const double2 a = Fw[(herm ? 10 : 8) * ns + sl];
        t0 = cadd(t0, cscale(-a.x, nxt[2 * (j + 1)]));
        t1 = cadd(t1, cscale(-a.y, nxt[2 * (j + 1) + 1]));
      }
      if (i < nx - 1) {
        const double2 a = Fw[(herm ? 11 : 9) * ns + sl];
        t0 = cadd(t0, cscale(-a.x, nxt[2 * j]));
        t1 = cadd(t1, cscale(-a.y, nxt[2 * j + 1]));
      }
      double2 u0, u1;
      mv2(dblock(sl), herm, t0, t1, u0, u1);
      const double2 y0 = csub(y[2 * p], u0), y1 = csub(y[2 * p + 1], u1);
      cur[2 * j] = y0;
      cur[2 * j + 1] = y1;
      y[2 * p] = y0;
      y[2 * p + 1] = y1;
    }
    __syncthreads();
  }
}

// The same sweeps with one thread per grid column j (ny <= kIluColMax):
// thread j walks its nodes (i, j), i = 0 .. nx-1 (backward: nx-1 .. 0), at
// anti-diagonal steps d = i + j.  Its own previous node, (i-1, j) (backward
// (i+1, j)), stays in registers; only the other neighbour, (i, j-1)
// (backward (i, j+1)), comes through LDS from the neighbouring thread's
// previous step.  A node's operands (x or the forward result, the two
// off-diagonal blocks, D^-1) do not depend on the sweep, so each thread loads
// its next node's while it computes the current one, into the other of two
// register sets (chosen by the parity of d, the same for every thread).  The
// loads are issued by every thread at every step (of a valid node, kept or
// not) and hold raw coefficients (signs applied at use): a load that is
// conditional, or whose value is transformed at once, makes the compiler
// wait for it, or for the loads around it, before the step's arithmetic.
// The arithmetic is the same, in the same order, as k_pc_ilu0_apply's.
constexpr int kIluColMax = 512;

struct IluOp {
  double2 v0, v1;      // x_p (forward) or w_p (backward)
  double a0, a1;       // minus the block to the (i, j -/+ 1) neighbour
  double b0, b1;       // minus the block to the (i -/+ 1, j) neighbour
  C2 D;
};

__global__ __launch_bounds__(kIluColMax) void k_pc_ilu0_apply_col(
    int nx, int ny, int k, int adjoint, const double* __restrict__ coef,
    const double2* __restrict__ Dinv, const double2* X, double2* Y, const uint32_t* active,
    const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  extern __shared__ __align__(16) char kc_smem[];
  double2* ring = reinterpret_cast<double2*>(kc_smem);  // [2][ny][2]
  const int c = blockIdx.x, w = blockIdx.y, nn = nx * ny;
  const int64_t q = (int64_t)w * k + c;
  if (active && !active[q]) return;
  const int64_t off = q * 2 * nn;
  const double2* x = X + off;
  double2* y = Y + off;
  const int64_t ns = ilu_slots(nx, ny);
  const double2* Fw = Dinv + (int64_t)w * kIluFields * ns;
  const bool herm = adjoint != 0;
  const int j = threadIdx.x;
  const bool col = j < ny;
  const int jc = col ? j : ny - 1;  // the column whose nodes this thread loads
  const int nd = nx + ny - 1;
  // raw loads of node (clamp(i), jc) (the blocks are minus the loaded
  // coefficients); D^-1 and the coefficients from the anti-diagonal layout
  auto node_load = [&](int i, IluOp& o, const double2* v, int fa, int fb) {
    i = min(max(i, 0), nx - 1);
    const int p = jc + ny * i;
    const int64_t sl = (int64_t)(i + jc) * ny + jc;
    o.v0 = v[2 * p];
    o.v1 = v[2 * p + 1];
    const double2 a = Fw[fa * ns + sl], b = Fw[fb * ns + sl];
    o.a0 = a.x;
    o.a1 = a.y;
    o.b0 = b.x;
    o.b1 = b.y;
#pragma unroll
    for (int e = 0; e < 4; e++) o.D.m[e] = Fw[e * ns + sl];
  };
  auto fwd_load = [&](int i, IluOp& o) { node_load(i, o, x, herm ? 6 : 4, herm ? 7 : 5); };
  auto bwd_load = [&](int i, IluOp& o) { node_load(i, o, y, herm ? 10 : 8, herm ? 11 : 9); };
  IluOp opA, opB;  // the register sets of even and odd steps
  double2 own0 = make_double2(0, 0), own1 = make_double2(0, 0);
  // forward: w_p = D_p^-1 (x_p - M_p,p-1 w_p-1 - M_p,p-ny w_p-ny)
  if (j & 1) fwd_load(0, opB);
  else fwd_load(0, opA);
  auto fwd_step = [&](int d, IluOp& use, IluOp& fill) {
    const int i = d - j;
    double2* cur = ring + (d & 1) * 2 * ny;
    const double2* prev = ring + ((d + 1) & 1) * 2 * ny;
    fwd_load(i + 1, fill);
    if (col && i >= 0 && i < nx) {
      double2 r0 = use.v0, r1 = use.v1;
      if (j > 0) {
        r0 = csub(r0, cscale(-use.a0, prev[2 * (j - 1)]));
        r1 = csub(r1, cscale(-use.a1, prev[2 * (j - 1) + 1]));
      }
      if (i > 0) {
        r0 = csub(r0, cscale(-use.b0, own0));
        r1 = csub(r1, cscale(-use.b1, own1));
      }
      double2 w0, w1;
      mv2(use.D, herm, r0, r1, w0, w1);
      cur[2 * j] = w0;
      cur[2 * j + 1] = w1;
      const int p = j + ny * i;
      y[2 * p] = w0;
      y[2 * p + 1] = w1;
      own0 = w0;
      own1 = w1;
    }
    __syncthreads();
  };
  int d = 0;
  for (; d + 1 < nd; d += 2) {
    fwd_step(d, opA, opB);
    fwd_step(d + 1, opB, opA);
  }
  if (d < nd) fwd_step(d, opA, opB);
  // backward: y_p = w_p - D_p^-1 (M_p,p+1 y_p+1 + M_p,p+ny y_p+ny); the
  // forward results of this thread's own column are its own stores
  if ((nx - 1 + j) & 1) bwd_load(nx - 1, opB);
  else bwd_load(nx - 1, opA);
  auto bwd_step = [&](int d, IluOp& use, IluOp& fill) {
    const int i = d - j;
    double2* cur = ring + (d & 1) * 2 * ny;
    const double2* nxt = ring + ((d + 1) & 1) * 2 * ny;
    bwd_load(i - 1, fill);
    if (col && i >= 0 && i < nx) {
      double2 t0 = make_double2(0, 0), t1 = make_double2(0, 0);
      if (j < ny - 1) {
        t0 = cadd(t0, cscale(-use.a0, nxt[2 * (j + 1)]));
        t1 = cadd(t1, cscale(-use.a1, nxt[2 * (j + 1) + 1]));
      }
      if (i < nx - 1) {
        t0 = cadd(t0, cscale(-use.b0, own0));
        t1 = cadd(t1, cscale(-use.b1, own1));
      }
      double2 u0, u1;
      mv2(use.D, herm, t0, t1, u0, u1);
      const double2 y0 = csub(use.v0, u0), y1 = csub(use.v1, u1);
      cur[2 * j] = y0;
      cur[2 * j + 1] = y1;
      const int p = j + ny * i;
      y[2 * p] = y0;
      y[2 * p + 1] = y1;
      own0 = y0;
      own1 = y1;
    }
    __syncthreads();
  };
  d = nd - 1;
  for (; d - 1 >= 0; d -= 2) {
    if (d & 1) {
      bwd_step(d, opB, opA);
      bwd_step(d - 1, opA, opB);
    } else {
      bwd_step(d, opA, opB);
      bwd_step(d - 1, opB, opA);
    }
  }
  if (d == 0) bwd_step(0, opA, opB);
}

// partial[(q * nchunk + chunk) * 2 + e] = sum over the chunk of conj(A_e) B_e
// for the npair (1 or 2) pairs, per system q = w * k + c.
__global__ __launch_bounds__(kKThreads) void k_kdot_partial(int64_t n, int k, int npair,
                                                           const double2* A0, const double2* B0,
                                                           const double2* A1, const double2* B1,
                                                           int nchunk, double2* partial,
                                                           const uint32_t* active,
                                                           const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ double2 red[2][kKThreads / 64];
  const int chunk = blockIdx.x, c = blockIdx.y, w = blockIdx.z;
  const int64_t q = (int64_t)w * k + c;
  if (active && !active[q]) return;
  const int64_t base = q * n, r0 = (int64_t)chunk * kKChunk, r1 = min(n, r0 + kKChunk);
  double2 s0 = make_double2(0, 0), s1 = make_double2(0, 0);
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kKThreads) {
    s0 = cadd(s0, cmulc(A0[base + r], B0[base + r]));
    if (npair > 1) s1 = cadd(s1, cmulc(A1[base + r], B1[base + r]));
  }
  for (int o = 32; o > 0; o >>= 1) {
    s0.x += __shfl_down(s0.x, o, 64);
    s0.y += __shfl_down(s0.y, o, 64);
    s1.x += __shfl_down(s1.x, o, 64);
    s1.y += __shfl_down(s1.y, o, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double2 t = make_double2(0, 0);
    for (int v = 0; v < kKThreads / 64; v++) t = cadd(t, red[threadIdx.x][v]);
    partial[(q * nchunk + chunk) * 2 + threadIdx.x] = t;
  }
}

__device__ __forceinline__ double2 dot_total(const double2* partial, int64_t q, int nchunk, int e) {
  double2 t = make_double2(0, 0);
  for (int ch = 0; ch < nchunk; ch++) t = cadd(t, partial[(q * nchunk + ch) * 2 + e]);
  return t;
}

// Per-system BiCGStab scalars: [0] rho, [1] alpha, [2] omega, [3] beta.
enum { KS_RHO = 0, KS_ALPHA = 1, KS_OMEGA = 2, KS_BETA = 3, KS_N = 4 };

// The scalar steps of one BiCGStab iteration, one thread per system, from
// the dot products just taken (mode):
//   0  start:  bnorm2 = ||b||^2 (a zero right-hand side is solved by x = 0)
//   1  rho:    rho = <rhat, r>, beta = (rho / rho_prev)(alpha / omega) (0 first)
//   2  alpha:  alpha = rho / <rhat, v>
//   3  omega:  omega = <t, s> / <t, t> (0 when t = 0)
//   4  check:  ||r||^2 <= tol^2 ||b||^2 ends the system; the last block of
//              the launch counts the systems left and marks the solve
//              converged when none are (later launches then skip).
// A zero denominator in a live system latches ST_BREAKDOWN and ends it.
__global__ __launch_bounds__(kKThreads) void k_bicg_scalars(int N, int nchunk, int mode, int it,
                                                           double tol2, const double2* partial,
                                                           double2* ks, double* bnorm2,
                                                           uint32_t* active, uint32_t* conv,
                                                           uint32_t* status,
                                                           const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ uint32_t live;
  if (threadIdx.x == 0) live = 0;
  __syncthreads();
  uint32_t mine = 0;
  for (int q = threadIdx.x; q < N; q += blockDim.x) {
    double2* s = ks + (int64_t)q * KS_N;
    if (mode == 0) {
      const double b2 = dot_total(partial, q, nchunk, 0).x;
      bnorm2[q] = b2;
      active[q] = b2 > 0.0 ? 1u : 0u;
      s[KS_RHO] = s[KS_ALPHA] = s[KS_OMEGA] = make_double2(1, 0);
      s[KS_BETA] = make_double2(0, 0);
      mine += active[q];
      continue;
    }
    if (!active[q]) continue;
    if (mode == 1) {
      const double2 rho = dot_total(partial, q, nchunk, 0);
      if (rho.x == 0.0 && rho.y == 0.0) {
        latch(status, ST_BREAKDOWN);
        active[q] = 0;
        continue;
      }
      s[KS_BETA] = it == 0 ? make_double2(0, 0)
                           : cmul(cdiv(rho, s[KS_RHO]), cdiv(s[KS_ALPHA], s[KS_OMEGA]));
      s[KS_RHO] = rho;
    } else if (mode == 2) {
      const double2 d = dot_total(partial, q, nchunk, 0);
      if (d.x == 0.0 && d.y == 0.0) {
        latch(status, ST_BREAKDOWN);
        active[q] = 0;
        continue;
      }
      s[KS_ALPHA] = cdiv(s[KS_RHO], d);
    } else if (mode == 3) {
      const double2 ts = dot_total(partial, q, nchunk, 0);
      const double tt = dot_total(partial, q, nchunk, 1).x;
      s[KS_OMEGA] = tt > 0.0 ? cscale(1.0 / tt, ts) : make_double2(0, 0);
    } else {
      const double r2 = dot_total(partial, q, nchunk, 0).x;
      if (!isfinite(r2)) {
        latch(status, ST_NONFINITE);
        active[q] = 0;
        continue;
      }
      if (r2 <= tol2 * bnorm2[q]) active[q] = 0;
      else mine++;
    }
  }
  if (mode == 0 || mode == 4) {
    atomicAdd(&live, mine);
    __syncthreads();
    if (threadIdx.x == 0 && live == 0) *conv = 1u;
  }
}

// p = r + beta (p - omega v)
__global__ void k_bicg_p(int64_t n, int k, const double2* ks, const double2* r, const double2* v,
                         double2* p, const uint32_t* active, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t q = (int64_t)blockIdx.z * k + blockIdx.y;
  if (e >= n || !active[q]) return;
  const double2* s = ks + q * KS_N;
  const int64_t o = q * n + e;
  p[o] = cadd(r[o], cmul(s[KS_BETA], csub(p[o], cmul(s[KS_OMEGA], v[o]))));
}

// r <- s = r - alpha v
__global__ void k_bicg_s(int64_t n, int k, const double2* ks, const double2* v, double2* r,
                         const uint32_t* active, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t q = (int64_t)blockIdx.z * k + blockIdx.y;
  if (e >= n || !active[q]) return;
  const int64_t o = q * n + e;
  r[o] = csub(r[o], cmul(ks[q * KS_N + KS_ALPHA], v[o]));
}

// x += alpha y + omega z,  r <- s - omega t
__global__ void k_bicg_xr(int64_t n, int k, const double2* ks, const double2* y,
                          const double2* z, const double2* t, double2* x, double2* r,
                          const uint32_t* active, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t q = (int64_t)blockIdx.z * k + blockIdx.y;
  if (e >= n || !active[q]) return;
  const double2* s = ks + q * KS_N;
  const int64_t o = q * n + e;
  x[o] = cadd(x[o], cadd(cmul(s[KS_ALPHA], y[o]), cmul(s[KS_OMEGA], z[o])));
  r[o] = csub(r[o], cmul(s[KS_OMEGA], t[o]));
}

// x += d for live systems
__global__ void k_kaxpy(int64_t n, int k, const double2* d, double2* x, const uint32_t* active,
                        const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t q = (int64_t)blockIdx.z * k + blockIdx.y;
  if (e >= n || !active[q]) return;
  x[q * n + e] = cadd(x[q * n + e], d[q * n + e]);
}

__global__ void k_kcopy(int64_t n, const double2* a, double2* b) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) b[e] = a[e];
}

__global__ void k_latch_live(int N, const uint32_t* active, uint32_t* status, uint32_t bit) {
  for (int q = threadIdx.x; q < N; q += blockDim.x)
    if (active[q]) {
      latch(status, bit);
      break;
    }
}

}  // namespace

int krylov_nchunk(int64_t n) { return (int)((n + kKChunk - 1) / kKChunk); }

size_t ilu0_lds(int ny) { return (size_t)2 * ny * sizeof(C2); }
// Bytes of a Krylov handle's preconditioner data (all shifts).
size_t pc_bytes(int precond, int nx, int ny, int n_omega) {
  if (precond == RR_PRECOND_ILU0)
    return (size_t)n_omega * kIluFields * ilu_slots(nx, ny) * sizeof(double2);
  return (size_t)n_omega * nx * ny * 4 * sizeof(double2);
}
size_t ilu0_apply_lds(int ny) { return (size_t)2 * ny * 2 * sizeof(double2); }

hipError_t prepare_krylov(int ny) {
  hipError_t e = hipFuncSetAttribute((const void*)k_pc_ilu0,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)ilu0_lds(ny));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_pc_ilu0_apply,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)ilu0_apply_lds(ny));
  if (e == hipSuccess && ny <= kIluColMax)
    e = hipFuncSetAttribute((const void*)k_pc_ilu0_apply_col,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)ilu0_apply_lds(ny));
  return e;
}

hipError_t launch_pc_setup(const OpDesc& op, int precond, const double* omega, int n_omega,
                           double* Dinv, uint32_t* status, hipStream_t s) {
  const int nn = op.nx * op.ny;
  if (precond == RR_PRECOND_ILU0)
    hipLaunchKernelGGL(k_pc_ilu0, dim3(n_omega), dim3(kKThreads), ilu0_lds(op.ny), s, op.nx,
                       op.ny, op.coef, omega, (double2*)Dinv, status);
  else
    hipLaunchKernelGGL(k_pc_jacobi, dim3((nn + 255) / 256, n_omega), dim3(256), 0, s, nn,
                       op.coef, omega, (double2*)Dinv, status);
  return hipGetLastError();
}

hipError_t launch_pc_apply(const OpDesc& op, int precond, int n_omega, int k, int adjoint,
                           const double* Dinv, const double* X, double* Y,
                           const uint32_t* active, const uint32_t* skip, hipStream_t s) {
  const int nn = op.nx * op.ny;
  if (precond == RR_PRECOND_ILU0 && op.ny <= kIluColMax)
    hipLaunchKernelGGL(k_pc_ilu0_apply_col, dim3(k, n_omega), dim3((op.ny + 63) / 64 * 64),
                       ilu0_apply_lds(op.ny), s, op.nx, op.ny, k, adjoint, op.coef,
                       (const double2*)Dinv, (const double2*)X, (double2*)Y, active, skip);
  else if (precond == RR_PRECOND_ILU0)
    hipLaunchKernelGGL(k_pc_ilu0_apply, dim3(k, n_omega), dim3(kKThreads), ilu0_apply_lds(op.ny),
                       s, op.nx, op.ny, k, adjoint, op.coef, (const double2*)Dinv,
                       (const double2*)X, (double2*)Y, active, skip);
  else
    hipLaunchKernelGGL(k_pc_jacobi_apply, dim3((nn + 255) / 256, k, n_omega), dim3(256), 0, s, nn,
                       k, adjoint, (const double2*)Dinv, (const double2*)X, (double2*)Y, active,
                       skip);
  return hipGetLastError();
}

hipError_t launch_kdot(int64_t n, int n_omega, int k, int npair, const double* A0,
                       const double* B0, const double* A1, const double* B1, double* partial,
                       const uint32_t* active, const uint32_t* skip, hipStream_t s) {
  const int nc = krylov_nchunk(n);
  hipLaunchKernelGGL(k_kdot_partial, dim3(nc, k, n_omega), dim3(kKThreads), 0, s, n, k, npair,
                     (const double2*)A0, (const double2*)B0, (const double2*)A1,
                     (const double2*)B1, nc, (double2*)partial, active, skip);
  return hipGetLastError();
}

hipError_t launch_bicg_scalars(int N, int64_t n, int mode, int it, double tol, const double* partial,
                               double* ks, double* bnorm2, uint32_t* active, uint32_t* conv,
                               uint32_t* status, const uint32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_scalars, dim3(1), dim3(kKThreads), 0, s, N, krylov_nchunk(n), mode,
                     it, tol * tol, (const double2*)partial, (double2*)ks, bnorm2, active, conv,
                     status, skip);
  return hipGetLastError();
}

hipError_t launch_bicg_vec(int which, int64_t n, int n_omega, int k, const double* ks,
                           const double* a, const double* b, const double* c, double* x,
                           double* y, const uint32_t* active, const uint32_t* skip,
                           hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), k, n_omega);
  if (which == 0)  // p = r + beta (p - omega v): a = r, b = v, y = p
    hipLaunchKernelGGL(k_bicg_p, grid, dim3(256), 0, s, n, k, (const double2*)ks,
                       (const double2*)a, (const double2*)b, (double2*)y, active, skip);
  else if (which == 1)  // r -= alpha v: b = v, y = r
    hipLaunchKernelGGL(k_bicg_s, grid, dim3(256), 0, s, n, k, (const double2*)ks,
                       (const double2*)b, (double2*)y, active, skip);
  else if (which == 2)  // x += alpha a + omega b, y(r) -= omega c
    hipLaunchKernelGGL(k_bicg_xr, grid, dim3(256), 0, s, n, k, (const double2*)ks,
                       (const double2*)a, (const double2*)b, (const double2*)c, (double2*)x,
                       (double2*)y, active, skip);
  else  // x += a
    hipLaunchKernelGGL(k_kaxpy, grid, dim3(256), 0, s, n, k, (const double2*)a, (double2*)x,
                       active, skip);
  return hipGetLastError();
}

hipError_t launch_kcopy(int64_t count, const double* a, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_kcopy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                     (const double2*)a, (double2*)b);
  return hipGetLastError();
}

hipError_t launch_latch_live(int N, const uint32_t* active, uint32_t* status, uint32_t bit,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_latch_live, dim3(1), dim3(256), 0, s, N, active, status, bit);
  return hipGetLastError();
}

}  // namespace rr
