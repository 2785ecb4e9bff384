// Operator-side kernels: Burgers stencil coefficients, matrix-free M X in
// FP64 (residuals of the mixed-precision refinement), and the physics-weighted
// complex Gaussian sketch (Algorithm 1 step 1 with eq. 10 weighting).
#include "rr_internal.h"

namespace rr {

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

// Linearised viscous Burgers about (U(x,y), V = 0), central differences:
//   u-row: nu Lap u - U u_x - U_x u - U_y v,    v-row: nu Lap v - U v_x
__global__ void k_burgers_coeffs(int nx, int ny, const double* __restrict__ U, double hx,
                                 double hy, double nu, double* __restrict__ coef,
                                 double* __restrict__ phi) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nx * ny) return;
  int i = p / ny + 1, j = p % ny + 1;  // 1-based node in the (nx+2) x (ny+2) array
  int ld = ny + 2;
  double Uc = U[i * ld + j];
  double Ux = (U[(i + 1) * ld + j] - U[(i - 1) * ld + j]) / (2.0 * hx);
  double Uy = (U[i * ld + j + 1] - U[i * ld + j - 1]) / (2.0 * hy);
  double ax = nu / (hx * hx), ay = nu / (hy * hy);
  double* c = coef + 12 * (int64_t)p;
  c[0] = -2.0 * (ax + ay) - Ux;
  c[1] = ax - Uc / (2.0 * hx);
  c[2] = ax + Uc / (2.0 * hx);
  c[3] = ay;
  c[4] = ay;
  c[5] = -Uy;
  c[6] = -2.0 * (ax + ay);
  c[7] = ax - Uc / (2.0 * hx);
  c[8] = ax + Uc / (2.0 * hx);
  c[9] = ay;
  c[10] = ay;
  c[11] = 0.0;
  if (phi) phi[p] = sqrt(Ux * Ux + Uy * Uy) + 0.1;
}

hipError_t launch_burgers_coeffs(int nx, int ny, const double* U, double hx, double hy,
                                 double nu, double* coef, double* phi, hipStream_t s) {
  int nn = nx * ny;
  hipLaunchKernelGGL(k_burgers_coeffs, dim3((nn + 255) / 256), dim3(256), 0, s, nx, ny, U, hx,
                     hy, nu, coef, phi);
  return hipGetLastError();
}

// Y = Bm - M X  (or Y = M X when Bm == NULL), M = i omega I - L, for all k
// columns of shift w (blockIdx.y); one thread per node (both components),
// which reads the node's stencil once and applies it to every column.
// Adjoint: M^H = conj(i omega) I - L^T, whose stencil reads the transposed
// coefficients from the neighbouring nodes.
__global__ void k_apply(int nx, int ny, const double* __restrict__ coef,
                        const double* __restrict__ omega, int k, int adjoint,
                        const double2* __restrict__ X, const double2* __restrict__ Bm,
                        int64_t bstride, double2* __restrict__ Y, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int nn = nx * ny;
  if (p >= nn) return;
  const int w = blockIdx.y;
  const int64_t n = 2 * (int64_t)nn;
  const int i = p / ny, jj = p % ny;
  const bool hE = i < nx - 1, hW = i > 0, hN = jj < ny - 1, hS = jj > 0;
  const int pE = p + ny, pW = p - ny, pN = p + 1, pS = p - 1;
  const double* c = coef + 12 * (int64_t)p;
  // (L x) or (L^T x) at rows 2p, 2p+1:
  //   u: au * x_u(p) + auv * x_v(p) + sum over neighbours q of eu[q] * x_u(q)
  //   v: av * x_v(p) + avu * x_u(p) + sum over neighbours q of ev[q] * x_v(q)
  // neighbours in the order E, W, N, S (forward) or W, E, S, N (adjoint)
  double au, auv, av, avu, eu[4], ev[4];
  int nb[4];
  bool has[4];
  if (!adjoint) {
    au = c[0]; auv = c[5]; av = c[6]; avu = c[11];
    nb[0] = pE; has[0] = hE; eu[0] = c[1]; ev[0] = c[7];
    nb[1] = pW; has[1] = hW; eu[1] = c[2]; ev[1] = c[8];
    nb[2] = pN; has[2] = hN; eu[2] = c[3]; ev[2] = c[9];
    nb[3] = pS; has[3] = hS; eu[3] = c[4]; ev[3] = c[10];
  } else {
    // (L^T x)_{2p} = uC_p xu_p + vCpl_p xv_p + uE_W xu_W + uW_E xu_E + uN_S xu_S + uS_N xu_N
    au = c[0]; auv = c[11]; av = c[6]; avu = c[5];
    const int qs[4] = {pW, pE, pS, pN};
    const bool hs[4] = {hW, hE, hS, hN};
    const int cu[4] = {1, 2, 3, 4};
#pragma unroll
    for (int d = 0; d < 4; d++) {
      nb[d] = qs[d];
      has[d] = hs[d];
      const double* cq = coef + 12 * (int64_t)(hs[d] ? qs[d] : p);
      eu[d] = cq[cu[d]];
      ev[d] = cq[cu[d] + 6];
    }
  }
  // shift: M = (i omega) I - L; i omega = -om_i + i om_r; M^H shift = conj of it
  const double sr = -omega[2 * w + 1], si = adjoint ? -omega[2 * w] : omega[2 * w];
  for (int j = 0; j < k; j++) {
    const int64_t off = ((int64_t)w * k + j) * n;
    const double2* x = X + off;
    const double2 xu = x[2 * p], xv = x[2 * p + 1];
    double lu_r = au * xu.x + auv * xv.x;
    double lu_i = au * xu.y + auv * xv.y;
    double lv_r = av * xv.x + avu * xu.x;
    double lv_i = av * xv.y + avu * xu.y;
#pragma unroll
    for (int d = 0; d < 4; d++) {
      if (!has[d]) continue;
      const double2 a = x[2 * nb[d]], b = x[2 * nb[d] + 1];
      lu_r += eu[d] * a.x;
      lu_i += eu[d] * a.y;
      lv_r += ev[d] * b.x;
      lv_i += ev[d] * b.y;
    }
    double2 mu, mv;
    mu.x = sr * xu.x - si * xu.y - lu_r;
    mu.y = sr * xu.y + si * xu.x - lu_i;
    mv.x = sr * xv.x - si * xv.y - lv_r;
    mv.y = sr * xv.y + si * xv.x - lv_i;
    if (Bm) {
      const double2* bb = Bm + (int64_t)w * bstride + (int64_t)j * n;
      const double2 bu = bb[2 * p], bv = bb[2 * p + 1];
      mu.x = bu.x - mu.x;
      mu.y = bu.y - mu.y;
      mv.x = bv.x - mv.x;
      mv.y = bv.y - mv.y;
    }
    double2* y = Y + off;
    y[2 * p] = mu;
    y[2 * p + 1] = mv;
  }
}

hipError_t launch_apply(const OpDesc& op, const double* omega, int n_omega, int k, int adjoint,
                        const double* X, const double* Bm, int64_t bstride, double* Y,
                        hipStream_t s, const uint32_t* skip) {
  int nn = op.nx * op.ny;
  dim3 grid((nn + 255) / 256, n_omega);
  hipLaunchKernelGGL(k_apply, grid, dim3(256), 0, s, op.nx, op.ny, op.coef, omega, k, adjoint,
                     (const double2*)X, (const double2*)Bm, bstride, (double2*)Y, skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 products
// on counter words 0 and 2, with the key bumped by the Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; r++) {
    if (r) { k0 += W0; k1 += W1; }
    uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__global__ void k_philox_raw(uint32_t* out, int64_t count, uint32_t c1, uint32_t c2,
                             uint32_t k0, uint32_t k1) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t c[4] = {(uint32_t)i, c1, c2, 0u};
  philox4x32_10(c, k0, k1);
  out[4 * i + 0] = c[0]; out[4 * i + 1] = c[1]; out[4 * i + 2] = c[2]; out[4 * i + 3] = c[3];
}

// Test matrix entry (r, j), weighted by phi[r/2] when phi is given:
//   Gaussian (and the orthonormal kind before its QR): sqrt(-ln u1) exp(2 pi i u2),
//     u1 = (m1+1) 2^-53, u2 = m2 2^-53 from the top 53 bits of (x0:x1) and
//     (x2:x3) at counter (r, j, 0, 0);
//   Rademacher: +-1, the sign being the top bit of x0 at that counter;
//   sparse sign: that +-1 if column j is among the zeta columns of row r with
//     the smallest keys (x0 at counter (r, j', 1, 0)), ties to the lower
//     column, else 0.
__global__ void k_sketch(int64_t n, int k, const double* __restrict__ phi, uint32_t k0,
                         uint32_t k1, int kind, int zeta, double2* __restrict__ theta) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (r >= n) return;
  uint32_t c[4] = {(uint32_t)r, (uint32_t)j, 0u, 0u};
  philox4x32_10(c, k0, k1);
  double2 v;
  if (kind == RR_TM_RADEMACHER || kind == RR_TM_SPARSE) {
    bool keep = true;
    if (kind == RR_TM_SPARSE) {
      uint32_t kc[4] = {(uint32_t)r, (uint32_t)j, 1u, 0u};
      philox4x32_10(kc, k0, k1);
      const uint32_t key = kc[0];
      int rank = 0;
      for (int jj = 0; jj < k; jj++) {
        if (jj == j) continue;
        uint32_t oc[4] = {(uint32_t)r, (uint32_t)jj, 1u, 0u};
        philox4x32_10(oc, k0, k1);
        rank += (oc[0] < key) || (oc[0] == key && jj < j);
      }
      keep = rank < zeta;
    }
    v = make_double2(keep ? ((c[0] >> 31) ? -1.0 : 1.0) : 0.0, 0.0);
  } else {
    uint64_t m1 = ((((uint64_t)c[0]) << 32) | c[1]) >> 11;
    uint64_t m2 = ((((uint64_t)c[2]) << 32) | c[3]) >> 11;
    const double two_m53 = 1.1102230246251565404e-16;
    double u1 = ((double)m1 + 1.0) * two_m53;
    double u2 = (double)m2 * two_m53;
    double rad = sqrt(-log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    v = make_double2(rad * cs, rad * sn);
  }
  double w = (phi && kind != RR_TM_ORTHONORMAL) ? phi[r >> 1] : 1.0;
  theta[(int64_t)j * n + r] = make_double2(w * v.x, w * v.y);
}

hipError_t launch_sketch(const OpDesc& op, const double* phi, int k, uint64_t seed, int kind,
                         int zeta, double* Theta, hipStream_t s) {
  int64_t n = op.n;
  dim3 grid((unsigned)((n + 255) / 256), k);
  hipLaunchKernelGGL(k_sketch, grid, dim3(256), 0, s, n, k, phi, (uint32_t)(seed & 0xffffffffu),
                     (uint32_t)(seed >> 32), kind, zeta, (double2*)Theta);
  return hipGetLastError();
}

__global__ void k_weight_rows(int64_t n, const double* __restrict__ phi, double2* theta) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double w = phi[r >> 1];
  double2* t = theta + (int64_t)blockIdx.y * n + r;
  double2 v = *t;
  *t = make_double2(w * v.x, w * v.y);
}

hipError_t launch_weight_rows(int64_t n, int k, const double* phi, double* Theta, hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), k);
  hipLaunchKernelGGL(k_weight_rows, grid, dim3(256), 0, s, n, phi, (double2*)Theta);
  return hipGetLastError();
}

}  // namespace rr

// Raw generator output for the known-answer test of the device generator:
// out[4*i .. 4*i+3] = Philox4x32-10 of counter (i, c1, c2, 0) under (k0, k1).
extern "C" rr_status rr_philox_raw(uint32_t* out_dev, int64_t count, uint32_t c1, uint32_t c2,
                                   uint32_t k0, uint32_t k1, void* stream) {
  if (!out_dev || count < 0) return RR_ERR_INVALID;
  if (count == 0) return RR_OK;
  hipLaunchKernelGGL(rr::k_philox_raw, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, out_dev, count, c1, c2, k0, k1);
  return hipGetLastError() == hipSuccess ? RR_OK : RR_ERR_HIP;
}

// Unweighted/weighted sketch written to a caller buffer (tests): Theta (k, n).
extern "C" rr_status rr_sketch(const rr_problem* p, int32_t k, uint64_t seed, rr_test_matrix kind,
                               int32_t zeta, double* theta, void* stream) {
  if (!p || !theta || k < 1 || p->nx < 1 || p->ny < 1) return RR_ERR_INVALID;
  if (kind != RR_TM_GAUSSIAN && kind != RR_TM_RADEMACHER && kind != RR_TM_SPARSE)
    return RR_ERR_INVALID;
  const int z = zeta <= 0 ? (k < 8 ? k : 8) : (zeta < k ? zeta : k);
  rr::OpDesc op{p->nx, p->ny, 2 * p->nx * p->ny, p->coef};
  return rr::launch_sketch(op, p->phi, k, seed, kind, z, theta, (hipStream_t)stream) ==
                 hipSuccess
             ? RR_OK
             : RR_ERR_HIP;
}
