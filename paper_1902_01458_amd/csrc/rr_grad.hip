// Gradient of the leading gain as a stencil reduction (FP64).
//
// For a simple sigma with H v = sigma u and u^H H = sigma v^H, perturbing
// M = i omega I - L gives d sigma = -sigma^2 Re(v^H dM u), so
//   d sigma / dp     = sigma^2 Re(v^H (dL/dp) u)      p = U at a node, nu
//   d sigma / domega = sigma^2 Im(v^H u)
// L depends on the interior nodal U through the convection coefficient at the
// node itself and through the central differences U_x, U_y at its four
// neighbours; a value on the boundary ring enters only through the central
// difference of its one interior neighbour (U_x for the west / east ring,
// U_y for the south / north ring; the corners through none); dL/dnu is the
// Dirichlet Laplacian on both components.  dU covers the whole
// (nx+2) x (ny+2) base-flow array, ring included, in U's own layout.
#include "rr_internal.h"

namespace rr {

constexpr int kGradBlock = 256;

__device__ __forceinline__ double re_cmulc(double2 a, double2 b) {  // Re(conj(a) b)
  return a.x * b.x + a.y * b.y;
}
__device__ __forceinline__ double im_cmulc(double2 a, double2 b) {  // Im(conj(a) b)
  return a.x * b.y - a.y * b.x;
}

// One thread per node q = J + (ny+2)*I of the (nx+2) x (ny+2) array (ring
// included); interior nodes are p = (J-1) + ny*(I-1).  u, v of shift w at
// stride.
__global__ __launch_bounds__(kGradBlock) void k_grad(int nx, int ny, double hx, double hy,
                                                     const double* __restrict__ sigma1,
                                                     const double2* __restrict__ u1,
                                                     const double2* __restrict__ v1,
                                                     int64_t stride, double* __restrict__ dU,
                                                     double* __restrict__ partial, int nchunk) {
  __shared__ double red[2][kGradBlock];
  const int w = blockIdx.y;
  const int NY = ny + 2;
  const int nfull = (nx + 2) * NY;
  const int q = blockIdx.x * kGradBlock + threadIdx.x;
  const double2* u = u1 + (int64_t)w * stride;
  const double2* v = v1 + (int64_t)w * stride;
  double s2 = sigma1[w] * sigma1[w];
  double lap_part = 0.0, vu_part = 0.0;
  const double ihx = 1.0 / (2.0 * hx), ihy = 1.0 / (2.0 * hy);
  const int I = q / NY, J = q % NY;
  const bool ring = q < nfull && (I == 0 || I == nx + 1 || J == 0 || J == ny + 1);
  if (ring) {
    // the one interior neighbour whose U_x (west / east) or U_y (south /
    // north) reads this node; corners have none
    double g = 0.0;
    const bool cornerless = (I == 0 || I == nx + 1) != (J == 0 || J == ny + 1);
    if (cornerless) {
      if (I == 0 || I == nx + 1) {  // U_x(nb) = (U(E) - U(W)) / 2hx; C carries -U_x
        const int p = (J - 1) + ny * (I == 0 ? 0 : nx - 1);
        const double sgn = I == 0 ? 1.0 : -1.0;
        g = sgn * re_cmulc(v[2 * p], u[2 * p]) * ihx;
      } else {                      // U_y(nb) = (U(N) - U(S)) / 2hy; Cpl = -U_y
        const int p = (J == 0 ? 0 : ny - 1) + ny * (I - 1);
        const double sgn = J == 0 ? 1.0 : -1.0;
        g = sgn * re_cmulc(v[2 * p], u[2 * p + 1]) * ihy;
      }
    }
    dU[(int64_t)w * nfull + q] = s2 * g;
  } else if (q < nfull) {
    const int i = I - 1, j = J - 1, p = j + ny * i;
    bool hE = i < nx - 1, hW = i > 0, hN = j < ny - 1, hS = j > 0;
    int pE = p + ny, pW = p - ny, pN = p + 1, pS = p - 1;
    const double2 z = make_double2(0, 0);
    double2 uu = u[2 * p], uv = u[2 * p + 1], vu = v[2 * p], vv = v[2 * p + 1];
    double2 uuE = hE ? u[2 * pE] : z, uuW = hW ? u[2 * pW] : z;
    double2 uvE = hE ? u[2 * pE + 1] : z, uvW = hW ? u[2 * pW + 1] : z;
    double2 uvN = hN ? u[2 * pN + 1] : z, uvS = hS ? u[2 * pS + 1] : z;
    double2 vuE = hE ? v[2 * pE] : z, vuW = hW ? v[2 * pW] : z;
    double2 vuN = hN ? v[2 * pN] : z, vuS = hS ? v[2 * pS] : z;
    // -U_p d/dx on both components at p
    double g = -re_cmulc(vu, make_double2((uuE.x - uuW.x) * ihx, (uuE.y - uuW.y) * ihx))
               - re_cmulc(vv, make_double2((uvE.x - uvW.x) * ihx, (uvE.y - uvW.y) * ihx));
    // -U_x u at W and E (U_x(W) = (U_p - ...)/2hx, U_x(E) = (... - U_p)/2hx)
    g += -re_cmulc(vuW, uuW) * ihx + re_cmulc(vuE, uuE) * ihx;
    // -U_y v at S and N
    g += -re_cmulc(vuS, uvS) * ihy + re_cmulc(vuN, uvN) * ihy;
    dU[(int64_t)w * nfull + q] = s2 * g;
    // Re(v^H Lap u) and Im(v^H u) contributions of rows 2p, 2p+1
    double2 uuN = hN ? u[2 * pN] : z, uuS = hS ? u[2 * pS] : z;
    double ax = 1.0 / (hx * hx), ay = 1.0 / (hy * hy);
    double2 lu = make_double2(ax * (uuE.x + uuW.x - 2 * uu.x) + ay * (uuN.x + uuS.x - 2 * uu.x),
                              ax * (uuE.y + uuW.y - 2 * uu.y) + ay * (uuN.y + uuS.y - 2 * uu.y));
    double2 lv = make_double2(ax * (uvE.x + uvW.x - 2 * uv.x) + ay * (uvN.x + uvS.x - 2 * uv.x),
                              ax * (uvE.y + uvW.y - 2 * uv.y) + ay * (uvN.y + uvS.y - 2 * uv.y));
    lap_part = re_cmulc(vu, lu) + re_cmulc(vv, lv);
    vu_part = im_cmulc(vu, uu) + im_cmulc(vv, uv);
  }
  red[0][threadIdx.x] = lap_part;
  red[1][threadIdx.x] = vu_part;
  __syncthreads();
  for (int o = kGradBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[((int64_t)w * nchunk + blockIdx.x) * 2 + 0] = red[0][0];
    partial[((int64_t)w * nchunk + blockIdx.x) * 2 + 1] = red[1][0];
  }
}

__global__ void k_grad_final(int nchunk, const double* __restrict__ sigma1,
                             const double* __restrict__ partial, double* dnu, double* domega) {
  const int w = blockIdx.x;
  if (threadIdx.x != 0) return;
  double a = 0, b = 0;
  for (int c = 0; c < nchunk; c++) {
    a += partial[((int64_t)w * nchunk + c) * 2 + 0];
    b += partial[((int64_t)w * nchunk + c) * 2 + 1];
  }
  double s2 = sigma1[w] * sigma1[w];
  dnu[w] = s2 * a;
  domega[w] = s2 * b;
}

hipError_t launch_grad(int nx, int ny, double hx, double hy, int n_omega, const double* omega,
                       const double* sigma1, const double* u1, const double* v1, int64_t stride,
                       double* dU, double* dnu, double* domega, double* partial, int nchunk,
                       hipStream_t s) {
  (void)omega;
  int nfull = (nx + 2) * (ny + 2);
  int nc = (nfull + kGradBlock - 1) / kGradBlock;
  if (nc > nchunk) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_grad, dim3(nc, n_omega), dim3(kGradBlock), 0, s, nx, ny, hx, hy, sigma1,
                     (const double2*)u1, (const double2*)v1, stride, dU, partial, nc);
  hipLaunchKernelGGL(k_grad_final, dim3(n_omega), dim3(64), 0, s, nc, sigma1, partial, dnu, domega);
  return hipGetLastError();
}

}  // namespace rr
