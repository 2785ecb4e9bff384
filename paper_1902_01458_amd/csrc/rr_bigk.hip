// Wide sketches: the k x k steps of Algorithm 1 for 32 < k <= 512.
//
// The paper studies the accuracy against the sketch width k from 2 to 500
// (Section 3.2, Fig. 7).  Past k = 32 the LDS-resident kernels of
// rr_small.hip no longer hold a k x k matrix, so these keep the small
// matrices in global memory (L2-resident at this size) and tile the tall
// products through LDS:
//   * Gram G = Y^H Y in 32 x 32 tiles per row chunk, then summed over chunks;
//   * Cholesky G = R^H R and R^-1, one workgroup per shift;
//   * k x k products (composing the two CholQR passes, R^-1 W) in 32 x 32 tiles;
//   * tall products Y S (n x k by k x k) in 64 x 32 output tiles;
//   * the one-sided Jacobi SVD of R^H, one workgroup per shift, one wave per
//     column pair of the round-robin order;
//   * column norms for eq. (9)'s sigma_j = ||M^-1 v_j||.
// Same steps and outputs as the narrow path (CholQR2, then the SVD of the
// k x k factor), with one difference: a Gram matrix that is not numerically
// positive definite latches ST_BREAKDOWN here (the narrow path falls back to
// shifted CholeskyQR3).
#include <algorithm>

#include "rr_internal.h"

namespace rr {

namespace {

constexpr int kBT = 32;          // tile edge of the k x k blocks
constexpr int kBigChunks = 16;   // row chunks of the tiled Gram matrix

__device__ __forceinline__ double2 bmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 bmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// part[w][chunk][i][j] = sum over the chunk's rows of conj(Y_i) Y_j for the
// 32 x 32 tile (I, J), J >= I, of every shift; Y is (n_omega, k, n).
__global__ __launch_bounds__(256) void k_gramb_partial(int64_t n, int k, const double2* Y,
                                                       int64_t rows, int nchunk, double2* part) {
  __shared__ double2 a[kBT][kBT + 1], b[kBT][kBT + 1];  // [row][col]
  const int nt = (k + kBT - 1) / kBT;
  const int I = blockIdx.x / nt, J = blockIdx.x % nt, chunk = blockIdx.y, w = blockIdx.z;
  if (J < I) return;
  const int64_t r0 = chunk * rows, r1 = min(n, r0 + rows);
  const double2* Yw = Y + (int64_t)w * k * n;
  const int t = threadIdx.x, oi = t >> 3, oj = (t & 7) * 4;  // outputs (oi, oj .. oj+3)
  double2 acc[4] = {};
  for (int64_t rb = r0; rb < r1; rb += kBT) {
    for (int e = t; e < kBT * kBT; e += 256) {
      const int c = e / kBT, rr = e % kBT;  // consecutive threads: consecutive rows
      const int64_t row = rb + rr;
      const int ca = kBT * I + c, cb = kBT * J + c;
      a[rr][c] = (row < r1 && ca < k) ? Yw[(int64_t)ca * n + row] : make_double2(0, 0);
      b[rr][c] = (row < r1 && cb < k) ? Yw[(int64_t)cb * n + row] : make_double2(0, 0);
    }
    __syncthreads();
    for (int rr = 0; rr < kBT; rr++) {
      const double2 x = a[rr][oi];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const double2 p = bmulc(x, b[rr][oj + q]);
        acc[q].x += p.x;
        acc[q].y += p.y;
      }
    }
    __syncthreads();
  }
  double2* out = part + ((int64_t)w * nchunk + chunk) * k * k;
  const int gi = kBT * I + oi;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int gj = kBT * J + oj + q;
    if (gi < k && gj < k) out[(int64_t)gi * k + gj] = acc[q];
  }
}

// G[w] (k x k, row-major, leading dimension k) = sum over chunks, the lower
// triangle mirrored from the upper one (G is Hermitian).
__global__ void k_gramb_reduce(int k, int nchunk, const double2* part, int64_t sG, double2* G) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int w = blockIdx.y;
  if (idx >= (int64_t)k * k) return;
  const int i = (int)(idx / k), j = (int)(idx % k);
  const bool up = j >= i;
  const int64_t src = up ? (int64_t)i * k + j : (int64_t)j * k + i;
  double2 s = make_double2(0, 0);
  for (int c = 0; c < nchunk; c++) {
    const double2 p = part[((int64_t)w * nchunk + c) * k * k + src];
    s.x += p.x;
    s.y += p.y;
  }
  G[w * sG + idx] = up ? s : make_double2(s.x, -s.y);
}

// G = R^H R (R upper, real positive diagonal) and R^-1, one workgroup per
// shift, in global memory: the right-looking Cholesky by rows, then each
// thread back-substitutes columns of R^-1.  A pivot that is not positive
// latches ST_BREAKDOWN and is taken as 1 (the results stay finite).
__global__ __launch_bounds__(1024) void k_cholb(int k, int64_t sM, const double2* G, double2* R,
                                                double2* Rinv, uint32_t* status) {
  __shared__ double piv;
  const int w = blockIdx.x;
  const double2* Gw = G + w * sM;
  double2* Rw = R + w * sM;
  double2* Xw = Rinv + w * sM;
  for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    Rw[e] = j >= i ? Gw[e] : make_double2(0, 0);
  }
  __syncthreads();
  for (int j = 0; j < k; j++) {
    if (threadIdx.x == 0) {
      double d = Rw[(int64_t)j * k + j].x;
      if (!(d > 0.0) || !isfinite(d)) {
        latch(status, ST_BREAKDOWN);
        d = 1.0;
      }
      piv = sqrt(d);
      Rw[(int64_t)j * k + j] = make_double2(piv, 0.0);
    }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int c = j + 1 + threadIdx.x; c < k; c += blockDim.x) {
      const double2 v = Rw[(int64_t)j * k + c];
      Rw[(int64_t)j * k + c] = make_double2(v.x * inv, v.y * inv);
    }
    __syncthreads();
    // trailing rows r > j: R[r][c] -= conj(R[j][r]) R[j][c], c >= r
    const int m = k - j - 1;
    for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
      const int r = j + 1 + (int)(e / m), c = j + 1 + (int)(e % m);
      if (c < r) continue;
      const double2 p = bmulc(Rw[(int64_t)j * k + r], Rw[(int64_t)j * k + c]);
      const double2 v = Rw[(int64_t)r * k + c];
      Rw[(int64_t)r * k + c] = make_double2(v.x - p.x, v.y - p.y);
    }
    __syncthreads();
  }
  // R^-1 column by column: X[c][c] = 1 / R[c][c], X[i][c] = -sum_{l=i+1..c} R[i][l] X[l][c] / R[i][i]
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    for (int i = 0; i < k; i++)
      if (i > c) Xw[(int64_t)i * k + c] = make_double2(0, 0);
    Xw[(int64_t)c * k + c] = make_double2(1.0 / Rw[(int64_t)c * k + c].x, 0.0);
    for (int i = c - 1; i >= 0; i--) {
      double2 s = make_double2(0, 0);
      for (int l = i + 1; l <= c; l++) {
        const double2 p = bmul(Rw[(int64_t)i * k + l], Xw[(int64_t)l * k + c]);
        s.x += p.x;
        s.y += p.y;
      }
      const double d = 1.0 / Rw[(int64_t)i * k + i].x;
      Xw[(int64_t)i * k + c] = make_double2(-s.x * d, -s.y * d);
    }
  }
}

// C[w] = A[w] B[w] (k x k, row-major, leading dimension k), 32 x 32 tiles.
__global__ __launch_bounds__(256) void k_sgemm(int k, int64_t sM, const double2* A,
                                               const double2* B, double2* C) {
  __shared__ double2 a[kBT][kBT + 1], b[kBT][kBT + 1];
  const int I = blockIdx.x, J = blockIdx.y, w = blockIdx.z;
  const int t = threadIdx.x, oi = t >> 3, oj = (t & 7) * 4;
  const double2* Aw = A + w * sM;
  const double2* Bw = B + w * sM;
  double2 acc[4] = {};
  for (int L = 0; L < k; L += kBT) {
    for (int e = t; e < kBT * kBT; e += 256) {
      const int i = e / kBT, j = e % kBT;
      const int ar = kBT * I + i, ac = L + j, br = L + i, bc = kBT * J + j;
      a[i][j] = (ar < k && ac < k) ? Aw[(int64_t)ar * k + ac] : make_double2(0, 0);
      b[i][j] = (br < k && bc < k) ? Bw[(int64_t)br * k + bc] : make_double2(0, 0);
    }
    __syncthreads();
    for (int l = 0; l < kBT; l++) {
      const double2 x = a[oi][l];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const double2 p = bmul(x, b[l][oj + q]);
        acc[q].x += p.x;
        acc[q].y += p.y;
      }
    }
    __syncthreads();
  }
  const int gi = kBT * I + oi;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int gj = kBT * J + oj + q;
    if (gi < k && gj < k) C[w * sM + (int64_t)gi * k + gj] = acc[q];
  }
}

// Out = Y S per shift: Y (n_omega, k, n), S (k x k, row-major), Out like Y
// (not aliasing it); 64 rows x 32 output columns per workgroup.
__global__ __launch_bounds__(256) void k_applyb(int64_t n, int k, const double2* Y, int64_t sS,
                                                const double2* S, double2* Out) {
  __shared__ double2 ya[kBT][64 + 1];  // [col][row]
  __shared__ double2 sa[kBT][kBT + 1];
  const int64_t r0 = blockIdx.x * (int64_t)64;
  const int J = blockIdx.y, w = blockIdx.z;
  const double2* Yw = Y + (int64_t)w * k * n;
  const double2* Sw = S + w * sS;
  const int t = threadIdx.x, orow = t & 63, oc = (t >> 6) * 8;  // 8 columns per thread
  double2 acc[8] = {};
  for (int L = 0; L < k; L += kBT) {
    for (int e = t; e < kBT * 64; e += 256) {
      const int c = e / 64, rr = e % 64;
      const int64_t row = r0 + rr;
      ya[c][rr] = (row < n && L + c < k) ? Yw[(int64_t)(L + c) * n + row] : make_double2(0, 0);
    }
    for (int e = t; e < kBT * kBT; e += 256) {
      const int i = e / kBT, j = e % kBT;
      sa[i][j] = (L + i < k && kBT * J + j < k) ? Sw[(int64_t)(L + i) * k + kBT * J + j]
                                               : make_double2(0, 0);
    }
    __syncthreads();
    for (int l = 0; l < kBT; l++) {
      const double2 x = ya[l][orow];
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const double2 p = bmul(x, sa[l][oc + q]);
        acc[q].x += p.x;
        acc[q].y += p.y;
      }
    }
    __syncthreads();
  }
  const int64_t row = r0 + orow;
  if (row >= n) return;
#pragma unroll
  for (int q = 0; q < 8; q++) {
    const int col = kBT * J + oc + q;
    if (col < k) Out[((int64_t)w * k + col) * n + row] = acc[q];
  }
}

// One-sided (Hestenes) Jacobi SVD of A = R^H (k x k) per shift, one
// workgroup of 16 waves: A and the accumulated rotations J live column-major
// in global scratch (column c contiguous), the pairs of each round follow the
// round-robin order and each wave takes pairs in turn, its 64 lanes splitting
// the column length.  The rotation is the narrow path's: with
// gamma = a_p^H a_q and e = gamma / |gamma|, the columns [a_p, conj(e) a_q]
// are rotated by the real Jacobi angle of [[alpha, |gamma|], [|gamma|, beta]].
// Then sigma_c = ||a_c||, sorted descending (ranks counted in parallel),
// Ut = A diag(1/sigma), W = J, both permuted; Rinv W is formed by k_sgemm.
__global__ __launch_bounds__(1024) void k_jacobib(int k, int64_t sM, const double2* R, double2* A,
                                                  double2* Jm, double* sigma, double2* Ut,
                                                  double2* W, double* sv, int* rank,
                                                  uint32_t* status, int max_sweeps) {
  __shared__ int rotated;
  const int w = blockIdx.x;
  const int m = (k + 1) & ~1;  // even number of players (a zero column pads odd k)
  const double2* Rw = R + w * sM;
  double2* Aw = A + (int64_t)w * m * m;
  double2* Jw = Jm + (int64_t)w * m * m;
  double* svw = sv + (int64_t)w * m;
  int* rk = rank + (int64_t)w * m;
  for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
    const int c = (int)(e / m), a = (int)(e % m);  // column c, row a
    double2 v = make_double2(0, 0);
    if (a < k && c < k) {
      const double2 rc = Rw[(int64_t)c * k + a];  // A[a][c] = conj(R[c][a])
      v = make_double2(rc.x, -rc.y);
    }
    Aw[e] = v;
    Jw[e] = make_double2(a == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwave = blockDim.x >> 6;
  const int npair = m / 2;
  int sweep = 0;
  for (; sweep < max_sweeps; sweep++) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < m - 1; rnd++) {
      for (int pr = wave; pr < npair; pr += nwave) {
        int p, q;
        if (pr == 0) {
          p = 0;
          q = 1 + rnd % (m - 1);
        } else {
          p = 1 + (pr + rnd) % (m - 1);
          q = 1 + (m - 1 - pr + rnd) % (m - 1);
        }
        if (p > q) { const int tt = p; p = q; q = tt; }
        double2* ap = Aw + (int64_t)p * m;
        double2* aq = Aw + (int64_t)q * m;
        double al = 0, be = 0, gr = 0, gi = 0;
        for (int a = lane; a < m; a += 64) {
          const double2 x = ap[a], y = aq[a];
          al += x.x * x.x + x.y * x.y;
          be += y.x * y.x + y.y * y.y;
          gr += x.x * y.x + x.y * y.y;
          gi += x.x * y.y - x.y * y.x;
        }
        for (int o = 32; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          gr += __shfl_xor(gr, o, 64);
          gi += __shfl_xor(gi, o, 64);
        }
        const double g = sqrt(gr * gr + gi * gi);
        if (g > 1e-15 * sqrt(al * be) && g > 0.0) {
          const double er = gr / g, ei = -gi / g;  // e^{-i phi}
          const double zeta = (be - al) / (2.0 * g);
          const double tn = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + tn * tn), sn = c * tn;
          double2* jp = Jw + (int64_t)p * m;
          double2* jq = Jw + (int64_t)q * m;
          for (int a = lane; a < m; a += 64) {
            double2 x = ap[a], y = aq[a];
            double2 yp = make_double2(y.x * er - y.y * ei, y.x * ei + y.y * er);
            ap[a] = make_double2(c * x.x - sn * yp.x, c * x.y - sn * yp.y);
            aq[a] = make_double2(sn * x.x + c * yp.x, sn * x.y + c * yp.y);
            x = jp[a];
            y = jq[a];
            yp = make_double2(y.x * er - y.y * ei, y.x * ei + y.y * er);
            jp[a] = make_double2(c * x.x - sn * yp.x, c * x.y - sn * yp.y);
            jq[a] = make_double2(sn * x.x + c * yp.x, sn * x.y + c * yp.y);
          }
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  if (threadIdx.x == 0 && rotated) latch(status, ST_SVD_NOT_CONVERGED);
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double s = 0;
    for (int a = 0; a < k; a++) {
      const double2 v = Aw[(int64_t)c * m + a];
      s += v.x * v.x + v.y * v.y;
    }
    svw[c] = sqrt(s);
    if (!isfinite(svw[c])) latch(status, ST_NONFINITE);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < k; c += blockDim.x) {  // stable descending rank
    int r = 0;
    for (int d = 0; d < k; d++) r += (svw[d] > svw[c]) || (svw[d] == svw[c] && d < c);
    rk[c] = r;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += blockDim.x) {
    const int src = (int)(e / k), a = (int)(e % k);  // source column, row
    const int c = rk[src];
    const double s = svw[src];
    const double2 u = Aw[(int64_t)src * m + a];
    Ut[w * sM + (int64_t)a * k + c] = s > 0 ? make_double2(u.x / s, u.y / s) : make_double2(0, 0);
    W[w * sM + (int64_t)a * k + c] = Jw[(int64_t)src * m + a];
    if (a == 0) sigma[(int64_t)w * k + c] = s;
  }
}

// sigma[w][c] = ||X_c|| and, when U != NULL, U_c = X_c / sigma (eq. 9), one
// workgroup per (column, shift).
__global__ __launch_bounds__(256) void k_colnormb(int64_t n, int k, const double2* X,
                                                  double* sigma, double2* U, uint32_t* status) {
  __shared__ double red[4];
  __shared__ double tot;
  const int c = blockIdx.x, w = blockIdx.y;
  const double2* x = X + ((int64_t)w * k + c) * n;
  double s = 0;
  for (int64_t r = threadIdx.x; r < n; r += 256) s += x[r].x * x[r].x + x[r].y * x[r].y;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    tot = sqrt(red[0] + red[1] + red[2] + red[3]);
    sigma[(int64_t)w * k + c] = tot;
    if (!isfinite(tot)) latch(status, ST_NONFINITE);
  }
  __syncthreads();
  if (!U) return;
  const double inv = tot > 0 ? 1.0 / tot : 0.0;
  double2* u = U + ((int64_t)w * k + c) * n;
  for (int64_t r = threadIdx.x; r < n; r += 256) u[r] = make_double2(x[r].x * inv, x[r].y * inv);
}

// Columns [c0, c0 + kg) of a wide block (shift w at w * wstride, k columns)
// to a narrow block (n_omega, kg, n) (gather), or back (scatter).
__global__ void k_cols_copy(int64_t n, int k, int64_t wstride, int c0, int kg, const double2* src,
                            double2* dst, int gather) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int c = blockIdx.y, w = blockIdx.z;
  if (r >= n) return;
  const int64_t wide = w * wstride + (int64_t)(c0 + c) * n + r;
  const int64_t narrow = ((int64_t)w * kg + c) * n + r;
  if (gather) dst[narrow] = src[wide];
  else dst[wide] = src[narrow];
}

}  // namespace

int gramb_chunks(int64_t n) { return (int)std::min<int64_t>(kBigChunks, (n + 2047) / 2048); }

namespace {

// Gram, Cholesky and R^-1 of Y into G, R, Rinv (k x k per shift, stride sM)
void gram_chol(int64_t n, int n_omega, int k, const double* Y, SmallWs& ws, double* G, double* R,
               double* Rinv, uint32_t* status, hipStream_t s) {
  const int nt = (k + kBT - 1) / kBT, nc = gramb_chunks(n);
  const int64_t rows = (n + nc - 1) / nc, sM = (int64_t)ws.kmax * ws.kmax;
  hipLaunchKernelGGL(k_gramb_partial, dim3(nt * nt, nc, n_omega), dim3(256), 0, s, n, k,
                     (const double2*)Y, rows, nc, (double2*)ws.partial);
  hipLaunchKernelGGL(k_gramb_reduce, dim3((unsigned)(((int64_t)k * k + 255) / 256), n_omega),
                     dim3(256), 0, s, k, nc, (const double2*)ws.partial, sM, (double2*)G);
  hipLaunchKernelGGL(k_cholb, dim3(n_omega), dim3(1024), 0, s, k, sM, (const double2*)G,
                     (double2*)R, (double2*)Rinv, status);
}

void sgemm(int n_omega, int k, int64_t sM, const double* A, const double* B, double* C,
           hipStream_t s) {
  const int nt = (k + kBT - 1) / kBT;
  hipLaunchKernelGGL(k_sgemm, dim3(nt, nt, n_omega), dim3(256), 0, s, k, sM, (const double2*)A,
                     (const double2*)B, (double2*)C);
}

void applyb(int64_t n, int n_omega, int k, const double* Y, int64_t sS, const double* S,
            double* Out, hipStream_t s) {
  const int nt = (k + kBT - 1) / kBT;
  hipLaunchKernelGGL(k_applyb, dim3((unsigned)((n + 63) / 64), nt, n_omega), dim3(256), 0, s, n,
                     k, (const double2*)Y, sS, (const double2*)S, (double2*)Out);
}

}  // namespace

// Y <- Q = Y R^-1 by two Cholesky QR passes (Y = Q R, R = R2 R1 into ws.R,
// R^-1 = R1^-1 R2^-1 into ws.Rinv); tmp: a block like Y.
hipError_t launch_cholqr2_big(int64_t n, int n_omega, int k, double* Y, double* tmp, SmallWs& ws,
                              uint32_t* status, hipStream_t s) {
  if (k > ws.kmax || k > kMaxWideK || !ws.big1 || !ws.big2) return hipErrorInvalidValue;
  const int64_t sM = (int64_t)ws.kmax * ws.kmax;
  gram_chol(n, n_omega, k, Y, ws, ws.G, ws.big1, ws.big2, status, s);   // R1, R1^-1
  applyb(n, n_omega, k, Y, sM, ws.big2, tmp, s);                          // Q1 = Y R1^-1
  gram_chol(n, n_omega, k, tmp, ws, ws.G, ws.W, ws.Ut, status, s);      // R2, R2^-1
  applyb(n, n_omega, k, tmp, sM, ws.Ut, Y, s);                            // Q = Q1 R2^-1
  sgemm(n_omega, k, sM, ws.W, ws.big1, ws.R, s);                          // R = R2 R1
  sgemm(n_omega, k, sM, ws.big2, ws.Ut, ws.Rinv, s);                      // R^-1 = R1^-1 R2^-1
  return hipGetLastError();
}

// The wide counterpart of launch_small_svd: Z = Qz R (two Cholesky QR passes
// on a copy in tmp), the Jacobi SVD R^H = Ut S W^H, V = Z R^-1 W and, when
// Uqu != NULL, U = Q Ut (eq. 8).
hipError_t launch_small_svd_big(int64_t n, int n_omega, int k, const double* Z, const double* Q,
                                double* sigma, double* V, double* Uqu, double* tmp,
                                SmallWs& ws, uint32_t* status, hipStream_t s) {
  if (k > ws.kmax || k > kMaxWideK || !ws.big1 || !ws.big2) return hipErrorInvalidValue;
  const int64_t sM = (int64_t)ws.kmax * ws.kmax;
  hipError_t e = launch_kcopy((int64_t)n_omega * k * n, Z, tmp, s);
  if (e != hipSuccess) return e;
  // V is free until the end: it holds the second pass's Q1 R2^-1 scratch
  gram_chol(n, n_omega, k, tmp, ws, ws.G, ws.big1, ws.big2, status, s);
  applyb(n, n_omega, k, tmp, sM, ws.big2, V, s);
  gram_chol(n, n_omega, k, V, ws, ws.G, ws.W, ws.Ut, status, s);
  sgemm(n_omega, k, sM, ws.W, ws.big1, ws.R, s);      // R = R2 R1
  sgemm(n_omega, k, sM, ws.big2, ws.Ut, ws.Rinv, s);  // R^-1 = R1^-1 R2^-1
  const int m = (k + 1) & ~1;
  // Jacobi scratch: A and J (m x m each; big1 / big2 hold (kmax + 1)^2 per
  // shift), the column norms and ranks in the partial-sum buffer
  double* sv = ws.partial;
  int* rank = reinterpret_cast<int*>(ws.partial + (size_t)n_omega * m);
  hipLaunchKernelGGL(k_jacobib, dim3(n_omega), dim3(1024), 0, s, k, sM, (const double2*)ws.R,
                     (double2*)ws.big1, (double2*)ws.big2, sigma, (double2*)ws.Ut,
                     (double2*)ws.W, sv, rank, status, ws.jacobi_sweeps);
  sgemm(n_omega, k, sM, ws.Rinv, ws.W, ws.G, s);  // Tv = R^-1 W
  applyb(n, n_omega, k, Z, sM, ws.G, V, s);        // V = Z Tv
  if (Uqu) applyb(n, n_omega, k, Q, sM, ws.Ut, Uqu, s);
  return hipGetLastError();
}

hipError_t launch_colnorm_big(int64_t n, int n_omega, int k, const double* X, double* sigma,
                              double* U, uint32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_colnormb, dim3(k, n_omega), dim3(256), 0, s, n, k, (const double2*)X,
                     sigma, (double2*)U, status);
  return hipGetLastError();
}

hipError_t launch_cols_copy(int64_t n, int n_omega, int k, int64_t wstride, int c0, int kg,
                            const double* src, double* dst, bool gather, hipStream_t s) {
  hipLaunchKernelGGL(k_cols_copy, dim3((unsigned)((n + 255) / 256), kg, n_omega), dim3(256), 0, s,
                     n, k, wstride, c0, kg, (const double2*)src, (double2*)dst, gather ? 1 : 0);
  return hipGetLastError();
}

}  // namespace rr
