// Tall-skinny and k x k kernels (all FP64): Cholesky QR applied twice for the
// orthonormal basis of Algorithm 1 step 3, the reduced SVD of step 5 (one-sided
// Jacobi on the k x k triangular factor), the tall-small products that form
// V = Qz W and U = Q Ut (eq. 8), the column norms of steps 7-9 and the
// convergence test of the mixed-precision refinement.
//
// Reductions over n use a fixed chunking and a fixed summation order, so the
// results are bitwise reproducible from run to run.
#include "rr_internal.h"

namespace rr {

constexpr int kChunkRows = 2048;  // rows per partial-sum chunk
constexpr int kSub = 64;          // rows staged in LDS at a time
constexpr int KM = 32;            // largest sketch width the k x k kernels take

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// partial[w][chunk] = (Y_c T)^H (Y_c T) over the chunk's rows, where T is the
// k x k matrix Tm[w] (identity when Tm == NULL).  Y: (n_omega, k, n).  The
// output is cut into 2 x 2 groups on and above the diagonal (the Cholesky
// reads the upper triangle only); each group is accumulated by S = 256 /
// groups threads that take every S-th row of a staged sub-block, and their S
// sums are added in a fixed order at the end, so results are bitwise
// reproducible.  With Tm, each staged sub-block is first multiplied by T in
// LDS, every thread taking one row and every fourth column.  The sketch width
// is at most KM = 32: at most 136 groups, so S >= 1.
// With only_if != NULL a shift whose only_if[w] is zero is skipped.
__device__ __forceinline__ void upper_group(int g, int ng, int& gi, int& gj) {
  int rem = g;
  gi = 0;
  while (rem >= ng - gi) { rem -= ng - gi; gi++; }
  gj = gi + rem;
}

__global__ __launch_bounds__(256) void k_gram_partial(int64_t n, int k, const double2* __restrict__ Y,
                                                      const double2* __restrict__ Tm, int kmax,
                                                      int nchunk, double2* __restrict__ partial,
                                                      const uint32_t* __restrict__ only_if) {
  __shared__ double2 ys[kSub][KM + 1];
  __shared__ double2 tm[KM][KM];
  const int w = blockIdx.y, chunk = blockIdx.x;
  if (only_if && only_if[w] == 0) return;
  const double2* Yw = Y + (int64_t)w * k * n;
  if (Tm) {
    for (int idx = threadIdx.x; idx < k * k; idx += 256)
      tm[idx / k][idx % k] = Tm[(int64_t)w * kmax * kmax + idx];  // tm[i][j] = T[i][j]
  }
  const int ng = (k + 1) / 2, nup = ng * (ng + 1) / 2, S = 256 / nup;
  const int t = threadIdx.x;
  const bool act = t < nup * S;
  const int g = t % nup, slice = t / nup;
  int gi, gj;
  upper_group(g, ng, gi, gj);
  const int i0 = 2 * gi, j0 = 2 * gj;
  double2 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int c = 0; c < 2; c++) acc[a][c] = make_double2(0, 0);
  int64_t r0 = (int64_t)chunk * kChunkRows, r1 = min(n, r0 + kChunkRows);
  // each stage's rows are loaded into registers during the previous stage's
  // products, then staged in LDS
  constexpr int NST = kSub * KM / 256;
  double2 pf[NST];
  auto fetch = [&](int64_t rb) {
    const int64_t rows = min((int64_t)kSub, r1 - rb);
#pragma unroll
    for (int q = 0; q < NST; q++) {
      const int idx = threadIdx.x + 256 * q, j = idx / kSub, rr = idx % kSub;
      pf[q] = (rr < rows && j < k) ? Yw[(int64_t)j * n + rb + rr] : make_double2(0, 0);
    }
  };
  fetch(r0);
  for (int64_t rb = r0; rb < r1; rb += kSub) {
    int rows = (int)min((int64_t)kSub, r1 - rb);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NST; q++) {
      const int idx = threadIdx.x + 256 * q;
      ys[idx % kSub][idx / kSub] = pf[q];
    }
    __syncthreads();
    fetch(rb + kSub);  // past the chunk: no rows, no loads
    if (Tm) {  // ys <- ys * T: thread (row rr, columns cg + 4 c)
      const int rr = t % kSub, cg = t / kSub;
      double2 o[KM / 4];
#pragma unroll
      for (int c = 0; c < KM / 4; c++) o[c] = make_double2(0, 0);
      for (int i = 0; i < k; i++) {
        const double2 a = ys[rr][i];
#pragma unroll
        for (int c = 0; c < KM / 4; c++) {
          const int j = cg + 4 * c;
          if (j < k) {
            const double2 p = cmul(a, tm[i][j]);
            o[c].x += p.x; o[c].y += p.y;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < KM / 4; c++)
        if (cg + 4 * c < k) ys[rr][cg + 4 * c] = o[c];
      __syncthreads();
    }
    if (act) {
      for (int rr = slice; rr < rows; rr += S) {
        const double2 a0 = ys[rr][i0], a1 = ys[rr][i0 + 1];
        const double2 b0 = ys[rr][j0], b1 = ys[rr][j0 + 1];
        double2 p;
        p = cmulc(a0, b0); acc[0][0].x += p.x; acc[0][0].y += p.y;
        p = cmulc(a0, b1); acc[0][1].x += p.x; acc[0][1].y += p.y;
        p = cmulc(a1, b0); acc[1][0].x += p.x; acc[1][0].y += p.y;
        p = cmulc(a1, b1); acc[1][1].x += p.x; acc[1][1].y += p.y;
      }
    }
  }
  // the S slice sums of every group, added in slice order (S * groups * 4 <=
  // 1024 entries, staged in ys)
  __syncthreads();
  double2* red = &ys[0][0];
  if (act) {
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
      for (int c = 0; c < 2; c++) red[(slice * nup + g) * 4 + a * 2 + c] = acc[a][c];
  }
  __syncthreads();
  for (int e = t; e < nup * 4; e += 256) {
    const int gg = e / 4, a = (e % 4) / 2, c = e % 2;
    double2 sum = make_double2(0, 0);
    for (int sl = 0; sl < S; sl++) {
      const double2 v = red[(sl * nup + gg) * 4 + e % 4];
      sum.x += v.x; sum.y += v.y;
    }
    int hi, hj;
    upper_group(gg, ng, hi, hj);
    const int ii = 2 * hi + a, jj = 2 * hj + c;
    if (ii < k && jj < k)
      partial[((int64_t)w * nchunk + chunk) * kmax * kmax + ii * k + jj] = sum;
  }
}

// Sum the partials (fixed order), Cholesky G = R^H R (R upper, real positive
// diagonal), Rinv = R^-1.  Passes 1 and 2 compose: R <- Rnew Rold,
// Rinv <- Rinv_old Rinv_new.
//
// Cholesky QR breaks down once cond(Y) passes about u^-1/2 (1e8): the Gram
// matrix is then not numerically positive definite.  Pass 0 then takes the
// Cholesky factor of G + s I instead, with the shift of Fukaya, Kannan,
// Nakatsukasa, Yamamoto & Yanagisawa (shifted CholeskyQR3, SISC 2020),
// s = 11 (m k + k (k + 1)) u ||Y||_F^2 (m + 2 in place of m for complex inner
// products; ||Y||_F^2 = trace G bounds ||Y||_2^2), and sets shifted[w]; Y R^-1
// then has a condition number near (u m k)^-1/2, which the two passes that
// follow make orthonormal.  Pass 2 runs only for shifts with shifted[w] set.
// A breakdown that remains latches ST_BREAKDOWN (the pivot is replaced by 1).
__global__ __launch_bounds__(256) void k_chol(int k, int kmax, int nchunk, int64_t m,
                                              const double2* __restrict__ partial,
                                              double2* __restrict__ Rg, double2* __restrict__ Rinvg,
                                              int pass, uint32_t* __restrict__ shifted,
                                              uint32_t* status) {
  __shared__ double2 G[KM][KM + 1];
  __shared__ double2 Rn[KM][KM + 1];
  __shared__ double2 Ri[KM][KM + 1];
  __shared__ int bad;
  __shared__ double shift;
  const int w = blockIdx.x;
  if (pass == 2 && shifted[w] == 0) return;
  int attempt = 0;
  for (;; attempt++) {
    for (int pr = threadIdx.x; pr < k * k; pr += 256) {  // upper triangle (all that is used)
      double2 s = make_double2(0, 0);
      if (pr % k >= pr / k) {
        for (int c = 0; c < nchunk; c++) {
          double2 v = partial[((int64_t)w * nchunk + c) * kmax * kmax + pr];
          s.x += v.x; s.y += v.y;
        }
        if (attempt && pr % k == pr / k) s.x += shift;
      }
      G[pr / k][pr % k] = s;
    }
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (attempt == 0 && threadIdx.x == 0) {
      double tr = 0;
      for (int j = 0; j < k; j++) tr += G[j][j].x;
      shift = 11.0 * ((double)(m + 2) * k + (double)k * (k + 1)) * 0x1p-53 * tr;
    }
    // right-looking Cholesky on the upper triangle: G = R^H R
    for (int j = 0; j < k; j++) {
      if (threadIdx.x == 0) {
        double d = G[j][j].x;
        if (!(d > 0.0) || !isfinite(d)) { bad = 1; d = 1.0; }
        G[j][j] = make_double2(sqrt(d), 0.0);
      }
      __syncthreads();
      double rjj = G[j][j].x;
      for (int c = j + 1 + threadIdx.x; c < k; c += 256) {
        G[j][c].x /= rjj; G[j][c].y /= rjj;
      }
      __syncthreads();
      int wd = k - 1 - j;
      for (int idx = threadIdx.x; idx < wd * wd; idx += 256) {
        int a = j + 1 + idx / wd, c = j + 1 + idx % wd;
        if (c < a) continue;
        double2 p = cmulc(G[j][a], G[j][c]);  // R[j][a]^* R[j][c]
        G[a][c].x -= p.x; G[a][c].y -= p.y;
      }
      __syncthreads();
    }
    if (!(bad && pass == 0 && attempt == 0)) break;  // bad is block-uniform here
    __syncthreads();
  }
  if (pass == 0 && threadIdx.x == 0) shifted[w] = attempt;
  const int compose = pass > 0;
  for (int idx = threadIdx.x; idx < k * k; idx += 256) {
    int a = idx / k, c = idx % k;
    Rn[a][c] = c >= a ? G[a][c] : make_double2(0, 0);
    Ri[a][c] = make_double2(a == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  // Rinv: solve R X = I by back substitution, one column per thread
  for (int c = threadIdx.x; c < k; c += 256) {
    for (int a = c; a >= 0; a--) {
      double2 s = make_double2(a == c ? 1.0 : 0.0, 0.0);
      for (int t = a + 1; t <= c; t++) {
        double2 p = cmul(Rn[a][t], Ri[t][c]);
        s.x -= p.x; s.y -= p.y;
      }
      double d = Rn[a][a].x;
      Ri[a][c] = make_double2(s.x / d, s.y / d);
    }
  }
  __syncthreads();
  double2* Rw = Rg + (int64_t)w * kmax * kmax;
  double2* Riw = Rinvg + (int64_t)w * kmax * kmax;
  if (compose) {
    // R <- Rn * Rold ; Rinv <- Riold * Ri  (Rold, Riold are the global inputs)
    double2 nr[4], ni[4];
    for (int q = 0; q < 4; q++) {
      int idx = threadIdx.x + 256 * q;
      if (idx >= k * k) break;
      int a = idx / k, c = idx % k;
      double2 s = make_double2(0, 0), t2 = make_double2(0, 0);
      for (int t = 0; t < k; t++) {
        double2 p = cmul(Rn[a][t], Rw[t * k + c]);
        s.x += p.x; s.y += p.y;
        double2 q2 = cmul(Riw[a * k + t], Ri[t][c]);
        t2.x += q2.x; t2.y += q2.y;
      }
      nr[q] = s;
      ni[q] = t2;
    }
    __syncthreads();
    for (int q = 0; q < 4; q++) {
      int idx = threadIdx.x + 256 * q;
      if (idx >= k * k) break;
      Rw[idx] = nr[q];
      Riw[idx] = ni[q];
    }
  } else {
    for (int idx = threadIdx.x; idx < k * k; idx += 256) {
      Rw[idx] = Rn[idx / k][idx % k];
      Riw[idx] = Ri[idx / k][idx % k];
    }
  }
  if (threadIdx.x == 0 && bad) latch(status, ST_BREAKDOWN);
}

// Out = Y * Tm[w]  (n x k times k x k), one row per thread (held in registers);
// Out may alias Y.  With only_if != NULL a shift whose only_if[w] is zero is
// skipped.
__global__ __launch_bounds__(256) void k_apply_small(int64_t n, int k, const double2* Y,
                                                     const double2* __restrict__ Tm, int kmax,
                                                     double2* Out,
                                                     const uint32_t* __restrict__ only_if) {
  __shared__ double2 tm[KM][KM];
  const int w = blockIdx.y;
  if (only_if && only_if[w] == 0) return;
  for (int idx = threadIdx.x; idx < k * k; idx += 256)
    tm[idx / k][idx % k] = Tm[(int64_t)w * kmax * kmax + idx];
  __syncthreads();
  int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (r >= n) return;
  const double2* Yw = Y + (int64_t)w * k * n;
  double2* Ow = Out + (int64_t)w * k * n;
  double2 row[KM];
#pragma unroll
  for (int i = 0; i < KM; i++) row[i] = i < k ? Yw[(int64_t)i * n + r] : make_double2(0, 0);
  for (int j = 0; j < k; j++) {
    double2 s = make_double2(0, 0);
#pragma unroll
    for (int i = 0; i < KM; i++) {
      if (i < k) {
        double2 p = cmul(row[i], tm[i][j]);
        s.x += p.x; s.y += p.y;
      }
    }
    Ow[(int64_t)j * n + r] = s;
  }
}

// T[w] = I for the shifts with only_if[w] set.
__global__ __launch_bounds__(256) void k_identity_if(int k, int kmax, double2* Tm,
                                                     const uint32_t* __restrict__ only_if) {
  const int w = blockIdx.x;
  if (only_if[w] == 0) return;
  for (int idx = threadIdx.x; idx < k * k; idx += 256)
    Tm[(int64_t)w * kmax * kmax + idx] = make_double2(idx / k == idx % k ? 1.0 : 0.0, 0.0);
}

static int nchunks(int64_t n) { return (int)((n + kChunkRows - 1) / kChunkRows); }

// Cholesky QR of Y (n_omega blocks of n x k) into ws.R and ws.Rinv: two
// passes, and for shifts whose first Cholesky broke down a shifted first pass
// and a third (shifted CholeskyQR3).  The launch sequence is the same either
// way (the third pass returns at once for the other shifts).  With
// explicit_q, a shifted shift's Y is replaced by Q1 = Y R1^-1 after the first
// pass and its R^-1 reset to I, so the two passes that follow orthonormalise
// Q1 itself and the final Q = Q1 R^-1 is orthonormal to O(u); otherwise Q is
// formed from Y through the composed R^-1 and orthonormal to about u cond(Y).
// R is the composed factor (Y = Q R) either way.
static void chol_passes(int n, int n_omega, int k, double* Y, bool explicit_q, SmallWs& ws,
                        uint32_t* status, hipStream_t s) {
  const int nc = nchunks(n);
  const dim3 g(nc, n_omega);
  double2* part = (double2*)ws.partial;
  for (int pass = 0; pass < 3; pass++) {
    hipLaunchKernelGGL(k_gram_partial, g, dim3(256), 0, s, (int64_t)n, k, (const double2*)Y,
                       pass ? (const double2*)ws.Rinv : (const double2*)nullptr, ws.kmax, nc,
                       part, pass == 2 ? (const uint32_t*)ws.shifted : (const uint32_t*)nullptr);
    hipLaunchKernelGGL(k_chol, dim3(n_omega), dim3(256), 0, s, k, ws.kmax, nc, (int64_t)n, part,
                       (double2*)ws.R, (double2*)ws.Rinv, pass, ws.shifted, status);
    if (pass == 0 && explicit_q) {
      hipLaunchKernelGGL(k_apply_small, dim3((n + 255) / 256, n_omega), dim3(256), 0, s,
                         (int64_t)n, k, (const double2*)Y, (const double2*)ws.Rinv, ws.kmax,
                         (double2*)Y, (const uint32_t*)ws.shifted);
      hipLaunchKernelGGL(k_identity_if, dim3(n_omega), dim3(256), 0, s, k, ws.kmax,
                         (double2*)ws.Rinv, (const uint32_t*)ws.shifted);
    }
  }
}

hipError_t launch_cholqr2(int n, int n_omega, int k, double* Y, SmallWs& ws, uint32_t* status,
                          hipStream_t s) {
  if (nchunks(n) > ws.nchunk || k > ws.kmax || k > KM) return hipErrorInvalidValue;
  chol_passes(n, n_omega, k, Y, true, ws, status, s);
  hipLaunchKernelGGL(k_apply_small, dim3((n + 255) / 256, n_omega), dim3(256), 0, s,
                     (int64_t)n, k, (const double2*)Y, (const double2*)ws.Rinv, ws.kmax,
                     (double2*)Y, (const uint32_t*)nullptr);
  return hipGetLastError();
}

// One-sided (Hestenes) Jacobi SVD of A = R^H (k x k, one workgroup per shift):
// columns are rotated pairwise until mutually orthogonal, A J = Ut S, so
// R^H = Ut S J^H.  Pairs follow the round-robin (circle) order, k/2 disjoint
// pairs per round, 8 threads per pair.  Outputs sorted by descending sigma.
// Also forms Tv = Rinv * W for V = Z Tv.
// A sweep that still rotated a pair after max_sweeps sweeps means the SVD has
// not converged: ST_SVD_NOT_CONVERGED is latched (the results are returned
// as they stand).
__global__ __launch_bounds__(256) void k_jacobi_svd(int k, int kmax, const double2* __restrict__ Rg,
                                                    const double2* __restrict__ Rinvg,
                                                    double* __restrict__ sigma,
                                                    double2* __restrict__ Utg, double2* __restrict__ Wg,
                                                    double2* __restrict__ Tvg, uint32_t* status,
                                                    int max_sweeps) {
  __shared__ double2 A[KM][KM + 1];  // A[row][col]
  __shared__ double2 J[KM][KM + 1];
  __shared__ double sv[KM];
  __shared__ int perm[KM];
  __shared__ int rotated;
  const int w = blockIdx.x;
  const double2* R = Rg + (int64_t)w * kmax * kmax;
  const int m = (k + 1) & ~1;  // even number of players (a zero column pads odd k)
  for (int idx = threadIdx.x; idx < m * m; idx += 256) {
    int a = idx / m, c = idx % m;
    double2 v = make_double2(0, 0);
    if (a < k && c < k) { double2 rc = R[c * k + a]; v = make_double2(rc.x, -rc.y); }  // R^H
    A[a][c] = v;
    J[a][c] = make_double2(a == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int npair = m / 2;
  const int pair = threadIdx.x >> 3, sub = threadIdx.x & 7;
  for (int sweep = 0; sweep < max_sweeps; sweep++) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int rnd = 0; rnd < m - 1; rnd++) {
      if (pair < npair) {
        int p, q;
        if (pair == 0) { p = 0; q = 1 + rnd % (m - 1); }
        else {
          p = 1 + (pair + rnd) % (m - 1);
          q = 1 + (m - 1 - pair + rnd) % (m - 1);
        }
        if (p > q) { int t = p; p = q; q = t; }
        double al = 0, be = 0, gr = 0, gi = 0;
        for (int a = sub; a < m; a += 8) {
          double2 x = A[a][p], y = A[a][q];
          al += x.x * x.x + x.y * x.y;
          be += y.x * y.x + y.y * y.y;
          gr += x.x * y.x + x.y * y.y;  // conj(x) y
          gi += x.x * y.y - x.y * y.x;
        }
        for (int o = 1; o < 8; o <<= 1) {
          al += __shfl_xor(al, o, 8);
          be += __shfl_xor(be, o, 8);
          gr += __shfl_xor(gr, o, 8);
          gi += __shfl_xor(gi, o, 8);
        }
        double g = sqrt(gr * gr + gi * gi);
        if (g > 1e-15 * sqrt(al * be) && g > 0.0) {
          // phase e^{i phi} = gamma/|gamma|; rotate [a_p, e^{-i phi} a_q]
          double er = gr / g, ei = -gi / g;  // e^{-i phi}
          double zeta = (be - al) / (2.0 * g);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
          for (int a = sub; a < m; a += 8) {
            double2 x = A[a][p], y = A[a][q];
            double2 yp = make_double2(y.x * er - y.y * ei, y.x * ei + y.y * er);
            A[a][p] = make_double2(c * x.x - sn * yp.x, c * x.y - sn * yp.y);
            A[a][q] = make_double2(sn * x.x + c * yp.x, sn * x.y + c * yp.y);
            x = J[a][p]; y = J[a][q];
            yp = make_double2(y.x * er - y.y * ei, y.x * ei + y.y * er);
            J[a][p] = make_double2(c * x.x - sn * yp.x, c * x.y - sn * yp.y);
            J[a][q] = make_double2(sn * x.x + c * yp.x, sn * x.y + c * yp.y);
          }
          if (sub == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // every thread read `rotated` after the last round's barrier; nothing has
  // written it since
  if (threadIdx.x == 0 && rotated) latch(status, ST_SVD_NOT_CONVERGED);
  for (int c = threadIdx.x; c < k; c += 256) {
    double s = 0;
    for (int a = 0; a < k; a++) s += A[a][c].x * A[a][c].x + A[a][c].y * A[a][c].y;
    sv[c] = sqrt(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < k; c++) perm[c] = c;
    for (int a = 0; a < k; a++) {  // selection sort, descending, stable
      int best = a;
      for (int c = a + 1; c < k; c++)
        if (sv[perm[c]] > sv[perm[best]]) best = c;
      int t = perm[a]; perm[a] = perm[best]; perm[best] = t;
    }
    for (int c = 0; c < k; c++)
      if (!isfinite(sv[c])) latch(status, ST_NONFINITE);
  }
  __syncthreads();
  double* sw = sigma + (int64_t)w * k;
  double2* Ut = Utg + (int64_t)w * kmax * kmax;
  double2* Wm = Wg + (int64_t)w * kmax * kmax;
  double2* Tv = Tvg + (int64_t)w * kmax * kmax;
  const double2* Ri = Rinvg + (int64_t)w * kmax * kmax;
  for (int idx = threadIdx.x; idx < k * k; idx += 256) {
    int a = idx / k, c = idx % k;  // row a, output column c
    int src = perm[c];
    double s = sv[src];
    double2 u = A[a][src];
    Ut[a * k + c] = s > 0 ? make_double2(u.x / s, u.y / s) : make_double2(0, 0);
    Wm[a * k + c] = J[a][src];
    double2 t = make_double2(0, 0);
    for (int b = 0; b < k; b++) {
      double2 p = cmul(Ri[a * k + b], J[b][src]);
      t.x += p.x; t.y += p.y;
    }
    Tv[a * k + c] = t;
    if (a == 0) sw[c] = s;
  }
}

hipError_t launch_small_svd(int n, int n_omega, int k, const double* Z, const double* Q,
                            double* sigma, double* V, double* Uqu, SmallWs& ws, uint32_t* status,
                            hipStream_t s) {
  if (nchunks(n) > ws.nchunk || k > ws.kmax || k > KM) return hipErrorInvalidValue;
  // Z = Qz R by Cholesky QR (R and R^-1 composed; Qz never formed)
  chol_passes(n, n_omega, k, const_cast<double*>(Z), false, ws, status, s);  // Z is not written
  // W and its product with R^-1 (ws.G holds Tv = R^-1 W)
  hipLaunchKernelGGL(k_jacobi_svd, dim3(n_omega), dim3(256), 0, s, k, ws.kmax,
                     (const double2*)ws.R, (const double2*)ws.Rinv, sigma, (double2*)ws.Ut,
                     (double2*)ws.W, (double2*)ws.G, status, ws.jacobi_sweeps);
  // V = Z R^-1 W = Qz W
  hipLaunchKernelGGL(k_apply_small, dim3((n + 255) / 256, n_omega), dim3(256), 0, s,
                     (int64_t)n, k, (const double2*)Z, (const double2*)ws.G, ws.kmax, (double2*)V,
                     (const uint32_t*)nullptr);
  if (Uqu)  // Halko et al.'s response modes U = Q Ut (eq. 8)
    hipLaunchKernelGGL(k_apply_small, dim3((n + 255) / 256, n_omega), dim3(256), 0, s,
                       (int64_t)n, k, (const double2*)Q, (const double2*)ws.Ut, ws.kmax,
                       (double2*)Uqu, (const uint32_t*)nullptr);
  return hipGetLastError();
}

// partial[w][chunk][j] = sum over the chunk of |X_j|^2 (and of |D_j|^2 into
// partial2 when D != NULL, after X += D).  Block (chunk, w, z) takes columns
// 4z .. 4z+3; each thread owns rows r0 + t + 256 i of the chunk and issues
// all of a column's loads before it adds them up (in i order), so a column
// costs one memory round trip.
constexpr int kColGroup = 4;
__global__ __launch_bounds__(256) void k_colnorm_partial(int64_t n, int k, double2* X,
                                                         const double2* __restrict__ D,
                                                         int nchunk, double* partial,
                                                         double* partial2, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  constexpr int RPT = kChunkRows / 256;
  __shared__ double red[2][256];
  const int w = blockIdx.y, chunk = blockIdx.x;
  const int64_t r0 = (int64_t)chunk * kChunkRows, r1 = min(n, r0 + kChunkRows);
  const int j1 = min(k, kColGroup * ((int)blockIdx.z + 1));
  for (int j = kColGroup * blockIdx.z; j < j1; j++) {
    double2* x = X + ((int64_t)w * k + j) * n;
    const double2* d = D ? D + ((int64_t)w * k + j) * n : nullptr;
    double2 xv[RPT], dv[RPT];
#pragma unroll
    for (int i = 0; i < RPT; i++) {
      const int64_t r = r0 + threadIdx.x + 256 * i;
      xv[i] = r < r1 ? x[r] : make_double2(0, 0);
      dv[i] = d && r < r1 ? d[r] : make_double2(0, 0);
    }
    double sx = 0, sd = 0;
#pragma unroll
    for (int i = 0; i < RPT; i++) {
      const int64_t r = r0 + threadIdx.x + 256 * i;
      if (r < r1) {
        double2 v = xv[i];
        if (d) {
          sd += dv[i].x * dv[i].x + dv[i].y * dv[i].y;
          v.x += dv[i].x; v.y += dv[i].y;
          x[r] = v;
        }
        sx += v.x * v.x + v.y * v.y;
      }
    }
    red[0][threadIdx.x] = sx;
    red[1][threadIdx.x] = sd;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        red[0][threadIdx.x] += red[0][threadIdx.x + o];
        red[1][threadIdx.x] += red[1][threadIdx.x + o];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      partial[((int64_t)w * nchunk + chunk) * 64 + j] = red[0][0];
      if (partial2) partial2[((int64_t)w * nchunk + chunk) * 64 + j] = red[1][0];
    }
    __syncthreads();
  }
}
static dim3 colnorm_grid(int nc, int n_omega, int k) {
  return dim3(nc, n_omega, (k + kColGroup - 1) / kColGroup);
}

__global__ void k_colnorm_final(int k, int nchunk, const double* partial, double* sigma,
                                uint32_t* status) {
  const int w = blockIdx.x;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double s = 0;
    for (int c = 0; c < nchunk; c++) s += partial[((int64_t)w * nchunk + c) * 64 + j];
    s = sqrt(s);
    if (!isfinite(s)) latch(status, ST_NONFINITE);
    sigma[(int64_t)w * k + j] = s;
  }
}

// U_j = W_j / sigma_j (divide; 0 where sigma_j = 0) or W_j * sigma_j.
// Each thread takes kScaleRows rows, 256 apart.
constexpr int kScaleRows = 8;
__global__ __launch_bounds__(256) void k_scale_cols(int64_t n, int k, const double2* W,
                                                    const double* sigma, double2* U, int divide) {
  const int j = blockIdx.y, w = blockIdx.z;
  const double s = sigma[(int64_t)w * k + j];
  const double c = divide ? (s > 0 ? 1.0 / s : 0.0) : s;
  const int64_t base = ((int64_t)w * k + j) * n;
  const int64_t r0 = blockIdx.x * (int64_t)(256 * kScaleRows) + threadIdx.x;
  double2 v[kScaleRows];
#pragma unroll
  for (int i = 0; i < kScaleRows; i++) {
    const int64_t r = r0 + 256 * i;
    v[i] = r < n ? W[base + r] : make_double2(0, 0);
  }
#pragma unroll
  for (int i = 0; i < kScaleRows; i++) {
    const int64_t r = r0 + 256 * i;
    if (r < n) U[base + r] = make_double2(v[i].x * c, v[i].y * c);
  }
}
static dim3 scale_grid(int n, int k, int n_omega) {
  return dim3((unsigned)((n + 256 * kScaleRows - 1) / (256 * kScaleRows)), k, n_omega);
}

hipError_t launch_scale_cols(int n, int n_omega, int k, const double* W, const double* scale,
                             double* U, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_cols, scale_grid(n, k, n_omega), dim3(256), 0, s,
                     (int64_t)n, k, (const double2*)W, scale, (double2*)U, 0);
  return hipGetLastError();
}

hipError_t launch_colnorm_scale(int n, int n_omega, int k, const double* W, double* sigma,
                                double* U, SmallWs& ws, uint32_t* status, hipStream_t s) {
  int nc = nchunks(n);
  if (nc > ws.nchunk || k > KM) return hipErrorInvalidValue;
  double* part = ws.partial;
  hipLaunchKernelGGL(k_colnorm_partial, colnorm_grid(nc, n_omega, k), dim3(256), 0, s,
                     (int64_t)n, k,
                     (double2*)W, (const double2*)nullptr, nc, part, (double*)nullptr,
                     (const uint32_t*)nullptr);
  hipLaunchKernelGGL(k_colnorm_final, dim3(n_omega), dim3(64), 0, s, k, nc, part, sigma, status);
  if (U)
    hipLaunchKernelGGL(k_scale_cols, scale_grid(n, k, n_omega), dim3(256), 0, s,
                       (int64_t)n, k, (const double2*)W, (const double*)sigma, (double2*)U, 1);
  return hipGetLastError();
}

// After X += D, per column j: e_j = ||D_j|| / ||X_j||, the size of the
// correction just applied.  Refinement shrinks the error by a contraction
// rho per correction, the rate of the iteration matrix I - M32^-1 M
// (forward) or I - M32^-H M^H (adjoint), so the error left is about rho e_j.
// rho is never assumed: it is measured, and kept per shift as the largest
// value seen since the factorisation (slot kRhoSlot of the shift's row; zero
// = not measured yet).  Two measurements: the ratio of two successive
// corrections, e_j / e_j,prev; and, on the first solve after a
// factorisation when the solve has spare columns, probe systems M x = M z
// with z known, solved beside the caller's columns, whose errors before and
// after the first correction are exact (k_probe_rho).  Both directions share it: the adjoint iteration matrix is
// the conjugate transpose of I - M M32^-1 = M (I - M32^-1 M) M^-1, similar
// to the forward one, so the two have the same eigenvalues and the ratios
// converge to the same rate.  A column has converged when e_j <= tol, or
// when the error it leaves, estimated with rho (this solve's own ratio from
// the second correction on, else the kept one), is at most tol / 2.  So the
// first solve after a factorisation takes a second correction unless the
// first already meets tol or its probes measured rho, and later ones, in
// either direction, stop after one when the measured contraction allows it.  Unconverged columns are
// counted into *fail_count (reset by the caller per correction).
__global__ void k_refine_check(int k, int nchunk, const double* px, const double* pd, double tol,
                               int it, int adjoint, double* rho, uint32_t* fail_count,
                               uint32_t* status, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ double ratio_max;
  const int w = blockIdx.x;
  double* rw = rho + (int64_t)w * kRhoStride;
  double e = 0.0, ratio = 0.0;
  const int j = threadIdx.x;
  if (threadIdx.x == 0) ratio_max = 0.0;
  __syncthreads();
  if (j < k) {
    double sx = 0, sd = 0;
    for (int c = 0; c < nchunk; c++) {
      sx += px[((int64_t)w * nchunk + c) * 64 + j];
      sd += pd[((int64_t)w * nchunk + c) * 64 + j];
    }
    if (!isfinite(sx) || !isfinite(sd)) latch(status, ST_NONFINITE);
    e = sx > 0 ? sqrt(sd / sx) : (sd > 0 ? INFINITY : 0.0);
    if (it > 0) {
      const double prev = rw[j];
      ratio = prev > 0 ? e / prev : (e > 0 ? INFINITY : 0.0);
      // doubles compare as their bit patterns when non-negative
      atomicMax(reinterpret_cast<unsigned long long*>(&ratio_max),
                (unsigned long long)__double_as_longlong(ratio));
    }
  }
  __syncthreads();
  double* kept = rw + kRhoSlot;
  (void)adjoint;
  const double rho_kept = *kept;
  if (j < k) {
    rw[j] = e;
    const double r = it > 0 ? fmax(ratio, rho_kept) : rho_kept;
    const bool ok = e <= tol || (r > 0.0 && 2.0 * e * r <= tol);
    if (!ok) atomicAdd(fail_count, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0 && it > 0) *kept = fmax(rho_kept, ratio_max);
}

// partial[w][chunk][q] = sum over the chunk of |X_{k0+q} - Z_q|^2, q < p: the
// errors of the probe columns (X: kk columns per shift, Z: p per shift).
__global__ __launch_bounds__(256) void k_probe_partial(int64_t n, int kk, int k0, int p,
                                                       const double2* __restrict__ X,
                                                       const double2* __restrict__ Z, int nchunk,
                                                       double* partial, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  constexpr int RPT = kChunkRows / 256;
  __shared__ double red[256];
  const int w = blockIdx.y, chunk = blockIdx.x;
  const int64_t r0 = (int64_t)chunk * kChunkRows, r1 = min(n, r0 + kChunkRows);
  for (int q = 0; q < p; q++) {
    const double2* x = X + ((int64_t)w * kk + k0 + q) * n;
    const double2* z = Z + ((int64_t)w * p + q) * n;
    double2 xv[RPT], zv[RPT];
#pragma unroll
    for (int i = 0; i < RPT; i++) {
      const int64_t r = r0 + threadIdx.x + 256 * i;
      xv[i] = r < r1 ? x[r] : make_double2(0, 0);
      zv[i] = r < r1 ? z[r] : make_double2(0, 0);
    }
    double se = 0;
#pragma unroll
    for (int i = 0; i < RPT; i++) {
      const double dx = xv[i].x - zv[i].x, dy = xv[i].y - zv[i].y;
      se += dx * dx + dy * dy;
    }
    red[threadIdx.x] = se;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[((int64_t)w * nchunk + chunk) * 64 + q] = red[0];
    __syncthreads();
  }
}

// The probes' errors e_q: after the first solve (stage 0) kept in the slots
// kProbeSlot + q; after the first correction (stage 1) their ratio to those,
// whose largest is the measured contraction rho (kept as in k_refine_check).
__global__ void k_probe_rho(int p, int nchunk, const double* partial, int stage, double* rho,
                            uint32_t* status, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ double ratio_max;
  const int w = blockIdx.x, q = threadIdx.x;
  double* rw = rho + (int64_t)w * kRhoStride;
  if (q == 0) ratio_max = 0.0;
  __syncthreads();
  if (q < p) {
    double s = 0;
    for (int c = 0; c < nchunk; c++) s += partial[((int64_t)w * nchunk + c) * 64 + q];
    if (!isfinite(s)) latch(status, ST_NONFINITE);
    const double e = sqrt(s);
    if (stage == 0) {
      rw[kProbeSlot + q] = e;
    } else {
      const double e0 = rw[kProbeSlot + q];
      const double ratio = e0 > 0 ? e / e0 : (e > 0 ? INFINITY : 0.0);
      atomicMax(reinterpret_cast<unsigned long long*>(&ratio_max),
                (unsigned long long)__double_as_longlong(ratio));
    }
  }
  __syncthreads();
  if (q == 0 && stage == 1) rw[kRhoSlot] = fmax(rw[kRhoSlot], ratio_max);
}

hipError_t launch_probe_errors(int n, int n_omega, int kk, int k0, int p, const double* X,
                               const double* Z, SmallWs& ws, uint32_t* status, hipStream_t s) {
  const int nc = nchunks(n);
  if (nc > ws.nchunk || p < 1 || p > 32 || k0 + p > kk || !ws.rho) return hipErrorInvalidValue;
  double* pz = ws.partial + 2 * (size_t)n_omega * nc * 64;
  hipLaunchKernelGGL(k_probe_partial, dim3(nc, n_omega), dim3(256), 0, s, (int64_t)n, kk, k0, p,
                     (const double2*)X, (const double2*)Z, nc, pz, (const uint32_t*)nullptr);
  hipLaunchKernelGGL(k_probe_rho, dim3(n_omega), dim3(64), 0, s, p, nc, (const double*)pz, 0,
                     ws.rho, status, (const uint32_t*)nullptr);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_cols_place(int64_t n, const double2* src, int64_t sws,
                                                    int sc0, double2* dst, int64_t dws, int dc0) {
  const int c = blockIdx.y, w = blockIdx.z;
  const double2* a = src + w * sws + (int64_t)(sc0 + c) * n;
  double2* b = dst + w * dws + (int64_t)(dc0 + c) * n;
  const int64_t r0 = blockIdx.x * (int64_t)(256 * kScaleRows) + threadIdx.x;
  double2 v[kScaleRows];
#pragma unroll
  for (int i = 0; i < kScaleRows; i++) {
    const int64_t r = r0 + 256 * i;
    v[i] = r < n ? a[r] : make_double2(0, 0);
  }
#pragma unroll
  for (int i = 0; i < kScaleRows; i++) {
    const int64_t r = r0 + 256 * i;
    if (r < n) b[r] = v[i];
  }
}

hipError_t launch_cols_place(int64_t n, int n_omega, int ncols, const double* src, int64_t sws,
                             int sc0, double* dst, int64_t dws, int dc0, hipStream_t s) {
  if (ncols < 1) return hipSuccess;
  hipLaunchKernelGGL(k_cols_place, scale_grid((int)n, ncols, n_omega), dim3(256), 0, s, n,
                     (const double2*)src, sws, sc0, (double2*)dst, dws, dc0);
  return hipGetLastError();
}

// Forget the measured contractions (a new factorisation).
__global__ void k_refine_reset(int n_omega, double* rho) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < n_omega) {
    rho[(int64_t)w * kRhoStride + kRhoSlot] = 0.0;
    rho[(int64_t)w * kRhoStride + kRhoSlot + 1] = 0.0;
  }
}

hipError_t launch_refine_reset(int n_omega, double* rho, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_reset, dim3((n_omega + 255) / 256), dim3(256), 0, s, n_omega, rho);
  return hipGetLastError();
}

hipError_t launch_refine_update(int n, int n_omega, int k, double* X, const double* D, double tol,
                                int it, int adjoint, SmallWs& ws, uint32_t* status,
                                uint32_t* fail_count, hipStream_t s, const uint32_t* skip, int kk,
                                int p, const double* Z) {
  int nc = nchunks(n);
  if (kk < k) kk = k;
  if (nc > ws.nchunk || kk > KM || (p > 0 && (!Z || k + p > kk))) return hipErrorInvalidValue;
  double* px = ws.partial;
  double* pd = ws.partial + (size_t)n_omega * nc * 64;
  hipLaunchKernelGGL(k_colnorm_partial, colnorm_grid(nc, n_omega, kk), dim3(256), 0, s,
                     (int64_t)n, kk,
                     (double2*)X, (const double2*)D, nc, px, pd, skip);
  if (p > 0 && it == 0) {  // the probes' errors after the first correction: rho
    double* pz = ws.partial + 2 * (size_t)n_omega * nc * 64;
    hipLaunchKernelGGL(k_probe_partial, dim3(nc, n_omega), dim3(256), 0, s, (int64_t)n, kk, k, p,
                       (const double2*)X, (const double2*)Z, nc, pz, skip);
    hipLaunchKernelGGL(k_probe_rho, dim3(n_omega), dim3(64), 0, s, p, nc, pz, 1, ws.rho, status,
                       skip);
  }
  hipLaunchKernelGGL(k_refine_check, dim3(n_omega), dim3(64), 0, s, k, nc, px, pd, tol, it,
                     adjoint, ws.rho, fail_count, status, skip);
  return hipGetLastError();
}

}  // namespace rr
