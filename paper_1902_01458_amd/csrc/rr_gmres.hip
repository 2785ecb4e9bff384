// GMRES-based iterative refinement (GMRES-IR, Carson & Higham, SISC 2017 and
// 2018) for the mixed-precision solves: where the correction of plain
// refinement, d = M32^-1 r, stops contracting (kappa(M) * eps_32 around one
// or more), the correction is taken from m steps of GMRES on the
// preconditioned system M32^-1 M d = M32^-1 r instead, with M applied in FP64
// from the stencil.  Every (shift, column) pair is its own Krylov space; the
// kernels below hold the batched pieces of one cycle:
//   * projections h_i = v_i^H w, i <= j (classical Gram-Schmidt, applied
//     twice by the caller), as partial sums over row chunks and their total,
//     accumulated into column j of the Hessenberg matrix;
//   * the update w -= sum_i v_i h_i;
//   * the small least-squares problem min || beta e_1 - H y || per column by
//     Givens rotations, and the correction d = sum_i v_i y_i.
// The Krylov blocks V_i are laid out like every other block, (n_omega, k, n)
// complex, vstride complex elements apart.
#include "rr_internal.h"

namespace rr {

namespace {

constexpr int kGsChunkRows = 2048;

__device__ __forceinline__ double2 cmul_conj(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// partial[((w*k + c)*nchunk + chunk)*M1 + i] = sum over the chunk of conj(V_i) x
__global__ __launch_bounds__(256) void k_gs_dots_partial(int64_t n, int k, int j, int M1,
                                                         int64_t vstride, const double2* V,
                                                         const double2* x, int nchunk,
                                                         double2* partial,
                                                         const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ double red[2][4];
  const int chunk = blockIdx.x, c = blockIdx.y, w = blockIdx.z;
  const int64_t col = ((int64_t)w * k + c) * n;
  const int64_t r0 = (int64_t)chunk * kGsChunkRows, r1 = min(n, r0 + kGsChunkRows);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double2* out = partial + (((int64_t)w * k + c) * nchunk + chunk) * M1;
  for (int i = 0; i <= j; i++) {
    const double2* v = V + i * vstride + col;
    double sr = 0, si = 0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
      double2 p = cmul_conj(v[r], x[col + r]);
      sr += p.x;
      si += p.y;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      red[0][wave] = sr;
      red[1][wave] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      out[i] = make_double2(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                            red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    __syncthreads();
  }
}

// h[(w*k + c)*M1 + i] = sum over chunks; H[((w*k + c)*M1 + i)*m + j] += h
__global__ void k_gs_dots_final(int N, int j, int M1, int m, int nchunk, const double2* partial,
                                double2* h, double2* H, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int q = blockIdx.x;  // column (w*k + c)
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    double2 s = make_double2(0, 0);
    for (int ch = 0; ch < nchunk; ch++) {
      double2 p = partial[((int64_t)q * nchunk + ch) * M1 + i];
      s.x += p.x;
      s.y += p.y;
    }
    h[(int64_t)q * M1 + i] = s;
    double2* e = H + ((int64_t)q * M1 + i) * m + j;
    *e = make_double2(e->x + s.x, e->y + s.y);
  }
  (void)N;
}

// x -= sum_{i <= j} V_i h_i
__global__ __launch_bounds__(256) void k_gs_update(int64_t n, int k, int j, int M1,
                                                   int64_t vstride, const double2* V,
                                                   const double2* h, double2* x,
                                                   const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int c = blockIdx.y, w = blockIdx.z;
  if (r >= n) return;
  const int64_t q = (int64_t)w * k + c, off = q * n + r;
  double2 acc = x[off];
  for (int i = 0; i <= j; i++) {
    const double2 hv = h[q * M1 + i], v = V[i * vstride + off];
    acc.x -= v.x * hv.x - v.y * hv.y;
    acc.y -= v.x * hv.y + v.y * hv.x;
  }
  x[off] = acc;
}

// H[j+1][j] = norm (the norm of the new Krylov vector before its scaling)
__global__ void k_store_subdiag(int N, int j, int M1, int m, const double* norm, double2* H,
                                const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  H[((int64_t)q * M1 + j + 1) * m + j] = make_double2(norm[q], 0.0);
}

// Per column: the Givens QR of the (m+1) x m Hessenberg matrix (in place),
// g = Q^H beta e_1, then y = R^-1 g[0..m-1] (a zero diagonal, a breakdown
// column, gives y_j = 0).  Rotation on (a, b): c = |a| / rho,
// s = (a / |a|) conj(b) / rho, rho = sqrt(|a|^2 + |b|^2), so that
// (c a + s b, -conj(s) a + c b) = ((a / |a|) rho, 0).
__global__ void k_gmres_ls(int N, int m, int M1, const double* beta, double2* H, double2* y,
                           const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N) return;
  double2* Hq = H + (int64_t)q * M1 * m;
  double2* yq = y + (int64_t)q * m;
  double2 g[kGmresMaxRestart + 1];
  double cs[kGmresMaxRestart];
  double2 sn[kGmresMaxRestart];
  for (int i = 0; i <= m; i++) g[i] = make_double2(0, 0);
  g[0] = make_double2(beta[q], 0.0);
  for (int jj = 0; jj < m; jj++) {
    for (int i = 0; i < jj; i++) {  // earlier rotations on column jj
      double2 a = Hq[i * m + jj], b = Hq[(i + 1) * m + jj];
      double2 s = sn[i];
      double c = cs[i];
      Hq[i * m + jj] = make_double2(c * a.x + s.x * b.x - s.y * b.y, c * a.y + s.x * b.y + s.y * b.x);
      Hq[(i + 1) * m + jj] = make_double2(-(s.x * a.x + s.y * a.y) + c * b.x,
                                          -(s.x * a.y - s.y * a.x) + c * b.y);
    }
    double2 a = Hq[jj * m + jj], b = Hq[(jj + 1) * m + jj];
    double aa = sqrt(a.x * a.x + a.y * a.y), bb = sqrt(b.x * b.x + b.y * b.y);
    double rho = sqrt(aa * aa + bb * bb);
    double c;
    double2 s;
    if (rho == 0.0) {
      c = 1.0;
      s = make_double2(0, 0);
    } else if (aa == 0.0) {
      c = 0.0;
      s = make_double2(b.x / bb, -b.y / bb);  // conj(b) / |b|
    } else {
      c = aa / rho;
      double2 ph = make_double2(a.x / aa, a.y / aa);
      s = make_double2((ph.x * b.x + ph.y * b.y) / rho, (ph.y * b.x - ph.x * b.y) / rho);
    }
    cs[jj] = c;
    sn[jj] = s;
    Hq[jj * m + jj] = make_double2(c * a.x + s.x * b.x - s.y * b.y, c * a.y + s.x * b.y + s.y * b.x);
    Hq[(jj + 1) * m + jj] = make_double2(0, 0);
    double2 g0 = g[jj], g1 = g[jj + 1];
    g[jj] = make_double2(c * g0.x + s.x * g1.x - s.y * g1.y, c * g0.y + s.x * g1.y + s.y * g1.x);
    g[jj + 1] = make_double2(-(s.x * g0.x + s.y * g0.y) + c * g1.x,
                             -(s.x * g0.y - s.y * g0.x) + c * g1.y);
  }
  for (int i = m - 1; i >= 0; i--) {
    double2 t = g[i];
    for (int l = i + 1; l < m; l++) {
      double2 h = Hq[i * m + l], v = yq[l];
      t.x -= h.x * v.x - h.y * v.y;
      t.y -= h.x * v.y + h.y * v.x;
    }
    double2 d = Hq[i * m + i];
    double dd = d.x * d.x + d.y * d.y;
    yq[i] = dd == 0.0 ? make_double2(0, 0)
                      : make_double2((t.x * d.x + t.y * d.y) / dd, (t.y * d.x - t.x * d.y) / dd);
  }
}

// out = sum_{i < m} V_i y_i
__global__ __launch_bounds__(256) void k_gmres_combine(int64_t n, int k, int m, int64_t vstride,
                                                       const double2* V, const double2* y,
                                                       double2* out, const uint32_t* skip) {
  if (skip && __hip_atomic_load(skip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int c = blockIdx.y, w = blockIdx.z;
  if (r >= n) return;
  const int64_t q = (int64_t)w * k + c, off = q * n + r;
  double2 acc = make_double2(0, 0);
  for (int i = 0; i < m; i++) {
    const double2 yv = y[q * m + i], v = V[i * vstride + off];
    acc.x += v.x * yv.x - v.y * yv.y;
    acc.y += v.x * yv.y + v.y * yv.x;
  }
  out[off] = acc;
}

}  // namespace

int gmres_nchunk(int64_t n) { return (int)((n + kGsChunkRows - 1) / kGsChunkRows); }

hipError_t launch_gs_project(int64_t n, int n_omega, int k, int j, const GmresWs& g,
                             double* x, const uint32_t* skip, hipStream_t s) {
  const int M1 = g.m + 1, nc = gmres_nchunk(n), N = n_omega * k;
  const int64_t vstride = (int64_t)n_omega * k * n;
  hipLaunchKernelGGL(k_gs_dots_partial, dim3(nc, k, n_omega), dim3(256), 0, s, n, k, j, M1,
                     vstride, (const double2*)g.V, (const double2*)x, nc, (double2*)g.partial,
                     skip);
  hipLaunchKernelGGL(k_gs_dots_final, dim3(N), dim3(64), 0, s, N, j, M1, g.m, nc,
                     (const double2*)g.partial, (double2*)g.h, (double2*)g.H, skip);
  hipLaunchKernelGGL(k_gs_update, dim3((unsigned)((n + 255) / 256), k, n_omega), dim3(256), 0, s,
                     n, k, j, M1, vstride, (const double2*)g.V, (const double2*)g.h, (double2*)x,
                     skip);
  return hipGetLastError();
}

hipError_t launch_store_subdiag(int n_omega, int k, int j, const GmresWs& g, const double* norm,
                                const uint32_t* skip, hipStream_t s) {
  const int N = n_omega * k;
  hipLaunchKernelGGL(k_store_subdiag, dim3((N + 63) / 64), dim3(64), 0, s, N, j, g.m + 1, g.m,
                     norm, (double2*)g.H, skip);
  return hipGetLastError();
}

hipError_t launch_gmres_finish(int64_t n, int n_omega, int k, const GmresWs& g, double* out,
                               const uint32_t* skip, hipStream_t s) {
  const int N = n_omega * k;
  hipLaunchKernelGGL(k_gmres_ls, dim3((N + 63) / 64), dim3(64), 0, s, N, g.m, g.m + 1,
                     (const double*)g.beta, (double2*)g.H, (double2*)g.y, skip);
  hipLaunchKernelGGL(k_gmres_combine, dim3((unsigned)((n + 255) / 256), k, n_omega), dim3(256),
                     0, s, n, k, g.m, (int64_t)n_omega * k * n, (const double2*)g.V,
                     (const double2*)g.y, (double2*)out, skip);
  return hipGetLastError();
}

}  // namespace rr
