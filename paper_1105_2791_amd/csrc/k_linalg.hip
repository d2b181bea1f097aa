// FP64 dense linear algebra for the modal covariance and the estimator.
//
//   zeta = (1/(6N)) sum_i b_i b_i^T                         (eq. linearterm)
//   zeta = L L^T, y = L^-1 alpha, z_s = L^-1 beta_s          (eq. Cholrot)
//   E_s = y.z_s / y.y,  sigma^2 = 6 / y.y                    (eqs. modalest, modalvariance)
//
// MI355X runs FP64 FMA on the vector ALUs at the same rate as its FP64 matrix
// cores (78.6 TFLOP/s each), so these kernels are register-tiled VALU code:
// 64x64 output tiles, 4x4 per thread, k-chunks of 16 staged in LDS.
// The Cholesky is right-looking with 64-wide panels: diagonal block factored in
// LDS by one workgroup, panel solved row-per-thread, trailing lower triangle
// updated tile by tile.  A non-positive (or NaN) pivot is recorded in flag[0]
// as 1 + its index; later steps then carry NaN and the host reports ENOTPD.
#include "common.h"

namespace modal {
namespace {

constexpr int NB = 64;
constexpr int KC = 16;

// C[i][j] = alpha * sum_k X[k][i] X[k][j] over rows k of X [N][n], for the
// tile (bi, bj), bi >= bj; mirrored into the upper triangle.
__global__ __launch_bounds__(256) void k_syrk_t(int n, int N, const double* __restrict__ X, double alpha,
                                                double* __restrict__ C) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  const int i0 = bi * NB, j0 = bj * NB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ double Xi[KC][NB + 1];
  __shared__ double Xj[KC][NB + 1];
  double acc[4][4] = {};
  for (int k0 = 0; k0 < N; k0 += KC) {
    for (int e = threadIdx.x; e < KC * NB; e += 256) {
      const int kk = e / NB, c = e - kk * NB;
      const int k = k0 + kk;
      Xi[kk][c] = (k < N && i0 + c < n) ? X[(size_t)k * n + i0 + c] : 0.0;
      Xj[kk][c] = (k < N && j0 + c < n) ? X[(size_t)k * n + j0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Xi[kk][ty * 4 + u];
        b[u] = Xj[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
      if (i < n && j < n) {
        C[(size_t)i * n + j] = alpha * acc[u][v];
        C[(size_t)j * n + i] = alpha * acc[u][v];
      }
    }
}

// Factor the diagonal block A[k0:k0+kb, k0:k0+kb] in place (lower triangle).
__global__ __launch_bounds__(256) void k_potrf_diag(int n, double* __restrict__ A, int k0, int kb, int* flag) {
  __shared__ double a[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, j = e - i * NB;
    a[i][j] = (i < kb && j < kb) ? A[(size_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (threadIdx.x == 0) {
      const double d = a[j][j];
      if (!(d > 0.0)) {
        atomicCAS(flag, 0, k0 + j + 1);
        a[j][j] = __builtin_nan("");
      } else {
        a[j][j] = sqrt(d);
      }
    }
    __syncthreads();
    const double djj = a[j][j];
    for (int i = j + 1 + threadIdx.x; i < kb; i += 256) a[i][j] /= djj;
    __syncthreads();
    // trailing update inside the block: a[i][c] -= a[i][j] a[c][j], j < c <= i
    for (int e = threadIdx.x; e < kb * kb; e += 256) {
      const int i = e / kb, c = e - i * kb;
      if (c > j && i >= c) a[i][c] -= a[i][j] * a[c][j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kb * kb; e += 256) {
    const int i = e / kb, j = e - i * kb;
    if (j <= i) A[(size_t)(k0 + i) * n + k0 + j] = a[i][j];
  }
}

// Panel: rows i >= k0 + kb, A[i, k0:k0+kb] <- A[i, k0:k0+kb] L_kk^-T (one row per thread).
__global__ __launch_bounds__(64) void k_trsm_panel(int n, double* __restrict__ A, int k0, int kb) {
  __shared__ double L[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += 64) {
    const int i = e / NB, j = e - i * NB;
    L[i][j] = (i < kb && j < kb) ? A[(size_t)(k0 + i) * n + k0 + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int i = k0 + kb + blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  double x[NB];
  double* row = A + (size_t)i * n + k0;
#pragma unroll
  for (int c = 0; c < NB; ++c) x[c] = c < kb ? row[c] : 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    double v = x[c];
#pragma unroll
    for (int cp = 0; cp < c; ++cp) v -= x[cp] * L[c][cp];
    x[c] = v / L[c][c];
  }
#pragma unroll
  for (int c = 0; c < NB; ++c)
    if (c < kb) row[c] = x[c];
}

// Trailing update of the lower triangle: A[i][j] -= sum_c A[i][k0+c] A[j][k0+c], i >= j >= k1.
__global__ __launch_bounds__(256) void k_chol_update(int n, double* __restrict__ A, int k0, int kb) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  const int k1 = k0 + kb;
  const int i0 = k1 + bi * NB, j0 = k1 + bj * NB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ double Pi[KC][NB + 1];
  __shared__ double Pj[KC][NB + 1];
  double acc[4][4] = {};
  for (int c0 = 0; c0 < kb; c0 += KC) {
    for (int e = threadIdx.x; e < KC * NB; e += 256) {
      const int r = e / KC, cc = e - r * KC;
      const int c = c0 + cc;
      Pi[cc][r] = (c < kb && i0 + r < n) ? A[(size_t)(i0 + r) * n + k0 + c] : 0.0;
      Pj[cc][r] = (c < kb && j0 + r < n) ? A[(size_t)(j0 + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < KC; ++cc) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Pi[cc][ty * 4 + u];
        b[u] = Pj[cc][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
      if (i < n && j < n && j <= i) A[(size_t)i * n + j] -= acc[u][v];
    }
}

// Forward substitution on the diagonal block for every right-hand side row.
__global__ __launch_bounds__(64) void k_trsv_diag(int n, const double* __restrict__ A, int k0, int kb,
                                                  double* __restrict__ B) {
  __shared__ double L[NB][NB + 1];
  __shared__ double y[NB];
  for (int e = threadIdx.x; e < NB * NB; e += 64) {
    const int i = e / NB, j = e - i * NB;
    L[i][j] = (i < kb && j < kb) ? A[(size_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  double* b = B + (size_t)blockIdx.x * n + k0;
  if (threadIdx.x < kb) y[threadIdx.x] = b[threadIdx.x];
  __syncthreads();
  for (int c = 0; c < kb; ++c) {
    if (threadIdx.x == 0) y[c] = y[c] / L[c][c];
    __syncthreads();
    const int i = threadIdx.x;
    if (i > c && i < kb) y[i] -= L[i][c] * y[c];
    __syncthreads();
  }
  if (threadIdx.x < kb) b[threadIdx.x] = y[threadIdx.x];
}

// B[r][i] -= sum_c A[i][k0+c] B[r][k0+c] for i >= k0 + kb, all rows r < nrhs (chunks of 64).
__global__ __launch_bounds__(256) void k_trsv_update(int n, const double* __restrict__ A, int k0, int kb, int nrhs,
                                                     double* __restrict__ B) {
  __shared__ double y[64][NB];
  const int r0 = blockIdx.y * 64;
  const int nr = min(64, nrhs - r0);
  for (int e = threadIdx.x; e < 64 * NB; e += 256) {
    const int r = e / NB, c = e - r * NB;
    y[r][c] = (r < nr && c < kb) ? B[(size_t)(r0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  const int i = k0 + kb + blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double l[NB];
  const double* row = A + (size_t)i * n + k0;
#pragma unroll
  for (int c = 0; c < NB; ++c) l[c] = c < kb ? row[c] : 0.0;
  for (int r = 0; r < nr; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < NB; ++c) acc += l[c] * y[r][c];
    B[(size_t)(r0 + r) * n + i] -= acc;
  }
}

// out[0] = y.y, out[1+s] = y.z_s with y = rows[0], z_s = rows[1+s].
__global__ __launch_bounds__(256) void k_dots(int n, const double* __restrict__ rows, double* __restrict__ out) {
  const double* y = rows;
  const double* z = rows + (size_t)blockIdx.x * n;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += y[i] * z[i];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_copy_lower(int n, const double* __restrict__ src, double* __restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const size_t i = e / n, j = e - i * n;
  dst[e] = j <= i ? src[e] : 0.0;
}

}  // namespace

// C[i][k] = B[i][k] - (1/N) sum_j B[j][k] (rows of B [N][n]); one thread per column
__global__ __launch_bounds__(256) void k_center_rows(int n, int N, const double* __restrict__ B,
                                                     double* __restrict__ C) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double m = 0.0;
  for (int i = 0; i < N; ++i) m += B[(size_t)i * n + k];
  m /= N;
  for (int i = 0; i < N; ++i) C[(size_t)i * n + k] = B[(size_t)i * n + k] - m;
}

hipError_t launch_center_rows(int n, int N, const double* B, double* C, hipStream_t st) {
  hipLaunchKernelGGL(k_center_rows, dim3((n + 255) / 256), dim3(256), 0, st, n, N, B, C);
  return hipGetLastError();
}

hipError_t launch_syrk(int n, int N, const double* B, double scale, double* Z, hipStream_t st) {
  const int nb = (n + NB - 1) / NB;
  hipLaunchKernelGGL(k_syrk_t, dim3(nb, nb), dim3(256), 0, st, n, N, B, scale, Z);
  return hipGetLastError();
}

hipError_t launch_copy_lower(int n, const double* src, double* dst, hipStream_t st) {
  const size_t tot = (size_t)n * n;
  hipLaunchKernelGGL(k_copy_lower, dim3((tot + 255) / 256), dim3(256), 0, st, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_cholesky(int n, double* A, int* flag, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = n - k0 < NB ? n - k0 : NB;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, n, A, k0, kb, flag);
    const int rem = n - k0 - kb;
    if (rem > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3((rem + 63) / 64), dim3(64), 0, st, n, A, k0, kb);
      const int nb = (rem + NB - 1) / NB;
      hipLaunchKernelGGL(k_chol_update, dim3(nb, nb), dim3(256), 0, st, n, A, k0, kb);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_trsm_rows(int n, const double* L, int nrhs, double* B, hipStream_t st) {
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = n - k0 < NB ? n - k0 : NB;
    hipLaunchKernelGGL(k_trsv_diag, dim3(nrhs), dim3(64), 0, st, n, L, k0, kb, B);
    const int rem = n - k0 - kb;
    if (rem > 0)
      hipLaunchKernelGGL(k_trsv_update, dim3((rem + 255) / 256, (nrhs + 63) / 64), dim3(256), 0, st, n, L, k0, kb,
                         nrhs, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_estimator(int n, const double* rows, const double* /*unused*/, int S, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dots, dim3(S + 1), dim3(256), 0, st, n, rows, out);
  return hipGetLastError();
}

}  // namespace modal
