// Truncated orthonormal mode frame: diagonally pivoted, truncated Cholesky of a symmetric
// positive semi-definite n x n matrix (the ideal covariance zeta0 of the separable modes).
//
// Sec. II works in an orthonormal basis truncated to the modes that span the space of
// interest, and eq. (Cholrot) re-orthonormalises by a Cholesky factor.  The separable
// q-product modes are linearly dependent in floating point for large P (zeta0 is singular
// to FP64), so the factor is pivoted and truncated:
//
//   Pi^T zeta0 Pi ~= L L^T,  L = [L11; L21] (n x k),  L11 lower triangular (k x k),
//
// taking at step j the mode with the largest remaining diagonal d and stopping once
// d_max <= tol * max(diag zeta0).  The frame T = L11^-1 [I_k 0] Pi^T is orthonormal under
// zeta0 (T zeta0 T^T = I_k), and eqs. (modalest, modalvariance) restricted to the k kept
// modes are the estimator in that frame.
//
// Left-looking, one column per step, three launches a step:
//   k_pivot   one workgroup: argmax of d over the modes not yet kept; at step 0 the value
//             is max(diag zeta0), the scale of the stopping rule; stores the pivot or the
//             stop (k = j);
//   k_colpart split dot products: part[ks][i] = sum over t in split ks of Lc[t][i] Lc[t][p]
//             (Lc holds the columns of L, one contiguous row of n per column; threads run
//             over i, so the loads are coalesced);
//   k_colfin  Lc[j][i] = (zeta[i][p] - sum_ks part[ks][i]) / sqrt(d_p), d_i -= Lc[j][i]^2;
//             rows already kept get 0 (they lie on the triangle).
// The host checks the stop flag every 64 steps; steps after the stop return at once.
#include "common.h"

namespace modal {
namespace {

constexpr int KSPLIT = 16;    // splits of the dot products over earlier columns
constexpr int CT = 256;       // threads per workgroup of the column kernels

struct FrameState {
  int k;          // number of kept modes once stopped (else the step count)
  int done;       // stop flag
  int piv;        // this step's pivot
  int pad;
  double dmax;    // max diag zeta0
  double s;       // sqrt of the pivot's remaining diagonal
};

__global__ void k_frame_init(int n, const double* __restrict__ Z, double* __restrict__ d, int* __restrict__ kept,
                             FrameState* stt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    d[i] = Z[(size_t)i * n + i];
    kept[i] = 0;
  }
  if (i == 0) {
    stt->k = 0;
    stt->done = 0;
    stt->piv = 0;
    stt->dmax = 0.0;
    stt->s = 0.0;
  }
}

__global__ __launch_bounds__(1024) void k_pivot(int n, int j, double tol, const double* __restrict__ d,
                                                int* __restrict__ kept, int* __restrict__ perm, FrameState* stt) {
  if (stt->done) return;
  __shared__ double bv[1024];
  __shared__ int bi[1024];
  double best = -1.0;
  int arg = -1;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (!kept[i] && d[i] > best) {   // NaN never wins: the comparison is false
      best = d[i];
      arg = i;
    }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double o = bv[threadIdx.x + h];
      const int oi = bi[threadIdx.x + h];
      // largest value; ties go to the smaller index (deterministic)
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi >= 0 && (bi[threadIdx.x] < 0 || oi < bi[threadIdx.x]))) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double v = bv[0];
    const int p = bi[0];
    if (j == 0) stt->dmax = v > 0.0 ? v : 0.0;
    if (p < 0 || !(v > tol * stt->dmax) || !(v > 0.0)) {
      stt->done = 1;
      stt->k = j;
    } else {
      perm[j] = p;
      kept[p] = 1;
      stt->piv = p;
      stt->s = sqrt(v);
      stt->k = j + 1;
    }
  }
}

// part[ks][i] = sum_{t in split ks, t < j} Lc[t][i] * Lc[t][p]
__global__ __launch_bounds__(CT) void k_colpart(int n, int j, const double* __restrict__ Lc, double* __restrict__ part,
                                                const FrameState* stt) {
  if (stt->done) return;
  const int i = blockIdx.x * CT + threadIdx.x;
  const int ks = blockIdx.y;
  const int p = stt->piv;
  const int per = (j + KSPLIT - 1) / KSPLIT;
  const int t0 = ks * per, t1 = min(j, t0 + per);
  __shared__ double lp[CT];
  double acc = 0.0;
  for (int c0 = t0; c0 < t1; c0 += CT) {
    const int m = min(CT, t1 - c0);
    if (threadIdx.x < m) lp[threadIdx.x] = Lc[(size_t)(c0 + threadIdx.x) * n + p];
    __syncthreads();
    if (i < n)
      for (int t = 0; t < m; ++t) acc += Lc[(size_t)(c0 + t) * n + i] * lp[t];
    __syncthreads();
  }
  if (i < n) part[(size_t)ks * n + i] = acc;
}

__global__ __launch_bounds__(CT) void k_colfin(int n, int j, const double* __restrict__ Z, const double* __restrict__ part,
                                               const int* __restrict__ kept, double* __restrict__ Lc,
                                               double* __restrict__ d, const FrameState* stt) {
  if (stt->done) return;
  const int i = blockIdx.x * CT + threadIdx.x;
  if (i >= n) return;
  const int p = stt->piv;
  const double s = stt->s;
  double v;
  if (i == p) {
    v = s;                             // (d_p) / sqrt(d_p)
  } else if (kept[i]) {
    v = 0.0;                           // an earlier pivot: on the triangle
  } else {
    double acc = Z[(size_t)i * n + p];
    for (int ks = 0; ks < KSPLIT; ++ks) acc -= part[(size_t)ks * n + i];
    v = acc / s;
  }
  Lc[(size_t)j * n + i] = v;
  d[i] = (i == p || kept[i]) ? 0.0 : d[i] - v * v;
}

// L11[r][c] = Lc[c][perm[r]] (k x k, row-major, lower triangle; upper zeroed)
__global__ void k_frame_l11(int n, int k, const double* __restrict__ Lc, const int* __restrict__ perm,
                            double* __restrict__ L11) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)k * k) return;
  const int r = (int)(e / k), c = (int)(e % k);
  L11[e] = c <= r ? Lc[(size_t)c * n + perm[r]] : 0.0;
}

// y[r][t] = x[r][perm[t]] for rows r (gather of the kept modes)
__global__ void k_gather_cols(int n, int k, int R, const double* __restrict__ x, const int* __restrict__ perm,
                              double* __restrict__ y) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)R * k) return;
  const int r = (int)(e / k), t = (int)(e % k);
  y[e] = x[(size_t)r * n + perm[t]];
}

// Zk[a][b] = Z[perm[a]][perm[b]]
__global__ void k_gather_sym(int n, int k, const double* __restrict__ Z, const int* __restrict__ perm,
                             double* __restrict__ Zk) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)k * k) return;
  const int a = (int)(e / k), b = (int)(e % k);
  Zk[e] = Z[(size_t)perm[a] * n + perm[b]];
}

}  // namespace

size_t frame_ws_bytes(int n) {
  // columns of L (up to n of n), d, kept flags, split partials, state
  return align256((size_t)n * n * 8) + align256((size_t)n * 8) + align256((size_t)n * 4) +
         align256((size_t)KSPLIT * n * 8) + align256(sizeof(FrameState));
}

hipError_t launch_frame(int n, const double* Z, double tol, int* perm, double* L11, int* k_host, void* ws,
                        hipStream_t st) {
  char* w = static_cast<char*>(ws);
  double* Lc = reinterpret_cast<double*>(w);
  w += align256((size_t)n * n * 8);
  double* d = reinterpret_cast<double*>(w);
  w += align256((size_t)n * 8);
  int* kept = reinterpret_cast<int*>(w);
  w += align256((size_t)n * 4);
  double* part = reinterpret_cast<double*>(w);
  w += align256((size_t)KSPLIT * n * 8);
  FrameState* stt = reinterpret_cast<FrameState*>(w);
  hipLaunchKernelGGL(k_frame_init, dim3((n + 255) / 256), dim3(256), 0, st, n, Z, d, kept, stt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 gpart((n + CT - 1) / CT, KSPLIT), gfin((n + CT - 1) / CT);
  FrameState h{};
  for (int j = 0; j < n; ++j) {
    hipLaunchKernelGGL(k_pivot, dim3(1), dim3(1024), 0, st, n, j, tol, d, kept, perm, stt);
    hipLaunchKernelGGL(k_colpart, gpart, dim3(CT), 0, st, n, j, Lc, part, stt);
    hipLaunchKernelGGL(k_colfin, gfin, dim3(CT), 0, st, n, j, Z, part, kept, Lc, d, stt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((j & 63) == 63 || j == n - 1) {
      if ((e = hipMemcpyAsync(&h, stt, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
      if (h.done) break;
    }
  }
  if (!h.done) {
    if ((e = hipMemcpyAsync(&h, stt, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  }
  const int k = h.k;
  *k_host = k;
  if (k > 0) {
    const size_t kk = (size_t)k * k;
    hipLaunchKernelGGL(k_frame_l11, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, st, n, k, Lc, perm, L11);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipStreamSynchronize(st);
}

hipError_t launch_gather_cols(int n, int k, int R, const double* x, const int* perm, double* y, hipStream_t st) {
  const size_t tot = (size_t)R * k;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, k, R, x, perm, y);
  return hipGetLastError();
}

hipError_t launch_gather_sym(int n, int k, const double* Z, const int* perm, double* Zk, hipStream_t st) {
  const size_t tot = (size_t)k * k;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_sym, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, k, Z, perm, Zk);
  return hipGetLastError();
}

}  // namespace modal
