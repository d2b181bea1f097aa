// FP64 dense linear algebra for the modal covariance and the estimator.
//
//   zeta = (1/(6N)) sum_i b_i b_i^T                         (eq. linearterm)
//   zeta = L L^T, y = L^-1 alpha, z_s = L^-1 beta_s          (eq. Cholrot)
//   E_s = y.z_s / y.y,  sigma^2 = 6 / y.y                    (eqs. modalest, modalvariance)
//
// The products run on the FP64 matrix cores (v_mfma_f64_16x16x4_f64: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16], accumulator register r is
// D[4 r + l / 16][l % 16], checked on the device).  The sample covariance and the Cholesky's trailing update
// are one lower-triangle tile kernel (64 x 64 tiles, four waves of 32 x 32, 16 k per
// LDS stage).  The Cholesky is right-looking with 64-wide panels: the diagonal block is
// factored in LDS by one workgroup, which also inverts it (W = L_kk^-1, kept in the
// block's unused upper triangle); the panel is then the product A_panel W^T on the matrix
// cores instead of a row-by-row substitution.  A non-positive (or NaN) pivot is recorded
// in flag[0] as 1 + its index; later steps then carry NaN and the host reports ENOTPD.
#include "common.h"

namespace modal {
namespace {

constexpr int NB = 64;

// Factor the diagonal block A[k0:k0+kb, k0:k0+kb] in place (lower triangle) and invert it,
// blocked by 16 so that the dependent chain is 4 x 16 short steps instead of 64 long ones.
// The block is in LDS; for each 16-column sub-block:
//   1. wave 0 factors its 16 x 16 diagonal block D (lane r holds row r in registers; the
//      pivot and the column of each step are broadcast by shuffles, no barrier) and inverts
//      it (lane c forms column c of D^-1);
//   2. the rows below it in the block become A_panel D^-T;
//   3. the trailing rows and columns of the block are updated.
// Then W = L^-1 from the four inverted diagonal blocks, by block distance:
//   W_IJ = -D_I^-1 (sum_{J <= K < I} L_IK W_KJ).
// L goes back to the lower triangle and W's strictly lower part, transposed, to the
// block's upper triangle (A[k0 + c][k0 + q] = W[q][c]).  Rows and columns past kb are an
// identity block.  A non-positive pivot is recorded in flag and turns into NaN.
constexpr int SB = 16;   // sub-block

__global__ __launch_bounds__(256) void k_potrf_diag(int n, double* __restrict__ A, int k0, int kb, int* flag) {
  __shared__ double a[NB][NB + 1];
  __shared__ double Wf[NB][NB + 1];   // W = L^-1 (diagonal blocks first, then the rest)
  __shared__ double T[NB][NB + 1];    // block products of the inverse
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e - r * NB;
    const double v = A[(size_t)(k0 + min(r, kb - 1)) * n + k0 + min(c, kb - 1)];
    a[r][c] = (r < kb && c < kb && c <= r) ? v : (c == r ? 1.0 : 0.0);
    Wf[r][c] = 0.0;
  }
  __syncthreads();
  for (int kk = 0; kk < NB / SB; ++kk) {
    const int c0 = SB * kk;
    if (wv == 0) {   // 1. factor and invert the 16 x 16 diagonal block (lanes 0..15 own rows)
      const int r = lane & (SB - 1);
      double d[SB];
#pragma unroll
      for (int c = 0; c < SB; ++c) d[c] = a[c0 + r][c0 + c];
#pragma unroll
      for (int j = 0; j < SB; ++j) {
        const double p = __shfl(d[j], j);
        const bool ok = p > 0.0;
        if (lane == 0 && !ok && c0 + j < kb) atomicCAS(flag, 0, k0 + c0 + j + 1);
        const double sd = ok ? sqrt(p) : __builtin_nan("");
        const double l = r > j ? d[j] / sd : (r == j ? sd : 0.0);
        d[j] = l;
#pragma unroll
        for (int c = j + 1; c < SB; ++c) d[c] -= l * __shfl(l, c);   // entries past the diagonal are never read
      }
      if (lane < SB) {
#pragma unroll
        for (int c = 0; c < SB; ++c)
          if (c <= r) a[c0 + r][c0 + c] = d[c];
      }
      // column c = r of D^-1: w_q = -(sum_{c <= k < q} L_qk w_k) / L_qq
      double Ld[SB];   // this lane's row of L (for broadcasting L_qk below)
#pragma unroll
      for (int c = 0; c < SB; ++c) Ld[c] = d[c];
      double w[SB];
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < q; ++k) {
          const double lqk = __shfl(Ld[k], q);
          v += k >= r ? lqk * w[k] : 0.0;
        }
        const double lqq = __shfl(Ld[q], q);
        w[q] = q > r ? -v / lqq : (q == r ? 1.0 / lqq : 0.0);
      }
      if (lane < SB) {
#pragma unroll
        for (int q = 0; q < SB; ++q) Wf[c0 + q][c0 + r] = w[q];
      }
    }
    __syncthreads();
    // 2. panel rows below: X[i][j] = sum_{k <= j} a[i][c0 + k] W_D[j][k]
    const int r0 = c0 + SB, nr = NB - r0;
    double xo[3];
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      xo[u] = 0.0;
      if (e < nr * SB) {
        const int i = r0 + e / SB, j = e % SB;
        double v = 0.0;
        for (int k = 0; k <= j; ++k) v += a[i][c0 + k] * Wf[c0 + j][c0 + k];
        xo[u] = v;
      }
    }
    __syncthreads();
    for (int u = 0; u < 3; ++u) {
      const int e = t + 256 * u;
      if (e < nr * SB) a[r0 + e / SB][c0 + e % SB] = xo[u];
    }
    __syncthreads();
    // 3. trailing update inside the block: a[i][j] -= sum_k a[i][c0 + k] a[j][c0 + k], r0 <= j <= i
    for (int e = t; e < nr * nr; e += 256) {
      const int i = r0 + e / nr, j = r0 + e % nr;
      if (j <= i) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < SB; ++k) v += a[i][c0 + k] * a[j][c0 + k];
        a[i][j] -= v;
      }
    }
    __syncthreads();
  }
  // the off-diagonal blocks of W, by block distance
  for (int dist = 1; dist < NB / SB; ++dist) {
    const int nbk = NB / SB - dist;   // blocks (I, J = I - dist)
    for (int e = t; e < nbk * SB * SB; e += 256) {   // T_IJ = sum_{J <= K < I} L_IK W_KJ
      const int b = e / (SB * SB), rc = e - b * SB * SB, I = b + dist, J = b;
      const int i = SB * I + rc / SB, j = SB * J + rc % SB;
      double v = 0.0;
      for (int k = SB * J; k < SB * I; ++k) v += a[i][k] * Wf[k][j];
      T[i][j] = v;
    }
    __syncthreads();
    for (int e = t; e < nbk * SB * SB; e += 256) {   // W_IJ = -D_I^-1 T_IJ
      const int b = e / (SB * SB), rc = e - b * SB * SB, I = b + dist, J = b;
      const int i = SB * I + rc / SB, j = SB * J + rc % SB;
      double v = 0.0;
      for (int k = SB * I; k <= i; ++k) v += Wf[i][k] * T[k][j];
      Wf[i][j] = -v;
    }
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e / NB, c = e - r * NB;
    if (r < kb && c < kb) A[(size_t)(k0 + r) * n + k0 + c] = c <= r ? a[r][c] : Wf[c][r];
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

// One step of the blocked forward substitution with the inverted diagonal blocks that
// k_potrf_diag leaves in the upper triangles: for the right-hand sides r (rows of B
// [nrhs][n]), y_r = W b_r[k0:k0+kb] (W = L_kk^-1), written to Y by workgroup 0; the other
// workgroups each form the same y (a 64 x 64 product, cheaper than a second launch) and
// update their 256 rows below: B[r][i] -= sum_c L[i][k0 + c] y_r[c].  B's block rows are
// only read, so no workgroup writes what another still reads.
constexpr int TRS_R = 16;   // right-hand sides per workgroup
__global__ __launch_bounds__(256) void k_trsv_inv_step(int n, const double* __restrict__ A, int k0, int kb, int nrhs,
                                                       double* __restrict__ B, double* __restrict__ Y) {
  __shared__ double W[NB][NB + 1];
  __shared__ double b[TRS_R][NB];
  __shared__ double y[TRS_R][NB];
  const int tid = threadIdx.x;
  const int r0 = blockIdx.y * TRS_R, nr = min(TRS_R, nrhs - r0);
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u, i = e / NB, k = e - i * NB;   // W[i][k], k <= i
    const int ic = min(i, kb - 1), kc = min(k, kb - 1);   // clamped into the block
    const double v = A[(size_t)(k0 + min(kc, ic)) * n + k0 + max(kc, ic)];   // L_ii on the diagonal
    W[i][k] = (i < kb && k < kb) ? (k == i ? 1.0 / v : (k < i ? v : 0.0)) : 0.0;
  }
  for (int e = tid; e < TRS_R * NB; e += 256) {
    const int r = e / NB, c = e - r * NB;
    b[r][c] = (r < nr && c < kb) ? B[(size_t)(r0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < TRS_R * NB; e += 256) {
    const int r = e / NB, i = e - r * NB;
    double v = 0.0;
    for (int k = 0; k <= i; ++k) v += W[i][k] * b[r][k];
    y[r][i] = v;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int e = tid; e < TRS_R * NB; e += 256) {
      const int r = e / NB, c = e - r * NB;
      if (r < nr && c < kb) Y[(size_t)(r0 + r) * n + k0 + c] = y[r][c];
    }
    return;
  }
  const int i = k0 + kb + (blockIdx.x - 1) * 256 + tid;
  if (i >= n) return;
  const double* row = A + (size_t)i * n + k0;
  double l[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) l[c] = row[c];   // kb == NB whenever rows remain below
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

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int TK = 16;     // k per LDS stage of the matrix-core update kernel

// Lower-triangle tile update on the matrix cores, tile (bi, bj), bi >= bj:
//   C[i][j] = alpha sum_k P(i, k) P(j, k) (+ C[i][j] when ACCUM),
// with P(i, k) = X[k][i] (COLS: rows of X [K][n] are the samples) or
// P(i, k) = X[(r0 + i) ld + k] (rows of a panel).  Rows and columns start at r0 for C.
// MIRROR: the upper triangle gets the same values (a symmetric result).
template <int TT, bool COLS, bool ACCUM, bool MIRROR>
__global__ __launch_bounds__(256) void k_tile_update(int n, int K, int r0, const double* __restrict__ X, int ld,
                                                     double alpha, double* __restrict__ C) {
  constexpr int WT = TT / 2, MT = WT / 16;   // wave tile, 16 x 16 MFMA tiles per wave side
  constexpr int NL = TK * TT / 256;           // staged values per thread and operand
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;   // whole workgroup, before any barrier
  const int i0 = r0 + bi * TT, j0 = r0 + bj * TT;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int wr = wv >> 1, wc = wv & 1, l16 = lane & 15, kq = lane >> 4;
  __shared__ double Pi[TK][TT + 1];
  __shared__ double Pj[TK][TT + 1];
  // this thread's outputs; with ACCUM their old values are loaded first and stay in flight
  // through the contraction (indices clamped, the loads unconditional)
  double cold[MT][MT][4];
#pragma unroll
  for (int ta = 0; ta < MT; ++ta)
#pragma unroll
    for (int tb = 0; tb < MT; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = min(i0 + WT * wr + 16 * ta + 4 * r + kq, n - 1), j = min(j0 + WT * wc + 16 * tb + l16, n - 1);
        cold[ta][tb][r] = ACCUM ? C[(size_t)i * n + j] : 0.0;
      }
  d4 acc[MT][MT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < MT; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // the next stage's operands are loaded into registers while this stage multiplies
  double pi[NL], pj[NL];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = tid + 256 * u;
      int kk, c;
      if (COLS) { kk = e / TT; c = e - kk * TT; }   // consecutive threads: consecutive columns of X
      else { c = e / TK; kk = e - c * TK; }          // consecutive threads: consecutive k of a row
      const int k = k0 + kk, kc = min(k, K - 1), ic = min(i0 + c, n - 1), jc = min(j0 + c, n - 1);
      const double vi = COLS ? X[(size_t)kc * ld + ic] : X[(size_t)ic * ld + kc];
      const double vj = COLS ? X[(size_t)kc * ld + jc] : X[(size_t)jc * ld + kc];
      pi[u] = (k < K && i0 + c < n) ? vi : 0.0;
      pj[u] = (k < K && j0 + c < n) ? vj : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = tid + 256 * u;
      int kk, c;
      if (COLS) { kk = e / TT; c = e - kk * TT; }
      else { c = e / TK; kk = e - c * TK; }
      Pi[kk][c] = pi[u];
      Pj[kk][c] = pj[u];
    }
    __syncthreads();
    if (k0 + TK < K) load(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kk = 4 * ks + kq;
      double a[MT], b[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        a[t] = Pi[kk][WT * wr + 16 * t + l16];
        b[t] = Pj[kk][WT * wc + 16 * t + l16];
      }
#pragma unroll
      for (int ta = 0; ta < MT; ++ta)
#pragma unroll
        for (int tb = 0; tb < MT; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ta = 0; ta < MT; ++ta)
#pragma unroll
    for (int tb = 0; tb < MT; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + WT * wr + 16 * ta + 4 * r + kq, j = j0 + WT * wc + 16 * tb + l16;
        if (i < n && j < n && j <= i) {
          const double v = cold[ta][tb][r] + alpha * acc[ta][tb][r];
          C[(size_t)i * n + j] = v;
          if (MIRROR && j < i) C[(size_t)j * n + i] = v;
        }
      }
}

// Panel: rows i >= k0 + kb, A[i, k0:k0+kb] <- A[i, k0:k0+kb] W^T with W = L_kk^-1, whose
// strictly lower part k_potrf_diag left transposed in the block's upper triangle and
// whose diagonal is 1 / L_jj.  64 rows per workgroup, four waves of 32 x 32.
__global__ __launch_bounds__(256) void k_panel_mfma(int n, double* __restrict__ A, int k0, int kb) {
  __shared__ double Ar[NB][NB + 1];   // the workgroup's panel rows
  __shared__ double Wt[NB][NB + 1];   // Wt[k][c] = W[c][k]
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int rbase = k0 + kb + blockIdx.x * NB;
  // loads unconditional (clamped indices, values selected after); kb == NB for a panel
#pragma unroll
  for (int u = 0; u < NB * NB / 256; ++u) {
    const int e = tid + 256 * u;
    const int r = e / NB, c = e - r * NB;
    const double av = A[(size_t)min(rbase + r, n - 1) * n + k0 + c];
    // Wt[k][c] = W[c][k]: W[c][k] for k < c sits at A[k0 + k][k0 + c]; W[c][c] = 1 / L_cc
    const int k = r;
    const double wv_ = A[(size_t)(k0 + min(k, c)) * n + k0 + c];
    Ar[r][c] = rbase + r < n ? av : 0.0;
    Wt[k][c] = k == c ? 1.0 / wv_ : (k < c ? wv_ : 0.0);
  }
  __syncthreads();
  const int wr = wv >> 1, wc = wv & 1;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int ks = 0; ks < NB / 4; ++ks) {
    const int kk = 4 * ks + kq;
    double a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = Ar[32 * wr + 16 * t + l16][kk];
      b[t] = Wt[kk][32 * wc + 16 * t + l16];
    }
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
  }
  // every read of the rows is done (the stores below overwrite them)
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = rbase + 32 * wr + 16 * ta + 4 * r + kq, c = 32 * wc + 16 * tb + l16;
        if (i < n && c < kb) A[(size_t)i * n + k0 + c] = acc[ta][tb][r];
      }
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
  constexpr int T = 64;
  const int nb = (n + T - 1) / T;
  hipLaunchKernelGGL((k_tile_update<T, true, false, true>), dim3(nb, nb), dim3(256), 0, st, n, N, 0, B, n, scale, Z);
  return hipGetLastError();
}

hipError_t launch_copy_lower(int n, const double* src, double* dst, hipStream_t st) {
  const size_t tot = (size_t)n * n;
  hipLaunchKernelGGL(k_copy_lower, dim3((tot + 255) / 256), dim3(256), 0, st, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_cholesky_lookahead(int n, double* A, int* flag, hipStream_t st, hipStream_t side, hipEvent_t ev_a,
                                     hipEvent_t ev_p, int nrhs, double* B, double* Y) {
  constexpr int T = 64;
  // A[i][j] -= sum_c A[i][k0 + c] A[j][k0 + c], i >= j >= r0, tile columns [bj0, ...) of the
  // (n - r0)-square trailing grid; nbx tile columns
  auto update = [&](int k0, int kb, int r0, int nbx, hipStream_t s) {
    const int nb = (n - r0 + T - 1) / T;
    hipLaunchKernelGGL((k_tile_update<T, false, true, false>), dim3(nbx, nb), dim3(256), 0, s, n, kb, r0, A + k0, n,
                       -1.0, A);
  };
  // Factor the block column [k, k + 2 NB) (its two NB-wide halves), all updates from the
  // columns left of k applied: diagonal block and panel of the first half, its update of the
  // second half's columns, then the second half's diagonal block and panel.
  auto factor2 = [&](int k, hipStream_t s) {
    const int kb = n - k < NB ? n - k : NB;
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, n, A, k, kb, flag);
    if (n - k - kb > 0) hipLaunchKernelGGL(k_panel_mfma, dim3((n - k - kb + NB - 1) / NB), dim3(256), 0, s, n, A, k, kb);
    const int k2 = k + NB;
    if (k2 < n) {
      update(k, NB, k2, 1, s);
      const int kb2 = n - k2 < NB ? n - k2 : NB;
      hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, n, A, k2, kb2, flag);
      if (n - k2 - kb2 > 0)
        hipLaunchKernelGGL(k_panel_mfma, dim3((n - k2 - kb2 + NB - 1) / NB), dim3(256), 0, s, n, A, k2, kb2);
    }
  };
  // The solve steps of a factored block column (Y_k = W_kk B_k, and the rows below updated
  // with its panel): they need only that block column, so they run on the stream that
  // factored it, after the event that releases the main stream, and overlap the trailing
  // updates instead of following the whole factorization.
  auto solve2 = [&](int k, hipStream_t s) {
    for (int kk = k; kk < k + 2 * NB && kk < n; kk += NB) {
      const int kb = n - kk < NB ? n - kk : NB, rem = n - kk - kb;
      hipLaunchKernelGGL(k_trsv_inv_step, dim3(1 + (rem + 255) / 256, (nrhs + TRS_R - 1) / TRS_R), dim3(256), 0, s, n,
                         A, kk, kb, nrhs, B, Y);
    }
  };
  // The trailing updates take both halves of a factored block column at once (K = 2 NB), so
  // each trailing tile is read and written once per 2 NB columns instead of per NB.
  factor2(0, st);
  if (nrhs > 0) solve2(0, st);
  for (int k0 = 0; k0 + 2 * NB < n; k0 += 2 * NB) {
    const int k1 = k0 + 2 * NB;   // the next block column (both halves of [k0, k1) are NB wide)
    const int w1 = n - k1 < 2 * NB ? n - k1 : 2 * NB;
    const int nb1 = (w1 + T - 1) / T;   // its tile columns
    // the next block column's tiles first, then the rest of the trailing matrix
    update(k0, 2 * NB, k1, nb1, st);
    hipError_t e = hipEventRecord(ev_a, st);
    if (e != hipSuccess) return e;
    if (n - k1 > 2 * NB) update(k0, 2 * NB, k1 + 2 * NB, (n - k1 - 2 * NB + T - 1) / T, st);
    if ((e = hipStreamWaitEvent(side, ev_a, 0)) != hipSuccess) return e;
    factor2(k1, side);
    if ((e = hipEventRecord(ev_p, side)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, ev_p, 0)) != hipSuccess) return e;
    if (nrhs > 0) solve2(k1, side);   // in order on the side stream, after ev_p
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (nrhs > 0 && n > 2 * NB) {   // the last solve steps ran on the side stream
    hipError_t e = hipEventRecord(ev_p, side);
    if (e != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(st, ev_p, 0)) != hipSuccess) return e;
  }
  return hipGetLastError();
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
