// Low-rank modal covariance, Sec. III B: zeta ~= I + sum_j b_j b_j^T (eq. ic_bivector
// for one vector, the principal-component form for several).
//
// Noise vectors.  The k leading eigenpairs of the sample covariance
// zeta = B^T B / (6N) (rows of B [N][n] are beta^hat_i, eq. linearterm) are found
// without forming zeta: the N x N Gram matrix G = B B^T / (6N) has the same
// nonzero eigenvalues, and G u = mu u gives zeta (B^T u) = mu (B^T u) with
// |B^T u|^2 = 6 N mu.  A block of kb <= 16 columns is iterated, X <- orth(G X)
// (Cholesky QR applied twice), then one Rayleigh-Ritz step diagonalises
// H = X^T G X by cyclic Jacobi.  b_j = sqrt(max(mu_j - 1, 0)) B^T u_j / sqrt(6 N mu_j),
// signed so that its entry of largest magnitude is positive.
//
// Estimator.  With K = [b_1 .. b_k] and M = I_k + K^T K, Woodbury gives
// x^T zeta^-1 y = x.y - (K^T x)^T M^-1 (K^T y) (eq. ic_bivectorinv for k = 1);
// E_s = alpha^T zeta^-1 beta_s / alpha^T zeta^-1 alpha (eq. modalest).
//
// Rotation by the closed-form Cholesky factor of I + b b^T (Sec. III B).  With
// D_i = 1 + sum_{l <= i} b_l^2 (D_{-1} = 1) and U_i = sum_{j < i} b_j x_j, forward
// substitution with that factor telescopes to
//   y_i = (x_i - b_i U_i / D_{i-1}) sqrt(D_{i-1} / D_i),
// so a rotation is two prefix sums, one workgroup per vector.
//
// All of it is FP64 on the vector ALUs; the Gram matrix (N^2 n / 2 FMAs) is the
// only part with real work, the rest is latency-bound small kernels.
#include "common.h"

#include <cmath>

namespace modal {
namespace {

constexpr int KB = 16;     // iterated block width (max noise vectors plus oversampling)
constexpr int GT = 64;     // Gram output tile
constexpr int GK = 16;     // Gram column chunk staged in LDS
constexpr int GXR = 16;    // rows i of G X per workgroup (N = 1000: 63 x 4 workgroups)
constexpr int GXP = 256 / GXR;   // phases over the rows l of G in a workgroup
constexpr int GXL = 256;   // rows l of G summed per workgroup
constexpr int RC = 256;    // rows staged per chunk in the one-workgroup kernels

constexpr int GKS = 16;    // most column splits of the Gram matrix

// Partial Gram tiles: Gp[ks][tp][64][64] = B_i . B_j over the columns of split ks, for the
// lower tile pair tp = bi (bi + 1) / 2 + bj (bj <= bi).  Splitting the columns gives the
// N = 1000 case (136 tile pairs) about a thousand workgroups; the next chunk's loads are
// issued into registers before this chunk's products.
__global__ __launch_bounds__(256) void k_gram_part(int N, int n, int kc, int ntp, const double* __restrict__ B,
                                                   double* __restrict__ Gp) {
  const int tp = blockIdx.x, ks = blockIdx.y;
  int bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= tp) ++bi;
  const int bj = tp - bi * (bi + 1) / 2;
  const int i0 = bi * GT, j0 = bj * GT;
  const int c_begin = ks * kc, c_end = min(n, c_begin + kc);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ double Bi[GK][GT + 1];
  __shared__ double Bj[GK][GT + 1];
  constexpr int NL = GK * GT / 256;   // elements of each tile chunk per thread (4)
  double pa[NL], pb[NL];
  auto load = [&](int c0) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = threadIdx.x + 256 * u, r = e / GK, c = c0 + (e - r * GK);
      pa[u] = (i0 + r < N && c < c_end) ? B[(size_t)(i0 + r) * n + c] : 0.0;
      pb[u] = (j0 + r < N && c < c_end) ? B[(size_t)(j0 + r) * n + c] : 0.0;
    }
  };
  double acc[4][4] = {};
  if (c_begin < c_end) load(c_begin);
  for (int c0 = c_begin; c0 < c_end; c0 += GK) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = threadIdx.x + 256 * u, r = e / GK, kk = e - r * GK;
      Bi[kk][r] = pa[u];
      Bj[kk][r] = pb[u];
    }
    __syncthreads();
    if (c0 + GK < c_end) load(c0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Bi[kk][ty * 4 + u];
        b[u] = Bj[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
  }
  double* dst = Gp + ((size_t)ks * ntp + tp) * GT * GT;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[(ty * 4 + u) * GT + tx * 4 + v] = acc[u][v];
}

// G[i][j] = G[j][i] = scale * (sum over the splits of the partial tiles), j <= i, in a
// fixed order (deterministic).
__global__ __launch_bounds__(256) void k_gram_reduce(int N, int ntp, int nks, const double* __restrict__ Gp,
                                                     double scale, double* __restrict__ G) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)N * N) return;
  const int i = (int)(e / N), j = (int)(e - (size_t)i * N);
  if (j > i) return;
  const int bi = i / GT, bj = j / GT, tp = bi * (bi + 1) / 2 + bj;
  const size_t o = (size_t)tp * GT * GT + (size_t)(i - bi * GT) * GT + (j - bj * GT);
  double sum = 0.0;
  for (int k = 0; k < nks; ++k) sum += Gp[(size_t)k * ntp * GT * GT + o];
  G[(size_t)i * N + j] = scale * sum;
  G[(size_t)j * N + i] = scale * sum;
}

// column splits of the Gram matrix: about a thousand workgroups, at most GKS, at least one
// GK-column chunk each
int gram_splits_max(int N) {
  const int nt = (N + GT - 1) / GT, ntp = nt * (nt + 1) / 2;
  return std::max(1, std::min(GKS, (1024 + ntp - 1) / ntp));
}
int gram_splits(int N, int n) { return std::max(1, std::min(gram_splits_max(N), (n + GK - 1) / GK)); }

// Starting block: a fixed hash of (i, j) mapped to [-1, 1), columns >= kb zero.
__global__ void k_start_block(int N, int kb, double* __restrict__ X) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * KB) return;
  const int j = e % KB;
  uint64_t z = (uint64_t)e * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;   // SplitMix64 finaliser
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[e] = j < kb ? (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0 : 0.0;
}

// Yp[split][i][j] = sum over l in this split of G[l][i] X[l][j] (G symmetric, so the
// reads G[l][i] are consecutive across the lanes).  X [N][KB].
__global__ __launch_bounds__(256) void k_gx(int N, const double* __restrict__ G, const double* __restrict__ X,
                                            double* __restrict__ Yp) {
  __shared__ double xs[GXL][KB];
  __shared__ double red[GXP][GXR][KB + 1];
  const int i0 = blockIdx.x * GXR, l0 = blockIdx.y * GXL;
  const int ri = threadIdx.x % GXR, ph = threadIdx.x / GXR;
  const int lend = min(N, l0 + GXL);
  for (int e = threadIdx.x; e < GXL * KB; e += 256) {
    const int l = e / KB;
    xs[l][e % KB] = l0 + l < N ? X[(size_t)l0 * KB + e] : 0.0;
  }
  __syncthreads();
  const int i = i0 + ri;
  double acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = 0.0;
  if (i < N)
    for (int l = l0 + ph; l < lend; l += GXP) {
      const double g = G[(size_t)l * N + i];
#pragma unroll
      for (int j = 0; j < KB; ++j) acc[j] = fma(g, xs[l - l0][j], acc[j]);
    }
#pragma unroll
  for (int j = 0; j < KB; ++j) red[ph][ri][j] = acc[j];
  __syncthreads();
  // one thread per (row, column) of the block: the phases added in a fixed order
  const int orow = threadIdx.x / KB, oj = threadIdx.x % KB;
  const int oi = i0 + orow;
  if (orow < GXR && oi < N) {
    double sm = 0.0;
    for (int p = 0; p < GXP; ++p) sm += red[p][orow][oj];
    Yp[((size_t)blockIdx.y * N + oi) * KB + oj] = sm;
  }
}

// C[a][b] = sum_i X[i][a] Y[i][b] (a, b < kb) for one workgroup (Y may be X: then only X
// is staged).  Thread t owns the entry t % kb^2 for the rows of row group t / kb^2; the
// groups' partial sums are added in LDS at the end.
template <int RCT>
__device__ void block_gram(int N, int kb, const double* __restrict__ X, const double* __restrict__ Y,
                           double (*xs)[KB + 1], double (*ys)[KB + 1], double (*C)[KB], double* part) {
  const int tid = threadIdx.x;
  const int kk = kb * kb, ng = 256 / kk;
  const int grp = tid / kk, ent = tid - grp * kk;
  const int a = ent / kb, b = ent - (ent / kb) * kb;
  const bool same = X == Y;
  double c = 0.0;
  for (int r0 = 0; r0 < N; r0 += RCT) {
    for (int e = tid; e < RCT * KB; e += 256) {
      const int r = e / KB, j = e - r * KB;
      xs[r][j] = r0 + r < N ? X[(size_t)(r0 + r) * KB + j] : 0.0;
      if (!same) ys[r][j] = r0 + r < N ? Y[(size_t)(r0 + r) * KB + j] : 0.0;
    }
    __syncthreads();
    if (grp < ng) {
      const double(*yy)[KB + 1] = same ? xs : ys;
      for (int r = grp; r < RCT; r += ng) c = fma(xs[r][a], yy[r][b], c);
    }
    __syncthreads();
  }
  if (grp < ng) part[tid] = c;
  __syncthreads();
  if (tid < kk) {
    double s = 0.0;
    for (int g = 0; g < ng; ++g) s += part[g * kk + tid];
    C[a][b] = s;
  }
  __syncthreads();
}

// Sum over the nsplit partial blocks of Yp (columns >= kb zero), by one workgroup; each
// entry e < N KB is handed to put(e, value).  EU entries of four blocks per thread are
// loaded at a time, unconditionally (clamped indices, values selected afterwards), so
// that 4 EU loads are in flight per wait instead of one.
template <int EU, typename F, int NB = 256>
__device__ void sum_partials_with(int N, int kb, int nsplit, const double* __restrict__ Yp, F put) {
  constexpr int PU = 4;
  const int tot = N * KB;
  for (int e0 = threadIdx.x; e0 < tot; e0 += NB * EU) {
    double sv[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) sv[u] = 0.0;
    for (int p0 = 0; p0 < nsplit; p0 += PU) {
      double v[PU][EU];
#pragma unroll
      for (int q = 0; q < PU; ++q) {
        const size_t base = (size_t)min(p0 + q, nsplit - 1) * tot;
#pragma unroll
        for (int u = 0; u < EU; ++u) v[q][u] = Yp[base + min(e0 + NB * u, tot - 1)];
      }
#pragma unroll
      for (int q = 0; q < PU; ++q)
#pragma unroll
        for (int u = 0; u < EU; ++u) sv[u] += p0 + q < nsplit ? v[q][u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EU; ++u) {
      const int e = e0 + NB * u;
      if (e < tot) put(e, e % KB < kb ? sv[u] : 0.0);
    }
  }
}

template <int EU>
__device__ void sum_partials(int N, int kb, int nsplit, const double* __restrict__ Yp, double* __restrict__ Y) {
  sum_partials_with<EU>(N, kb, nsplit, Yp, [&](int e, double v) { Y[e] = v; });
}

// One workgroup: X = sum of the nsplit partial blocks, then made orthonormal by two
// rounds of Cholesky QR (C = X^T X = R^T R, X <- X R^-1).  The Cholesky runs column by
// column across the workgroup; each row then solves y R = x.  A column whose pivot falls
// below 1e-26 of the largest diagonal entry of C (numerically dependent) is set to zero.
__global__ __launch_bounds__(256) void k_orth(int N, int kb, int nsplit, const double* __restrict__ Yp,
                                              double* __restrict__ X) {
  __shared__ double xs[RC][KB + 1];
  __shared__ double C[KB][KB];
  __shared__ double R[KB][KB];
  __shared__ double part[256];
  __shared__ int drop[KB];
  const int tid = threadIdx.x;
  sum_partials<8>(N, kb, nsplit, Yp, X);
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    block_gram<RC>(N, kb, X, X, xs, nullptr, C, part);
    double dmax = 0.0;
    for (int j = 0; j < kb; ++j) dmax = fmax(dmax, C[j][j]);
    for (int j = 0; j < kb; ++j) {   // right-looking: row j of R, then the trailing update of C
      const double d = C[j][j];
      const bool dj = !(d > 1e-26 * dmax);
      const double rjj = dj ? 1.0 : sqrt(d);
      if (tid == j) {
        R[j][j] = rjj;
        drop[j] = dj ? 1 : 0;
      } else if (tid > j && tid < kb) {
        R[j][tid] = dj ? 0.0 : C[j][tid] / rjj;
      }
      __syncthreads();
      for (int e = tid; e < kb * kb; e += 256) {
        const int a = e / kb, b = e - (e / kb) * kb;
        if (a > j && b > j) C[a][b] -= R[j][a] * R[j][b];
      }
      __syncthreads();
    }
    for (int i = tid; i < N; i += 256) {
      double x[KB], y[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) x[j] = X[(size_t)i * KB + j];
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        y[j] = 0.0;
        if (j < kb) {   // uniform
          double s = x[j];
#pragma unroll
          for (int p = 0; p < j; ++p) s -= y[p] * R[p][j];
          y[j] = drop[j] ? 0.0 : s / R[j][j];
          X[(size_t)i * KB + j] = y[j];
        }
      }
    }
    __syncthreads();
  }
}

constexpr int ORN = 1024;   // largest N whose block k_orth_res keeps resident in LDS
constexpr int ORT = 1024;   // threads of k_orth_res: one row each

// k_orth with the whole N x KB block resident in LDS (N <= ORN, N (KB + 1) doubles of
// dynamic LDS): the partial blocks are summed straight into LDS, both Cholesky QR rounds
// read and write LDS only, and X goes to HBM once at the end.  Same arithmetic as
// k_orth (the Gram sums run over the rows in another order).
__global__ __launch_bounds__(ORT) void k_orth_res(int N, int kb, int nsplit, const double* __restrict__ Yp,
                                                  double* __restrict__ X) {
  extern __shared__ __attribute__((aligned(16))) double ores[];
  double(*xs)[KB + 1] = reinterpret_cast<double(*)[KB + 1]>(ores);   // [N][KB + 1]
  __shared__ double C[KB][KB];
  __shared__ double R[KB][KB];
  __shared__ double part[ORT];
  __shared__ double rinv[KB];   // 1 / R[j][j], 0 for a dropped column
  const int tid = threadIdx.x;
  const int tot = N * KB;
  auto put_x = [&](int e, double v) { xs[e / KB][e % KB] = v; };
  sum_partials_with<8, decltype(put_x), ORT>(N, kb, nsplit, Yp, put_x);
  __syncthreads();
  const int kk = kb * kb, ng = ORT / kk;
  const int grp = tid / kk, ent = tid - grp * kk;
  const int a = ent / kb, b = ent - (ent / kb) * kb;
  for (int pass = 0; pass < 2; ++pass) {
    if (grp < ng) {
      // four independent chains so that the LDS reads are in flight together
      double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
      int r = grp;
      for (; r + 3 * ng < N; r += 4 * ng) {
        c0 = fma(xs[r][a], xs[r][b], c0);
        c1 = fma(xs[r + ng][a], xs[r + ng][b], c1);
        c2 = fma(xs[r + 2 * ng][a], xs[r + 2 * ng][b], c2);
        c3 = fma(xs[r + 3 * ng][a], xs[r + 3 * ng][b], c3);
      }
      for (; r < N; r += ng) c0 = fma(xs[r][a], xs[r][b], c0);
      part[tid] = (c0 + c1) + (c2 + c3);
    }
    __syncthreads();
    if (tid < kk) {
      double sm = 0.0;
      for (int g = 0; g < ng; ++g) sm += part[g * kk + tid];
      C[a][b] = sm;
    }
    __syncthreads();
    double dmax = 0.0;
    for (int j = 0; j < kb; ++j) dmax = fmax(dmax, C[j][j]);
    for (int j = 0; j < kb; ++j) {   // right-looking: row j of R, then the trailing update of C
      const double d = C[j][j];
      const bool dj = !(d > 1e-26 * dmax);
      const double rjj = dj ? 1.0 : sqrt(d);
      if (tid == j) {
        R[j][j] = rjj;
        rinv[j] = dj ? 0.0 : 1.0 / rjj;
      } else if (tid > j && tid < kb) {
        R[j][tid] = dj ? 0.0 : C[j][tid] / rjj;
      }
      __syncthreads();
      for (int e = tid; e < kk; e += ORT) {
        const int ea = e / kb, eb = e - (e / kb) * kb;
        if (ea > j && eb > j) C[ea][eb] -= R[j][ea] * R[j][eb];
      }
      __syncthreads();
    }
    {
      // y R = x for the thread's rows tid + ORT r (N <= ORN: all of them)
      constexpr int NR = ORN / ORT;
      double y[NR][KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        if (j < kb) {   // uniform
          const double rj = rinv[j];
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int i = tid + ORT * r;
            double sm = i < N ? xs[i][j] : 0.0;
#pragma unroll
            for (int p = 0; p < j; ++p) sm -= y[r][p] * R[p][j];
            y[r][j] = sm * rj;
            if (i < N) xs[i][j] = y[r][j];
          }
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < tot; e += ORT) X[e] = xs[e / KB][e % KB];
}

// Cyclic Jacobi for the symmetric kb x kb matrix A (destroyed): eigenvalues w and
// eigenvectors V (columns), sorted by decreasing eigenvalue.  Single thread.
__device__ void jacobi_eig(int kb, double (*A)[KB], double (*V)[KB], double* w) {
  for (int i = 0; i < kb; ++i)
    for (int j = 0; j < kb; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < kb; ++i)
      for (int j = 0; j < kb; ++j) {
        tot += A[i][j] * A[i][j];
        if (i != j) off += A[i][j] * A[i][j];
      }
    if (!(off > 1e-32 * tot)) break;
    for (int p = 0; p < kb - 1; ++p)
      for (int q = p + 1; q < kb; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        // rotation angle from the stable tangent formula (Rutishauser)
        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < kb; ++r) {   // A <- A J (columns p, q)
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = c * arp - s * arq;
          A[r][q] = s * arp + c * arq;
        }
        for (int r = 0; r < kb; ++r) {   // A <- J^T A (rows p, q)
          const double apr = A[p][r], aqr = A[q][r];
          A[p][r] = c * apr - s * aqr;
          A[q][r] = s * apr + c * aqr;
        }
        for (int r = 0; r < kb; ++r) {   // V <- V J
          const double vrp = V[r][p], vrq = V[r][q];
          V[r][p] = c * vrp - s * vrq;
          V[r][q] = s * vrp + c * vrq;
        }
      }
  }
  for (int i = 0; i < kb; ++i) w[i] = A[i][i];
  for (int i = 0; i < kb; ++i) {   // selection sort, decreasing
    int m = i;
    for (int j = i + 1; j < kb; ++j)
      if (w[j] > w[m]) m = j;
    if (m != i) {
      const double tw = w[i];
      w[i] = w[m];
      w[m] = tw;
      for (int r = 0; r < kb; ++r) {
        const double tv = V[r][i];
        V[r][i] = V[r][m];
        V[r][m] = tv;
      }
    }
  }
}

// One workgroup: H = X^T (G X) (partials summed on the fly), symmetrised, diagonalised;
// X <- X V, mu = eigenvalues (decreasing).
__global__ __launch_bounds__(256) void k_rayleigh_ritz(int N, int kb, int nsplit, const double* __restrict__ Yp,
                                                       double* __restrict__ Y, double* __restrict__ X,
                                                       double* __restrict__ mu) {
  __shared__ double xs[RC / 2][KB + 1];
  __shared__ double ys[RC / 2][KB + 1];
  __shared__ double H[KB][KB];
  __shared__ double V[KB][KB];
  __shared__ double w[KB];
  __shared__ double part[256];
  const int tid = threadIdx.x;
  sum_partials<4>(N, kb, nsplit, Yp, Y);
  __syncthreads();
  block_gram<RC / 2>(N, kb, X, Y, xs, ys, H, part);
  if (tid == 0) {
    for (int i = 0; i < kb; ++i)
      for (int j = i + 1; j < kb; ++j) H[i][j] = H[j][i] = 0.5 * (H[i][j] + H[j][i]);
    jacobi_eig(kb, H, V, w);
    for (int j = 0; j < kb; ++j) mu[j] = w[j];
  }
  __syncthreads();
  for (int i = tid; i < N; i += 256) {
    double x[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) x[j] = X[(size_t)i * KB + j];
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < kb) {   // uniform
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < KB; ++a)
          if (a < kb) s = fma(x[a], V[a][j], s);
        X[(size_t)i * KB + j] = s;
      }
  }
}

constexpr int NBC = 32;            // columns of B per workgroup of k_noise_from_block
constexpr int NBP = 256 / NBC;     // row phases per workgroup (8)

// bt[j][c] = sqrt(max(mu_j - 1, 0) / (6N mu_j)) sum_i B[i][c] X[i][j], j < k.
__global__ __launch_bounds__(256) void k_noise_from_block(int N, int n, int k, const double* __restrict__ B,
                                                          const double* __restrict__ X, const double* __restrict__ mu,
                                                          double sixN, double* __restrict__ bt) {
  __shared__ double xs[RC][KB];
  __shared__ double red[NBP][NBC][KB + 1];
  const int cl = threadIdx.x % NBC, ph = threadIdx.x / NBC;
  const int c = blockIdx.x * NBC + cl;
  double acc[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) acc[j] = 0.0;
  for (int r0 = 0; r0 < N; r0 += RC) {
    for (int e = threadIdx.x; e < RC * KB; e += 256) {
      const int r = e / KB;
      xs[r][e % KB] = r0 + r < N ? X[(size_t)r0 * KB + e] : 0.0;
    }
    __syncthreads();
    const int nr = min(RC, N - r0);
    if (c < n)
      for (int r = ph; r < nr; r += NBP) {
        const double b = B[(size_t)(r0 + r) * n + c];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = fma(b, xs[r][j], acc[j]);
      }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < KB; ++j) red[ph][cl][j] = acc[j];
  __syncthreads();
  // one thread per (vector j, column): the row phases added in a fixed order
  for (int e = threadIdx.x; e < KB * NBC; e += 256) {
    const int j = e / NBC, oc = e - j * NBC, cc = blockIdx.x * NBC + oc;
    if (j < k && cc < n) {
      double sm = 0.0;
      for (int p = 0; p < NBP; ++p) sm += red[p][oc][j];
      const double m = mu[j];
      const double coef = m > 1.0 ? sqrt((m - 1.0) / (sixN * m)) : 0.0;
      bt[(size_t)j * n + cc] = coef * sm;
    }
  }
}

// Sign of vector j: its entry of largest magnitude (first one on ties) made positive.
__global__ __launch_bounds__(256) void k_sign_fix(int n, double* __restrict__ bt) {
  double* v = bt + (size_t)blockIdx.x * n;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int c = threadIdx.x; c < n; c += 256) {
    const double a = fabs(v[c]);
    if (a > best) {
      best = a;
      bi = c;
    }
  }
  __shared__ double sb[256];
  __shared__ int si[256];
  sb[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = sb[threadIdx.x + s];
      const int oi = si[threadIdx.x + s];
      if (o > sb[threadIdx.x] || (o == sb[threadIdx.x] && oi < si[threadIdx.x])) {
        sb[threadIdx.x] = o;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int im = si[0];
  const bool flip = im < n && v[im] < 0.0;
  __syncthreads();
  if (flip)
    for (int c = threadIdx.x; c < n; c += 256) v[c] = -v[c];
}

__device__ inline double block_sum(double v, double* red) {
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// D[r][0] = v_r . alpha and D[r][1 + j] = v_r . b_j for the rows
// v = (alpha, beta_1 .. beta_S, b_1 .. b_k), one workgroup per row.
__global__ __launch_bounds__(256) void k_lowrank_dots(int n, int S, int k, const double* __restrict__ alpha,
                                                      const double* __restrict__ beta, const double* __restrict__ bt,
                                                      double* __restrict__ D) {
  const int r = blockIdx.x;
  const double* v = r == 0 ? alpha : (r <= S ? beta + (size_t)(r - 1) * n : bt + (size_t)(r - 1 - S) * n);
  double acc[KB + 1];
#pragma unroll
  for (int j = 0; j <= KB; ++j) acc[j] = 0.0;
  for (int c = threadIdx.x; c < n; c += 256) {
    const double x = v[c];
    acc[0] = fma(x, alpha[c], acc[0]);
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < k) acc[1 + j] = fma(x, bt[(size_t)j * n + c], acc[1 + j]);
  }
  __shared__ double red[4];
#pragma unroll
  for (int j = 0; j <= KB; ++j)
    if (j <= k) {   // uniform
      const double s = block_sum(acc[j], red);
      if (threadIdx.x == 0) D[(size_t)r * (KB + 1) + j] = s;
    }
}

// out[r] = D[r][0] - w^T D[r][1..k] with w = (I + K^T K)^-1 K^T alpha: out[0] is
// alpha^T zeta^-1 alpha and out[1 + s] is alpha^T zeta^-1 beta_s.  One workgroup.
__global__ __launch_bounds__(256) void k_lowrank_finish(int S, int k, const double* __restrict__ D,
                                                        double* __restrict__ out) {
  __shared__ double w[KB];
  if (threadIdx.x == 0) {
    double M[KB][KB], Lc[KB][KB], y[KB];
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) M[a][b] = (a == b ? 1.0 : 0.0) + D[(size_t)(S + 1 + a) * (KB + 1) + 1 + b];
    for (int j = 0; j < k; ++j) {   // M = Lc Lc^T (M >= I, so the pivots are >= 1)
      double d = M[j][j];
      for (int p = 0; p < j; ++p) d -= Lc[j][p] * Lc[j][p];
      Lc[j][j] = sqrt(d);
      for (int i = j + 1; i < k; ++i) {
        double s = M[i][j];
        for (int p = 0; p < j; ++p) s -= Lc[i][p] * Lc[j][p];
        Lc[i][j] = s / Lc[j][j];
      }
    }
    for (int i = 0; i < k; ++i) {
      double s = D[1 + i];
      for (int p = 0; p < i; ++p) s -= Lc[i][p] * y[p];
      y[i] = s / Lc[i][i];
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = y[i];
      for (int p = i + 1; p < k; ++p) s -= Lc[p][i] * w[p];
      w[i] = s / Lc[i][i];
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r <= S; r += 256) {
    double q = D[(size_t)r * (KB + 1)];
    for (int j = 0; j < k; ++j) q -= w[j] * D[(size_t)r * (KB + 1) + 1 + j];
    out[r] = q;
  }
}

// Inclusive scan of v over the 256 threads of the workgroup; total in *tot.
__device__ inline double block_incl_scan(double v, double* sh, double* tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int d = 1; d < 64; d <<= 1) {
    const double t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  __syncthreads();
  if (lane == 63) sh[wv] = v;
  __syncthreads();
  double off = 0.0;
  for (int u = 0; u < wv; ++u) off += sh[u];
  *tot = sh[0] + sh[1] + sh[2] + sh[3];
  return v + off;
}

// y = lambda~^-1 x for every row of x [R][n] (see the file comment); one workgroup per
// row, 1024 entries per round, 4 consecutive per thread.
__global__ __launch_bounds__(256) void k_bivector_rotate(int n, const double* __restrict__ b,
                                                         const double* __restrict__ x, double* __restrict__ y) {
  __shared__ double sh2[4], shu[4];
  const double* xr = x + (size_t)blockIdx.x * n;
  double* yr = y + (size_t)blockIdx.x * n;
  double carryD = 1.0, carryU = 0.0;
  for (int base = 0; base < n; base += 1024) {
    const int i0 = base + 4 * threadIdx.x;
    double bb[4], xx[4], s2 = 0.0, su = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const bool in = i0 + e < n;
      bb[e] = in ? b[i0 + e] : 0.0;
      xx[e] = in ? xr[i0 + e] : 0.0;
      s2 = fma(bb[e], bb[e], s2);
      su = fma(bb[e], xx[e], su);
    }
    double t2, tu;
    const double i2 = block_incl_scan(s2, sh2, &t2);
    const double iu = block_incl_scan(su, shu, &tu);
    double D = carryD + (i2 - s2);   // D_{i0 - 1}
    double U = carryU + (iu - su);   // U_{i0}
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const double Dn = fma(bb[e], bb[e], D);
      if (i0 + e < n) yr[i0 + e] = (xx[e] - bb[e] * U / D) * sqrt(D / Dn);
      D = Dn;
      U = fma(bb[e], xx[e], U);
    }
    carryD += t2;
    carryU += tu;
  }
}

}  // namespace

size_t noise_ws_bytes(int N) {
  const size_t nsplit = (size_t)(N + GXL - 1) / GXL;
  const size_t nt = (N + GT - 1) / GT, ntp = nt * (nt + 1) / 2;
  return align256((size_t)N * N * 8) + align256((size_t)N * KB * 8) * 2 + align256(nsplit * N * KB * 8) +
         align256((size_t)gram_splits_max(N) * ntp * GT * GT * 8) + align256(KB * 8);
}

int noise_block_max() { return KB; }

hipError_t launch_noise_vectors(int N, int n, int k, int iters, const double* B, double* bt, double* ws,
                                double* mu_dev, hipStream_t st) {
  const int kb = std::min(std::min(k + 4, KB), std::min(N, n));
  const int nsplit = (N + GXL - 1) / GXL;
  char* p = (char*)ws;
  double* G = (double*)p;
  p += align256((size_t)N * N * 8);
  double* X = (double*)p;
  p += align256((size_t)N * KB * 8);
  double* Y = (double*)p;
  p += align256((size_t)N * KB * 8);
  double* Yp = (double*)p;
  p += align256((size_t)nsplit * N * KB * 8);
  double* Gp = (double*)p;   // partial Gram tiles, before the final slot (the eigenvalues)
  const int nt = (N + GT - 1) / GT, ntp = nt * (nt + 1) / 2;
  const int nks = gram_splits(N, n);
  const int kc = ((n + nks - 1) / nks + GK - 1) / GK * GK;
  hipLaunchKernelGGL(k_gram_part, dim3(ntp, nks), dim3(256), 0, st, N, n, kc, ntp, B, Gp);
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)(((size_t)N * N + 255) / 256)), dim3(256), 0, st, N, ntp, nks, Gp,
                     1.0 / (6.0 * N), G);
  hipLaunchKernelGGL(k_start_block, dim3((N * KB + 255) / 256), dim3(256), 0, st, N, kb, Yp);
  // the block stays in LDS through the orthonormalisation when it fits
  const bool res = N <= ORN;
  const size_t res_lds = (size_t)N * (KB + 1) * 8;
  if (res) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_orth_res, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)((size_t)ORN * (KB + 1) * 8));
    if (e != hipSuccess) return e;
  }
  auto orth = [&](int ns) {
    if (res)
      hipLaunchKernelGGL(k_orth_res, dim3(1), dim3(ORT), res_lds, st, N, kb, ns, Yp, X);
    else
      hipLaunchKernelGGL(k_orth, dim3(1), dim3(256), 0, st, N, kb, ns, Yp, X);
  };
  orth(1);
  const dim3 ggx((N + GXR - 1) / GXR, nsplit);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_gx, ggx, dim3(256), 0, st, N, G, X, Yp);
    orth(nsplit);
  }
  hipLaunchKernelGGL(k_gx, ggx, dim3(256), 0, st, N, G, X, Yp);
  hipLaunchKernelGGL(k_rayleigh_ritz, dim3(1), dim3(256), 0, st, N, kb, nsplit, Yp, Y, X, mu_dev);
  hipLaunchKernelGGL(k_noise_from_block, dim3((n + NBC - 1) / NBC), dim3(256), 0, st, N, n, k, B, X, mu_dev,
                     6.0 * N, bt);
  hipLaunchKernelGGL(k_sign_fix, dim3(k), dim3(256), 0, st, n, bt);
  return hipGetLastError();
}

size_t lowrank_ws_bytes(int S) { return align256((size_t)(S + 1 + KB) * (KB + 1) * 8) + align256((size_t)(S + 1) * 8); }

hipError_t launch_fnl_lowrank(int n, int k, const double* bt, const double* alpha, const double* beta, int S,
                              double* ws, double* out, hipStream_t st) {
  double* D = ws;
  hipLaunchKernelGGL(k_lowrank_dots, dim3(S + 1 + k), dim3(256), 0, st, n, S, k, alpha, beta, bt, D);
  hipLaunchKernelGGL(k_lowrank_finish, dim3(1), dim3(256), 0, st, S, k, D, out);
  return hipGetLastError();
}

hipError_t launch_bivector_rotate(int n, const double* b, const double* x, int R, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_bivector_rotate, dim3(R), dim3(256), 0, st, n, b, x, y);
  return hipGetLastError();
}

}  // namespace modal
