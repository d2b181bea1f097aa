// Theory mode coefficients of separable bispectra, eq. (abispect), and the ideal
// (full-sky, isotropic) covariance of the separable modes, eq. (cbispect) with a
// diagonal covariance, which is also their Gram matrix: its Cholesky factor
// orthonormalises the basis (Sec. II).
//
// Both are triple sums over (l1, l2, l3) weighted by
//   h^2_{l1 l2 l3} = (2l1+1)(2l2+1)(2l3+1)/(8 pi) int_{-1}^{1} P_l1 P_l2 P_l3 dmu,
// since the squared 3j symbol (l1 l2 l3; 0 0 0)^2 is half the Legendre triple
// integral.  The sums then factor into one-dimensional Legendre series on a
// Gauss-Legendre rule in mu with ceil((3 lmax + 1) / 2) nodes, exact because the
// integrand has degree at most 3 lmax:
//   F_{f,a}(mu_k) = sum_l (2l+1) U_f(l) B_a(l) P_l(mu_k)
//   alpha_(pqr) = 1/(48 pi) sum_k w_k sum_t sum_{sigma in S3} F_{t,sigma1,p} F_{t,sigma2,q} F_{t,sigma3,r}
//       U = (X_t, Y_t, Z_t) for b = sum_t X_t Y_t Z_t, B_a = q_a / sqrt(C)
//   zeta0_(abc),(def) = 1/(48 pi) sum_k w_k sum_{sigma in S3} Q_{a,sigma d} Q_{b,sigma e} Q_{c,sigma f}
//       Q_ab = F_{b,a} with U_b = c q_b, B_a = q_a (c_l = <|a~_lm|^2> of the whitened sky)
// FP64 throughout.  The series are O(nf P nmu lmax); alpha is O(n_max nmu T); the
// covariance, n_max^2 nmu / 2 sums of six triple products, is the only large one
// and is tiled 64 x 64 with the Q(mu) slices staged in LDS.
#include "common.h"

#include <algorithm>

namespace modal {
namespace {

constexpr int SL = 64;   // l per staged chunk of the series kernel

// F[f][k][a] = sum_l (2l+1) U[f][l] B[a][l] P_l(mu_k); one thread per node for the modes
// a0 .. a0 + NP - 1, a0 = NP blockIdx.z (each group of modes repeats the cheap recurrence).
template <int NP>
__global__ __launch_bounds__(64) void k_legendre_series(int L, int nmu, int P, const double* __restrict__ U,
                                                        const double* __restrict__ B, const double* __restrict__ mu,
                                                        double* __restrict__ F) {
  __shared__ double bs[SL][NP];
  __shared__ double us[SL];
  const int f = blockIdx.y, a0 = blockIdx.z * NP;
  const int k = blockIdx.x * 64 + threadIdx.x;
  const double x = k < nmu ? mu[k] : 0.0;
  double acc[NP];
#pragma unroll
  for (int a = 0; a < NP; ++a) acc[a] = 0.0;
  double pm = 0.0, pl = 1.0;   // P_{l-1}, P_l
  for (int l0 = 0; l0 < L; l0 += SL) {
    __syncthreads();
    for (int e = threadIdx.x; e < SL * NP; e += 64) {
      const int i = e / NP, a = e - i * NP;
      bs[i][a] = (a0 + a < P && l0 + i < L) ? B[(size_t)(a0 + a) * L + l0 + i] : 0.0;
    }
    us[threadIdx.x] = l0 + (int)threadIdx.x < L ? U[(size_t)f * L + l0 + threadIdx.x] : 0.0;
    __syncthreads();
    const int n = min(SL, L - l0);
    for (int i = 0; i < n; ++i) {
      const int l = l0 + i;
      const double g = (2.0 * l + 1.0) * us[i] * pl;
#pragma unroll
      for (int a = 0; a < NP; ++a) acc[a] = fma(g, bs[i][a], acc[a]);
      const double pn = ((2.0 * l + 1.0) * x * pl - l * pm) / (l + 1.0);   // Bonnet's recurrence
      pm = pl;
      pl = pn;
    }
  }
  if (k >= nmu) return;
  double* out = F + ((size_t)f * nmu + k) * P;
#pragma unroll
  for (int a = 0; a < NP; ++a)
    if (a0 + a < P) out[a0 + a] = acc[a];
}

// alpha[n] = 1/(48 pi) sum_k w_k sum_t sum_sigma F[3t + sigma1][k][p] F[3t + sigma2][k][q] F[3t + sigma3][k][r]
// A workgroup takes AMC modes, its threads AMP phases of the nodes k; the phases are added
// in a fixed order through LDS.
constexpr int AMC = 32;
constexpr int AMP = 256 / AMC;

__global__ __launch_bounds__(256) void k_alpha_modes(int nmax, int P, int T, int nmu, const int* __restrict__ tri,
                                                     const double* __restrict__ F, const double* __restrict__ wmu,
                                                     double* __restrict__ alpha) {
  __shared__ double red[AMP][AMC];
  const int ml = threadIdx.x % AMC, ph = threadIdx.x / AMC;
  const int n = blockIdx.x * AMC + ml;
  double acc = 0.0;
  if (n < nmax) {
    const int p = tri[6 * n], q = tri[6 * n + 1], r = tri[6 * n + 2];
    for (int k = ph; k < nmu; k += AMP) {
      double sm = 0.0;
      for (int t = 0; t < T; ++t) {
        const double* X = F + ((size_t)(3 * t) * nmu + k) * P;
        const double* Y = X + (size_t)nmu * P;
        const double* Z = Y + (size_t)nmu * P;
        const double xp = X[p], xq = X[q], xr = X[r], yp = Y[p], yq = Y[q], yr = Y[r], zp = Z[p], zq = Z[q], zr = Z[r];
        sm += xp * (yq * zr + zq * yr) + yp * (xq * zr + zq * xr) + zp * (xq * yr + yq * xr);
      }
      acc = fma(wmu[k], sm, acc);
    }
  }
  red[ph][ml] = acc;
  __syncthreads();
  if (ph == 0 && n < nmax) {
    double s = 0.0;
    for (int i = 0; i < AMP; ++i) s += red[i][ml];
    alpha[n] = s * (1.0 / (48.0 * 3.14159265358979323846));
  }
}

// zeta0 over the padded row order (runs of equal (p, r), each a multiple of 4 rows):
// tile (bi, bj), bj <= bi, mirrored; Q slices [KC][P][P+1] staged in dynamic LDS.
// Each thread owns 4 rows (a, b, c_u) and 4 columns (d, e, f_v) of one aligned group, so
// the permanent of the 3 x 3 block, expanded along its third row,
//   perm = Q_cf (Q_ad Q_be + Q_ae Q_bd) + Q_ce (Q_ad Q_bf + Q_af Q_bd) + Q_cd (Q_ae Q_bf + Q_af Q_be),
// shares its 2 x 2 permanents across the thread's rows: 36 LDS reads per node for the
// 16 entries instead of 144.
__global__ __launch_bounds__(256) void k_ideal_cov(int nmax, int P, int nmu, int KC, int nrows,
                                                   const int4* __restrict__ zrows, const double* __restrict__ F,
                                                   const double* __restrict__ wmu, double* __restrict__ Z) {
  extern __shared__ double qs_raw[];
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  const int PP = P + 1;
  double* wk = qs_raw + (size_t)KC * P * PP;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  // groups past the table (whole groups: nrows % 4 == 0) take a dummy row of mode -1
  int4 rr[4], cc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = bi * 64 + ty * 4 + u, j = bj * 64 + tx * 4 + u;
    rr[u] = i < nrows ? zrows[i] : make_int4(0, 0, 0, -1);
    cc[u] = j < nrows ? zrows[j] : make_int4(0, 0, 0, -1);
  }
  const int ra = rr[0].x * PP, rb = rr[0].y * PP, d = cc[0].x, e = cc[0].y;
  int rc[4], cf[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    rc[u] = rr[u].z * PP;
    cf[u] = cc[u].z;
  }
  double acc[4][4] = {};
  for (int k0 = 0; k0 < nmu; k0 += KC) {
    const int kn = min(KC, nmu - k0);
    __syncthreads();
    for (int x = threadIdx.x; x < kn * P * P; x += 256) {
      const int kk = x / (P * P), rem = x - kk * P * P, b = rem / P, a = rem - b * P;
      qs_raw[(size_t)kk * P * PP + a * PP + b] = F[((size_t)b * nmu + k0 + kk) * P + a];   // Q_ab(mu_k)
    }
    if ((int)threadIdx.x < kn) wk[threadIdx.x] = wmu[k0 + threadIdx.x];
    __syncthreads();
    for (int kk = 0; kk < kn; ++kk) {
      const double* Q = qs_raw + (size_t)kk * P * PP;
      const double w = wk[kk];
      const double qad = Q[ra + d], qae = Q[ra + e], qbd = Q[rb + d], qbe = Q[rb + e];
      const double t0 = qad * qbe + qae * qbd;
      double t1[4], t2[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double qaf = Q[ra + cf[v]], qbf = Q[rb + cf[v]];
        t1[v] = qad * qbf + qaf * qbd;
        t2[v] = qae * qbf + qaf * qbe;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double qcd = Q[rc[u] + d], qce = Q[rc[u] + e];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double s = Q[rc[u] + cf[v]] * t0 + qce * t1[v] + qcd * t2[v];
          acc[u][v] = fma(w, s, acc[u][v]);
        }
      }
    }
  }
  const double scale = 1.0 / (48.0 * 3.14159265358979323846);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int n = rr[u].w, m = cc[v].w;
      if (n >= 0 && m >= 0 && m <= n) {   // one writer per symmetric pair
        Z[(size_t)n * nmax + m] = scale * acc[u][v];
        Z[(size_t)m * nmax + n] = scale * acc[u][v];
      }
    }
}

}  // namespace

int shapes_nmu(int lmax) { return (3 * lmax + 2) / 2; }

hipError_t launch_legendre_series(int L, int nmu, int P, int nf, const double* U, const double* B, const double* mu,
                                  double* F, hipStream_t st) {
  constexpr int NG = 16;   // modes per thread
  const dim3 grid((nmu + 63) / 64, nf, (P + NG - 1) / NG);
  hipLaunchKernelGGL(k_legendre_series<NG>, grid, dim3(64), 0, st, L, nmu, P, U, B, mu, F);
  return hipGetLastError();
}

hipError_t launch_alpha_modes(int nmax, int P, int T, int nmu, const int* tri, const double* F, const double* wmu,
                              double* alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_alpha_modes, dim3((nmax + AMC - 1) / AMC), dim3(256), 0, st, nmax, P, T, nmu, tri, F, wmu, alpha);
  return hipGetLastError();
}

hipError_t launch_ideal_cov(int nmax, int P, int nmu, int nrows, const int4* zrows, const double* F,
                            const double* wmu, double* Z, hipStream_t st) {
  const size_t slice = (size_t)P * (P + 1) * 8 + 8;
  const int KC = (int)std::max<size_t>(1, std::min<size_t>(8, 65536 / slice));
  const size_t lds = (size_t)KC * slice;
  const int nt = (nrows + 63) / 64;
  hipLaunchKernelGGL(k_ideal_cov, dim3(nt, nt), dim3(256), lds, st, nmax, P, nmu, KC, nrows, zrows, F, wmu, Z);
  return hipGetLastError();
}

}  // namespace modal
