// Linear term evaluated in harmonic space.
//
// The Monte-Carlo linear term needs, for every pair (ab), map s and mode t,
//   L_{(ab),s,t} = sum_x w(x) V_ab(x) M^s_t(x)
// (lin_prs = L_{(pr),s} + L_{(ps),r} + L_{(rs),p}, eq. bbispect with the three
// pairings of the "3 C a" term of eq. bispectrumest).  The filtered map is itself a
// finite harmonic sum on the grid, M^s_t(x) = sum_lm qw_t(l) a^s_lm Y_lm(x) with
// qw = q / sqrt(C_l), so exchanging the two finite sums gives, exactly,
//   L_{(ab),s,t} = sum_l qw_t(l) X_{s,(ab)}(l),
//   X_{s,(ab)}(l) = sum_{m=0}^{l} (Re a^s_lm Re Z_ab,lm + Im a^s_lm Im Z_ab,lm),
//   Z_ab,lm = c_m sum_j lambda_lm(theta_j) sum_k w V_ab (theta_j, phi_k) e^{-i m phi_k}
// (c_m = 2 - delta_m0).  Z depends on the state only, so it is computed once when
// the state is finalised (weighted planes -> ring r2c FFT -> per-column adjoint
// Legendre), and each batch costs one pass over Z instead of a pixel-space
// contraction of npairs planes against S P maps.  No band-limit or quadrature
// property is used: it is a reordering of the same finite sums.
#include "common.h"

namespace modal {
namespace {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

// G[k][x] = w(x) V[k][x] for nk consecutive pair planes.
template <typename T>
__global__ __launch_bounds__(256) void k_weight_planes(int npix, int nk, const T* __restrict__ V,
                                                       const T* __restrict__ w, T* __restrict__ G) {
  // grid-stride (the launch is capped below the 2^32 work-items of one dispatch dimension)
  const size_t n = (size_t)nk * npix, step = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += step) {
    const int x = (int)(i % (size_t)npix);
    G[i] = T((double)V[i] * (double)w[x]);
  }
}

// X[s][pair][l] = sum_{m <= l} (Re a Re Z + Im a Im Z) at index (l, m), FP64 sums.
// A workgroup covers LT consecutive l (one per lane) x PT pairs x ST maps (grid x: the pair
// group, y: the l tile), so that every Z and a_lm element it loads feeds PT or ST products; its MW waves take the m of the
// sum in turn (m = w, w + MW, ...) and their partial sums are added through LDS.  The
// lanes of a wave read consecutive l of one m row of the m-major packing: coalesced.
constexpr int PT = 8;
constexpr int ST = 8;
constexpr int LT = 64;
constexpr int MW = 4;
constexpr int RED = 16;   // accumulators per LDS reduction round

template <typename T>
__global__ __launch_bounds__(LT * MW) void k_lin_x(int lmax, int nalm, int npairs, int S,
                                                   const typename vec2<T>::type* __restrict__ Z,
                                                   const typename vec2<T>::type* __restrict__ alm,
                                                   double* __restrict__ X) {
  using T2 = typename vec2<T>::type;
  __shared__ double red[MW - 1][RED][LT];
  const int lane = threadIdx.x % LT, w = threadIdx.x / LT;
  const int l = blockIdx.y * LT + lane;
  const int lc = min(l, lmax);
  const int mend = min((int)blockIdx.y * LT + LT - 1, lmax);   // largest l of the workgroup
  const int p0 = blockIdx.x * PT, s0 = blockIdx.z * ST;
  double acc[PT][ST];
#pragma unroll
  for (int k = 0; k < PT; ++k)
#pragma unroll
    for (int q = 0; q < ST; ++q) acc[k][q] = 0.0;
  const T2* zr[PT];
  const T2* ar[ST];
#pragma unroll
  for (int k = 0; k < PT; ++k) zr[k] = Z + (size_t)min(p0 + k, npairs - 1) * nalm;
#pragma unroll
  for (int q = 0; q < ST; ++q) ar[q] = alm + (size_t)min(s0 + q, S - 1) * nalm;
#pragma unroll 2
  for (int m = w; m <= mend; m += MW) {
    // lanes with l < m (or past lmax) read a valid element of the row and add zero
    const bool on = m <= l && l <= lmax;
    const size_t idx = (size_t)m * (2 * lmax + 3 - m) / 2 + (max(lc, m) - m);   // m-major packing
    double zx[PT], zy[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const T2 z = zr[k][idx];
      zx[k] = on ? (double)z.x : 0.0;
      zy[k] = on ? (double)z.y : 0.0;
    }
#pragma unroll
    for (int q = 0; q < ST; ++q) {
      const T2 a = ar[q][idx];
      const double ax = (double)a.x, ay = (double)a.y;
#pragma unroll
      for (int k = 0; k < PT; ++k) acc[k][q] = fma(ax, zx[k], fma(ay, zy[k], acc[k][q]));
    }
  }
  // add the partial sums of waves 1 .. MW-1 into wave 0, RED accumulators at a time
#pragma unroll
  for (int r0 = 0; r0 < PT * ST; r0 += RED) {
    __syncthreads();
    if (w > 0) {
#pragma unroll
      for (int i = 0; i < RED; ++i) red[w - 1][i][lane] = acc[(r0 + i) / ST][(r0 + i) % ST];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int i = 0; i < RED; ++i)
#pragma unroll
        for (int v = 0; v < MW - 1; ++v) acc[(r0 + i) / ST][(r0 + i) % ST] += red[v][i][lane];
    }
  }
  if (w != 0 || l > lmax) return;
#pragma unroll
  for (int q = 0; q < ST; ++q) {
    if (s0 + q >= S) break;
#pragma unroll
    for (int k = 0; k < PT; ++k)
      if (p0 + k < npairs) X[((size_t)(s0 + q) * npairs + p0 + k) * (lmax + 1) + l] = acc[k][q];
  }
}

// L[s][pair][t] = sum_l qw_t(l) X[s][pair][l]; one workgroup per (map, pair), one
// thread per mode, the X row staged in LDS.
__global__ __launch_bounds__(64) void k_lin_l(int lmax, int npairs, int P, const double* __restrict__ qw,
                                              const double* __restrict__ X, double* __restrict__ L) {
  const int pair = blockIdx.x, s = blockIdx.y;
  const int t = threadIdx.x;
  __shared__ double xs[256];
  const double* xrow = X + ((size_t)s * npairs + pair) * (lmax + 1);
  double acc = 0.0;
  for (int l0 = 0; l0 <= lmax; l0 += 256) {
    const int n = min(256, lmax + 1 - l0);
    __syncthreads();
    for (int i = t; i < n; i += 64) xs[i] = xrow[l0 + i];
    __syncthreads();
    if (t < P) {
      const double* q = qw + (size_t)t * (lmax + 1) + l0;
      for (int i = 0; i < n; ++i) acc = fma(q[i], xs[i], acc);
    }
  }
  if (t < P) L[((size_t)s * npairs + pair) * P + t] = acc;
}

// The adjoint of the linear term with respect to a_lm.  With the slot matrix K of the
// adjoint (K[s][u][pair]: dL/dlin summed onto the leg u of each triple),
//   dL/da^s_lm (linear part) = - sum_pair H_{s,pair}(l) Z_pair,lm,
//   H_{s,pair}(l) = sum_u K[s][u][pair] qw_u(l),
// the transpose of the X contraction above: the same reordering of finite sums, so the
// pixel-space adjoint needs only the cubic part w sum K M_a M_b.
template <typename T>
__global__ __launch_bounds__(256) void k_lin_vjp_h(int lmax, int P, int npairs, const double* __restrict__ qw,
                                                   const double* __restrict__ K, T* __restrict__ H) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  const int pair = blockIdx.y, s = blockIdx.z;
  if (l > lmax) return;
  const double* k = K + (size_t)s * P * npairs + pair;
  double acc = 0.0;
  for (int u = 0; u < P; ++u) acc = fma(k[(size_t)u * npairs], qw[(size_t)u * (lmax + 1) + l], acc);
  H[((size_t)s * npairs + pair) * (lmax + 1) + l] = T(acc);
}

// grad[s][lm] -= sum_pair H[s][pair][l] Z[pair][lm], FP64 sums.  A workgroup covers VL
// consecutive l (one per lane) x VM consecutive m x VS maps; its VW waves take the pairs
// in turn (pair = w, w + VW, ...) and their partial sums are added through LDS, so that
// every wave runs a short loop and many waves are in flight.  Each Z element is read
// once; lanes with l < m read a valid element and add nothing.
constexpr int VL = 64;
constexpr int VW = 4;
constexpr int VM = 4;
constexpr int VS = 8;
constexpr int VRED = 16;   // accumulators per LDS reduction round

template <typename T>
__global__ __launch_bounds__(VL * VW) void k_lin_vjp(int lmax, int nalm, int npairs, int S, const T* __restrict__ H,
                                                     const typename vec2<T>::type* __restrict__ Z,
                                                     typename vec2<T>::type* __restrict__ grad) {
  using T2 = typename vec2<T>::type;
  __shared__ double red[VW - 1][VRED][VL];
  const int lane = threadIdx.x % VL, w = threadIdx.x / VL;
  const int l = blockIdx.x * VL + lane;
  const int lc = min(l, lmax);
  const int m0 = blockIdx.y * VM;
  const int s0 = blockIdx.z * VS;
  if (m0 > min((int)blockIdx.x * VL + VL - 1, lmax)) return;   // whole workgroup: no l >= m in the tile
  size_t idx[VM];
  bool on[VM];
#pragma unroll
  for (int j = 0; j < VM; ++j) {
    const int m = min(m0 + j, lmax);
    on[j] = m0 + j <= l && l <= lmax;
    idx[j] = (size_t)m * (2 * lmax + 3 - m) / 2 + (max(lc, m) - m);   // m-major packing
  }
  double acc[2 * VM * VS];   // [re/im][j][q]
#pragma unroll
  for (int k = 0; k < 2 * VM * VS; ++k) acc[k] = 0.0;
  const T* hr[VS];
#pragma unroll
  for (int q = 0; q < VS; ++q) hr[q] = H + (size_t)min(s0 + q, S - 1) * npairs * (lmax + 1) + lc;
  for (int pair = w; pair < npairs; pair += VW) {
    double h[VS];
#pragma unroll
    for (int q = 0; q < VS; ++q) h[q] = (double)hr[q][(size_t)pair * (lmax + 1)];
    const T2* zp = Z + (size_t)pair * nalm;
#pragma unroll
    for (int j = 0; j < VM; ++j) {
      const T2 z = zp[idx[j]];
      const double zx = on[j] ? (double)z.x : 0.0, zy = on[j] ? (double)z.y : 0.0;
#pragma unroll
      for (int q = 0; q < VS; ++q) {
        acc[(0 * VM + j) * VS + q] = fma(h[q], zx, acc[(0 * VM + j) * VS + q]);
        acc[(1 * VM + j) * VS + q] = fma(h[q], zy, acc[(1 * VM + j) * VS + q]);
      }
    }
  }
  // add the partial sums of waves 1 .. VW-1 into wave 0, VRED accumulators at a time
#pragma unroll
  for (int r0 = 0; r0 < 2 * VM * VS; r0 += VRED) {
    __syncthreads();
    if (w > 0) {
#pragma unroll
      for (int i = 0; i < VRED; ++i) red[w - 1][i][lane] = acc[r0 + i];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int i = 0; i < VRED; ++i)
#pragma unroll
        for (int v = 0; v < VW - 1; ++v) acc[r0 + i] += red[v][i][lane];
    }
  }
  if (w != 0) return;
#pragma unroll
  for (int j = 0; j < VM; ++j) {
    if (!on[j]) continue;
#pragma unroll
    for (int q = 0; q < VS; ++q) {
      if (s0 + q >= S) break;
      T2* g = grad + (size_t)(s0 + q) * nalm + idx[j];
      T2 v = *g;
      v.x = T((double)v.x - acc[(0 * VM + j) * VS + q]);
      v.y = T((double)v.y - acc[(1 * VM + j) * VS + q]);
      *g = v;
    }
  }
}

}  // namespace

hipError_t launch_weight_planes(const modal_ctx* c, const void* V, int nk, void* G, hipStream_t st) {
  const size_t n = (size_t)nk * c->npix;
  if (n == 0) return hipSuccess;
  const size_t blocks = std::min((n + 255) / 256, (size_t)65536);
  if (is_f64(c))
    hipLaunchKernelGGL(k_weight_planes<double>, dim3(blocks), dim3(256), 0, st, c->npix, nk, (const double*)V,
                       c->t.w64, (double*)G);
  else
    hipLaunchKernelGGL(k_weight_planes<float>, dim3(blocks), dim3(256), 0, st, c->npix, nk, (const float*)V,
                       c->t.w32, (float*)G);
  return hipGetLastError();
}

hipError_t launch_lin_harmonic(const modal_ctx* c, const void* Z, const void* alm, int S, double* X, double* L,
                               hipStream_t st) {
  if (c->P > 64) return hipErrorInvalidValue;
  // pair groups fastest: the workgroups running together share one l tile of a_lm in L2
  dim3 gx((c->npairs + PT - 1) / PT, (c->lmax + LT) / LT, (S + ST - 1) / ST);
  if (is_f64(c))
    hipLaunchKernelGGL(k_lin_x<double>, gx, dim3(LT * MW), 0, st, c->lmax, c->nalm, c->npairs, S, (const double2*)Z,
                       (const double2*)alm, X);
  else
    hipLaunchKernelGGL(k_lin_x<float>, gx, dim3(LT * MW), 0, st, c->lmax, c->nalm, c->npairs, S, (const float2*)Z,
                       (const float2*)alm, X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lin_l, dim3(c->npairs, S), dim3(64), 0, st, c->lmax, c->npairs, c->P, c->t.qw64, X, L);
  return hipGetLastError();
}

hipError_t launch_lin_vjp(const modal_ctx* c, const double* K, const void* Z, int S, void* H, void* grad,
                          hipStream_t st) {
  const dim3 gh((c->lmax + 256) / 256, c->npairs, S);
  const dim3 gv((c->lmax + VL) / VL, (c->lmax + VM) / VM, (S + VS - 1) / VS);
  if (is_f64(c)) {
    hipLaunchKernelGGL(k_lin_vjp_h<double>, gh, dim3(256), 0, st, c->lmax, c->P, c->npairs, c->t.qw64, K,
                       (double*)H);
    hipLaunchKernelGGL(k_lin_vjp<double>, gv, dim3(VL * VW), 0, st, c->lmax, c->nalm, c->npairs, S,
                       (const double*)H, (const double2*)Z, (double2*)grad);
  } else {
    hipLaunchKernelGGL(k_lin_vjp_h<float>, gh, dim3(256), 0, st, c->lmax, c->P, c->npairs, c->t.qw64, K,
                       (float*)H);
    hipLaunchKernelGGL(k_lin_vjp<float>, gv, dim3(VL * VW), 0, st, c->lmax, c->nalm, c->npairs, S,
                       (const float*)H, (const float2*)Z, (float2*)grad);
  }
  return hipGetLastError();
}

}  // namespace modal
