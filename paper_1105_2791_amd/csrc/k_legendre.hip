// Associated-Legendre synthesis and its adjoint (FP64 recurrence on the fly).
//
// F_{s,p,m}(theta_j) = sum_{l>=m} qw_p(l) a_{s,lm} lambda_lm(theta_j),  qw = q / sqrt(C_l)
//
// is the harmonic half of the filtered maps M_p (separable form of eq. bbispect):
// for each m it is a contraction over l.  lambda_lm is produced by the normalised
// three-term recurrence in l, carried in FP64 from per-(m, ring) seeds that a setup
// kernel finds with a log-scaled FP64 recurrence (values below 2^-90 are dropped).
// Rings are processed in north/south mirror pairs: lambda_lm(-x) = (-1)^{l+m}
// lambda_lm(x), so even and odd (l - m) are summed separately and F_north = E + O,
// F_south = E - O.
#include "common.h"

namespace modal {
namespace {

// ---------------------------------------------------------------------------
// seeds: first significant l per (m, ring) and lambda there (log-scaled FP64)
// ---------------------------------------------------------------------------
__global__ void k_seeds(int lmax, int nrp, const double* __restrict__ x, const double* __restrict__ rec,
                        const double* __restrict__ logpref, double* __restrict__ seed, int* __restrict__ lstart) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (j >= nrp) return;
  const double xx = x[j];
  const double st = sqrt((1.0 - xx) * (1.0 + xx));
  double E = logpref[m] + (m > 0 ? m * log(st) : 0.0);  // log scale of the scaled value
  double s1 = (m & 1) ? -1.0 : 1.0;                     // scaled lambda_l
  double s2 = 0.0;                                      // scaled lambda_{l-1}
  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;  // alm index of (m, m)
  int l = m;
  int ls = lmax + 1;
  double v0 = 0.0, v1 = 0.0;
  for (;;) {
    if (s1 != 0.0 && E + log(fabs(s1)) >= kLogSeedFloor) {
      ls = l;
      v0 = s1 * exp(E);
      if (l < lmax) {
        const double* rc = rec + 2 * (off + (l + 1 - m));
        v1 = (rc[0] * xx * s1 - rc[1] * s2) * exp(E);
      }
      break;
    }
    if (l == lmax) break;
    const double* rc = rec + 2 * (off + (l + 1 - m));
    const double sn = rc[0] * xx * s1 - rc[1] * s2;
    s2 = s1;
    s1 = sn;
    ++l;
    if (fabs(s1) > 1e100) {
      s1 *= 1e-100;
      s2 *= 1e-100;
      E += 230.25850929940458;  // ln(1e100)
    }
  }
  seed[2 * ((size_t)m * nrp + j) + 0] = v0;
  seed[2 * ((size_t)m * nrp + j) + 1] = v1;
  lstart[(size_t)m * nrp + j] = ls;
}

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

// Per-lane recurrence state for one ring.
struct Rec {
  double l1, l2;   // lambda_{l-1}, lambda_{l-2}
  double s0, s1;   // seeds at ls, ls+1
  int ls;
  __device__ inline double step(int l, double xx, const double* rc) {
    double v;
    if (l < ls) v = 0.0;
    else if (l == ls) v = s0;
    else if (l == ls + 1) v = s1;
    else v = rc[0] * xx * l1 - rc[1] * l2;
    l2 = l1;
    l1 = v;
    return v;
  }
};

// ---------------------------------------------------------------------------
// forward synthesis (VALU): one wave = 64 north rings, NSEQ (s,p) sequences
// ---------------------------------------------------------------------------
constexpr int kLch = 64;

template <typename T, int NSEQ>
__global__ __launch_bounds__(64) void k_legendre(int lmax, int ntheta, int nrp, int P, int nseq, int nalm,
                                                 const double* __restrict__ x, const double* __restrict__ rec,
                                                 const double* __restrict__ seed, const int* __restrict__ lstart,
                                                 const T* __restrict__ qw,
                                                 const typename vec2<T>::type* __restrict__ alm,
                                                 typename vec2<T>::type* __restrict__ F) {
  using T2 = typename vec2<T>::type;
  const int m = blockIdx.z;
  const int lane = threadIdx.x;
  const int j = blockIdx.y * 64 + lane;
  const int seq0 = blockIdx.x * NSEQ;
  const bool ring_ok = j < nrp;
  __shared__ T2 coef[kLch][NSEQ];
  __shared__ int lmin_s;

  Rec r;
  double xx = 0.0;
  r.l1 = r.l2 = 0.0;
  r.ls = lmax + 1;
  r.s0 = r.s1 = 0.0;
  if (ring_ok) {
    xx = x[j];
    r.ls = lstart[(size_t)m * nrp + j];
    r.s0 = seed[2 * ((size_t)m * nrp + j)];
    r.s1 = seed[2 * ((size_t)m * nrp + j) + 1];
  }
  if (lane == 0) lmin_s = lmax + 1;
  __syncthreads();
  atomicMin(&lmin_s, r.ls);
  __syncthreads();
  const int lmin = lmin_s;

  T er[NSEQ], ei[NSEQ], orr[NSEQ], oi[NSEQ];
#pragma unroll
  for (int q = 0; q < NSEQ; ++q) er[q] = ei[q] = orr[q] = oi[q] = T(0);

  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;
  for (int l0 = lmin; l0 <= lmax; l0 += kLch) {
    {
      const int l = l0 + lane;
#pragma unroll
      for (int q = 0; q < NSEQ; ++q) {
        T2 v;
        v.x = T(0);
        v.y = T(0);
        const int sq = seq0 + q;
        if (l <= lmax && sq < nseq) {
          const int s = sq / P, p = sq - s * P;
          const T2 a = alm[(size_t)s * nalm + off + (l - m)];
          const T wq = qw[(size_t)p * (lmax + 1) + l];
          v.x = a.x * wq;
          v.y = a.y * wq;
        }
        coef[lane][q] = v;
      }
    }
    __syncthreads();
    const int nl = min(kLch, lmax + 1 - l0);
    for (int tt = 0; tt < nl; ++tt) {
      const int l = l0 + tt;
      const double lam = r.step(l, xx, rec + 2 * (off + (l - m)));
      const T lf = T(lam);
      if ((l - m) & 1) {
#pragma unroll
        for (int q = 0; q < NSEQ; ++q) {
          orr[q] += coef[tt][q].x * lf;
          oi[q] += coef[tt][q].y * lf;
        }
      } else {
#pragma unroll
        for (int q = 0; q < NSEQ; ++q) {
          er[q] += coef[tt][q].x * lf;
          ei[q] += coef[tt][q].y * lf;
        }
      }
    }
    __syncthreads();
  }
  if (!ring_ok) return;
  const int js = ntheta - 1 - j;
#pragma unroll
  for (int q = 0; q < NSEQ; ++q) {
    const int sq = seq0 + q;
    if (sq >= nseq) break;
    const int nrb8 = f_ring_blocks(ntheta);
    T2 vn, vs;
    vn.x = er[q] + orr[q];
    vn.y = ei[q] + oi[q];
    vs.x = er[q] - orr[q];
    vs.y = ei[q] - oi[q];
    F[f_index(sq, j, m, lmax, nrb8)] = vn;
    if (js != j) F[f_index(sq, js, m, lmax, nrb8)] = vs;
  }
}

// ---------------------------------------------------------------------------
// lambda table for the adjoint: lam[m][j][l - m] (north rings), T precision.  A workgroup
// runs the recurrences of 64 rings (one per thread) 64 steps at a time into LDS and writes
// each ring's run of 64 l back as one contiguous row segment, so the stores are coalesced
// (a thread writing its own ring's row would touch 64 rows per store instruction).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_lambda_table(int lmax, int nrp, const double* __restrict__ x,
                                                     const double* __restrict__ rec, const double* __restrict__ seed,
                                                     const int* __restrict__ lstart, T* __restrict__ lam) {
  __shared__ T buf[64][65];
  const int t = threadIdx.x, j0 = blockIdx.x * 64;
  const int jc = min(j0 + t, nrp - 1);   // rings past nrp run a valid recurrence, not stored
  const int m = blockIdx.y;
  const int L = lmax + 1 - m;
  Rec r;
  r.l1 = r.l2 = 0.0;
  r.ls = lstart[(size_t)m * nrp + jc];
  r.s0 = seed[2 * ((size_t)m * nrp + jc)];
  r.s1 = seed[2 * ((size_t)m * nrp + jc) + 1];
  const double xx = x[jc];
  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;
  T* out = lam + off * nrp;   // rows j of length L
  const int nr = min(64, nrp - j0);
  for (int l0 = 0; l0 < L; l0 += 64) {
    const int nl = min(64, L - l0);
    for (int i = 0; i < nl; ++i) buf[t][i] = T(r.step(m + l0 + i, xx, rec + 2 * (off + l0 + i)));
    __syncthreads();
    if (t < nl)
      for (int rr = 0; rr < nr; ++rr) out[(size_t)(j0 + rr) * L + l0 + t] = buf[rr][t];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// mode combination after the adjoint Legendre contraction of every (sky, mode) column
// (k_adj_legendre_cols: Z[s P + u][lm] = c_m sum_j lambda_lm(theta_j) Gh_{s,u,m}(theta_j),
// mirror rings folded, imaginary part zero at m = 0):
//   grad_{s,lm} = sum_u q_u(l) / sqrt(C_l) Z[s P + u][lm].
// One thread per (l, s) of one m; the column reads are coalesced along l.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_adj_combine(int lmax, int P, int S, int nalm, const T* __restrict__ qw,
                                                     const typename vec2<T>::type* __restrict__ Z,
                                                     typename vec2<T>::type* __restrict__ grad) {
  using T2 = typename vec2<T>::type;
  const int m = blockIdx.y, s = blockIdx.z;
  const int li = blockIdx.x * 256 + threadIdx.x;
  if (li > lmax - m) return;
  const int l = m + li;
  const size_t o = (size_t)m * (2 * lmax + 3 - m) / 2 + li;
  double gr = 0.0, gi = 0.0;
  for (int u = 0; u < P; ++u) {
    const double q = (double)qw[(size_t)u * (lmax + 1) + l];
    const T2 z = Z[((size_t)s * P + u) * nalm + o];
    gr += q * (double)z.x;
    gi += q * (double)z.y;
  }
  T2 g;
  g.x = T(gr);
  g.y = T(gi);
  grad[(size_t)s * nalm + o] = g;
}

}  // namespace

hipError_t launch_seeds(const modal_ctx* c, const double* logpref, hipStream_t st) {
  dim3 grid((c->nrp + 127) / 128, c->lmax + 1);
  hipLaunchKernelGGL(k_seeds, grid, dim3(128), 0, st, c->lmax, c->nrp, c->t.x, c->t.rec, logpref, c->t.seed,
                     c->t.lstart);
  return hipGetLastError();
}

hipError_t launch_legendre(const modal_ctx* c, const void* alm, int S, void* F, hipStream_t st) {
  const int nseq = S * c->P;
  constexpr int NS = 8;
  dim3 grid((nseq + NS - 1) / NS, (c->nrp + 63) / 64, c->lmax + 1);
  if (is_f64(c)) {
    hipLaunchKernelGGL((k_legendre<double, NS>), grid, dim3(64), 0, st, c->lmax, c->ntheta, c->nrp, c->P, nseq,
                       c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw64, (const double2*)alm,
                       (double2*)F);
  } else {
    hipLaunchKernelGGL((k_legendre<float, NS>), grid, dim3(64), 0, st, c->lmax, c->ntheta, c->nrp, c->P, nseq,
                       c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw32, (const float2*)alm,
                       (float2*)F);
  }
  return hipGetLastError();
}

hipError_t launch_lambda_table(const modal_ctx* c, void* lam, hipStream_t st) {
  dim3 grid((c->nrp + 63) / 64, c->lmax + 1);
  if (is_f64(c))
    hipLaunchKernelGGL(k_lambda_table<double>, grid, dim3(64), 0, st, c->lmax, c->nrp, c->t.x, c->t.rec, c->t.seed,
                       c->t.lstart, (double*)lam);
  else
    hipLaunchKernelGGL(k_lambda_table<float>, grid, dim3(64), 0, st, c->lmax, c->nrp, c->t.x, c->t.rec, c->t.seed,
                       c->t.lstart, (float*)lam);
  return hipGetLastError();
}

hipError_t launch_adj_combine(const modal_ctx* c, const void* Z, int S, void* grad, hipStream_t st) {
  dim3 grid((c->lmax + 1 + 255) / 256, c->lmax + 1, S);
  if (is_f64(c))
    hipLaunchKernelGGL(k_adj_combine<double>, grid, dim3(256), 0, st, c->lmax, c->P, S, c->nalm, c->t.qw64,
                       (const double2*)Z, (double2*)grad);
  else
    hipLaunchKernelGGL(k_adj_combine<float>, grid, dim3(256), 0, st, c->lmax, c->P, S, c->nalm, c->t.qw32,
                       (const float2*)Z, (float2*)grad);
  return hipGetLastError();
}

}  // namespace modal
