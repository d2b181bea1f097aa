// Modal power-spectrum estimator (Sec. IV): the quadratic analogue of the cubic
// reduction, for every pair p <= r
//   beta_pr = sum_x w(x) (M_p(x) M_r(x) - V_pr(x)),
// with the filtered maps M of the bispectrum path and the Monte-Carlo pair means V
// of its linear-term state.  The mean term needs no pass over V: the state's
// harmonic transform holds Z_pr,00 = sum_x w V_pr lambda_00 with lambda_00 = 1/sqrt(4 pi),
// so sum_x w V_pr = sqrt(4 pi) Re Z_pr,00.
//
// The pixel sum is a symmetric rank-npix update, bound by reading the maps once
// (4 or 8 bytes per map value).  A workgroup takes a chunk of pixels of one sky,
// stages M and w M for 128 pixels at a time in LDS, and register-blocks the upper
// triangle of the P x P result in 4 x 4 blocks: nb (nb + 1) / 2 blocks, nb = ceil(P/4),
// each held by one thread per pixel phase (256 / blocks phases share the pixels of a
// stage).  Partial sums per (chunk, block) go to a buffer that one FP64 pass reduces.
#include "common.h"

#include <type_traits>

namespace modal {
namespace {

constexpr int PKC = 128;   // pixels per staged step (32 groups of 4)

// LDS row stride in elements: 16 bytes of padding move consecutive rows to different
// banks (the threads of a wave read different rows at the same pixel group)
template <typename T>
__host__ __device__ constexpr int pks() { return PKC + 16 / (int)sizeof(T); }

// thread -> (phase, block (rb, cb), rb <= cb); nblk = nb (nb + 1) / 2
__device__ inline void block_of(int b, int nb, int& rb, int& cb) {
  rb = 0;
  int left = nb;
  while (b >= left) {
    b -= left;
    ++rb;
    --left;
  }
  cb = rb + b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pair_sums(int P, int npix, int chunk_px, int nchunk, int vec,
                                                   const T* __restrict__ maps, const T* __restrict__ w,
                                                   double* __restrict__ part) {
  typedef typename std::conditional<sizeof(T) == 4, float4, double4>::type T4;
  extern __shared__ __attribute__((aligned(16))) unsigned char praw[];
  const int nb = (P + 3) / 4, PR = 4 * nb, nblk = nb * (nb + 1) / 2;
  const int nph = max(1, 256 / nblk);
  constexpr int PKS = pks<T>();
  T* Ms = reinterpret_cast<T*>(praw);        // [PR][PKS]
  T* Ws = Ms + (size_t)PR * PKS;              // [PR][PKS]  w * M
  const int chunk = blockIdx.x, s = blockIdx.y;
  const int tid = threadIdx.x;
  const int ph = tid / nblk, bk = tid - ph * nblk;
  const bool on = ph < nph;
  int rb = 0, cb = 0;
  if (on) block_of(bk, nb, rb, cb);
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0;
  const T* Msky = maps + (size_t)s * P * npix;
  const int x0 = chunk * chunk_px, x1 = min(npix, x0 + chunk_px);
  // 4-pixel groups: chunks start at multiples of 4 and npix % 4 == 0, so a group is
  // wholly inside or wholly past the chunk end; rows >= P stage zeros.  The next step's
  // groups are loaded into registers before this step's products, so that their latency
  // is hidden behind them.
  // (the group e = tid + 256 k has pixel group tid % 32 for every k: one weight group)
  constexpr int NPF = kMaxP * (PKC / 4) / 256;   // groups per thread at most (8)
  T4 pm[NPF], pw;
  auto load_step = [&](int xs) {
    const int x = xs + 4 * (tid % (PKC / 4));
    pw.x = pw.y = pw.z = pw.w = T(0);
    if (x < x1) pw = *reinterpret_cast<const T4*>(w + x);
#pragma unroll
    for (int k = 0; k < NPF; ++k) {
      const int r = (tid + 256 * k) / (PKC / 4);
      pm[k].x = pm[k].y = pm[k].z = pm[k].w = T(0);
      if (r < P && x < x1) pm[k] = *reinterpret_cast<const T4*>(Msky + (size_t)r * npix + x);
    }
  };
  if (vec) load_step(x0);
  for (int xs = x0; xs < x1; xs += PKC) {
    __syncthreads();
    if (vec) {
#pragma unroll
      for (int k = 0; k < NPF; ++k) {
        const int e = tid + 256 * k, r = e / (PKC / 4), g = e - r * (PKC / 4);
        if (r < PR) {
          *reinterpret_cast<T4*>(Ms + (size_t)r * PKS + 4 * g) = pm[k];
          T4 wm;
          wm.x = pw.x * pm[k].x;
          wm.y = pw.y * pm[k].y;
          wm.z = pw.z * pm[k].z;
          wm.w = pw.w * pm[k].w;
          *reinterpret_cast<T4*>(Ws + (size_t)r * PKS + 4 * g) = wm;
        }
      }
    } else {
      for (int e = tid; e < PR * PKC; e += 256) {
        const int r = e / PKC, i = e - r * PKC, x = xs + i;
        const bool in = r < P && x < x1;
        const T m = in ? Msky[(size_t)r * npix + x] : T(0);
        const T ww = x < x1 ? w[x] : T(0);
        Ms[(size_t)r * PKS + i] = m;
        Ws[(size_t)r * PKS + i] = ww * m;
      }
    }
    __syncthreads();
    if (vec && xs + PKC < x1) load_step(xs + PKC);
    if (on)
      for (int g = ph; g < PKC / 4; g += nph) {
        T4 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          a[i] = *reinterpret_cast<const T4*>(Ms + (size_t)(4 * rb + i) * PKS + 4 * g);
          b[i] = *reinterpret_cast<const T4*>(Ws + (size_t)(4 * cb + i) * PKS + 4 * g);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[i][j] = fma(a[i].x, b[j].x, acc[i][j]);
            acc[i][j] = fma(a[i].y, b[j].y, acc[i][j]);
            acc[i][j] = fma(a[i].z, b[j].z, acc[i][j]);
            acc[i][j] = fma(a[i].w, b[j].w, acc[i][j]);
          }
      }
  }
  // sum the phases of each block in LDS (FP64), then one thread per block entry writes
  __syncthreads();
  double* red = reinterpret_cast<double*>(praw);   // [nblk][16]
  for (int e = tid; e < nblk * 16; e += 256) red[e] = 0.0;
  __syncthreads();
  for (int p = 0; p < nph; ++p) {
    if (on && ph == p)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[bk * 16 + 4 * i + j] += (double)acc[i][j];
    __syncthreads();
  }
  double* dst = part + ((size_t)s * nchunk + chunk) * nblk * 16;
  for (int e = tid; e < nblk * 16; e += 256) dst[e] = red[e];
}

// beta[s][pair(a, b)] = sum over chunks of the block entry (a, b) minus sqrt(4 pi) Re Z_ab,00.
template <typename Z>
__global__ __launch_bounds__(256) void k_pair_reduce(int P, int npairs, int nchunk, int S, const double* __restrict__ part,
                                                     const int* __restrict__ pair_a, const int* __restrict__ pair_b,
                                                     const Z* __restrict__ zst, size_t zstride, double* __restrict__ beta) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= S * npairs) return;
  const int s = e / npairs, pr = e - s * npairs;
  const int a = pair_a[pr], b = pair_b[pr];
  const int nb = (P + 3) / 4, nblk = nb * (nb + 1) / 2;
  const int rb = a / 4, cb = b / 4;
  const int blk = rb * nb - rb * (rb - 1) / 2 + (cb - rb);
  const int slot = blk * 16 + 4 * (a - 4 * rb) + (b - 4 * cb);
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += part[((size_t)s * nchunk + c) * nblk * 16 + slot];
  if (zst) acc -= 3.5449077018110320546 * (double)zst[(size_t)pr * zstride];   // sqrt(4 pi) Re Z_ab,00
  beta[e] = acc;
}

// The estimator's modes are the isotropic R_n(l) = q_0(l) q_n(l), n < P: the pairs (0, n),
// the first P entries of each row of pair sums.
// alpha[n] = sum_l (2l + 1) qw_0(l) qw_n(l) dcl(l)   (qw = q / sqrt(C))
__global__ __launch_bounds__(256) void k_power_alpha(int lmax, int P, const double* __restrict__ qw,
                                                     const double* __restrict__ dcl, double* __restrict__ alpha) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= P) return;
  const double* q0 = qw;
  const double* qn = qw + (size_t)n * (lmax + 1);
  double acc = 0.0;
  for (int l = 0; l <= lmax; ++l) acc = fma((2.0 * l + 1.0) * q0[l] * qn[l], dcl[l], acc);
  alpha[n] = acc;
}

// X[l][n] = sqrt(2l + 1) c_l q_0(l) q_n(l): zeta = X^T X is the ideal covariance
__global__ __launch_bounds__(256) void k_power_rows(int lmax, int P, const double* __restrict__ q,
                                                    const double* __restrict__ c, double* __restrict__ X) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= (lmax + 1) * P) return;
  const int l = e / P, n = e - l * P;
  X[e] = sqrt(2.0 * l + 1.0) * c[l] * q[l] * q[(size_t)n * (lmax + 1) + l];
}

}  // namespace

int power_chunk_px() { return 16384; }

size_t power_part_bytes(int P, int npix, int S) {
  const int nb = (P + 3) / 4, nblk = nb * (nb + 1) / 2;
  const size_t nchunk = (npix + power_chunk_px() - 1) / power_chunk_px();
  return (size_t)S * nchunk * nblk * 16 * 8;
}

size_t power_lds(int P, bool f64) {
  const int nb = (P + 3) / 4;
  const size_t stage = f64 ? (size_t)2 * 4 * nb * pks<double>() * 8 : (size_t)2 * 4 * nb * pks<float>() * 4;
  const size_t red = (size_t)nb * (nb + 1) / 2 * 16 * 8;
  return stage > red ? stage : red;
}

hipError_t power_set_lds() {
  const size_t mx = power_lds(kMaxP, true);
  hipError_t e = hipFuncSetAttribute((const void*)k_pair_sums<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)mx);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_pair_sums<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx);
}

hipError_t launch_power_beta(const modal_ctx* c, const void* maps, int S, const void* zstate, double* part,
                             double* beta, hipStream_t st) {
  const bool f64 = c->prec == MODAL_F64;
  const int cpx = power_chunk_px();
  const int nchunk = (c->npix + cpx - 1) / cpx;
  const size_t lds = power_lds(c->P, f64);
  const int vec = c->npix % 4 == 0 ? 1 : 0;
  if (f64)
    hipLaunchKernelGGL(k_pair_sums<double>, dim3(nchunk, S), dim3(256), lds, st, c->P, c->npix, cpx, nchunk, vec,
                       (const double*)maps, c->t.w64, part);
  else
    hipLaunchKernelGGL(k_pair_sums<float>, dim3(nchunk, S), dim3(256), lds, st, c->P, c->npix, cpx, nchunk, vec,
                       (const float*)maps, c->t.w32, part);
  const int tot = S * c->npairs;
  const size_t zstride = (size_t)c->nalm * 2;   // complex entries: real part of entry 0 of each pair row
  if (f64)
    hipLaunchKernelGGL(k_pair_reduce<double>, dim3((tot + 255) / 256), dim3(256), 0, st, c->P, c->npairs, nchunk, S,
                       part, c->t.pair_a, c->t.pair_b, (const double*)zstate, zstride, beta);
  else
    hipLaunchKernelGGL(k_pair_reduce<float>, dim3((tot + 255) / 256), dim3(256), 0, st, c->P, c->npairs, nchunk, S,
                       part, c->t.pair_a, c->t.pair_b, (const float*)zstate, zstride, beta);
  return hipGetLastError();
}

hipError_t launch_power_alpha(const modal_ctx* c, const double* dcl, double* alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_power_alpha, dim3((c->P + 255) / 256), dim3(256), 0, st, c->lmax, c->P, c->t.qw64, dcl, alpha);
  return hipGetLastError();
}

hipError_t launch_power_rows(const modal_ctx* c, const double* q, const double* cw, double* X, hipStream_t st) {
  const int tot = (c->lmax + 1) * c->P;
  hipLaunchKernelGGL(k_power_rows, dim3((tot + 255) / 256), dim3(256), 0, st, c->lmax, c->P, q, cw, X);
  return hipGetLastError();
}

}  // namespace modal
