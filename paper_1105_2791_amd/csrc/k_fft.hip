// Ring FFTs in LDS (Stockham autosort, mixed radix).
//
// c2r (synthesis):  M(theta_j, phi_k) = Re F_0 + 2 Re sum_{m=1}^{lmax} F_m e^{i m phi_k},
//                   phi_k = 2 pi k / N, N = nphi even, lmax < N/2.
// The length-N real transform is one complex transform of length K = N/2:
//   Z_m = (X_m + X*_{K-m}) + i e^{2 pi i m / N} (X_m - X*_{K-m}),  z = sum_m Z_m e^{2 pi i m n / K},
//   M_{2n} = Re z_n, M_{2n+1} = Im z_n,
// with X_m = F_m (m <= lmax), 0 otherwise, and X_0 real.
// r2c (adjoint):    Gh_m = sum_k G_k e^{-i m phi_k} for m <= lmax, from
//   z_n = G_{2n} + i G_{2n+1}, Z = sum_n z_n e^{-2 pi i m n / K},
//   Gh_m = (Z_m + Z*_{K-m}) / 2 - (i/2) e^{-2 pi i m / N} (Z_m - Z*_{K-m}).
// One workgroup per ring row; twiddles tw[t] = e^{2 pi i t / N} come from an FP64
// table (rounded to the working precision).
#include "common.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace modal {
namespace {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

template <typename T2>
__device__ inline T2 cmul(T2 a, T2 b) {
  T2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// One Stockham stage of an odd prime radix R known at compile time, float data.  Each
// butterfly's R inputs are twiddled once into registers (stage twiddle index kept
// incrementally, no division), then the R-point DFT pairs r with R - r:
//   out_q = a_0 + sum_{j=1}^{(R-1)/2} [(a_j + a_{R-j}) Re w^{jq} + i (a_j - a_{R-j}) Im w^{jq}],
// w = exp(sign 2 pi i / R), whose powers are held in registers (the indices j q mod R are
// compile-time).  R^2 / 2 complex multiply-adds per butterfly, no LDS re-reads.
template <typename T2, int SIGN, int R>
__device__ inline void prime_stage(const T2* __restrict__ in0, T2* __restrict__ out0, int K, int Ns,
                                   const T2* __restrict__ tw, int nring) {
  constexpr int H = (R - 1) / 2;
  const int KR = K / R;
  const int step = K / (Ns * R);
  T2 wr[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    wr[m] = tw[2 * m * KR];                 // exp(2 pi i m / R) = exp(2 pi i m KR / K)
    if (SIGN < 0) wr[m].y = -wr[m].y;
  }
  // the butterflies of all nring rings are dealt to the threads together (a ring alone has
  // K / R of them: 64 for R = 47 at K = 3008, a quarter of the workgroup)
  for (int bb = threadIdx.x; bb < nring * KR; bb += blockDim.x) {
    const int ring = bb / KR, b = bb - ring * KR;
    const T2* in = in0 + (size_t)ring * K;
    T2* out = out0 + (size_t)ring * K;
    const int k = b % Ns;
    const int obase = (b / Ns) * Ns * R + k;
    const int dt = k * step;                // < K: the stage twiddle of input r is exp(2 pi i r dt / K)
    const T2 a0 = in[b];
    T2 s[H], d[H], hi[H];
    int t = 0;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      t += dt;
      if (t >= K) t -= K;
      T2 w = tw[2 * t];
      if (SIGN < 0) w.y = -w.y;
      const T2 a = cmul(in[b + r * KR], w);
      if (r <= H) {
        hi[r - 1] = a;
      } else {
        const T2 lo = hi[R - r - 1];       // a_{R-r}, R - r <= H
        s[R - r - 1].x = lo.x + a.x; s[R - r - 1].y = lo.y + a.y;
        d[R - r - 1].x = lo.x - a.x; d[R - r - 1].y = lo.y - a.y;
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      T2 acc = a0;
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const T2 w = wr[(j * q) % R];
        acc.x += s[j - 1].x * w.x - d[j - 1].y * w.y;
        acc.y += s[j - 1].y * w.x + d[j - 1].x * w.y;
      }
      out[obase + q * Ns] = acc;
    }
  }
}

// One Stockham stage of radix R on K points: out = stage(in).  sign = +1 for
// e^{+i}, -1 for e^{-i}.  Twiddle exp(sign 2 pi i t / K) = tw[2 t] (conjugated for sign -1).
// PR: a large prime radix with its own compiled stage (0: none).
template <typename T2, int SIGN, int PR>
__device__ inline void stockham_stage(const T2* __restrict__ in0, T2* __restrict__ out0, int K, int Ns, int R,
                                      const T2* __restrict__ tw, int nring) {
  if constexpr (sizeof(T2) == 8) {   // float data: compiled odd-prime stages
    if (R == 3) return prime_stage<T2, SIGN, 3>(in0, out0, K, Ns, tw, nring);
    if (R == 5) return prime_stage<T2, SIGN, 5>(in0, out0, K, Ns, tw, nring);
    if (R == 7) return prime_stage<T2, SIGN, 7>(in0, out0, K, Ns, tw, nring);
    if constexpr (PR > 7)
      if (R == PR) return prime_stage<T2, SIGN, PR>(in0, out0, K, Ns, tw, nring);
  }
  const int KR = K / R;
  const int step = K / (Ns * R);  // exp(2 pi i u / (Ns R)) = exp(2 pi i u step / K)
  for (int bb = threadIdx.x; bb < nring * KR; bb += blockDim.x) {
    const int ring = bb / KR, b = bb - ring * KR;
    const T2* in = in0 + (size_t)ring * K;
    T2* out = out0 + (size_t)ring * K;
    const int k = b % Ns;
    const int obase = (b / Ns) * Ns * R + k;
    if (R == 2) {
      const T2 a0 = in[b];
      T2 a1 = in[b + KR];
      T2 w = tw[2 * ((k * step) % K)];
      if (SIGN < 0) w.y = -w.y;
      a1 = cmul(a1, w);
      T2 y0, y1;
      y0.x = a0.x + a1.x; y0.y = a0.y + a1.y;
      y1.x = a0.x - a1.x; y1.y = a0.y - a1.y;
      out[obase] = y0;
      out[obase + Ns] = y1;
    } else if (R == 4) {
      T2 a[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a[r] = in[b + r * KR];
        if (r) {
          T2 w = tw[2 * ((r * k * step) % K)];
          if (SIGN < 0) w.y = -w.y;
          a[r] = cmul(a[r], w);
        }
      }
      // radix-4 DFT with e^{sign i pi/2} = sign * i
      T2 s02, d02, s13, d13;
      s02.x = a[0].x + a[2].x; s02.y = a[0].y + a[2].y;
      d02.x = a[0].x - a[2].x; d02.y = a[0].y - a[2].y;
      s13.x = a[1].x + a[3].x; s13.y = a[1].y + a[3].y;
      d13.x = a[1].x - a[3].x; d13.y = a[1].y - a[3].y;
      // j * d13 where j = sign * i
      T2 jd;
      jd.x = -SIGN * d13.y;
      jd.y = SIGN * d13.x;
      T2 y0, y1, y2, y3;
      y0.x = s02.x + s13.x; y0.y = s02.y + s13.y;
      y2.x = s02.x - s13.x; y2.y = s02.y - s13.y;
      y1.x = d02.x + jd.x;  y1.y = d02.y + jd.y;
      y3.x = d02.x - jd.x;  y3.y = d02.y - jd.y;
      out[obase] = y0;
      out[obase + Ns] = y1;
      out[obase + 2 * Ns] = y2;
      out[obase + 3 * Ns] = y3;
    } else {
      // generic radix: direct DFT with the combined twiddle exp(sign 2 pi i r (k + q Ns) / (Ns R)),
      // its index r (k + q Ns) step mod K advanced incrementally over r
      for (int q = 0; q < R; ++q) {
        T2 acc;
        acc.x = 0;
        acc.y = 0;
        const int dt = (int)(((long long)(k + q * Ns) * step) % K);
        int t = 0;
        for (int r = 0; r < R; ++r) {
          const T2 a = in[b + r * KR];
          T2 w = tw[2 * t];
          if (SIGN < 0) w.y = -w.y;
          const T2 p = cmul(a, w);
          acc.x += p.x;
          acc.y += p.y;
          t += dt;
          if (t >= K) t -= K;
        }
        out[obase + q * Ns] = acc;
      }
    }
  }
}

// Stage over R independent transforms of length K stored back to back.
template <typename T2, int SIGN, int PR>
__device__ inline void stockham_stage_multi(const T2* __restrict__ in, T2* __restrict__ out, int K, int R, int Ns,
                                            int Rf, const T2* __restrict__ tw) {
  stockham_stage<T2, SIGN, PR>(in, out, K, Ns, Rf, tw, R);
}

// c2r, generic radices: one workgroup per (sequence, block of R consecutive rings),
// two LDS buffers (Stockham ping-pong).  Used for FP64 and for ring lengths whose
// factors the register kernel below does not cover.
template <typename T, int PR>
__global__ __launch_bounds__(256) void k_fft_c2r(FftPlan plan, int lmax, int ntheta, int R,
                                                 const typename vec2<T>::type* __restrict__ F,
                                                 T* __restrict__ maps, const typename vec2<T>::type* __restrict__ tw) {
  using T2 = typename vec2<T>::type;
  extern __shared__ char smem[];
  const int K = plan.K;
  T2* b0 = reinterpret_cast<T2*>(smem);
  T2* b1 = b0 + (size_t)R * K;
  const int nrb = (ntheta + R - 1) / R;
  const int seq = blockIdx.x / nrb;
  const int j0 = (blockIdx.x - seq * nrb) * R;
  const int nr = min(R, ntheta - j0);
  const int nrb8 = f_ring_blocks(ntheta);
  // X_m (zero beyond lmax, X_0 real) into b1, ring-major
  for (int e = threadIdx.x; e < R * K; e += blockDim.x) {
    const int m = e / R, r = e - m * R;
    T2 x;
    x.x = x.y = T(0);
    if (m <= lmax && r < nr) x = F[f_index(seq, j0 + r, m, lmax, nrb8)];
    if (m == 0) x.y = T(0);
    b1[(size_t)r * K + m] = x;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < R * K; e += blockDim.x) {
    const int r = e / K, m = e - r * K;
    const T2 xm = b1[(size_t)r * K + m];
    T2 xk;
    xk.x = xk.y = T(0);
    if (m > 0) xk = b1[(size_t)r * K + (K - m)];   // X_K = 0 since lmax < K
    T2 a, d;
    a.x = xm.x + xk.x; a.y = xm.y - xk.y;   // X_m + conj(X_{K-m})
    d.x = xm.x - xk.x; d.y = xm.y + xk.y;   // X_m - conj(X_{K-m})
    const T2 ew = tw[m];
    T2 z;
    z.x = a.x - (ew.x * d.y + ew.y * d.x);
    z.y = a.y + (ew.x * d.x - ew.y * d.y);
    b0[(size_t)r * K + m] = z;
  }
  __syncthreads();
  T2* in = b0;
  T2* out = b1;
  int Ns = 1;
  for (int f = 0; f < plan.nf; ++f) {
    const int Rf = plan.radix[f];
    stockham_stage_multi<T2, +1, PR>(in, out, K, R, Ns, Rf, tw);
    __syncthreads();
    T2* tmp = in; in = out; out = tmp;
    Ns *= Rf;
  }
  for (int r = 0; r < nr; ++r) {
    T2* dst = reinterpret_cast<T2*>(maps + ((size_t)seq * ntheta + j0 + r) * plan.N);
    for (int n = threadIdx.x; n < K; n += blockDim.x) dst[n] = in[(size_t)r * K + n];
  }
}

// r2c: G rows [seq][ring][pixel] -> Gh [seq][m][ring], m <= lmax.
template <typename T, int PR>
__global__ __launch_bounds__(256) void k_fft_r2c(FftPlan plan, int lmax, int ntheta, int R, const T* __restrict__ G,
                                                 typename vec2<T>::type* __restrict__ Gh,
                                                 const typename vec2<T>::type* __restrict__ tw) {
  using T2 = typename vec2<T>::type;
  extern __shared__ char smem[];
  const int K = plan.K;
  T2* b0 = reinterpret_cast<T2*>(smem);
  T2* b1 = b0 + (size_t)R * K;
  const int nrb = (ntheta + R - 1) / R;
  const int seq = blockIdx.x / nrb;
  const int j0 = (blockIdx.x - seq * nrb) * R;
  const int nr = min(R, ntheta - j0);
  for (int r = 0; r < R; ++r) {
    const T2* src = reinterpret_cast<const T2*>(G + ((size_t)seq * ntheta + j0 + min(r, nr - 1)) * plan.N);
    for (int n = threadIdx.x; n < K; n += blockDim.x) {
      T2 v = src[n];
      if (r >= nr) v.x = v.y = T(0);
      b0[(size_t)r * K + n] = v;
    }
  }
  __syncthreads();
  T2* in = b0;
  T2* out = b1;
  int Ns = 1;
  for (int f = 0; f < plan.nf; ++f) {
    const int Rf = plan.radix[f];
    stockham_stage_multi<T2, -1, PR>(in, out, K, R, Ns, Rf, tw);
    __syncthreads();
    T2* tmp = in; in = out; out = tmp;
    Ns *= Rf;
  }
  T2* dst = Gh + (size_t)seq * (lmax + 1) * ntheta;
  for (int e = threadIdx.x; e < (lmax + 1) * R; e += blockDim.x) {
    const int m = e / R, r = e - m * R;
    if (r >= nr) continue;
    const T2 zk = in[(size_t)r * K + (m % K)];
    const T2 zm = in[(size_t)r * K + ((K - m) % K)];
    T2 a, d;
    a.x = zk.x + zm.x; a.y = zk.y - zm.y;   // Z_m + conj(Z_{K-m})
    d.x = zk.x - zm.x; d.y = zk.y + zm.y;   // Z_m - conj(Z_{K-m})
    const T2 ew = tw[m];                    // e^{+2 pi i m / N}; use its conjugate (c, -s)
    // -(i/2) (c - i s) d = 0.5 (c d.y - s d.x) - 0.5 i (c d.x + s d.y)
    T2 g;
    g.x = T(0.5) * (a.x + (ew.x * d.y - ew.y * d.x));
    g.y = T(0.5) * (a.y - (ew.x * d.x + ew.y * d.y));
    dst[(size_t)m * ntheta + j0 + r] = g;
  }
}


// ---------------------------------------------------------------------------
// c2r, register passes: one wave per ring, 4 rings per workgroup (half of one
// f_index ring group).  The group's spectra are one contiguous block of F; the two
// halves of a group run on the same XCD back to back (block b -> XCD b % 8), so a
// cache line of F is fetched once.  Each pass of the mixed-radix (8, 4, 2, 3, 5)
// Stockham transform reads all of a lane's butterfly inputs from the ring's LDS
// buffer into registers, then writes the outputs in place: one wave owns the
// buffer, and its LDS accesses complete in program order, so no barrier is needed
// between passes.  LDS indices are padded by one element per 16 against bank
// conflicts of the strided early passes.
// ---------------------------------------------------------------------------
constexpr int RG_RINGS = 4;            // rings (waves) per workgroup
constexpr int RG_KMAX = 2048;          // longest complex transform of the register kernel

// LDS padding of the register-pass ring buffers: one slot after every 8 points, so that
// the strided writes of the early passes and the interleaved spectrum stores hit
// distinct banks
__device__ inline int padr(int i) { return i + (i >> 3); }

__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cmulf(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cmuli(float2 a) { return make_float2(-a.y, a.x); }            // i a
__device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// y_q = sum_r x_r e^{+2 pi i r q / R}, in place
template <int R>
__device__ inline void dft_plus(float2* x) {
  if (R == 2) {
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if (R == 4) {
    const float2 s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    const float2 s13 = cadd(x[1], x[3]), d13 = cmuli(csub(x[1], x[3]));
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, d13);
    x[3] = csub(d02, d13);
  } else if (R == 8) {
    const float h = 0.70710678118654752f;
    float2 a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = cadd(x[r], x[r + 4]);
      b[r] = csub(x[r], x[r + 4]);
    }
    b[1] = make_float2(h * (b[1].x - b[1].y), h * (b[1].x + b[1].y));    // e^{i pi / 4}
    b[2] = cmuli(b[2]);                                                  // e^{i pi / 2}
    b[3] = make_float2(-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y));   // e^{3 i pi / 4}
    dft_plus<4>(a);
    dft_plus<4>(b);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[2 * q] = a[q];
      x[2 * q + 1] = b[q];
    }
  } else if (R == 3) {
    const float s3 = 0.86602540378443865f;
    const float2 t = cadd(x[1], x[2]), d = cscale(cmuli(csub(x[1], x[2])), s3);
    const float2 m = csub(x[0], cscale(t, 0.5f));
    x[0] = cadd(x[0], t);
    x[1] = cadd(m, d);
    x[2] = csub(m, d);
  } else if (R == 5) {
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
    const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
    const float2 t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    const float2 d1 = csub(x[1], x[4]), d2 = csub(x[2], x[3]);
    const float2 a1 = cadd(x[0], cadd(cscale(t1, c1), cscale(t2, c2)));
    const float2 a2 = cadd(x[0], cadd(cscale(t1, c2), cscale(t2, c1)));
    const float2 b1 = cmuli(cadd(cscale(d1, s1), cscale(d2, s2)));
    const float2 b2 = cmuli(csub(cscale(d1, s2), cscale(d2, s1)));
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(a1, b1);
    x[4] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[3] = csub(a2, b2);
  } else if (R == 24) {
    // 24 = 3 x 8 (Cooley-Tukey): input index 8 n1 + n2, output index k1 + 3 k2;
    //   y[k1][n2] = e^{2 pi i n2 k1 / 24} sum_n1 x[8 n1 + n2] e^{2 pi i n1 k1 / 3},
    //   X[k1 + 3 k2] = sum_n2 y[k1][n2] e^{2 pi i n2 k2 / 8}.
    // e^{i pi j / 12} = (cos 15 j deg, sin 15 j deg), j = n2 k1 <= 14
    const float cw[15] = {1.f, 0.96592582628906829f, 0.86602540378443865f, 0.70710678118654752f, 0.5f,
                          0.25881904510252076f, 0.f, -0.25881904510252076f, -0.5f, -0.70710678118654752f,
                          -0.86602540378443865f, -0.96592582628906829f, -1.f, -0.96592582628906829f,
                          -0.86602540378443865f};
    const float sw[15] = {0.f, 0.25881904510252076f, 0.5f, 0.70710678118654752f, 0.86602540378443865f,
                          0.96592582628906829f, 1.f, 0.96592582628906829f, 0.86602540378443865f,
                          0.70710678118654752f, 0.5f, 0.25881904510252076f, 0.f, -0.25881904510252076f, -0.5f};
    float2 y[3][8];
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) {
      float2 t[3] = {x[n2], x[8 + n2], x[16 + n2]};
      dft_plus<3>(t);
      y[0][n2] = t[0];
#pragma unroll
      for (int k1 = 1; k1 < 3; ++k1)
        y[k1][n2] = (n2 == 0) ? t[k1] : cmulf(t[k1], make_float2(cw[n2 * k1], sw[n2 * k1]));
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      dft_plus<8>(y[k1]);
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) x[k1 + 3 * k2] = y[k1][k2];
    }
  }
}

// one Stockham pass of radix R over the ring buffer b (length K); twp is this pass's
// twiddle table, twp[(q - 1) Ns + k] = e^{2 pi i q k / (Ns R)}, laid out so that the
// lanes of a wave (consecutive k) read consecutive entries
// PTS: the most points a lane holds in any pass of the plan (register budget)
// OUT: the last pass writes its (natural-order) output to the global row out instead
// of back to b (nothing when out is null: a padding ring)
// KC, NSC: the ring length and the pass's stride when known at compile time (0: from
// the arguments), so that the index arithmetic of a specialised plan folds to constants
template <int R, int PTS, bool OUT = false, int KC = 0, int NSC = 0>
__device__ inline void rg_pass(float2* b, int K_, int Ns_, int lane, const float2* twp, float2* out = nullptr) {
  constexpr int NB = KC ? (KC / R + 63) / 64 : (PTS + R - 1) / R;
  const int K = KC ? KC : K_;
  const int Ns = NSC ? NSC : Ns_;
  const int KR = K / R;
  float2 v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int bi = lane + 64 * i;
    if (bi < KR) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[i][q] = b[padr(bi + q * KR)];
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int bi = lane + 64 * i;
    if (bi < KR) {
      const int k = bi % Ns;
      if (NSC != 1) {   // (the first pass's twiddles are all 1)
#pragma unroll
        for (int q = 1; q < R; ++q) v[i][q] = cmulf(v[i][q], twp[(q - 1) * Ns + k]);
      }
      dft_plus<R>(v[i]);
      const int ob = (bi / Ns) * Ns * R + k;
      if (OUT) {
        if (out) {
#pragma unroll
          for (int q = 0; q < R; ++q) out[ob + q * Ns] = v[i][q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) b[padr(ob + q * Ns)] = v[i][q];
      }
    }
  }
}

// cos and sin of 2 pi j / 47, j < 47, rounded to float
__device__ constexpr float kC47[47] = {
    1.0f, 0.991077488f, 0.964469175f, 0.920649887f, 0.860401579f, 0.784799385f, 0.695192428f,
    0.593179745f, 0.480581755f, 0.359407773f, 0.23182015f, 0.100095692f, -0.033414977f, -0.166329355f,
    -0.296275581f, -0.420934762f, -0.538082353f, -0.645627852f, -0.741652106f, -0.82444156f, -0.892518836f,
    -0.944669092f, -0.979961705f, -0.997766879f, -0.997766879f, -0.979961705f, -0.944669092f, -0.892518836f,
    -0.82444156f, -0.741652106f, -0.645627852f, -0.538082353f, -0.420934762f, -0.296275581f, -0.166329355f,
    -0.033414977f, 0.100095692f, 0.23182015f, 0.359407773f, 0.480581755f, 0.593179745f, 0.695192428f,
    0.784799385f, 0.860401579f, 0.920649887f, 0.964469175f, 0.991077488f};
__device__ constexpr float kS47[47] = {
    0.0f, 0.133286955f, 0.264195402f, 0.390389275f, 0.509616643f, 0.619749889f, 0.718823684f,
    0.805070053f, 0.876949928f, 0.933180611f, 0.972758664f, 0.994977815f, 0.999441564f, 0.986070254f,
    0.955102497f, 0.907090914f, 0.842892271f, 0.763652197f, 0.67078473f, 0.565947094f, 0.451010119f,
    0.328024858f, 0.199185985f, 0.0667926337f, -0.0667926337f, -0.199185985f, -0.328024858f, -0.451010119f,
    -0.565947094f, -0.67078473f, -0.763652197f, -0.842892271f, -0.907090914f, -0.955102497f, -0.986070254f,
    -0.999441564f, -0.994977815f, -0.972758664f, -0.933180611f, -0.876949928f, -0.805070053f, -0.718823684f,
    -0.619749889f, -0.509616643f, -0.390389275f, -0.264195402f, -0.133286955f};

// The first pass of a ring of K = 47 x 64 points (stride 1, so no twiddles): one
// 47-point DFT per lane, y_q = sum_r x_r e^{+2 pi i r q / 47} of x_r = b[lane + 64 r],
// into b[47 lane + q].  The inputs r and 47 - r are paired, s_r = x_r + x_{47-r},
// d_r = x_r - x_{47-r} (r = 1..23), so that one cosine sum and one sine sum give two
// outputs:
//   y_q = A_q + i B_q,  y_{47-q} = A_q - i B_q,
//   A_q = x_0 + sum_r s_r cos(2 pi r q / 47),  B_q = sum_r d_r sin(2 pi r q / 47),
// each pair stored as soon as it is formed.  All the wave's loads precede its stores in
// program order, and LDS accesses of one wave complete in order, so the pass is in place.
__device__ inline void rg_pass47_first(float2* b, int lane) {
  float2 x[47];
#pragma unroll
  for (int r = 0; r < 47; ++r) x[r] = b[padr(lane + 64 * r)];
#pragma unroll
  for (int r = 1; r < 24; ++r) {
    const float2 sr = cadd(x[r], x[47 - r]), dr = csub(x[r], x[47 - r]);
    x[r] = sr;
    x[47 - r] = dr;
  }
  const int ob = 47 * lane;
  float2 y0 = x[0];
#pragma unroll
  for (int r = 1; r < 24; ++r) y0 = cadd(y0, x[r]);
  b[padr(ob)] = y0;
#pragma unroll
  for (int q = 1; q < 24; ++q) {
    float2 A = x[0], B = make_float2(0.f, 0.f);
#pragma unroll
    for (int r = 1; r < 24; ++r) {
      const int j = (r * q) % 47;
      A.x = fmaf(x[r].x, kC47[j], A.x);
      A.y = fmaf(x[r].y, kC47[j], A.y);
      B.x = fmaf(x[47 - r].x, kS47[j], B.x);
      B.y = fmaf(x[47 - r].y, kS47[j], B.y);
    }
    b[padr(ob + q)] = make_float2(A.x - B.y, A.y + B.x);
    b[padr(ob + 47 - q)] = make_float2(A.x + B.y, A.y - B.x);
  }
}

template <int PTS, int KC>
__device__ __forceinline__ void c2r_rg_body(FftPlan plan, int lmax, int ntheta, int nseq,
                                            const float2* __restrict__ F, float* __restrict__ maps,
                                            const float2* __restrict__ twg, const float2* __restrict__ twpg) {
  extern __shared__ __attribute__((aligned(16))) float2 rbuf[];
  const int K = KC ? KC : plan.K;   // KC: a plan compiled in (24 x 8 x 8 of K = 1536, 47 x 8 x 8 of 3008)
  const int KP = padr(K) + 1;
  float2* tw = rbuf + RG_RINGS * KP;   // e^{2 pi i t / N}, t <= K / 2, shared by the workgroup's rings
  float2* twp = tw + K / 2 + 1;          // the passes' twiddle tables, K - 1 entries in all
  const int nrb8 = f_ring_blocks(ntheta);
  const int units = nseq * nrb8;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: the ring row base stays scalar
  for (int t = tid; t <= K / 2; t += 64 * RG_RINGS) tw[t] = twg[t];
  for (int t = tid; t < K - 1; t += 64 * RG_RINGS) twp[t] = twpg[t];
  // persistent: workgroups b and b + 8 (one XCD) take the two halves of the same ring
  // groups, xcd + 8 (slot + k nslot), k = 0, 1, ...
  const int b = blockIdx.x;
  const int xcd = b & 7, half = (b >> 3) & 1, slot = b >> 4;
  const int nslot = gridDim.x >> 4;
  for (int unit = xcd + 8 * slot; unit < units; unit += 8 * nslot) {
    const int seq = unit / nrb8, rb = unit - seq * nrb8;
    // previous unit's buffers (and the twiddle table) are settled; its map stores stay in
    // flight (the workgroup never reads them back)
    lds_barrier();
    // spectra of the four rings (F block of ring group rb, rings 4 half .. 4 half + 3;
    // float4 = rings (2 rp, 2 rp + 1) at one m) go straight into the buffers as the input
    // of the half-length complex transform:
    //   Z_m = (X_m + conj X_{K-m}) + i e^{2 pi i m / N} (X_m - conj X_{K-m}),  m < K,
    // with X_m = F_m for m <= lmax (X_0 real) and 0 otherwise.  Element e = (m, rp), both
    // loads unconditional (index clamped, value selected after), ZE elements per thread
    // per round.
    const float4* src = reinterpret_cast<const float4*>(F + (size_t)unit * (lmax + 1) * 8 + RG_RINGS * half);
    constexpr int ZE = 4;
    for (int e0 = 0; e0 < 2 * K; e0 += ZE * 64 * RG_RINGS) {
      float4 xa[ZE], xb[ZE];
#pragma unroll
      for (int i = 0; i < ZE; ++i) {
        const int e = min(e0 + tid + i * 64 * RG_RINGS, 2 * K - 1);
        const int m = e >> 1, rp = e & 1;
        xa[i] = src[(size_t)min(m, lmax) * 4 + rp];
        xb[i] = src[(size_t)min(K - m, lmax) * 4 + rp];
      }
#pragma unroll
      for (int i = 0; i < ZE; ++i) {
        const int e = e0 + tid + i * 64 * RG_RINGS;
        if (e < 2 * K) {
          const int m = e >> 1, rp = e & 1;
          const bool ha = m <= lmax, hb = m > 0 && K - m <= lmax;
          const float2 ew = (m <= K / 2) ? tw[m] : make_float2(-tw[K - m].x, tw[K - m].y);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            float2 X = ha ? (j ? make_float2(xa[i].z, xa[i].w) : make_float2(xa[i].x, xa[i].y)) : make_float2(0.f, 0.f);
            if (m == 0) X.y = 0.f;
            const float2 Y = hb ? (j ? make_float2(xb[i].z, xb[i].w) : make_float2(xb[i].x, xb[i].y)) : make_float2(0.f, 0.f);
            const float2 sa = make_float2(X.x + Y.x, X.y - Y.y), d = make_float2(X.x - Y.x, X.y + Y.y);
            rbuf[(2 * rp + j) * KP + padr(m)] =
                make_float2(sa.x - (ew.x * d.y + ew.y * d.x), sa.y + (ew.x * d.x - ew.y * d.y));
          }
        }
      }
    }
    __syncthreads();

    float2* bw = rbuf + w * KP;
    // z = sum_m Z_m e^{+2 pi i m n / K}; the last pass writes the map row directly:
    // M_{2n} = Re z_n, M_{2n+1} = Im z_n
    const int j = rb * 8 + RG_RINGS * half + w;
    float2* dst = (j < ntheta) ? reinterpret_cast<float2*>(maps + ((size_t)seq * ntheta + j) * plan.N) : nullptr;
    if constexpr (KC == 1536) {
      // passes 24, 8, 8 (strides 1, 24, 192; twiddle tables at 0, 23, 23 + 7 * 24)
      rg_pass<24, PTS, false, KC, 1>(bw, K, 1, lane, twp);
      rg_pass<8, PTS, false, KC, 24>(bw, K, 24, lane, twp + 23);
      rg_pass<8, PTS, true, KC, 192>(bw, K, 192, lane, twp + 23 + 7 * 24, dst);
    } else if constexpr (KC == 3008) {
      // passes 47, 8, 8 (strides 1, 47, 376; twiddle tables at 46, 46 + 7 * 47)
      rg_pass47_first(bw, lane);
      rg_pass<8, PTS, false, KC, 47>(bw, K, 47, lane, twp + 46);
      rg_pass<8, PTS, true, KC, 376>(bw, K, 376, lane, twp + 46 + 7 * 47, dst);
    } else {
      int Ns = 1;
      const float2* tf = twp;
      // (a last pass of radix 8, the common case, stores straight to the row; other plans
      // finish in LDS and copy the row out)
      const bool direct = plan.radix[plan.nf - 1] == 8;
      for (int f = 0; f < plan.nf; ++f) {
        const int R = plan.radix[f];
        if (direct && f == plan.nf - 1) rg_pass<8, PTS, true>(bw, K, Ns, lane, tf, dst);
        else if (R == 24) rg_pass<24, PTS>(bw, K, Ns, lane, tf);
        else if (R == 8) rg_pass<8, PTS>(bw, K, Ns, lane, tf);
        else if (R == 4) rg_pass<4, PTS>(bw, K, Ns, lane, tf);
        else if (R == 2) rg_pass<2, PTS>(bw, K, Ns, lane, tf);
        else if (R == 3) rg_pass<3, PTS>(bw, K, Ns, lane, tf);
        else rg_pass<5, PTS>(bw, K, Ns, lane, tf);
        tf += (R - 1) * Ns;
        Ns *= R;
      }
      if (!direct && dst) {
        for (int n = lane; n < K; n += 64) dst[n] = bw[padr(n)];
      }
    }
  }
}

template <int PTS>
__global__ __launch_bounds__(64 * RG_RINGS) void k_fft_c2r_rg(FftPlan plan, int lmax, int ntheta, int nseq,
                                                              const float2* __restrict__ F, float* __restrict__ maps,
                                                              const float2* __restrict__ twg,
                                                              const float2* __restrict__ twpg) {
  c2r_rg_body<PTS, 0>(plan, lmax, ntheta, nseq, F, maps, twg, twpg);
}

// the plan 24 x 8 x 8 of K = 1536 compiled in (the constant index arithmetic lets the
// compiler keep more in registers: held to two waves per SIMD)
__global__ __launch_bounds__(64 * RG_RINGS) __attribute__((amdgpu_waves_per_eu(2))) void k_fft_c2r_rg_k1536(
    FftPlan plan, int lmax, int ntheta, int nseq, const float2* __restrict__ F, float* __restrict__ maps,
    const float2* __restrict__ twg, const float2* __restrict__ twpg) {
  c2r_rg_body<24, 1536>(plan, lmax, ntheta, nseq, F, maps, twg, twpg);
}

// the plan 47 x 8 x 8 of K = 3008 (the rings of nphi 6016, the l_max 2000 grid): its
// LDS (about 141 KB) holds one workgroup per CU, so registers are not limited
__global__ __launch_bounds__(64 * RG_RINGS) void k_fft_c2r_rg_k3008(
    FftPlan plan, int lmax, int ntheta, int nseq, const float2* __restrict__ F, float* __restrict__ maps,
    const float2* __restrict__ twg, const float2* __restrict__ twpg) {
  c2r_rg_body<48, 3008>(plan, lmax, ntheta, nseq, F, maps, twg, twpg);
}

// r2c, register passes (the adjoint of k_fft_c2r_rg): same persistent ring-group order,
// one wave per ring.  z_n = G_{2n} + i G_{2n+1} goes into the ring buffer conjugated, so
// the e^{+i} passes above give conj of Z_m = sum_n z_n e^{-2 pi i m n / K}; after a
// workgroup barrier every thread forms Gh_m of one (m, ring) of the four rings from
// Z_m and Z_{K-m} (see the top of the file), and consecutive threads write the four
// rings of one m, the contiguous run of the [seq][m][ring] layout.
template <int PTS, int KC = 0>
__global__ __launch_bounds__(64 * RG_RINGS) void k_fft_r2c_rg(FftPlan plan, int lmax, int ntheta, int nseq,
                                                              const float* __restrict__ G, float2* __restrict__ Gh,
                                                              const float2* __restrict__ twg,
                                                              const float2* __restrict__ twpg) {
  extern __shared__ __attribute__((aligned(16))) float2 rbuf[];
  const int K = KC ? KC : plan.K;   // KC: a plan compiled in (24 x 8 x 8 of K = 1536, 47 x 8 x 8 of 3008)
  const int KP = padr(K) + 1;
  float2* tw = rbuf + RG_RINGS * KP;
  float2* twp = tw + K / 2 + 1;
  const int nrb8 = f_ring_blocks(ntheta);
  const int units = nseq * nrb8;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int t = tid; t <= K / 2; t += 64 * RG_RINGS) tw[t] = twg[t];
  for (int t = tid; t < K - 1; t += 64 * RG_RINGS) twp[t] = twpg[t];
  const int b = blockIdx.x;
  const int xcd = b & 7, half = (b >> 3) & 1, slot = b >> 4;
  const int nslot = gridDim.x >> 4;
  for (int unit = xcd + 8 * slot; unit < units; unit += 8 * nslot) {
    const int seq = unit / nrb8, rb = unit - seq * nrb8;
    // the previous unit's reads of all four buffers (and the twiddle tables) are settled
    lds_barrier();
    const int jb = rb * 8 + RG_RINGS * half;
    const int j = jb + w;
    float2* bw = rbuf + w * KP;
    if (j < ntheta) {   // wave-uniform
      const float2* src = reinterpret_cast<const float2*>(G + ((size_t)seq * ntheta + j) * plan.N);
      if constexpr (PTS <= 24) {
        // the row in rounds of 8 loads per lane issued before their stores (64 PTS >= K):
        // a round trip per 512 points instead of per 64 (at more points per lane the extra
        // registers would cost the second wave per SIMD)
        const float2* srcl = src + lane;
        float2* dstb = bw + padr(lane);   // padr(n + 64) = padr(n) + 72: constant offsets
        constexpr int RL = 8;
#pragma unroll
        for (int i0 = 0; i0 < PTS; i0 += RL) {
          float2 v[RL];
#pragma unroll
          for (int i = 0; i < RL; ++i)
            if (i0 + i < PTS && lane + 64 * (i0 + i) < K) v[i] = srcl[64 * (i0 + i)];
#pragma unroll
          for (int i = 0; i < RL; ++i)
            if (i0 + i < PTS && lane + 64 * (i0 + i) < K) dstb[72 * (i0 + i)] = make_float2(v[i].x, -v[i].y);
        }
      } else {
        for (int n = lane; n < K; n += 64) {
          const float2 v = src[n];
          bw[padr(n)] = make_float2(v.x, -v.y);
        }
      }
      if constexpr (KC == 1536) {
        rg_pass<24, PTS, false, KC, 1>(bw, K, 1, lane, twp);
        rg_pass<8, PTS, false, KC, 24>(bw, K, 24, lane, twp + 23);
        rg_pass<8, PTS, false, KC, 192>(bw, K, 192, lane, twp + 23 + 7 * 24);
      } else if constexpr (KC == 3008) {
        rg_pass47_first(bw, lane);
        rg_pass<8, PTS, false, KC, 47>(bw, K, 47, lane, twp + 46);
        rg_pass<8, PTS, false, KC, 376>(bw, K, 376, lane, twp + 46 + 7 * 47);
      } else {
        int Ns = 1;
        const float2* tf = twp;
        for (int f = 0; f < plan.nf; ++f) {
          const int R = plan.radix[f];
          if (R == 24) rg_pass<24, PTS>(bw, K, Ns, lane, tf);
          else if (R == 8) rg_pass<8, PTS>(bw, K, Ns, lane, tf);
          else if (R == 4) rg_pass<4, PTS>(bw, K, Ns, lane, tf);
          else if (R == 2) rg_pass<2, PTS>(bw, K, Ns, lane, tf);
          else if (R == 3) rg_pass<3, PTS>(bw, K, Ns, lane, tf);
          else rg_pass<5, PTS>(bw, K, Ns, lane, tf);
          tf += (R - 1) * Ns;
          Ns *= R;
        }
      }
    }
    lds_barrier();   // the four rings' spectra are in LDS
    float2* dst = Gh + (size_t)seq * (lmax + 1) * ntheta;
    for (int e = tid; e < (lmax + 1) * RG_RINGS; e += 64 * RG_RINGS) {
      const int m = e / RG_RINGS, r = e - m * RG_RINGS;
      if (jb + r >= ntheta) continue;
      const float2* br = rbuf + r * KP;
      const float2 cz = br[padr(m)], cw = br[padr((K - m) % K)];   // conj Z_m, conj Z_{K-m}
      const float2 zk = make_float2(cz.x, -cz.y);
      const float2 a = make_float2(zk.x + cw.x, zk.y + cw.y);   // Z_m + conj Z_{K-m}
      const float2 d = make_float2(zk.x - cw.x, zk.y - cw.y);   // Z_m - conj Z_{K-m}
      const float2 ew = (m <= K / 2) ? tw[m] : make_float2(-tw[K - m].x, tw[K - m].y);   // e^{2 pi i m / N}
      float2 g;
      g.x = 0.5f * (a.x + (ew.x * d.y - ew.y * d.x));
      g.y = 0.5f * (a.y - (ew.x * d.x + ew.y * d.y));
      dst[(size_t)m * ntheta + j - w + r] = g;
    }
  }
}

}  // namespace

int fft_rings_max(const modal_ctx* c) {
  // as many rings per workgroup as fit in LDS (two buffers), at most 4
  const size_t per = 2 * (size_t)c->fft.K * 2 * real_bytes(c);
  int R = 4;
  while (R > 1 && (size_t)R * per > c->max_lds) R >>= 1;
  return R;
}

int fft_rings_per_block(const modal_ctx* c) {
  const int R = fft_rings_max(c);
  return (c->tune_fft_rings > 0 && c->tune_fft_rings <= R) ? c->tune_fft_rings : R;
}

// The register kernel's plan: 24 first where it fits, then radices 8, 4, 2, 3, 5
// (largest first); false if the ring length has other factors or exceeds the
// register kernel's size.
int fft_rg_points(const FftPlan& p);

bool fft_plan_rg(int N, FftPlan& p) {
  p.N = N;
  p.K = N / 2;
  p.nf = 0;
  if (p.K == 3008) {   // 47 x 8 x 8, compiled in (the one plan with a radix-47 pass)
    p.radix[0] = 47;
    p.radix[1] = p.radix[2] = 8;
    p.nf = 3;
    return true;
  }
  if (p.K > RG_KMAX || p.K < 1) return false;
  int K = p.K;
  // a first radix-24 pass (a 24-point DFT in registers) saves one LDS round trip when a
  // pass of 24 points per lane still keeps every lane of the wave busy
  if (K % 24 == 0 && K / 24 >= 64) {
    p.radix[p.nf++] = 24;
    K /= 24;
  }
  for (int r : {8, 4, 2, 3, 5})
    while (K % r == 0) {
      if (p.nf >= kMaxFactors) return false;
      p.radix[p.nf++] = r;
      K /= r;
    }
  if (K != 1) return false;
  return fft_rg_points(p) <= 48;
}

// The register kernel's per-pass twiddles, in pass order: for the pass of radix R
// after Ns points, e^{2 pi i q k / (Ns R)} at (q - 1) Ns + k, q = 1..R-1, k < Ns
// (K - 1 entries in all: the (R - 1) Ns telescope to K - 1).
std::vector<float> fft_rg_twiddles(const FftPlan& p) {
  std::vector<float> out;
  int Ns = 1;
  for (int f = 0; f < p.nf; ++f) {
    const int R = p.radix[f];
    for (int q = 1; q < R; ++q)
      for (int k = 0; k < Ns; ++k) {
        const double a = 2.0 * 3.14159265358979323846 * (double)(q * k) / (double)(Ns * R);
        out.push_back((float)std::cos(a));
        out.push_back((float)std::sin(a));
      }
    Ns *= R;
  }
  return out;
}

// the most points one lane holds in a pass: ceil(K / R / 64) R
int fft_rg_points(const FftPlan& p) {
  int pts = 0;
  for (int f = 0; f < p.nf; ++f) pts = std::max(pts, (p.K / p.radix[f] + 63) / 64 * p.radix[f]);
  return pts;
}

size_t fft_rg_lds(const modal_ctx* c) {
  const int K = c->fft.K;
  return ((size_t)RG_RINGS * (K + (K >> 3) + 1) + (size_t)(K / 2 + 1) + (size_t)(K - 1)) * sizeof(float2);
}

hipError_t fft_rg_set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_fft_c2r_rg<16>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_fft_c2r_rg<24>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_fft_c2r_rg<32>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_fft_c2r_rg<48>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_fft_c2r_rg_k1536, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_fft_c2r_rg_k3008, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  const void* r2c[] = {(const void*)k_fft_r2c_rg<16>,       (const void*)k_fft_r2c_rg<24>,
                       (const void*)k_fft_r2c_rg<32>,       (const void*)k_fft_r2c_rg<48>,
                       (const void*)k_fft_r2c_rg<24, 1536>, (const void*)k_fft_r2c_rg<48, 3008>};
  for (const void* f : r2c)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return e;
}

namespace {
bool plan_has_radix(const FftPlan& p, int r) {
  for (int f = 0; f < p.nf; ++f)
    if (p.radix[f] == r) return true;
  return false;
}

// the register plan compiled in (K = 1536: the rings of nphi 3072, the l_max 1000 grid)
bool plan_is_k1536(const FftPlan& p) {
  return p.K == 1536 && p.nf == 3 && p.radix[0] == 24 && p.radix[1] == 8 && p.radix[2] == 8;
}

// K = 3008 (nphi 6016, the l_max 2000 grid); the register kernels run it only compiled in
bool plan_is_k3008(const FftPlan& p) {
  return p.K == 3008 && p.nf == 3 && p.radix[0] == 47 && p.radix[1] == 8 && p.radix[2] == 8;
}
}  // namespace

hipError_t launch_fft_c2r(const modal_ctx* c, const void* F, int S, void* maps, hipStream_t st) {
  if (c->fft_rg) {
    // persistent: two workgroups per CU, in pairs (b, b + 8) per XCD
    const int nseq = S * c->P;
    const int units = nseq * f_ring_blocks(c->ntheta);
    int blocks = 16 * ((units + 7) / 8);
    blocks = std::min(blocks, 16 * 64);   // 1024 workgroups: 256 CUs x 4 rings x 2 x 2
    const int pts = fft_rg_points(c->fft_rg_plan);
#define LAUNCH(PT)                                                                                                \
  hipLaunchKernelGGL(k_fft_c2r_rg<PT>, dim3(blocks), dim3(64 * RG_RINGS), fft_rg_lds(c), st, c->fft_rg_plan,        \
                     c->lmax, c->ntheta, nseq, (const float2*)F, (float*)maps, (const float2*)c->t.tw32,        \
                     (const float2*)c->t.twp32)
    if (plan_is_k1536(c->fft_rg_plan) && pts == 24)
      hipLaunchKernelGGL(k_fft_c2r_rg_k1536, dim3(blocks), dim3(64 * RG_RINGS), fft_rg_lds(c), st,
                         c->fft_rg_plan, c->lmax, c->ntheta, nseq, (const float2*)F, (float*)maps,
                         (const float2*)c->t.tw32, (const float2*)c->t.twp32);
    else if (plan_is_k3008(c->fft_rg_plan))   // one workgroup per CU: 256 of them
      hipLaunchKernelGGL(k_fft_c2r_rg_k3008, dim3(std::min(blocks, 256)), dim3(64 * RG_RINGS), fft_rg_lds(c), st,
                         c->fft_rg_plan, c->lmax, c->ntheta, nseq, (const float2*)F, (float*)maps,
                         (const float2*)c->t.tw32, (const float2*)c->t.twp32);
    else if (pts <= 16) LAUNCH(16);
    else if (pts <= 24) LAUNCH(24);
    else if (pts <= 32) LAUNCH(32);
    else LAUNCH(48);
#undef LAUNCH
    return hipGetLastError();
  }
  const int R = fft_rings_per_block(c);
  const size_t blocks = (size_t)S * c->P * ((c->ntheta + R - 1) / R);
  const size_t lds = (size_t)R * 2 * c->fft.K * 2 * real_bytes(c);
  if (is_f64(c))
    hipLaunchKernelGGL((k_fft_c2r<double, 0>), dim3(blocks), dim3(256), lds, st, c->fft, c->lmax, c->ntheta, R,
                       (const double2*)F, (double*)maps, (const double2*)c->t.tw64);
  else if (plan_has_radix(c->fft, 47))
    hipLaunchKernelGGL((k_fft_c2r<float, 47>), dim3(blocks), dim3(256), lds, st, c->fft, c->lmax, c->ntheta, R,
                       (const float2*)F, (float*)maps, (const float2*)c->t.tw32);
  else
    hipLaunchKernelGGL((k_fft_c2r<float, 0>), dim3(blocks), dim3(256), lds, st, c->fft, c->lmax, c->ntheta, R,
                       (const float2*)F, (float*)maps, (const float2*)c->t.tw32);
  return hipGetLastError();
}

hipError_t launch_fft_r2c(const modal_ctx* c, const void* G, int S, void* Gh, hipStream_t st) {
  return launch_fft_r2c_rows(c, G, (size_t)S * c->P, Gh, st);
}

// nseq sequences of ntheta ring rows each
hipError_t launch_fft_r2c_rows(const modal_ctx* c, const void* G, size_t nseq, void* Gh, hipStream_t st) {
  if (c->fft_rg) {
    const int units = (int)nseq * f_ring_blocks(c->ntheta);
    int blocks = 16 * ((units + 7) / 8);
    blocks = std::min(blocks, 16 * 64);
    const int pts = fft_rg_points(c->fft_rg_plan);
#define LAUNCH(PT)                                                                                                \
  hipLaunchKernelGGL(k_fft_r2c_rg<PT>, dim3(blocks), dim3(64 * RG_RINGS), fft_rg_lds(c), st, c->fft_rg_plan,        \
                     c->lmax, c->ntheta, (int)nseq, (const float*)G, (float2*)Gh, (const float2*)c->t.tw32,       \
                     (const float2*)c->t.twp32)
    if (plan_is_k1536(c->fft_rg_plan) && pts == 24)
      hipLaunchKernelGGL((k_fft_r2c_rg<24, 1536>), dim3(blocks), dim3(64 * RG_RINGS), fft_rg_lds(c), st,
                         c->fft_rg_plan, c->lmax, c->ntheta, (int)nseq, (const float*)G, (float2*)Gh,
                         (const float2*)c->t.tw32, (const float2*)c->t.twp32);
    else if (plan_is_k3008(c->fft_rg_plan))
      hipLaunchKernelGGL((k_fft_r2c_rg<48, 3008>), dim3(std::min(blocks, 256)), dim3(64 * RG_RINGS), fft_rg_lds(c),
                         st, c->fft_rg_plan, c->lmax, c->ntheta, (int)nseq, (const float*)G, (float2*)Gh,
                         (const float2*)c->t.tw32, (const float2*)c->t.twp32);
    else if (pts <= 16) LAUNCH(16);
    else if (pts <= 24) LAUNCH(24);
    else if (pts <= 32) LAUNCH(32);
    else LAUNCH(48);
#undef LAUNCH
    return hipGetLastError();
  }
  const int R = fft_rings_per_block(c);
  const size_t blocks = nseq * ((c->ntheta + R - 1) / R);
  const size_t lds = (size_t)R * 2 * c->fft.K * 2 * real_bytes(c);
  if (is_f64(c))
    hipLaunchKernelGGL((k_fft_r2c<double, 0>), dim3(blocks), dim3(256), lds, st, c->fft, c->lmax, c->ntheta, R,
                       (const double*)G, (double2*)Gh, (const double2*)c->t.tw64);
  else if (plan_has_radix(c->fft, 47))
    hipLaunchKernelGGL((k_fft_r2c<float, 47>), dim3(blocks), dim3(256), lds, st, c->fft, c->lmax, c->ntheta, R,
                       (const float*)G, (float2*)Gh, (const float2*)c->t.tw32);
  else
    hipLaunchKernelGGL((k_fft_r2c<float, 0>), dim3(blocks), dim3(256), lds, st, c->fft, c->lmax, c->ntheta, R,
                       (const float*)G, (float2*)Gh, (const float2*)c->t.tw32);
  return hipGetLastError();
}

// Called once per context to allow LDS above the 64 KB default.
hipError_t fft_set_lds_limit(size_t bytes) {
  const void* fns[] = {(const void*)k_fft_c2r<double, 0>, (const void*)k_fft_c2r<float, 0>,
                       (const void*)k_fft_c2r<float, 47>, (const void*)k_fft_r2c<double, 0>,
                       (const void*)k_fft_r2c<float, 0>, (const void*)k_fft_r2c<float, 47>};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace modal
