// Legendre synthesis on the matrix cores, recurrence computed on the fly.
//
// For each m: F_c(theta_j) = sum_l Lambda[j][l] Coef[l][c],
//   Lambda[j][l] = lambda_lm(theta_j)  (north rings j, FP64 three-term recurrence),
//   Coef[l][c]   = qw_p(l) Re/Im a_{s,lm}  (column c = (s, p, re/im)),
// a GEMM with M = rings, N = columns, K = l, split by the parity of l - m so that
// F_north = E + O and F_south = E - O (lambda_lm(-x) = (-1)^{l+m} lambda_lm(x)).
//
// Workgroup = 4 waves = 256 north rings (64 per wave, one lane per ring in the
// recurrence) x 64 columns, one m.  Per chunk of 64 consecutive l (32 of each
// parity): every lane advances its ring's recurrence (FP64) and writes lambda to the
// wave's LDS tile; the workgroup writes the coefficient tile; then each wave runs
// the 2 parities x 4 ring tiles x 4 column tiles of 16x16 MFMAs.
//   BF16X3: v_mfma_f32_16x16x32_bf16 on hi/lo splits, all four products
//           (hi.hi + hi.lo + lo.hi + lo.lo): every map enters the cubic three
//           times, so the synthesis keeps the lo.lo term (error ~2^-18 per term
//           instead of ~2^-16); FP32 accumulation.
//   F16X3 : v_mfma_f32_16x16x32_f16 on fp16 hi/lo splits (22 bits; hi.hi + hi.lo +
//           lo.hi).  lambda is bounded by sqrt((2l+1)/4pi) and whitened
//           coefficients are O(1), so no scaling is needed; lo parts that fall
//           into fp16 subnormals carry absolute errors below 1e-7.
//   F32   : v_mfma_f32_16x16x4_f32.
// Output goes through LDS so that F (f_index layout) is written in runs of rings.
#include "common.h"

namespace modal {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int LCH = 64;    // l per chunk
constexpr int LH = 32;     // l per parity per chunk
constexpr int RW = 64;     // rings per wave
constexpr int NCOL = 64;   // columns per workgroup
constexpr int NWAVE = 4;

__device__ inline uint32_t bf2(float a, float b) {
  typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
  bf16x2 h;
  h[0] = (__bf16)a;
  h[1] = (__bf16)b;
  return __builtin_bit_cast(uint32_t, h);
}

// hi/lo split of one float into two 16-bit words (bf16 or fp16, RNE each).
// The value a split starts from must be one rounded FP32 number: the backend may
// otherwise fuse the producing multiply into the hi conversion (a mixed-precision
// FMA rounding the exact product) in one place and not in another, so that hi and
// lo no longer add up.  An empty asm statement makes the rounded value opaque.
template <int PREC>
__device__ inline void split1(float v, uint16_t& hi, uint16_t& lo) {
  asm("" : "+v"(v));
  if (PREC == MODAL_F16X3) {
    const _Float16 h = (_Float16)v;
    const _Float16 l = (_Float16)(v - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  } else {
    const uint32_t hb = bf2(v, 0.f);
    const float h = __builtin_bit_cast(float, hb << 16);
    hi = (uint16_t)(hb & 0xffffu);
    lo = (uint16_t)(bf2(v - h, 0.f) & 0xffffu);
  }
}

struct RecState {
  double l1, l2, s0, s1;
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

// LDS layout (dynamic):
//   BF16X3: coefH/coefL [2][NCOL][LH] u16, lamH/lamL [NWAVE][2][RW][LH] u16
//   F32   : coef [2][NCOL][LH] f32, lam [NWAVE][2][RW][LH] f32
// After the chunk loop the lambda area is reused as output staging, [RW][NCOL+1]
// f32 per wave (disjoint slabs).
template <int PREC>
__global__ __launch_bounds__(256) void k_legendre_mfma(int lmax, int ntheta, int nrp, int P, int ncols, int nalm,
                                                       const double* __restrict__ x, const double* __restrict__ rec,
                                                       const double* __restrict__ seed,
                                                       const int* __restrict__ lstart, const float* __restrict__ qw,
                                                       const float2* __restrict__ alm, float2* __restrict__ F) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const int m = blockIdx.z;
  const int c0 = blockIdx.x * NCOL;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int row = lane & 15, kg = lane >> 4;
  const int jring = blockIdx.y * (NWAVE * RW) + wv * RW + lane;
  const bool ring_ok = jring < nrp;
  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;

  constexpr bool BF = (PREC == MODAL_BF16X3 || PREC == MODAL_F16X3);   // 16-bit split tiles
  constexpr int ES = BF ? 2 : 4;                       // element bytes of a tile
  constexpr size_t COEF_B = 2 * NCOL * LH * ES;         // one coef plane
  constexpr size_t LAM_B = 2 * RW * LH * ES;            // one lambda plane per wave
  unsigned char* coefH = lds;
  unsigned char* coefL = lds + COEF_B;                  // BF16X3 only
  unsigned char* lamBase = lds + (BF ? 2 : 1) * COEF_B;
  unsigned char* lamH = lamBase + (size_t)wv * (BF ? 2 : 1) * LAM_B;
  unsigned char* lamL = lamH + LAM_B;                   // BF16X3 only
  __shared__ int lmin_blk;
  __shared__ int lmin_wave[NWAVE];

  RecState rs;
  rs.l1 = rs.l2 = 0.0;
  rs.s0 = rs.s1 = 0.0;
  rs.ls = lmax + 1;
  double xx = 0.0;
  if (ring_ok) {
    xx = x[jring];
    rs.ls = lstart[(size_t)m * nrp + jring];
    rs.s0 = seed[2 * ((size_t)m * nrp + jring)];
    rs.s1 = seed[2 * ((size_t)m * nrp + jring) + 1];
  }
  if (tid == 0) lmin_blk = lmax + 1;
  if (lane == 0) lmin_wave[wv] = lmax + 1;
  __syncthreads();
  atomicMin(&lmin_blk, rs.ls);
  atomicMin(&lmin_wave[wv], rs.ls);
  __syncthreads();
  const int lmin = lmin_blk;
  const int wlmin = lmin_wave[wv];

  f32x4 acc[2][4][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[a][b][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  // chunks start at l = m + 64 k so that parity(l - m) = parity(l - l0)
  const int kfirst = (lmin > m) ? (lmin - m) / LCH : 0;
  for (int l0 = m + kfirst * LCH; l0 <= lmax; l0 += LCH) {
    // ---- coefficient tile [par][col][idx]
    for (int e = tid; e < NCOL * LH; e += 256) {
      const int col = e / LH, idx = e - col * LH;
      const int cg = c0 + col;
      float v[2] = {0.f, 0.f};
      if (cg < ncols) {
        const int sq = cg >> 1, reim = cg & 1;
        const int s = sq / P, p = sq - s * P;
#pragma unroll
        for (int par = 0; par < 2; ++par) {
          const int l = l0 + 2 * idx + par;
          if (l <= lmax) {
            const float2 a = alm[(size_t)s * nalm + off + (l - m)];
            v[par] = qw[(size_t)p * (lmax + 1) + l] * (reim ? a.y : a.x);
          }
        }
      }
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const size_t at = ((size_t)par * NCOL + col) * LH + idx;
        if (BF) {
          split1<PREC>(v[par], reinterpret_cast<uint16_t*>(coefH)[at], reinterpret_cast<uint16_t*>(coefL)[at]);
        } else {
          reinterpret_cast<float*>(coefH)[at] = v[par];
        }
      }
    }
    // ---- lambda tile of this wave's rings [par][ring][idx] (recurrence, FP64)
    for (int t = 0; t < LCH; ++t) {
      const int l = l0 + t;
      double lam = 0.0;
      if (l <= lmax) lam = rs.step(l, xx, rec + 2 * (off + (l - m)));
      const int par = t & 1, idx = t >> 1;
      const size_t at = ((size_t)par * RW + lane) * LH + idx;
      const float lf = (float)lam;
      if (BF) {
        split1<PREC>(lf, reinterpret_cast<uint16_t*>(lamH)[at], reinterpret_cast<uint16_t*>(lamL)[at]);
      } else {
        reinterpret_cast<float*>(lamH)[at] = lf;
      }
    }
    __syncthreads();
    // ---- MFMA (uniform per wave: skipped when all its rings are still below l_start)
    if (l0 + LCH - 1 >= wlmin) {
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        if (PREC == MODAL_BF16X3) {
          bf16x8 bh[4], bl[4];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const size_t at = ((size_t)par * NCOL + 16 * ct + row) * LH + 8 * kg;
            bh[ct] = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const uint16_t*>(coefH) + at);
            bl[ct] = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const uint16_t*>(coefL) + at);
          }
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            const size_t at = ((size_t)par * RW + 16 * rt + row) * LH + 8 * kg;
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const uint16_t*>(lamH) + at);
            const bf16x8 al = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const uint16_t*>(lamL) + at);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
              acc[par][rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[par][rt][ct], 0, 0, 0);
              acc[par][rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[par][rt][ct], 0, 0, 0);
              acc[par][rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[par][rt][ct], 0, 0, 0);
              acc[par][rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bl[ct], acc[par][rt][ct], 0, 0, 0);
            }
          }
        } else if (PREC == MODAL_F16X3) {
          f16x8 bh[4], bl[4];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const size_t at = ((size_t)par * NCOL + 16 * ct + row) * LH + 8 * kg;
            bh[ct] = *reinterpret_cast<const f16x8*>(reinterpret_cast<const uint16_t*>(coefH) + at);
            bl[ct] = *reinterpret_cast<const f16x8*>(reinterpret_cast<const uint16_t*>(coefL) + at);
          }
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            const size_t at = ((size_t)par * RW + 16 * rt + row) * LH + 8 * kg;
            const f16x8 ah = *reinterpret_cast<const f16x8*>(reinterpret_cast<const uint16_t*>(lamH) + at);
            const f16x8 al = *reinterpret_cast<const f16x8*>(reinterpret_cast<const uint16_t*>(lamL) + at);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
              // the chunk's products start from zero and join the running sum with a
              // round-to-nearest vector add
              f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[ct], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
              t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[ct], t, 0, 0, 0);
              t = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[ct], t, 0, 0, 0);
              acc[par][rt][ct] += t;
            }
          }
        } else {
          const float* cf = reinterpret_cast<const float*>(coefH);
          const float* lf = reinterpret_cast<const float*>(lamH);
          float bv[4][8];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int k = 0; k < 8; ++k) bv[ct][k] = cf[((size_t)par * NCOL + 16 * ct + row) * LH + 8 * kg + k];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) {
            float av[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) av[k] = lf[((size_t)par * RW + 16 * rt + row) * LH + 8 * kg + k];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
              f32x4 t = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
              for (int k = 0; k < 8; ++k) t = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k], bv[ct][k], t, 0, 0, 0);
              acc[par][rt][ct] += t;
            }
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- output: stage N = E + O then S = E - O through the (now idle) lambda area,
  // one disjoint [RW][NCOL + 1] float slab per wave
  constexpr int SS = NCOL + 1;
  float* stg = reinterpret_cast<float*>(lamBase) + (size_t)wv * RW * SS;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const float sg = half ? -1.f : 1.f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          stg[(16 * rt + 4 * kg + r) * SS + 16 * ct + row] = acc[0][rt][ct][r] + sg * acc[1][rt][ct][r];
    __syncthreads();
    if (ring_ok) {
      const int jw = half ? ntheta - 1 - jring : jring;
      if (!(half && jw == jring)) {
        for (int cc = 0; cc < NCOL; cc += 2) {
          const int cg = c0 + cc;
          if (cg >= ncols) break;
          float2 v;
          v.x = stg[lane * SS + cc];
          v.y = stg[lane * SS + cc + 1];
          F[f_index(cg >> 1, jw, m, lmax, f_ring_blocks(ntheta))] = v;
        }
      }
    }
    __syncthreads();
  }
}

size_t lds_bytes(int prec) {
  const bool bf = prec == MODAL_BF16X3 || prec == MODAL_F16X3;
  const size_t es = bf ? 2 : 4;
  const size_t coef = 2 * NCOL * LH * es * (bf ? 2 : 1);
  const size_t lam = (size_t)NWAVE * 2 * RW * LH * es * (bf ? 2 : 1);
  const size_t stage = (size_t)NWAVE * RW * (NCOL + 1) * 4;
  return coef + (lam > stage ? lam : stage);
}

}  // namespace

size_t legendre_mfma_lds(const modal_ctx* c) { return lds_bytes(c->prec); }

hipError_t legendre_mfma_set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_legendre_mfma<MODAL_BF16X3>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_legendre_mfma<MODAL_F16X3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_legendre_mfma<MODAL_F32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

hipError_t launch_legendre_mfma(const modal_ctx* c, const void* alm, int S, void* F, hipStream_t st) {
  const int ncols = 2 * S * c->P;
  dim3 grid((ncols + NCOL - 1) / NCOL, (c->nrp + NWAVE * RW - 1) / (NWAVE * RW), c->lmax + 1);
  const size_t lds = lds_bytes(c->prec);
  if (c->prec == MODAL_F16X3)
    hipLaunchKernelGGL(k_legendre_mfma<MODAL_F16X3>, grid, dim3(256), lds, st, c->lmax, c->ntheta, c->nrp, c->P,
                       ncols, c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw32, (const float2*)alm,
                       (float2*)F);
  else if (c->prec == MODAL_BF16X3)
    hipLaunchKernelGGL(k_legendre_mfma<MODAL_BF16X3>, grid, dim3(256), lds, st, c->lmax, c->ntheta, c->nrp, c->P,
                       ncols, c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw32, (const float2*)alm,
                       (float2*)F);
  else
    hipLaunchKernelGGL(k_legendre_mfma<MODAL_F32>, grid, dim3(256), lds, st, c->lmax, c->ntheta, c->nrp, c->P, ncols,
                       c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw32, (const float2*)alm, (float2*)F);
  return hipGetLastError();
}

}  // namespace modal
