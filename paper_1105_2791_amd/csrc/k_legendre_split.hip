// Legendre synthesis on the matrix cores with split 16-bit operands, 32x32 tiles,
// recurrence computed on the fly and kept in registers.
//
// For each m: F_c(theta_j) = sum_l Lambda[j][l] Coef[l][c],
//   Lambda[j][l] = lambda_lm(theta_j)  (north rings j, FP64 three-term recurrence),
//   Coef[l][c]   = qw_p(l) Re/Im a_{s,lm}  (column c = (s, p, re/im)),
// a GEMM with M = rings, N = columns, K = l, split by the parity of l - m so that
// F_north = E + O and F_south = E - O (lambda_lm(-x) = (-1)^{l+m} lambda_lm(x)).
//
// Workgroup = 4 waves = 256 north rings (one per lane: 64 per wave) x 64 columns,
// one m.  Per chunk of 64 consecutive l (32 of each parity):
//   * every lane advances its ring's recurrence 64 steps (FP64) and splits the values
//     into hi/lo words held in registers.  The A operand of
//     v_mfma_f32_32x32x16_{bf16,f16} wants, in lane l, ring l % 32 of a 32-ring tile
//     at l-index 8 (l / 32) + i: lanes 0-31 keep their first 8 indices, lanes 32-63
//     their last 8, and one v_permlane32_swap per register hands the other halves
//     across, so lambda never goes through LDS;
//   * the workgroup stages the coefficient tile (hi/lo, padded rows) in LDS;
//   * each wave runs 2 parities x 2 ring tiles x 2 column tiles, accumulating
//     2 K steps x 3 products (hi.hi + hi.lo + lo.hi; lo.lo is below the operand
//     split error) per chunk in place: an output takes at most about 130
//     accumulations, so the matrix core's addend truncation stays far below the split
//     error.
// Output goes through LDS so that F (f_index layout) is written in runs of rings.
#include "common.h"

#include <type_traits>

namespace modal {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

constexpr int LCH = 64;     // l per chunk
constexpr int LH = 32;      // l per parity per chunk
constexpr int LHP = LH + 8; // padded LDS row (16-bit elements)
constexpr int NCOL = 64;    // columns per workgroup
constexpr int NWAVE = 4;
constexpr int RW = 64;      // rings per wave
constexpr int SS = NCOL + 1;  // output staging row (floats)

struct CoefTile {
  uint16_t h[2][NCOL][LHP];
  uint16_t l[2][NCOL][LHP];
};
constexpr size_t kStageBytes = (size_t)NWAVE * RW * SS * 4;
constexpr size_t kLdsBytes = sizeof(CoefTile) > kStageBytes ? sizeof(CoefTile) : kStageBytes;

__device__ inline uint32_t bf16x2_bits(float a, float b) {
  typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
  bf16x2 h;
  h[0] = (__bf16)a;
  h[1] = (__bf16)b;
  return __builtin_bit_cast(uint32_t, h);
}

// hi/lo words of two values (RNE each; the split starts from the rounded FP32 value)
template <int PREC>
__device__ inline void split2(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  asm("" : "+v"(v0), "+v"(v1));
  if (PREC == MODAL_F16X3) {
    const _Float16 h0 = (_Float16)v0, h1 = (_Float16)v1;
    const _Float16 l0 = (_Float16)(v0 - (float)h0), l1 = (_Float16)(v1 - (float)h1);
    hi = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    lo = (uint32_t)__builtin_bit_cast(uint16_t, l0) | ((uint32_t)__builtin_bit_cast(uint16_t, l1) << 16);
  } else {
    uint32_t hb = bf16x2_bits(v0, v1);
    asm("" : "+v"(hb));
    hi = hb;
    lo = bf16x2_bits(v0 - __builtin_bit_cast(float, hb << 16), v1 - __builtin_bit_cast(float, hb & 0xffff0000u));
  }
}

// 64 recurrence steps of one lane's ring from l0, split into hi/lo words: Lh/Ll
// [par][ks][half][k] hold l-indices 16 ks + 8 half + 2 k and + 1 of parity par.
// wave-uniform value of lane t of a register pair (lo, hi) as a double
__device__ inline double lane_double(uint32_t lo, uint32_t hi, int t) {
  const uint64_t v = (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)lo, t) |
                     ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)hi, t) << 32);
  return __builtin_bit_cast(double, v);
}

template <int PREC, bool FAST>
__device__ inline void lambda_chunk(int l0, int m, int lmax, const uint32_t (&rr)[4], double xx, int ls,
                                    double s0, double s1, double& l1, double& l2, uint32_t (&Lh)[2][2][2][4],
                                    uint32_t (&Ll)[2][2][2][4]) {
  // rr: lane t holds (A, B) of l0 + t for this m (one vector load per lane per chunk,
  // issued with the coefficient loads); each step reads its pair back as wave-uniform
  // values, so the recurrence never waits on the scalar cache
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    // 8 steps: l-indices 4 g .. 4 g + 3 of each parity, i.e. [ks = g / 4][half = (g / 2) % 2]
    // at k = 2 (g % 2) and 2 (g % 2) + 1
    float lam[2][4];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int l = l0 + 8 * g + t;
      const double A = lane_double(rr[0], rr[1], 8 * g + t), B = lane_double(rr[2], rr[3], 8 * g + t);
      double v = fma(A * xx, l1, -B * l2);
      if (!FAST) {
        v = (l < ls) ? 0.0 : v;
        v = (l == ls) ? s0 : v;
        v = (l == ls + 1) ? s1 : v;
      }
      l2 = l1;
      l1 = v;
      lam[t & 1][t >> 1] = (FAST || l <= lmax) ? (float)v : 0.f;
    }
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int k = 0; k < 2; ++k)
        split2<PREC>(lam[par][2 * k], lam[par][2 * k + 1], Lh[par][g >> 2][(g >> 1) & 1][2 * (g & 1) + k],
                     Ll[par][g >> 2][(g >> 1) & 1][2 * (g & 1) + k]);
  }
}

constexpr int RECUR = 0, BUILD = 1, TABLE = 2;

// MODE: RECUR computes lambda in the kernel; BUILD only computes it and stores the
// operand words in the context's lambda table; TABLE reads them from the table.
template <int PREC, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_legendre_split(
    int lmax, int ntheta, int nrp, int P, int ncols, int nalm, const double* __restrict__ x,
    const double* __restrict__ rec, const double* __restrict__ seed, const int* __restrict__ lstart,
    const float* __restrict__ qw, const float2* __restrict__ alm, float2* __restrict__ F, uint4* __restrict__ tab,
    const long long* __restrict__ tab_off) {
  constexpr bool F16 = PREC == MODAL_F16X3;
  typedef typename std::conditional<F16, f16x8, bf16x8>::type vec8;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  CoefTile& C = *reinterpret_cast<CoefTile*>(lds);
  __shared__ int lmin_blk;
  __shared__ int lmax_ls_wave[NWAVE];

  int m, rbk, cbk;
  if (MODE == TABLE) {
    // 1-D grid, XCD-aware: unit (m, ring block) u goes to XCD u % 8, and its column blocks
    // follow each other there, so they read its lambda records from the same L2
    const int nrb = (nrp + NWAVE * RW - 1) / (NWAVE * RW), ncb = (ncols + NCOL - 1) / NCOL;
    const int b = blockIdx.x, idx = b >> 3;
    const int unit = (b & 7) + 8 * (idx / ncb);
    if (unit >= nrb * (lmax + 1)) return;   // whole workgroup
    cbk = idx - (idx / ncb) * ncb;
    m = unit / nrb;
    rbk = unit - m * nrb;
  } else {
    m = blockIdx.z;
    rbk = blockIdx.y;
    cbk = blockIdx.x;
  }
  const int c0 = cbk * NCOL;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int lrow = lane & 31, kh = lane >> 5;
  const int jring = rbk * (NWAVE * RW) + wv * RW + lane;
  // lambda records of this wave: one per chunk k (from l = m), 16 x 64 lanes x 16 bytes
  const int nkm = (lmax + 1 - m + LCH - 1) / LCH;
  const long long rec0 = (MODE == RECUR) ? 0 : tab_off[m] + (long long)(rbk * NWAVE + wv) * nkm;
  const bool ring_ok = jring < nrp;
  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;

  // recurrence state of this lane's ring: lambda_{l-1}, lambda_{l-2}, seeds at l_start
  double xx = 0.0, l1 = 0.0, l2 = 0.0, s0 = 0.0, s1 = 0.0;
  int ls = lmax + 1;
  if (ring_ok) {
    xx = x[jring];
    ls = lstart[(size_t)m * nrp + jring];
    s0 = seed[2 * ((size_t)m * nrp + jring)];
    s1 = seed[2 * ((size_t)m * nrp + jring) + 1];
  }
  if (tid == 0) lmin_blk = lmax + 1;
  if (lane == 0) lmax_ls_wave[wv] = 0;
  __syncthreads();
  atomicMin(&lmin_blk, ls);
  atomicMax(&lmax_ls_wave[wv], ring_ok ? ls : 0);
  __syncthreads();
  const int lmin = lmin_blk;
  const int wls = lmax_ls_wave[wv];   // past l = wls + 1 no lane of the wave needs its seeds

  f32x16 acc[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][b][c][r] = 0.f;

  // this thread's coefficient column (col, quarter q): pointers offset so that element l
  // of the column is pa2[l] (a_{s,lm}, of which the column takes Re or Im) and pq[l]
  // (qw_p(l)) for l = 16 q + i of a chunk starting at 0; a chunk at l0 adds l0
  const int ccol = tid >> 2, cq = tid & 3;
  const bool col_ok = c0 + ccol < ncols;
  const float2* pa2;
  const float* pq;
  const int creim = min(c0 + ccol, ncols - 1) & 1;
  {
    const int sq = min(c0 + ccol, ncols - 1) >> 1;
    const int s = sq / P, p = sq - s * P;
    pa2 = alm + (size_t)s * nalm + off + 16 * cq - m;
    pq = qw + (size_t)p * (lmax + 1) + 16 * cq;
  }

  // chunks start at l = m + 64 k so that parity(l - m) = parity(l - l0)
  const int kfirst = (lmin > m) ? (lmin - m) / LCH : 0;
  // recurrence coefficients of a chunk, lane t <- (A, B) of l0 + t (the table is padded
  // past the last m, so l0 + 63 may run past lmax); loaded one chunk ahead
  uint32_t rr[4];
  auto load_rr = [&](int l0n) {
    const uint4 r4 = *reinterpret_cast<const uint4*>(rec + 2 * (off + (size_t)(l0n - m + lane)));
    rr[0] = r4.x;
    rr[1] = r4.y;
    rr[2] = r4.z;
    rr[3] = r4.w;
  };
  if (MODE != TABLE && m + kfirst * LCH <= lmax) load_rr(m + kfirst * LCH);

  for (int l0 = m + kfirst * LCH; l0 <= lmax; l0 += LCH) {
    uint4* trec = tab + (size_t)(rec0 + (l0 - m) / LCH) * 16 * 64 + lane;
    if (MODE != BUILD) __syncthreads();
    // ---- coefficient loads: thread (col, quarter) takes 16 consecutive l of one column.
    //      All 16 pairs are unconditional (index clamped in the last chunk, value selected
    //      after) and in flight together while the recurrence below runs.
    const int col = ccol, q = cq;
    float va[16], vq[16];
    const float* pa = reinterpret_cast<const float*>(pa2) + creim;
    if (MODE == BUILD) {
#pragma unroll
      for (int i = 0; i < 16; ++i) va[i] = vq[i] = 0.f;
    } else if (l0 + LCH - 1 <= lmax) {   // wave-uniform: one base, immediate offsets
      const float* a = pa + 2 * l0;
      const float* b = pq + l0;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        va[i] = a[2 * i];
        vq[i] = b[i];
      }
    } else {
      // the last chunk of an m: clamped indices, and the product is formed here (vq = 1),
      // which also keeps this path from being merged with the one above
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int li = min(l0 + 16 * q + i, lmax) - 16 * q;
        va[i] = pq[li] * pa[2 * li];
        vq[i] = 1.f;
      }
    }

    // ---- lambda for this lane's ring, l0 .. l0 + 63, as hi/lo words: lw index
    //      [par][ks][half][k] holds l-indices 16 ks + 8 half + 2 k, + 1
    uint32_t Lh[2][2][2][4], Ll[2][2][2][4];
    if (MODE == TABLE) {
      // record word i: Lh (i < 8) or Ll (i >= 8) at [par][ks][half] = i % 8
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const uint4 u = trec[i * 64];
        uint32_t(&dst)[4] = (i < 8) ? Lh[(i >> 2) & 1][(i >> 1) & 1][i & 1] : Ll[(i >> 2) & 1][(i >> 1) & 1][i & 1];
        dst[0] = u.x;
        dst[1] = u.y;
        dst[2] = u.z;
        dst[3] = u.w;
      }
    } else {
      // wave-uniform: every lane is past its seeds and the chunk ends inside l <= lmax,
      // so the steps need no selects (the general form handles seeds and the tail)
      if (l0 > wls + 1 && l0 + LCH - 1 <= lmax) {
        lambda_chunk<PREC, true>(l0, m, lmax, rr, xx, ls, s0, s1, l1, l2, Lh, Ll);
      } else {
        lambda_chunk<PREC, false>(l0, m, lmax, rr, xx, ls, s0, s1, l1, l2, Lh, Ll);
      }
      // hand half 1 of lanes 0-31 and half 0 of lanes 32-63 across: afterwards
      // half 0 is the ring tile 0 operand and half 1 the ring tile 1 operand
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            auto sh = __builtin_amdgcn_permlane32_swap(Lh[par][ks][0][k], Lh[par][ks][1][k], false, false);
            Lh[par][ks][0][k] = sh[0];
            Lh[par][ks][1][k] = sh[1];
            auto sl = __builtin_amdgcn_permlane32_swap(Ll[par][ks][0][k], Ll[par][ks][1][k], false, false);
            Ll[par][ks][0][k] = sl[0];
            Ll[par][ks][1][k] = sl[1];
          }
      if (l0 + LCH <= lmax) load_rr(l0 + LCH);
    }
    if (MODE == BUILD) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const uint32_t(&w)[4] = (i < 8) ? Lh[(i >> 2) & 1][(i >> 1) & 1][i & 1] : Ll[(i >> 2) & 1][(i >> 1) & 1][i & 1];
        trec[i * 64] = make_uint4(w[0], w[1], w[2], w[3]);
      }
      continue;
    }

    // ---- coefficient tile: qw_p(l) Re/Im a_lm, split, stored; l = l0 + 16 q + i has
    //      parity i & 1 and index 8 q + i / 2 (zero past lmax and for padding columns)
    {
      float v[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = (col_ok && l0 + 16 * q + i <= lmax) ? vq[i] * va[i] : 0.f;
      uint32_t h[2][4], lw[2][4];
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int k = 0; k < 4; ++k) split2<PREC>(v[4 * k + par], v[4 * k + 2 + par], h[par][k], lw[par][k]);
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        *reinterpret_cast<u32x4*>(&C.h[par][col][8 * q]) = u32x4{h[par][0], h[par][1], h[par][2], h[par][3]};
        *reinterpret_cast<u32x4*>(&C.l[par][col][8 * q]) = u32x4{lw[par][0], lw[par][1], lw[par][2], lw[par][3]};
      }
    }
    __syncthreads();

    // ---- MFMA: per (parity, ring tile, column tile) a chain over the 2 K steps
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        vec8 bh[2], bl[2];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          bh[ks] = *reinterpret_cast<const vec8*>(&C.h[par][32 * ct + lrow][16 * ks + 8 * kh]);
          bl[ks] = *reinterpret_cast<const vec8*>(&C.l[par][32 * ct + lrow][16 * ks + 8 * kh]);
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
          f32x16& t = acc[par][rt][ct];
#pragma unroll
          for (int ks = 0; ks < 2; ++ks) {
            const u32x4 hv = {Lh[par][ks][rt][0], Lh[par][ks][rt][1], Lh[par][ks][rt][2], Lh[par][ks][rt][3]};
            const u32x4 lv = {Ll[par][ks][rt][0], Ll[par][ks][rt][1], Ll[par][ks][rt][2], Ll[par][ks][rt][3]};
            const vec8 ah = __builtin_bit_cast(vec8, hv), al = __builtin_bit_cast(vec8, lv);
            if (F16) {
              t = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh[ks], t, 0, 0, 0);
              t = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl[ks], t, 0, 0, 0);
              t = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh[ks], t, 0, 0, 0);
            } else {
              t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[ks], t, 0, 0, 0);
              t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[ks], t, 0, 0, 0);
              t = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[ks], t, 0, 0, 0);
            }
          }
        }
      }
  }

  if (MODE == BUILD) return;

  // ---- output: stage N = E + O then S = E - O through LDS, one [RW][SS] slab per wave;
  // acc[par][rt][ct][j] is ring 32 rt + 8 (j / 4) + 4 kh + j % 4, column 32 ct + lrow
  __syncthreads();
  float* stg = reinterpret_cast<float*>(lds) + (size_t)wv * RW * SS;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const float sg = half ? -1.f : 1.f;
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int j = 0; j < 16; ++j)
          stg[(32 * rt + 8 * (j >> 2) + 4 * kh + (j & 3)) * SS + 32 * ct + lrow] =
              acc[0][rt][ct][j] + sg * acc[1][rt][ct][j];
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

}  // namespace

size_t legendre_split_lds() { return kLdsBytes; }

hipError_t legendre_split_set_lds(size_t bytes) {
#define SETLDS(PR, MD)                                                                                        \
  {                                                                                                           \
    hipError_t e = hipFuncSetAttribute((const void*)k_legendre_split<PR, MD>,                                 \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);              \
    if (e != hipSuccess) return e;                                                                            \
  }
  SETLDS(MODAL_BF16X3, RECUR) SETLDS(MODAL_BF16X3, TABLE) SETLDS(MODAL_F16X3, RECUR) SETLDS(MODAL_F16X3, TABLE)
#undef SETLDS
  return hipSuccess;
}

// lambda table: per m, per wave of 64 north rings, per chunk of 64 l from l = m, one
// record of 16 x 64 lanes x 16 bytes (the wave's hi/lo operand words of the chunk)
static int lam_waves(const modal_ctx* c) { return 4 * ((c->nrp + 255) / 256); }

size_t lambda_table_records(const modal_ctx* c, std::vector<long long>* off) {
  long long n = 0;
  if (off) off->resize(c->lmax + 1);
  for (int m = 0; m <= c->lmax; ++m) {
    if (off) (*off)[m] = n;
    n += (long long)lam_waves(c) * ((c->lmax + 1 - m + LCH - 1) / LCH);
  }
  return (size_t)n;
}

size_t lambda_table_bytes(const modal_ctx* c) { return lambda_table_records(c, nullptr) * 16 * 64 * sizeof(uint4); }

hipError_t build_lambda_table(modal_ctx* c, hipStream_t st) {
  dim3 grid(1, (c->nrp + NWAVE * RW - 1) / (NWAVE * RW), c->lmax + 1);
#define LAUNCH(PR)                                                                                                  \
  hipLaunchKernelGGL((k_legendre_split<PR, BUILD>), grid, dim3(256), 0, st, c->lmax, c->ntheta, c->nrp, c->P, 0,      \
                     c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw32, (const float2*)nullptr,          \
                     (float2*)nullptr, c->t.lamtab, c->t.lamtab_off)
  if (c->prec == MODAL_F16X3) LAUNCH(MODAL_F16X3);
  else LAUNCH(MODAL_BF16X3);
#undef LAUNCH
  return hipGetLastError();
}

hipError_t launch_legendre_split(const modal_ctx* c, const void* alm, int S, void* F, hipStream_t st) {
  const int ncols = 2 * S * c->P;
  const int nrb = (c->nrp + NWAVE * RW - 1) / (NWAVE * RW), ncb = (ncols + NCOL - 1) / NCOL;
  if (c->t.lamtab) {
    const int nunits = nrb * (c->lmax + 1);
    dim3 grid((unsigned)(8 * ((nunits + 7) / 8) * ncb));
#define LAUNCH(PR)                                                                                                  \
  hipLaunchKernelGGL((k_legendre_split<PR, TABLE>), grid, dim3(256), kLdsBytes, st, c->lmax, c->ntheta, c->nrp, c->P, \
                     ncols, c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw32, (const float2*)alm,         \
                     (float2*)F, c->t.lamtab, c->t.lamtab_off)
    if (c->prec == MODAL_F16X3) LAUNCH(MODAL_F16X3);
    else LAUNCH(MODAL_BF16X3);
#undef LAUNCH
    return hipGetLastError();
  }
  dim3 grid(ncb, nrb, c->lmax + 1);
#define LAUNCH(PR)                                                                                                  \
  hipLaunchKernelGGL((k_legendre_split<PR, RECUR>), grid, dim3(256), kLdsBytes, st, c->lmax, c->ntheta, c->nrp, c->P, \
                     ncols, c->nalm, c->t.x, c->t.rec, c->t.seed, c->t.lstart, c->t.qw32, (const float2*)alm,         \
                     (float2*)F, (uint4*)nullptr, (const long long*)nullptr)
  if (c->prec == MODAL_F16X3) LAUNCH(MODAL_F16X3);
  else LAUNCH(MODAL_BF16X3);
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace modal
