// Cubic pixel reduction on the CDNA4 matrix cores.
//
//   E_{(ab),t} = sum_x A_ab(x) B_t(x),  A_ab = M_a M_b,  B_t = w M_t
//
// is a GEMM with M = pairs, N = modes and K = pixels (split into chunks whose
// FP32 partial sums are reduced in FP64 by k_cubic.hip).  The A operand is formed
// on the vector ALUs from maps staged in LDS and never stored; B is split once
// per K step into LDS.
//
// Pair tiling: lane-row i of a wave owns a 2 x 4 block of pairs, a in {a0, a0+1},
// b in {b0..b0+3}, so one K step needs 6 map rows per lane (instead of 2 per pair)
// and the eight 16-row tiles of a wave are its eight (a, b) combinations.  Blocks
// that straddle the diagonal carry invalid pairs (a > b) whose A is zero.
//
// Precisions
//   F32    : v_mfma_f32_16x16x4_f32, A and B in FP32 (short chunks: the FP32
//            accumulation length sets this path's error).
//   BF16X3 : v_mfma_f32_16x16x32_bf16 on hi/lo splits, A B ~ Ah Bh + Ah Bl + Al Bh
//            (hi = RNE bf16, lo = RNE bf16 of the residual), FP32 accumulation.
//   F16X3  : the same on fp16 hi/lo splits (22-bit operands).  Maps are staged
//            scaled by exact powers of two s_p ~ 1/sigma_p and w by s_w ~ npix/4pi so
//            that pair products and B stay inside the fp16 range; the partial sums
//            are unscaled exactly (FP64) when written.
//
// Launch: one workgroup per (pixel chunk, block group, sky); chunk c runs on XCD
// c mod 8 with all skies of that chunk dispatched back to back.
#include "common.h"

namespace modal {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int KS = 32;          // pixels per K step
constexpr int MS_STRIDE = KS + 4;
// waves per workgroup: 8 for split-bf16 (two waves per SIMD to overlap the
// vector-ALU operand formation with the matrix cores); 4 for FP32 (compensated
// accumulation, twice the accumulator registers) and split-fp16 (scaling and the
// per-step product chains), which then have up to 512 registers per lane
template <int PREC> struct Waves { static constexpr int value = (PREC == MODAL_BF16X3) ? 8 : 4; };
constexpr int TCOLS = 48;       // modes padded to three 16-wide column tiles

struct Blocks {
  int nblk;      // valid blocks
  int ngroups;   // ceil(nblk / (16 * waves))
};

// The value a split starts from must be one rounded FP32 number: the backend may
// otherwise fuse the producing multiply into the hi conversion (a mixed-precision
// FMA rounding the exact product) in one place and not in another, so that hi and
// lo no longer add up.  An empty asm statement makes the rounded product opaque.
__device__ inline float rounded(float x) {
  asm("" : "+v"(x));
  return x;
}

__device__ inline uint32_t bf16x2_bits(float a, float b) {
  typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
  bf16x2 h;
  h[0] = (__bf16)a;
  h[1] = (__bf16)b;
  return __builtin_bit_cast(uint32_t, h);
}

// hi/lo split of 8 floats into two bf16x8 (hi = RNE(x), lo = RNE(x - hi)).
__device__ inline void split8(const float* v, bf16x8& hi, bf16x8& lo) {
  uint32_t h[4], l[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float v0 = rounded(v[2 * k]), v1 = rounded(v[2 * k + 1]);
    const uint32_t hb = bf16x2_bits(v0, v1);
    const float h0 = __builtin_bit_cast(float, hb << 16);
    const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
    h[k] = hb;
    l[k] = bf16x2_bits(v0 - h0, v1 - h1);
  }
  typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
  u32x4 hv = {h[0], h[1], h[2], h[3]};
  u32x4 lv = {l[0], l[1], l[2], l[3]};
  hi = __builtin_bit_cast(bf16x8, hv);
  lo = __builtin_bit_cast(bf16x8, lv);
}

// fp16 hi/lo split of 8 floats (hi = RNE fp16(x), lo = RNE fp16(x - hi)).
__device__ inline void split8h(const float* v, f16x8& hi, f16x8& lo) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float x = rounded(v[k]);
    const _Float16 h = (_Float16)x;
    hi[k] = h;
    lo[k] = (_Float16)(x - (float)h);
  }
}

template <int PREC>
__global__ __launch_bounds__(64 * Waves<PREC>::value) void k_cubic_mfma(int P, int npairs, int npix, int S, int nchunk, int chunk_px,
                                                   Blocks bk, const int2* __restrict__ blocks,
                                                   const int* __restrict__ pair_of, const float* __restrict__ maps,
                                                   const float* __restrict__ w, const float* __restrict__ mscale,
                                                   float wscale, double* __restrict__ part) {
  constexpr bool SCALED = (PREC == MODAL_F16X3);
  constexpr int NT = 64 * Waves<PREC>::value;
  constexpr int BLK_PER_GROUP = 16 * Waves<PREC>::value;
  // ---- XCD-aware decode: chunk c on XCD c % 8, its (group, sky) items consecutive there
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int i8 = b >> 3;
  const int per = bk.ngroups * S;
  const int chunk = xcd + 8 * (i8 / per);
  if (chunk >= nchunk) return;
  const int rem = i8 - (i8 / per) * per;
  const int group = rem / S;
  const int s = rem - group * S;

  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63;
  const int row = lane & 15, kg = lane >> 4;

  __shared__ float Ms[kMaxP][MS_STRIDE];
  __shared__ __attribute__((aligned(16))) uint16_t Bh[TCOLS][KS];   // bf16 / fp16 bits
  __shared__ __attribute__((aligned(16))) uint16_t Bl[TCOLS][KS];
  __shared__ float msc[kMaxP];
  if (tid < kMaxP) msc[tid] = (SCALED && tid < P) ? mscale[tid] : 1.f;
  __shared__ __attribute__((aligned(16))) float Bf[TCOLS][KS];      // FP32 path

  // this lane-row's block
  const int blk = group * BLK_PER_GROUP + wv * 16 + row;
  int a0 = -1, b0 = 0;
  if (blk < bk.nblk) {
    const int2 bb = blocks[blk];
    a0 = bb.x;
    b0 = bb.y;
  }
  __syncthreads();

  f32x4 acc[8][3];
  f32x4 cmp[PREC == MODAL_F32 ? 8 : 1][3];   // FP32: running compensation of acc (Fast2Sum)
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[j][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < (PREC == MODAL_F32 ? 8 : 1); ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) cmp[j][c] = f32x4{0.f, 0.f, 0.f, 0.f};

  const float* Msky = maps + (size_t)s * P * npix;
  const int x_begin = chunk * chunk_px;
  const int x_end = min(npix, x_begin + chunk_px);

  for (int x0 = x_begin; x0 < x_end; x0 += KS) {
    // ---- stage maps and the B operand for this K step
    for (int e = tid; e < P * KS; e += NT) {
      const int p = e / KS, xx = e - p * KS;
      const int x = x0 + xx;
      Ms[p][xx] = x < x_end ? Msky[(size_t)p * npix + x] * msc[p] : 0.f;
    }
    for (int e = tid; e < TCOLS * KS / 2; e += NT) {
      const int t = e / (KS / 2), xx = 2 * (e - t * (KS / 2));
      const int x = x0 + xx;
      float v0 = 0.f, v1 = 0.f;
      if (t < P) {
        const float sc = SCALED ? msc[t] * wscale : 1.f;
        if (x < x_end) v0 = w[x] * sc * Msky[(size_t)t * npix + x];
        if (x + 1 < x_end) v1 = w[x + 1] * sc * Msky[(size_t)t * npix + x + 1];
      }
      v0 = rounded(v0);
      v1 = rounded(v1);
      if (PREC == MODAL_F16X3) {
        const _Float16 h0 = (_Float16)v0, h1 = (_Float16)v1;
        const _Float16 l0 = (_Float16)(v0 - (float)h0), l1 = (_Float16)(v1 - (float)h1);
        Bh[t][xx] = __builtin_bit_cast(uint16_t, h0);
        Bh[t][xx + 1] = __builtin_bit_cast(uint16_t, h1);
        Bl[t][xx] = __builtin_bit_cast(uint16_t, l0);
        Bl[t][xx + 1] = __builtin_bit_cast(uint16_t, l1);
      } else if (PREC == MODAL_BF16X3) {
        const uint32_t hb = bf16x2_bits(v0, v1);
        const float h0 = __builtin_bit_cast(float, hb << 16);
        const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
        const uint32_t lb = bf16x2_bits(v0 - h0, v1 - h1);
        *reinterpret_cast<uint32_t*>(&Bh[t][xx]) = hb;
        *reinterpret_cast<uint32_t*>(&Bl[t][xx]) = lb;
      } else {
        Bf[t][xx] = v0;
        Bf[t][xx + 1] = v1;
      }
    }
    __syncthreads();

    {
      // Every lane runs this block: an MFMA reads its operands from all 64 lanes,
      // so no lane may skip it; lane-rows without a block contribute A = 0.
      // the six map rows this lane needs, at its 8 pixels (x0 + 8 kg .. + 7)
      float ma[2][8], mb[4][8];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int p = min(max(a0, 0) + u, P - 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) ma[u][k] = Ms[p][8 * kg + k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = min(b0 + u, P - 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) mb[u][k] = Ms[p][8 * kg + k];
      }
      if (PREC == MODAL_BF16X3) {
        bf16x8 bh[3], bl[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          bh[c] = *reinterpret_cast<const bf16x8*>(&Bh[16 * c + row][8 * kg]);
          bl[c] = *reinterpret_cast<const bf16x8*>(&Bl[16 * c + row][8 * kg]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          // rows of pairs outside the triangle (or of lanes without a block) hold
          // finite products that are never written out
          float av[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) av[k] = ma[j >> 2][k] * mb[j & 3][k];
          bf16x8 ah, al;
          split8(av, ah, al);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[c], acc[j][c], 0, 0, 0);
            acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[c], acc[j][c], 0, 0, 0);
            acc[j][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[c], acc[j][c], 0, 0, 0);
          }
        }
      } else if (PREC == MODAL_F16X3) {
        f16x8 bh[3], bl[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          bh[c] = *reinterpret_cast<const f16x8*>(&Bh[16 * c + row][8 * kg]);
          bl[c] = *reinterpret_cast<const f16x8*>(&Bl[16 * c + row][8 * kg]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          // rows of pairs outside the triangle (or of lanes without a block) hold
          // finite products that are never written out
          float av[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) av[k] = ma[j >> 2][k] * mb[j & 3][k];
          f16x8 ah, al;
          split8h(av, ah, al);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            // the three products of one K step start from zero and join the running
            // sum with a round-to-nearest vector add, so the long FP32 sum is not
            // accumulated inside the matrix unit
            f32x4 t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[c], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[c], t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[c], t, 0, 0, 0);
            acc[j][c] += t;
          }
        }
      } else {
        float bv[3][8];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 8; ++k) bv[c][k] = Bf[16 * c + row][8 * kg + k];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          // rows of pairs outside the triangle (or of lanes without a block) hold
          // finite products that are never written out
          float av[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) av[k] = ma[j >> 2][k] * mb[j & 3][k];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            // one K step (8 MFMAs of K = 4) from zero, then a round-to-nearest add
            f32x4 t = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 8; ++k) t = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k], bv[c][k], t, 0, 0, 0);
            // two-sum of the running total and this K step; the rounding error is kept
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float a = acc[j][c][r], b = t[r];
              const float sum = a + b;
              const float bb = sum - a;
              const float err = (a - (sum - bb)) + (b - bb);
              acc[j][c][r] = sum;
              cmp[(PREC == MODAL_F32) ? j : 0][c][r] += err;
            }
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- write this chunk's partial sums: acc[j][c][r] is output row 4 kg + r
  // (a lane-row of this wave), column t = 16 c + row
  double* dst = part + ((size_t)s * nchunk + chunk) * npairs * P;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int orow = 4 * kg + r;
    const int oblk = group * BLK_PER_GROUP + wv * 16 + orow;
    if (oblk >= bk.nblk) continue;
    const int2 bb = blocks[oblk];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int a = bb.x + (j >> 2), bm = bb.y + (j & 3);
      if (a >= P || bm >= P || a > bm) continue;
      const int pr = pair_of[a * P + bm];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int t = 16 * c + row;
        if (t < P) {
          double v = (double)acc[j][c][r];
          if (PREC == MODAL_F32) v += (double)cmp[(PREC == MODAL_F32) ? j : 0][c][r];
          if (SCALED) v /= (double)msc[a] * (double)msc[bm] * (double)msc[t] * (double)wscale;
          dst[(size_t)pr * P + t] = v;
        }
      }
    }
  }
}

int chunk_px_for(const modal_ctx* c, int target) {
  // nchunk a multiple of 8 (one chunk stream per XCD), chunks of about target pixels
  int nchunk = 8 * ((c->npix + 8 * target - 1) / (8 * target));
  int px = (c->npix + nchunk - 1) / nchunk;
  px = (px + 127) / 128 * 128;   // whole staged steps of both matrix-core kernels (64, 128 pixels)
  return px;
}

}  // namespace

// FP32 accumulates its exact products in FP32, so it uses short chunks; the split
// precisions carry a larger operand error and use long chunks (fewer partials).
// (defaults: the autotuner's choice at lmax 1000, P 40 on MI355X)
int chunk_target_default(const modal_ctx* c) { return c->prec == MODAL_F32 ? 4096 : 16384; }
int chunk_target_min(const modal_ctx* c) { return c->prec == MODAL_F32 ? 2048 : 8192; }

int cubic_chunk_px(const modal_ctx* c) {
  return chunk_px_for(c, c->tune_chunk_px > 0 ? c->tune_chunk_px : chunk_target_default(c));
}

int cubic_mfma_nchunk_max(const modal_ctx* c) {
  const int px = chunk_px_for(c, chunk_target_min(c));
  return (c->npix + px - 1) / px;
}

// The FP32 tiles cover the modes t < 48 (three 16-row tiles per wave); more modes in an
// FP32 context take the vector-ALU contraction.  The split precisions' own contraction
// covers every P <= kMaxP (this flag also picks their chunking).
bool cubic_mfma_available(const modal_ctx* c) {
  return (c->prec == MODAL_F32 && c->P <= 48) || c->prec == MODAL_BF16X3 || c->prec == MODAL_F16X3;
}

int cubic_mfma_nchunk(const modal_ctx* c) {
  const int px = chunk_px_for(c, c->tune_chunk_px > 0 ? c->tune_chunk_px : chunk_target_default(c));
  return (c->npix + px - 1) / px;
}

// Blocks of 2 x 4 pairs covering the triangle a <= b < P.
void make_pair_blocks(int P, std::vector<int2>& out) {
  out.clear();
  for (int u = 0; u < P; u += 2)
    for (int v = 0; v < P; v += 4) {
      bool any = false;
      for (int a = u; a < u + 2 && a < P; ++a)
        for (int b = v; b < v + 4 && b < P; ++b) any |= (a <= b);
      if (any) out.push_back(make_int2(u, v));
    }
}

hipError_t launch_cubic_mfma(const modal_ctx* c, const void* maps, int S, double* part, hipStream_t st) {
  Blocks bk;
  bk.nblk = c->t.nblk;
  const int waves = (c->prec == MODAL_BF16X3) ? Waves<MODAL_BF16X3>::value : Waves<MODAL_F32>::value;
  bk.ngroups = (bk.nblk + 16 * waves - 1) / (16 * waves);
  const int px = chunk_px_for(c, c->tune_chunk_px > 0 ? c->tune_chunk_px : chunk_target_default(c));
  const int nchunk = (c->npix + px - 1) / px;
  const int nslots = 8 * ((nchunk + 7) / 8);
  const size_t grid = (size_t)nslots * bk.ngroups * S;
#define LAUNCH(PR)                                                                                            \
  hipLaunchKernelGGL((k_cubic_mfma<PR>), dim3(grid), dim3(64 * Waves<PR>::value), 0, st, c->P, c->npairs,    \
                     c->npix, S, nchunk, px, bk, c->t.blk, c->t.pair_of, (const float*)maps, c->t.w32,        \
                     c->t.mscale, c->wscale, part)
  if (c->prec == MODAL_F16X3) LAUNCH(MODAL_F16X3);
  else if (c->prec == MODAL_BF16X3) LAUNCH(MODAL_BF16X3);
  else LAUNCH(MODAL_F32);
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace modal
