// Linear term as one GEMM over the whole batch (matrix cores).
//
//   L[(ab)][(s,t)] = sum_x V_ab(x) w(x) M^s_t(x)
//
// V (the Monte-Carlo pair means) is the same for every map of the batch, so this
// form reads the npairs pixel planes once per batch instead of once per map.  The
// three-pairing sum lin_prs = L[pr][s,s'] + L[ps][s,r] + L[rs][s,p] is formed by the
// split-K reduction (k_cubic.hip).  The column index (s,t) = s P + t is exactly the
// plane index of the map array [S][P][npix], so a column is one contiguous plane.
//
// Tile: ROWS pairs x COLS columns; 8 waves as 2 row halves x 4 column groups, each
// wave owning RT row tiles x CTW column tiles of 16x16 MFMAs.  Per K step of 32 pixels
// both operand tiles are staged in LDS (hi/lo splits for the split precisions; rows
// padded against bank conflicts), double-buffered so that the next step's global
// loads overlap this step's MFMAs.  A wave keeps its column-tile operands in
// registers for the step and streams its row tiles past them.
//   BF16X3: bf16 hi/lo, 3 products; F16X3: fp16 hi/lo with exact power-of-two
//   scaling (V by s_a s_b, w M by s_t s_w); both sum each step's products from zero
//   and add them to the running FP32 sum on the VALU.  F32: FP32 with
//   Fast2Sum-compensated per-step accumulation.
#include "common.h"

#include <type_traits>

namespace modal {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int KS = 32;     // pixels per K step
constexpr int WR = 2;      // row halves
constexpr int WC = 4;      // column groups
constexpr int NWV = WR * WC;
constexpr int NTH = 64 * NWV;
constexpr int GRP = NTH / KS;   // rows (or columns) one staging pass covers: 16
constexpr int KH = KS + 8;      // padded LDS row, 16-bit elements
constexpr int KF = KS + 4;      // padded LDS row, FP32

template <int PREC>
struct Tile {
  static constexpr bool SPLIT = PREC != MODAL_F32;
  static constexpr int RT = 4;                      // row tiles per wave
  static constexpr int CTW = SPLIT ? 5 : 3;         // column tiles per wave (F32 also holds compensations)
  static constexpr int ROWS = 16 * RT * WR;         // 128
  static constexpr int COLS = 16 * CTW * WC;        // 320 (split) / 192 (F32)
  static constexpr int VA = ROWS / GRP;             // staged A values per thread
  static constexpr int VB = COLS / GRP;             // staged B values per thread
  // split: [stage][hi/lo][rows|cols][KH] u16;  F32: [stage][rows|cols][KF] f32
  static constexpr size_t A_B = SPLIT ? 2 * ROWS * KH * 2 : ROWS * KF * 4;
  static constexpr size_t B_B = SPLIT ? 2 * COLS * KH * 2 : COLS * KF * 4;
  static constexpr size_t STAGE = A_B + B_B;
  static constexpr size_t TOTAL = 2 * STAGE;
};
static_assert(NTH % KS == 0, "staging assumes whole pixel rows per pass");
static_assert(Tile<MODAL_BF16X3>::ROWS % GRP == 0 && Tile<MODAL_BF16X3>::COLS % GRP == 0, "tile");
static_assert(Tile<MODAL_F32>::COLS % GRP == 0, "tile");

__device__ inline uint16_t bf16_bits(float v) {
  typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
  bf16x2 h;
  h[0] = (__bf16)v;
  h[1] = (__bf16)0.f;
  return (uint16_t)(__builtin_bit_cast(uint32_t, h) & 0xffffu);
}

template <int PREC>
__device__ inline void split_store(float v, uint16_t* hi, uint16_t* lo) {
  if (PREC == MODAL_F16X3) {
    const _Float16 h = (_Float16)v;
    *hi = __builtin_bit_cast(uint16_t, h);
    *lo = __builtin_bit_cast(uint16_t, (_Float16)(v - (float)h));
  } else {
    const uint16_t hb = bf16_bits(v);
    *hi = hb;
    *lo = bf16_bits(v - __builtin_bit_cast(float, (uint32_t)hb << 16));
  }
}

template <int PREC>
__global__ __launch_bounds__(NTH) void k_lin_gemm(int P, int npairs, int npix, int S, int nchunk, int chunk_px,
                                                  int nrb, int ncb, const int* __restrict__ pair_a,
                                                  const int* __restrict__ pair_b, const float* __restrict__ V,
                                                  const float* __restrict__ maps, const float* __restrict__ w,
                                                  const float* __restrict__ mscale, float wscale,
                                                  double* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  using T = Tile<PREC>;
  constexpr bool SCALED = PREC == MODAL_F16X3;
  constexpr int RT = T::RT, CTW = T::CTW, ROWS = T::ROWS, COLS = T::COLS, VA = T::VA, VB = T::VB;
  // XCD-aware decode: chunk c on XCD c % 8, its (row block, column block) items consecutive
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int i8 = b >> 3;
  const int per = nrb * ncb;
  const int chunk = xcd + 8 * (i8 / per);
  if (chunk >= nchunk) return;
  const int rem = i8 - (i8 / per) * per;
  const int rb = rem / ncb, cb = rem - (rem / ncb) * ncb;
  const int ncols = S * P;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int wr = wv & 1, wc = wv >> 1;
  const int row = lane & 15, kg = lane >> 4;
  const int x_begin = chunk * chunk_px;
  const int x_end = min(npix, x_begin + chunk_px);

  // staging: thread owns pixel xx of rows r0 + GRP i (A) and of columns r0 + GRP i (B)
  const int r0 = tid / KS, xx = tid - (tid / KS) * KS;
  const int row_base = rb * ROWS, col_base = cb * COLS;
  // F16X3 operand scales of this tile's rows and columns (kept in LDS, not registers)
  __shared__ float ascale[SCALED ? ROWS : 1], bscale[SCALED ? COLS : 1];
  if (SCALED) {
    for (int r = tid; r < ROWS; r += NTH) {
      const int pr = row_base + r;
      ascale[r] = pr < npairs ? mscale[pair_a[pr]] * mscale[pair_b[pr]] : 0.f;
    }
    for (int cc = tid; cc < COLS; cc += NTH) {
      const int col = col_base + cc;
      bscale[cc] = col < ncols ? mscale[col % P] * wscale : 0.f;
    }
    __syncthreads();
  }
  float sa[VA], sb[VB];
  // row/column plane offsets split into a block-uniform 64-bit part (scalar registers)
  // and this thread's 32-bit part r0 * npix
  const int roff = r0 * npix + xx;
  auto load_step = [&](int x0) {
    const bool in = x0 + xx < x_end;
    const float wx = in ? w[x0 + xx] : 0.f;
#pragma unroll
    for (int i = 0; i < VA; ++i) {
      const float* Vi = V + (size_t)(row_base + GRP * i) * npix + x0;
      float v = 0.f;
      if (in && row_base + GRP * i + r0 < npairs) v = Vi[roff];
      if (SCALED) v *= ascale[r0 + GRP * i];
      sa[i] = v;
    }
#pragma unroll
    for (int i = 0; i < VB; ++i) {
      const float* Mi = maps + (size_t)(col_base + GRP * i) * npix + x0;
      float v = 0.f;
      if (in && col_base + GRP * i + r0 < ncols) v = Mi[roff];
      v *= wx;
      if (SCALED) v *= bscale[r0 + GRP * i];
      sb[i] = v;
    }
  };
  auto store_step = [&](int stage) {
    unsigned char* base = lds + stage * T::STAGE;
#pragma unroll
    for (int i = 0; i < VA; ++i) {
      const int r = r0 + GRP * i;
      if (T::SPLIT) {
        uint16_t* hi = reinterpret_cast<uint16_t*>(base);
        split_store<PREC>(sa[i], hi + r * KH + xx, hi + ROWS * KH + r * KH + xx);
      } else {
        reinterpret_cast<float*>(base)[r * KF + xx] = sa[i];
      }
    }
#pragma unroll
    for (int i = 0; i < VB; ++i) {
      const int cc = r0 + GRP * i;
      if (T::SPLIT) {
        uint16_t* hi = reinterpret_cast<uint16_t*>(base + T::A_B);
        split_store<PREC>(sb[i], hi + cc * KH + xx, hi + COLS * KH + cc * KH + xx);
      } else {
        reinterpret_cast<float*>(base + T::A_B)[cc * KF + xx] = sb[i];
      }
    }
  };

  f32x4 acc[RT][CTW];
  f32x4 cmp[PREC == MODAL_F32 ? RT : 1][CTW];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CTW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < (PREC == MODAL_F32 ? RT : 1); ++i)
#pragma unroll
    for (int j = 0; j < CTW; ++j) cmp[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int ct0 = wc * CTW, rt0 = wr * RT;

  int stage = 0;
  load_step(x_begin);
  store_step(0);
  __syncthreads();
  for (int x0 = x_begin; x0 < x_end; x0 += KS) {
    const bool more = x0 + KS < x_end;
    if (more) load_step(x0 + KS);   // global loads in flight during this step's MFMAs
    const unsigned char* base = lds + stage * T::STAGE;
    if (T::SPLIT) {
      typedef typename std::conditional<PREC == MODAL_F16X3, f16x8, bf16x8>::type vec8;
      const uint16_t* Ah = reinterpret_cast<const uint16_t*>(base);
      const uint16_t* Al = Ah + ROWS * KH;
      const uint16_t* Bh = reinterpret_cast<const uint16_t*>(base + T::A_B);
      const uint16_t* Bl = Bh + COLS * KH;
      vec8 bh[CTW], bl[CTW];
#pragma unroll
      for (int j = 0; j < CTW; ++j) {
        const int bo = (16 * (ct0 + j) + row) * KH + 8 * kg;
        bh[j] = *reinterpret_cast<const vec8*>(Bh + bo);
        bl[j] = *reinterpret_cast<const vec8*>(Bl + bo);
      }
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int ao = (16 * (rt0 + i) + row) * KH + 8 * kg;
        const vec8 ah = *reinterpret_cast<const vec8*>(Ah + ao);
        const vec8 al = *reinterpret_cast<const vec8*>(Al + ao);
#pragma unroll
        for (int j = 0; j < CTW; ++j) {
          // each step's three products start from zero and join the running sum
          // through an RNE add: the matrix core aligns a chain's addends to its
          // largest and drops the bits below, which against a large running sum
          // would bias every step
          f32x4 t;
          if (PREC == MODAL_F16X3) {
            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[j], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[j], t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[j], t, 0, 0, 0);
          } else {
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], t, 0, 0, 0);
          }
          acc[i][j] += t;
        }
        __builtin_amdgcn_sched_barrier(0);   // at most CTW chains in flight (register budget)
      }
    } else {
      const float* A = reinterpret_cast<const float*>(base);
      const float* Bm = reinterpret_cast<const float*>(base + T::A_B);
      float bv[CTW][8];
#pragma unroll
      for (int j = 0; j < CTW; ++j)
#pragma unroll
        for (int k = 0; k < 8; ++k) bv[j][k] = Bm[(16 * (ct0 + j) + row) * KF + 8 * kg + k];
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        float av[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) av[k] = A[(16 * (rt0 + i) + row) * KF + 8 * kg + k];
#pragma unroll
        for (int j = 0; j < CTW; ++j) {
          f32x4 t = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int k = 0; k < 8; ++k) t = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k], bv[j][k], t, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float a = acc[i][j][r], bq = t[r];
            const float sum = a + bq;
            const float bb = sum - a;
            cmp[(PREC == MODAL_F32) ? i : 0][j][r] += (a - (sum - bb)) + (bq - bb);
            acc[i][j][r] = sum;
          }
        }
      }
    }
    if (more) store_step(stage ^ 1);
    __syncthreads();
    stage ^= 1;
  }

  // write partials [S][nchunk][npairs][P]:
  //   acc[i][j][r] = L[row 16 (rt0 + i) + 4 kg + r][column 16 (ct0 + j) + row]
#pragma unroll
  for (int j = 0; j < CTW; ++j) {
    const int col = col_base + 16 * (ct0 + j) + row;
    if (col >= ncols) continue;
    const int s = col / P, t = col - s * P;
    double* dst = part + ((size_t)s * nchunk + chunk) * npairs * P;
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pr = row_base + 16 * (rt0 + i) + 4 * kg + r;
        if (pr >= npairs) continue;
        double v = (double)acc[i][j][r];
        if (PREC == MODAL_F32) v += (double)cmp[(PREC == MODAL_F32) ? i : 0][j][r];
        if (SCALED)
          v /= (double)mscale[pair_a[pr]] * (double)mscale[pair_b[pr]] * (double)mscale[t] * (double)wscale;
        dst[(size_t)pr * P + t] = v;
      }
  }
}

}  // namespace

size_t lin_gemm_lds(const modal_ctx* c) {
  return c->prec == MODAL_F32 ? Tile<MODAL_F32>::TOTAL : Tile<MODAL_BF16X3>::TOTAL;
}

hipError_t lin_gemm_set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_lin_gemm<MODAL_F32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_lin_gemm<MODAL_BF16X3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_lin_gemm<MODAL_F16X3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

// Partials use the contraction's chunking so one reduction serves both.
hipError_t launch_lin_gemm(const modal_ctx* c, const void* maps, const void* V, int S, int nchunk, int chunk_px,
                           double* part, hipStream_t st) {
  const bool f32 = c->prec == MODAL_F32;
  const int rows = f32 ? Tile<MODAL_F32>::ROWS : Tile<MODAL_BF16X3>::ROWS;
  const int cols = f32 ? Tile<MODAL_F32>::COLS : Tile<MODAL_BF16X3>::COLS;
  const int nrb = (c->npairs + rows - 1) / rows;
  const int ncb = (S * c->P + cols - 1) / cols;
  if ((long long)nchunk * chunk_px < c->npix || chunk_px % KS != 0) return hipErrorInvalidValue;
  const int nslots = 8 * ((nchunk + 7) / 8);
  const size_t grid = (size_t)nslots * nrb * ncb;
  const size_t lds = lin_gemm_lds(c);
#define LAUNCH(PR)                                                                                             \
  hipLaunchKernelGGL((k_lin_gemm<PR>), dim3(grid), dim3(NTH), lds, st, c->P, c->npairs, c->npix, S, nchunk,     \
                     chunk_px, nrb, ncb, c->t.pair_a, c->t.pair_b, (const float*)V, (const float*)maps, c->t.w32, \
                     c->t.mscale, c->wscale, part)
  if (c->prec == MODAL_F16X3) LAUNCH(MODAL_F16X3);
  else if (c->prec == MODAL_BF16X3) LAUNCH(MODAL_BF16X3);
  else LAUNCH(MODAL_F32);
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace modal
