// Cubic pixel reduction on the matrix cores, 32x32 tiles over a cover of the triples:
// split 16-bit operands (32x32x16) for the bf16x3 and f16x3 contexts, FP32 operands
// (32x32x2) for FP32 contexts.
//
//   E_{(ab),t} = sum_x A_ab(x) B_t(x),  A_ab = M_a M_b,  B_t = w M_t,
//
// a GEMM with M = pairs, N = modes, K = pixels (chunked; FP32 partial sums are
// reduced in FP64 by k_cubic.hip).  beta_prs is the cell of any one of its three
// pairings, so only the cells of the cover are computed.
//
// Tiling (v_mfma_f32_32x32x16_{bf16,f16}; lane l holds A[l % 32][8 (l / 32) + i],
// B[8 (l / 32) + i][l % 32], and accumulator register j is D[8 (j / 4) + 4 (l / 32)
// + j % 4][l % 32]):
//   * lane-row i of a wave owns a 2 x 2 block of pairs (a0, a0+1) x (b0, b0+1); the
//     four 32-row tiles of a wave are the four positions in the block, so a K step
//     reads 4 map rows per lane for 4 pair products;
//   * a work item is 32 such blocks with one 32-mode window [s0, s0 + 32), and each
//     block carries the range [zlo, zhi) of window modes it writes.  The host covers
//     the triples with few items (make_cubic_cover): beta_{abz} is the cell of pair
//     (a, b) at mode z for any of the three ways to split the triple, so the pairs need
//     not be the two smallest modes.  The modes are grouped in two-mode vertices split
//     into two classes; pairs inside a class take the window that holds the modes of
//     the class, and by pigeonhole two modes of every triple share a class (for P 40:
//     4 items instead of the 8 that pairs (a <= b) with modes z >= b take);
//   * with fewer than eight items the waves of a workgroup share them: MULT waves run
//     one item, each on its own substeps of every staged step, and their sums are
//     added through LDS at the end;
//   * maps and the split B operand of a 128-pixel step are staged in LDS, double
//     buffered, with the next step's global loads issued before this step's MFMAs
//     (a step is long enough to cover the load latency).
// Precisions
//   FP32  : A formed in FP32 per lane, B = w M_t in FP32 in LDS; v_mfma_f32_32x32x2_f32 with
//           pixel 8 kh + i of a substep in MFMA i; each substep's 8 MFMAs start from zero
//           and join the running FP32 sum.
//   BF16X3: maps staged in FP32; A = M_a M_b in FP32 split as hi = RNE bf16, lo = RNE bf16
//           of the exact residual; Ah Bh + Ah Bl + Al Bh.
//   F16X3 : maps scaled by exact powers of two (s_p ~ 1/sigma_p, s_w ~ npix/4pi) and staged
//           as fp16 pairs m = h + l (h = f16(m), l = f16(m - h)).  A pair product is formed
//           with packed fp16 arithmetic, two pixels per instruction:
//             H = h_a h_b (rounded), r = fma(h_a, h_b, -H) (exact: the residual of a 22-bit
//             product fits in fp16), L = fma(l_a, h_b, fma(h_a, l_b, r)),
//           so A = H + L carries about 21 bits (the l_a l_b term, 2^-22, is dropped): four
//           packed instructions per two products.
// For F16X3 with one wave per item the substeps of 16 pixels are software-pipelined: the next substep's map rows
// are read and its pair products split while this substep's MFMAs run, so that the vector
// work issues between matrix-core instructions instead of after them (8.7 -> 8.0 ms per
// 8-sky batch at l_max 1000, P 40 with the packed products; the same order made the bf16
// split, twice the vector work, 3% slower, so bf16 keeps split-then-MFMA per substep).
// With waves sharing an item (four substeps each per staged step) the pipelined registers
// spilled (80 bytes per lane) and split-then-MFMA was faster for F16X3 too (5.35 -> 4.88 ms
// per 8-sky batch at l_max 1000, P 40, same box).
// The matrix core drops addend bits below the largest term of an accumulation, which
// against a long running sum biases every step; so the MFMAs accumulate a short
// chain of CHAIN x MULT staged steps from zero (48 MFMAs per tile whatever the number of
// waves sharing an item), and each chain joins the running FP32 sum
// with a round-to-nearest vector add.
#include "common.h"

#include <type_traits>

namespace modal {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

constexpr int KS = 128;            // pixels per staged step (eight MFMA K = 16 substeps)
constexpr int NW = 8;              // waves per workgroup
constexpr int NT = 64 * NW;
constexpr int BPW = 32;            // pair blocks per wave (one per lane-row)
constexpr int MSS = KS + 4;        // map row stride in LDS (floats)
constexpr int BSS = KS + 8;        // B row stride in LDS (16-bit)
constexpr int BROWS = 64;          // B rows: row r <-> mode P - 64 + r (rows of negative modes are zero)
constexpr int BSF = KS + 4;        // FP32 contexts: B row stride (floats) of the FP32 operand in the bh/bl area
constexpr int QSTEP = kMaxP * KS / (4 * NT);   // staged pixel quads per thread per step (4)
constexpr int CHAIN = 2;           // staged steps per MFMA accumulation chain with one wave per item

// LDS slot of map row r: even rows first, then odd rows.  The lane-rows of a wave
// read rows a0 (even, consecutive blocks) and a0 + 1, so consecutive even rows land
// in consecutive 16-byte bank groups (row stride MSS = 17 groups).
__device__ inline int ms_slot(int r) { return (r >> 1) + (r & 1) * (kMaxP / 2); }

struct Lds {
  float ms[2][kMaxP][MSS];
  uint16_t bh[2][BROWS][BSS];
  uint16_t bl[2][BROWS][BSS];
};
// FP32 contexts keep B as floats [2][BROWS][BSF] in the bh and bl arrays
static_assert((size_t)2 * BROWS * BSF * sizeof(float) <= 2 * sizeof(uint16_t[2][BROWS][BSS]), "FP32 B operand");
// the sums of the waves that share an item pass through the staging area (up to 7 waves)
static_assert(sizeof(Lds) >= (size_t)(NW - 1) * 64 * 64 * sizeof(float), "LDS too small for the wave sums");

// The value a split starts from must be one rounded FP32 number (see the bf16 path).
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

// bf16 hi/lo of the products x[k] y[k], k = 0..7.
__device__ inline void split_bf16(const float* x, const float* y, bf16x8& hi, bf16x8& lo) {
  u32x4 h, l;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float v0 = rounded(x[2 * k] * y[2 * k]), v1 = rounded(x[2 * k + 1] * y[2 * k + 1]);
    uint32_t hb = bf16x2_bits(v0, v1);
    asm("" : "+v"(hb));   // extract the hi words from this one conversion
    h[k] = hb;
    l[k] = bf16x2_bits(v0 - __builtin_bit_cast(float, hb << 16), v1 - __builtin_bit_cast(float, hb & 0xffff0000u));
  }
  hi = __builtin_bit_cast(bf16x8, h);
  lo = __builtin_bit_cast(bf16x8, l);
}

typedef __attribute__((__vector_size__(2 * sizeof(_Float16)))) _Float16 f16x2;

// fp16 hi/lo of the products (ha + la)(hb + lb) of eight pixels, two per packed instruction
__device__ inline void prod_f16(const u32x4& ha, const u32x4& la, const u32x4& hb, const u32x4& lb, f16x8& hi,
                                f16x8& lo) {
  u32x4 h, l;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // vector elements go through scalars first: a bit_cast of the element itself is dropped
    // by the compiler
    const uint32_t wa = ha[k], va = la[k], wb = hb[k], vb = lb[k];
    const f16x2 xa = __builtin_bit_cast(f16x2, wa), ya = __builtin_bit_cast(f16x2, va);
    const f16x2 xb = __builtin_bit_cast(f16x2, wb), yb = __builtin_bit_cast(f16x2, vb);
    f16x2 H = xa * xb;
    uint32_t Hb = __builtin_bit_cast(uint32_t, H);
    asm("" : "+v"(Hb));   // H is one rounded product, used as is below
    H = __builtin_bit_cast(f16x2, Hb);
    f16x2 r = __builtin_elementwise_fma(xa, xb, -H);
    r = __builtin_elementwise_fma(xa, yb, r);
    r = __builtin_elementwise_fma(ya, xb, r);
    const uint32_t rb = __builtin_bit_cast(uint32_t, r);
    h[k] = Hb;
    l[k] = rb;
  }
  hi = __builtin_bit_cast(f16x8, h);
  lo = __builtin_bit_cast(f16x8, l);
}

// hi/lo words of two B values (packed low half first); each split starts from one
// rounded FP32 value
template <int PREC>
__device__ inline void split_pair(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  v0 = rounded(v0);
  v1 = rounded(v1);
  if (PREC == MODAL_F16X3) {
    const _Float16 h0 = (_Float16)v0, h1 = (_Float16)v1;
    const _Float16 r0 = (_Float16)(v0 - (float)h0), r1 = (_Float16)(v1 - (float)h1);
    hi = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
    lo = (uint32_t)__builtin_bit_cast(uint16_t, r0) | ((uint32_t)__builtin_bit_cast(uint16_t, r1) << 16);
  } else {
    uint32_t hb = bf16x2_bits(v0, v1);
    asm("" : "+v"(hb));
    hi = hb;
    lo = bf16x2_bits(v0 - __builtin_bit_cast(float, hb << 16), v1 - __builtin_bit_cast(float, hb & 0xffff0000u));
  }
}

template <int PREC, typename V>
__device__ inline f32x16 mfma32(const V& a, const V& b, const f32x16& c) {
  if constexpr (PREC == MODAL_F16X3)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                   0);
}

// FP32 contexts: v_mfma_f32_32x32x2_f32, lane l holding A[l % 32][l / 32] and B[l / 32][l % 32]
__device__ inline f32x16 mfma32_f32(float a, float b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <int PREC, int MULT>
__global__ __launch_bounds__(NT) void k_cubic_split(int P, int npairs, int npix, int S, int nchunk, int chunk_px,
                                                    int nblk, int nitems, int ngroups, const int4* __restrict__ blocks,
                                                    const int2* __restrict__ items, const int* __restrict__ pair_of,
                                                    const float* __restrict__ maps, const float* __restrict__ w,
                                                    const float* __restrict__ mscale, float wscale, int vec,
                                                    double* __restrict__ part) {
  constexpr bool F16 = PREC == MODAL_F16X3;
  constexpr bool F32 = PREC == MODAL_F32;
  // MFMA accumulation chain in staged steps: 48 MFMAs per tile for the splits (FP32
  // contexts chain one 16-pixel substep, 8 MFMAs of K = 2, inside the substep loop)
  constexpr int CHAIN_STEPS = CHAIN * MULT;
  constexpr int NWI = NW / MULT;          // items per workgroup
  constexpr int NSUB = KS / 16 / MULT;    // substeps of a staged step per wave
  typedef typename std::conditional<F16, f16x8, bf16x8>::type vec8;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  Lds& L = *reinterpret_cast<Lds*>(lds_raw);
  __shared__ float msc[kMaxP];

  // XCD-aware decode: chunk c on XCD c % 8, its (group, sky) items consecutive there
  const int bid = blockIdx.x;
  const int xcd = bid & 7;
  const int i8 = bid >> 3;
  const int per = ngroups * S;
  const int chunk = xcd + 8 * (i8 / per);
  if (chunk >= nchunk) return;
  const int rem = i8 - (i8 / per) * per;
  const int group = rem / S;
  const int s = rem - group * S;

  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int lrow = lane & 31, kh = lane >> 5;

  if (tid < kMaxP) msc[tid] = (F16 && tid < P) ? mscale[tid] : 1.f;
  // rows of negative modes stay zero in both stages
  float* const bf = reinterpret_cast<float*>(&L.bh[0][0][0]);   // FP32 contexts: B as [2][BROWS][BSF]
  if constexpr (F32) {
    for (int e = tid; e < 2 * BROWS * BSF; e += NT)
      if ((e / BSF) % BROWS < BROWS - P) bf[e] = 0.f;
  } else {
    for (int e = tid; e < 2 * BROWS * BSS; e += NT) {
      const int st = e / (BROWS * BSS), r = (e / BSS) % BROWS, xx = e % BSS;
      if (r < BROWS - P) {
        L.bh[st][r][xx] = 0;
        L.bl[st][r][xx] = 0;
      }
    }
  }

  // this wave's work item (wave-uniform): 32 blocks from wfirst, window [s0, s0 + 32);
  // the MULT waves wi, wi + NWI, ... of an item take the substeps sub NSUB .. + NSUB - 1
  // of every staged step
  const int wi = wv % NWI, sub = wv / NWI;
  const int item = group * NWI + wi;
  const bool wave_on = item < nitems;
  int wfirst = 0, s0 = P - 32;
  if (wave_on) {
    const int2 it = items[item];
    wfirst = __builtin_amdgcn_readfirstlane(it.x);
    s0 = __builtin_amdgcn_readfirstlane(it.y);
  }
  const int myblk = wfirst + lrow;
  int a0 = 0, b0 = 0;
  if (myblk < nblk) {
    const int4 bb = blocks[myblk];
    a0 = bb.x;
    b0 = bb.y;
  }
  // LDS offsets (floats within a stage) of this lane's four map rows at its k-half
  const int oa[2] = {ms_slot(min(a0, P - 1)) * MSS + 8 * kh, ms_slot(min(a0 + 1, P - 1)) * MSS + 8 * kh};
  const int ob_[2] = {ms_slot(min(b0, P - 1)) * MSS + 8 * kh, ms_slot(min(b0 + 1, P - 1)) * MSS + 8 * kh};

  const float* Msky = maps + (size_t)s * P * npix;
  const int x_begin = chunk * chunk_px;
  const int x_end = min(npix, x_begin + chunk_px);

  // staging: thread owns quads e = tid + NT i -> (mode t = e / (KS / 4), pixels 4 (e % (KS / 4)) .. + 3).
  // Loads are float4 when rows are 16-byte aligned (npix % 4 == 0; chunks start at
  // multiples of 64 pixels, so a quad is then wholly inside or wholly past the chunk
  // end), element-wise otherwise; indices are clamped in range and the loads are
  // unconditional.  Past the chunk end w = 0 makes B = 0, so whatever A holds there
  // contributes nothing.  Rows t >= P (whole waves when P % 4 == 0) stage nothing.
  float4 pre[QSTEP];
  float4 wpre;
  const int sq4 = 4 * (tid % (KS / 4));
  auto load_step = [&](int x0) {
    const int x = x0 + sq4;
    if (vec) {
      const int xc = min(x, x_end - 4);
      const float4 wv_ = *reinterpret_cast<const float4*>(w + xc);
      wpre = x < x_end ? wv_ : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int i = 0; i < QSTEP; ++i) {
        const int t = min((tid + NT * i) / (KS / 4), P - 1);
        pre[i] = *reinterpret_cast<const float4*>(Msky + (size_t)t * npix + xc);
      }
    } else {
      float wq[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int xc = min(x + k, x_end - 1);
        const float wv_ = w[xc];
        wq[k] = x + k < x_end ? wv_ : 0.f;
      }
      wpre = make_float4(wq[0], wq[1], wq[2], wq[3]);
#pragma unroll
      for (int i = 0; i < QSTEP; ++i) {
        const float* row = Msky + (size_t)min((tid + NT * i) / (KS / 4), P - 1) * npix;
        pre[i] = make_float4(row[min(x, x_end - 1)], row[min(x + 1, x_end - 1)], row[min(x + 2, x_end - 1)],
                             row[min(x + 3, x_end - 1)]);
      }
    }
  };
  auto store_step = [&](int st) {
#pragma unroll
    for (int i = 0; i < QSTEP; ++i) {
      const int t = (tid + NT * i) / (KS / 4);
      if (t < P) {
        const float m = msc[t];
        const float sc = F16 ? m * wscale : 1.f;
        uint32_t h0, l0, h1, l1;
        if (F16) {
          // the row as halves: hi words at [0, KS), lo words at [KS, 2 KS)
          uint16_t* row = reinterpret_cast<uint16_t*>(&L.ms[st][ms_slot(t)][0]);
          split_pair<PREC>(pre[i].x * m, pre[i].y * m, h0, l0);
          split_pair<PREC>(pre[i].z * m, pre[i].w * m, h1, l1);
          *reinterpret_cast<uint2*>(row + sq4) = make_uint2(h0, h1);
          *reinterpret_cast<uint2*>(row + KS + sq4) = make_uint2(l0, l1);
        } else {
          *reinterpret_cast<float4*>(&L.ms[st][ms_slot(t)][sq4]) = pre[i];
        }
        if constexpr (F32) {
          *reinterpret_cast<float4*>(bf + ((size_t)st * BROWS + BROWS - P + t) * BSF + sq4) =
              make_float4(wpre.x * pre[i].x, wpre.y * pre[i].y, wpre.z * pre[i].z, wpre.w * pre[i].w);
          continue;
        }
        split_pair<PREC>(wpre.x * sc * pre[i].x, wpre.y * sc * pre[i].y, h0, l0);
        split_pair<PREC>(wpre.z * sc * pre[i].z, wpre.w * sc * pre[i].w, h1, l1);
        *reinterpret_cast<uint2*>(&L.bh[st][BROWS - P + t][sq4]) = make_uint2(h0, h1);
        *reinterpret_cast<uint2*>(&L.bl[st][BROWS - P + t][sq4]) = make_uint2(l0, l1);
      }
    }
  };

  f32x16 acc[4], cha[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = cha[j][r] = 0.f;
  const int brow = s0 - (P - BROWS) + lrow;   // this lane's B row (mode s0 + lrow)

  __syncthreads();   // msc and the zero rows
  load_step(x_begin);
  store_step(0);
  __syncthreads();
  int st = 0, link = 0;
  for (int x0 = x_begin; x0 < x_end; x0 += KS) {
    const bool more = x0 + KS < x_end;
    if (more) load_step(x0 + KS);
    if (wave_on) {
      // The lane's four map rows at its 8 pixels of substep ks (F16X3: fp16 hi and lo words;
      // BF16X3: FP32 values), and the split pair product of tile j = (a row j / 2, b row j % 2).
      struct Rows {
        u32x4 h[4], l[4];   // F16X3
        float v[4][8];      // BF16X3
      };
      auto load_rows = [&](int ks, Rows& R) {
        if constexpr (F16) {
          const uint16_t* rows = reinterpret_cast<const uint16_t*>(&L.ms[st][0][0]);
          // row offsets in halves: the slot's row start doubles (two halves per float of the
          // row), the lane's pixel offset 8 kh does not (one half per pixel)
          const int o[4] = {2 * oa[0] - 8 * kh, 2 * oa[1] - 8 * kh, 2 * ob_[0] - 8 * kh, 2 * ob_[1] - 8 * kh};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            R.h[u] = *reinterpret_cast<const u32x4*>(rows + o[u] + 16 * ks);
            R.l[u] = *reinterpret_cast<const u32x4*>(rows + o[u] + KS + 16 * ks);
          }
        } else {
          const float* msb = &L.ms[st][0][0] + 16 * ks;
          const int o[4] = {oa[0], oa[1], ob_[0], ob_[1]};
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float4 lo4 = reinterpret_cast<const float4*>(msb + o[u])[0];
            const float4 hi4 = reinterpret_cast<const float4*>(msb + o[u])[1];
            R.v[u][0] = lo4.x; R.v[u][1] = lo4.y; R.v[u][2] = lo4.z; R.v[u][3] = lo4.w;
            R.v[u][4] = hi4.x; R.v[u][5] = hi4.y; R.v[u][6] = hi4.z; R.v[u][7] = hi4.w;
          }
        }
      };
      auto split_tile = [&](const Rows& R, int j, vec8& ah, vec8& al) {
        if constexpr (F16)
          prod_f16(R.h[j >> 1], R.l[j >> 1], R.h[2 + (j & 1)], R.l[2 + (j & 1)], *reinterpret_cast<f16x8*>(&ah),
                   *reinterpret_cast<f16x8*>(&al));
        else
          split_bf16(R.v[j >> 1], R.v[2 + (j & 1)], *reinterpret_cast<bf16x8*>(&ah), *reinterpret_cast<bf16x8*>(&al));
      };
      if constexpr (F32) {
        // FP32: per substep the lane's 8 pixels as 8 MFMAs of K = 2 per tile (pixel 8 kh + i
        // in MFMA i, in A and B alike), the four tiles in turn.  Each substep's chain starts
        // from zero and joins the running sum (twice the accumulation steps per pixel of the
        // split forms' K = 16 tiles, so shorter chains keep the truncation of the addends
        // small)
#pragma unroll
        for (int i = 0; i < NSUB; ++i) {
          const int ks = sub * NSUB + i;
          const float* brw = bf + ((size_t)st * BROWS + brow) * BSF + 16 * ks + 8 * kh;
          const float4 b0 = reinterpret_cast<const float4*>(brw)[0];
          const float4 b1 = reinterpret_cast<const float4*>(brw)[1];
          const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
          Rows R;
          load_rows(ks, R);
          f32x16 ch[4];
#pragma unroll
          for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const float a = R.v[j >> 1][k] * R.v[2 + (j & 1)][k];
              ch[j] = mfma32_f32(a, bv[k], k == 0 ? f32x16{} : ch[j]);
            }
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[j] += ch[j];
        }
      } else if constexpr (!F16 || MULT >= 2) {
        // bf16: per substep, all four tiles' operands first, then the MFMAs product by product,
        // so that consecutive MFMAs feed different accumulators (measured faster than the
        // pipelined order for bf16, whose split is twice the vector work of the fp16 one)
#pragma unroll
        for (int i = 0; i < NSUB; ++i) {
          const int ks = sub * NSUB + i;
          const int kx = 16 * ks + 8 * kh;
          const vec8 bh = *reinterpret_cast<const vec8*>(&L.bh[st][brow][kx]);
          const vec8 bl = *reinterpret_cast<const vec8*>(&L.bl[st][brow][kx]);
          Rows R;
          load_rows(ks, R);
          vec8 ah[4], al[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) split_tile(R, j, ah[j], al[j]);
#pragma unroll
          for (int j = 0; j < 4; ++j) cha[j] = mfma32<PREC>(al[j], bh, cha[j]);
#pragma unroll
          for (int j = 0; j < 4; ++j) cha[j] = mfma32<PREC>(ah[j], bl, cha[j]);
#pragma unroll
          for (int j = 0; j < 4; ++j) cha[j] = mfma32<PREC>(ah[j], bh, cha[j]);
        }
      } else {
      vec8 ah[4], al[4];
      {
        Rows R0;
        load_rows(sub * NSUB, R0);
#pragma unroll
        for (int j = 0; j < 4; ++j) split_tile(R0, j, ah[j], al[j]);
      }
#pragma unroll
      for (int i = 0; i < NSUB; ++i) {
        const int ks = sub * NSUB + i;
        const int kx = 16 * ks + 8 * kh;
        const vec8 bh = *reinterpret_cast<const vec8*>(&L.bh[st][brow][kx]);
        const vec8 bl = *reinterpret_cast<const vec8*>(&L.bl[st][brow][kx]);
        Rows Rn;
        if (i + 1 < NSUB) load_rows(ks + 1, Rn);
        // tile by tile: its three products, then the next substep's split of the same tile
        // into the registers they have just read (issued among the following MFMAs)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cha[j] = mfma32<PREC>(al[j], bh, cha[j]);
          cha[j] = mfma32<PREC>(ah[j], bl, cha[j]);
          cha[j] = mfma32<PREC>(ah[j], bh, cha[j]);
          if (i + 1 < NSUB) split_tile(Rn, j, ah[j], al[j]);
        }
      }
      }
      if (!F32 && (++link == CHAIN_STEPS || !more)) {   // wave-uniform
        link = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[j] += cha[j];
#pragma unroll
          for (int r = 0; r < 16; ++r) cha[j][r] = 0.f;
        }
      }
    }
    if (more) store_step(st ^ 1);
    __syncthreads();
    st ^= 1;
  }
  if constexpr (MULT > 1) {
    // the item's other waves hand their sums to wave sub 0 through LDS (the staging
    // buffers are free after the loop's last barrier), added in the order of sub
    float* red = reinterpret_cast<float*>(lds_raw);
    if (sub > 0) {
      float* mine = red + (size_t)((sub - 1) * NWI + wi) * (64 * 64) + lane;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) mine[(16 * j + r) * 64] = acc[j][r];
    }
    __syncthreads();
    if (sub > 0) return;
#pragma unroll 1
    for (int u = 1; u < MULT; ++u) {
      const float* theirs = red + (size_t)((u - 1) * NWI + wi) * (64 * 64) + lane;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[j][r] += theirs[(16 * j + r) * 64];
    }
  }
  if (!wave_on) return;

  // partial sums: acc[j][r] = E[pair j of block wfirst + 8 (r/4) + 4 kh + r % 4][mode s0 + lrow];
  // each block writes the modes [zlo, zhi) of the window (a cell is written by one item)
  const int t = s0 + lrow;
  double* dst = part + ((size_t)s * nchunk + chunk) * npairs * P;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ob = wfirst + 8 * (r >> 2) + 4 * kh + (r & 3);
    if (ob >= nblk) continue;
    const int4 bb = blocks[ob];
    if (t < bb.z || t >= bb.w) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = bb.x + (j >> 1), b = bb.y + (j & 1);
      if (a >= P || b >= P || a > b) continue;
      double v = (double)acc[j][r];
      if (F16) v *= 1.0 / ((double)mscale[a] * (double)mscale[b] * (double)mscale[t] * (double)wscale);   // powers of two
      dst[(size_t)pair_of[a * P + b] * P + t] = v;
    }
  }
}

}  // namespace

// Cover of the triples p <= r <= s by the cells (pair, mode) that the work items write.
// A vertex v is the mode pair {2v, 2v + 1}; block (u, v), u <= v, holds the pairs of
// {2u, 2u + 1} x {2v, 2v + 1} with a <= b.  Windows: [P - 32, P) when P <= 32, else
// A = [0, 32) and B = [P - 32, P).  With L the vertices holding a mode below P - 32 and
// H those holding a mode from 32 on, the vertices are split into classes C_B = [0, k)
// (holding L) and C_A = [k, V) (holding H).  Blocks inside C_A take window A, blocks
// inside C_B window B.  A triple has two modes in one class (pigeonhole); their pair's
// window misses the third mode only when that mode lies in L (class B) or H (class A),
// i.e. in the same class, and then another pair of the triple works, unless all three
// modes are in L (or all in H).  Those triples take the blocks inside L with window A
// (inside H with window B); there the blocks of two halves suffice, since two of any
// three vertices fall in one half.  Within a single window (P <= 32) the same two
// halves cover everything.  A block in two windows writes each mode once: [zlo, zhi).
// For P = 40 this takes 122 blocks in 4 items (61 per window).
namespace {
struct BlockWin {
  int u, v, s0, zlo, zhi;
};
void add_clique(std::vector<BlockWin>& bw, int v0, int v1, int s0, int zlo, int zhi) {
  for (int v = v0; v < v1; ++v)
    for (int u = v0; u <= v; ++u) bw.push_back({u, v, s0, zlo, zhi});
}
void add_halves(std::vector<BlockWin>& bw, int v0, int v1, int s0, int zlo, int zhi) {
  const int h = v0 + (v1 - v0 + 1) / 2;
  add_clique(bw, v0, h, s0, zlo, zhi);
  add_clique(bw, h, v1, s0, zlo, zhi);
}
int clique_blocks(int n) { return n * (n + 1) / 2; }
int halves_blocks(int n) { return clique_blocks((n + 1) / 2) + clique_blocks(n / 2); }
int ceil32(int n) { return (n + BPW - 1) / BPW; }
}  // namespace

bool make_cubic_cover(int P, const std::vector<int>& pair_of, std::vector<int4>& slots, std::vector<int2>& items,
                      std::vector<int>& cell, int* mult) {
  slots.clear();
  items.clear();
  cell.clear();
  if (P < 1 || P > kMaxP) return false;
  const int V = (P + 1) / 2;
  std::vector<BlockWin> bw;
  if (P <= 32) {
    add_halves(bw, 0, V, P - 32, 0, P);
  } else {
    const int nL = (P - 31) / 2, hv = 16;   // L = [0, nL), H = [16, V)
    int best_k = nL, best = 1 << 30, best_imb = 1 << 30;
    for (int k = nL; k <= hv; ++k) {   // the class boundary with the fewest items, then the most even
      const int nA = clique_blocks(V - k) + halves_blocks(nL), nB = clique_blocks(k) + halves_blocks(V - hv);
      const int n = ceil32(nA) + ceil32(nB), imb = std::abs(nA - nB);
      if (n < best || (n == best && imb < best_imb)) {
        best = n;
        best_imb = imb;
        best_k = k;
      }
    }
    // the low and high blocks first: the item halves they open are then filled with the
    // class blocks whose vertices share no LDS bank group with them
    add_halves(bw, 0, nL, 0, 0, P - 32);
    add_clique(bw, best_k, V, 0, 0, 32);
    add_halves(bw, hv, V, P - 32, 32, P);
    add_clique(bw, 0, best_k, P - 32, P - 32, P);
  }
  // items: the blocks of one window, 32 at a time.  The map row of vertex u sits in the
  // 16-byte LDS bank group u mod 16 (even and odd rows alike, row stride 33 groups), so
  // each half item (the 16 lanes of one LDS read cycle) is filled greedily with the blocks
  // that add the fewest vertices sharing a group with a different vertex already there
  std::vector<std::vector<int>> lists;
  for (int w = 0; w < 2; ++w) {
    const int s0 = w == 0 ? std::min(0, P - 32) : P - 32;
    if (w == 1 && s0 == std::min(0, P - 32)) break;
    std::vector<int> left;
    for (int i = 0; i < (int)bw.size(); ++i)
      if (bw[i].s0 == s0) left.push_back(i);
    std::vector<int> order;
    while (!left.empty()) {
      unsigned long long seen_u = 0, seen_v = 0;   // vertices present in this half
      for (int k = 0; k < BPW / 2 && !left.empty(); ++k) {
        size_t best = 0;
        int best_cost = 1 << 30;
        for (size_t q = 0; q < left.size(); ++q) {
          const BlockWin& b = bw[left[q]];
          auto clash = [](unsigned long long seen, int x) {
            if (seen >> x & 1ull) return 0;   // the same row: one address
            for (int y = x % 16; y < 64; y += 16)
              if (seen >> y & 1ull) return 1;
            return 0;
          };
          const int cost = clash(seen_u, b.u) + clash(seen_v, b.v);
          if (cost < best_cost) {
            best_cost = cost;
            best = q;
          }
          if (cost == 0) break;
        }
        const BlockWin& b = bw[left[best]];
        seen_u |= 1ull << b.u;
        seen_v |= 1ull << b.v;
        order.push_back(left[best]);
        left.erase(left.begin() + best);
      }
    }
    for (size_t f = 0; f < order.size(); f += BPW)
      lists.emplace_back(order.begin() + f, order.begin() + std::min(order.size(), f + BPW));
  }
  // fewer than eight items: split the largest until the count divides the eight waves
  int n = (int)lists.size();
  int target = n;
  if (n <= 8) {
    target = 1;
    while (target < n) target *= 2;
  }
  while ((int)lists.size() < target) {
    size_t big = 0;
    for (size_t i = 1; i < lists.size(); ++i)
      if (lists[i].size() > lists[big].size()) big = i;
    if (lists[big].size() < 2) break;
    std::vector<int> tail(lists[big].begin() + lists[big].size() / 2, lists[big].end());
    lists[big].resize(lists[big].size() / 2);
    lists.push_back(tail);
  }
  n = (int)lists.size();
  *mult = (n <= 8 && 8 % n == 0) ? 8 / n : 1;
  for (const auto& li : lists) {
    items.push_back(make_int2((int)slots.size(), bw[li[0]].s0));
    for (int i : li) slots.push_back(make_int4(2 * bw[i].u, 2 * bw[i].v, bw[i].zlo, bw[i].zhi));
    // unused slots repeat the rows of the item's last block (one LDS address) and write nothing
    const int4 last = slots.back();
    while (slots.size() % BPW) slots.push_back(make_int4(last.x, last.y, 0, 0));
  }
  // written cells: block (u, v) -> modes, each written once
  std::vector<unsigned long long> wmask((size_t)V * V, 0ull);
  for (const auto& b : bw)
    for (int z = std::max(b.zlo, 0); z < std::min(b.zhi, P); ++z) {
      if (z < b.s0 || z >= b.s0 + 32) return false;
      unsigned long long& m = wmask[(size_t)b.u * V + b.v];
      if (m >> z & 1ull) return false;   // two items would write one cell
      m |= 1ull << z;
    }
  auto written = [&](int x, int y, int z) {
    return (wmask[(size_t)(x >> 1) * V + (y >> 1)] >> z & 1ull) != 0;
  };
  for (int p = 0; p < P; ++p)
    for (int r = p; r < P; ++r)
      for (int s = r; s < P; ++s) {
        int c = -1;
        if (written(p, r, s)) c = pair_of[(size_t)p * P + r] * P + s;
        else if (written(p, s, r)) c = pair_of[(size_t)p * P + s] * P + r;
        else if (written(r, s, p)) c = pair_of[(size_t)r * P + s] * P + p;
        if (c < 0) return false;
        cell.push_back(c);
      }
  return true;
}

namespace {
// Pixel chunks of the contraction: a multiple of 8 of them (one chunk stream per XCD), of
// about target pixels, in whole staged steps.
int chunk_px_for(const modal_ctx* c, int target) {
  int nchunk = 8 * ((c->npix + 8 * target - 1) / (8 * target));
  int px = (c->npix + nchunk - 1) / nchunk;
  px = (px + KS - 1) / KS * KS;
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

// The matrix-core contraction over the triple cover serves the split and FP32 contexts
// for every P <= kMaxP (this flag also picks their chunking); FP64 runs on the vector ALUs.
bool cubic_mfma_available(const modal_ctx* c) {
  return (c->prec == MODAL_F32 || c->prec == MODAL_BF16X3 || c->prec == MODAL_F16X3) && c->P <= kMaxP;
}

int cubic_mfma_nchunk(const modal_ctx* c) {
  const int px = chunk_px_for(c, c->tune_chunk_px > 0 ? c->tune_chunk_px : chunk_target_default(c));
  return (c->npix + px - 1) / px;
}

size_t cubic_split_lds() { return sizeof(Lds); }

hipError_t cubic_split_set_lds(size_t bytes) {
  const void* fns[] = {(const void*)k_cubic_split<MODAL_BF16X3, 1>, (const void*)k_cubic_split<MODAL_BF16X3, 2>,
                       (const void*)k_cubic_split<MODAL_BF16X3, 4>, (const void*)k_cubic_split<MODAL_BF16X3, 8>,
                       (const void*)k_cubic_split<MODAL_F16X3, 1>,  (const void*)k_cubic_split<MODAL_F16X3, 2>,
                       (const void*)k_cubic_split<MODAL_F16X3, 4>,  (const void*)k_cubic_split<MODAL_F16X3, 8>,
                       (const void*)k_cubic_split<MODAL_F32, 1>,    (const void*)k_cubic_split<MODAL_F32, 2>,
                       (const void*)k_cubic_split<MODAL_F32, 4>,    (const void*)k_cubic_split<MODAL_F32, 8>};
  for (const void* f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cubic_split(const modal_ctx* c, const void* maps, int S, int nchunk, int chunk_px, double* part,
                              hipStream_t st) {
  if (c->P > kMaxP || chunk_px % KS != 0 || (long long)nchunk * chunk_px < c->npix) return hipErrorInvalidValue;
  const int mult = c->t.cmult;
  if (mult != 1 && mult != 2 && mult != 4 && mult != 8) return hipErrorInvalidValue;
  if (mult > 1 && c->t.nitems * mult != NW) return hipErrorInvalidValue;
  const int ngroups = (c->t.nitems * mult + NW - 1) / NW;
  const int nslots = 8 * ((nchunk + 7) / 8);
  const size_t grid = (size_t)nslots * ngroups * S;
  const size_t lds = sizeof(Lds);
#define LAUNCH(PR, M)                                                                                           \
  hipLaunchKernelGGL((k_cubic_split<PR, M>), dim3(grid), dim3(NT), lds, st, c->P, c->npairs, c->npix, S, nchunk, \
                     chunk_px, c->t.ncslot, c->t.nitems, ngroups, c->t.cslot, c->t.items, c->t.pair_of,          \
                     (const float*)maps, c->t.w32, c->t.mscale, c->wscale, c->npix % 4 == 0 ? 1 : 0, part)
#define BY_MULT(PR)              \
  switch (mult) {                \
    case 1: LAUNCH(PR, 1); break; \
    case 2: LAUNCH(PR, 2); break; \
    case 4: LAUNCH(PR, 4); break; \
    default: LAUNCH(PR, 8); break; \
  }
  if (c->prec == MODAL_F16X3) BY_MULT(MODAL_F16X3) else if (c->prec == MODAL_F32) BY_MULT(MODAL_F32) else BY_MULT(MODAL_BF16X3)
#undef BY_MULT
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace modal
