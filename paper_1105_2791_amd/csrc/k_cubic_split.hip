// Cubic pixel reduction on the matrix cores with split 16-bit operands, 32x32 tiles.
//
//   E_{(ab),t} = sum_x A_ab(x) B_t(x),  A_ab = M_a M_b,  B_t = w M_t,
//
// a GEMM with M = pairs, N = modes, K = pixels (chunked; FP32 partial sums are
// reduced in FP64 by k_cubic.hip).  beta_prs = E_{(pr),s} for p <= r <= s, so only
// the modes t >= b of a pair (a, b) are needed.
//
// Tiling (v_mfma_f32_32x32x16_{bf16,f16}; lane l holds A[l % 32][8 (l / 32) + i],
// B[8 (l / 32) + i][l % 32], and accumulator register j is D[8 (j / 4) + 4 (l / 32)
// + j % 4][l % 32]):
//   * lane-row i of a wave owns a 2 x 2 block of pairs (a0, a0+1) x (b0, b0+1); the
//     four 32-row tiles of a wave are the four positions in the block, so a K step
//     reads 4 map rows per lane for 4 pair products;
//   * blocks are sorted by b0 and taken 32 at a time; a work item is such a group of
//     32 blocks with one 32-mode tile: the last 32 modes [P-32, P) always, and the
//     32 before them only when the group's smallest b0 is below P - 32 (for P = 40
//     that is one extra item; every wave runs one item);
//   * maps and the split B operand of a 128-pixel step are staged in LDS, double
//     buffered, with the next step's global loads issued before this step's MFMAs
//     (a step is long enough to cover the load latency).
// Precisions
//   BF16X3: maps staged in FP32; A = M_a M_b in FP32 split as hi = RNE bf16, lo = RNE bf16
//           of the exact residual; Ah Bh + Ah Bl + Al Bh.
//   F16X3 : maps scaled by exact powers of two (s_p ~ 1/sigma_p, s_w ~ npix/4pi) and staged
//           as fp16 pairs m = h + l (h = f16(m), l = f16(m - h)).  A pair product is formed
//           with packed fp16 arithmetic, two pixels per instruction:
//             H = h_a h_b (rounded), r = fma(h_a, h_b, -H) (exact: the residual of a 22-bit
//             product fits in fp16), L = fma(l_a, h_b, fma(h_a, l_b, r)),
//           so A = H + L carries about 21 bits (the l_a l_b term, 2^-22, is dropped): four
//           packed instructions per two products.
// For F16X3 the substeps of 16 pixels are software-pipelined: the next substep's map rows
// are read and its pair products split while this substep's MFMAs run, so that the vector
// work issues between matrix-core instructions instead of after them (8.7 -> 8.0 ms per
// 8-sky batch at l_max 1000, P 40 with the packed products; the same order made the bf16
// split, twice the vector work, 3% slower, so bf16 keeps split-then-MFMA per substep).
// The matrix core drops addend bits below the largest term of an accumulation, which
// against a long running sum biases every step; so the MFMAs accumulate a short
// chain of CHAIN staged steps from zero, and each chain joins the running FP32 sum
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
constexpr int QSTEP = kMaxP * KS / (4 * NT);   // staged pixel quads per thread per step (4)
constexpr int CHAIN = 2;           // staged steps per MFMA accumulation chain (48 MFMAs per tile)

// LDS slot of map row r: even rows first, then odd rows.  The lane-rows of a wave
// read rows a0 (even, consecutive blocks) and a0 + 1, so consecutive even rows land
// in consecutive 16-byte bank groups (row stride MSS = 17 groups).
__device__ inline int ms_slot(int r) { return (r >> 1) + (r & 1) * (kMaxP / 2); }

struct Lds {
  float ms[2][kMaxP][MSS];
  uint16_t bh[2][BROWS][BSS];
  uint16_t bl[2][BROWS][BSS];
};

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

template <int PREC>
__global__ __launch_bounds__(NT) void k_cubic_split(int P, int npairs, int npix, int S, int nchunk, int chunk_px,
                                                    int nblk, int nitems, int ngroups, const int2* __restrict__ blocks,
                                                    const int2* __restrict__ items, const int* __restrict__ pair_of,
                                                    const float* __restrict__ maps, const float* __restrict__ w,
                                                    const float* __restrict__ mscale, float wscale, int vec,
                                                    double* __restrict__ part) {
  constexpr bool F16 = PREC == MODAL_F16X3;
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
  for (int e = tid; e < 2 * BROWS * BSS; e += NT) {
    const int st = e / (BROWS * BSS), r = (e / BSS) % BROWS, xx = e % BSS;
    if (r < BROWS - P) {
      L.bh[st][r][xx] = 0;
      L.bl[st][r][xx] = 0;
    }
  }

  // this wave's work item (wave-uniform): 32 blocks from wfirst, mode tile ct
  const int item = group * NW + wv;
  const bool wave_on = item < nitems;
  int wfirst = 0, ct = 1;
  if (wave_on) {
    const int2 it = items[item];
    wfirst = __builtin_amdgcn_readfirstlane(it.x);
    ct = __builtin_amdgcn_readfirstlane(it.y);
  }
  const int myblk = wfirst + lrow;
  int a0 = 0, b0 = 0;
  if (myblk < nblk) {
    const int2 bb = blocks[myblk];
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
  const int brow = 32 * ct + lrow;   // this lane's B row (mode P - 64 + brow)

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
      if constexpr (!F16) {
        // bf16: per substep, all four tiles' operands first, then the MFMAs product by product,
        // so that consecutive MFMAs feed different accumulators (measured faster than the
        // pipelined order for bf16, whose split is twice the vector work of the fp16 one)
#pragma unroll
        for (int ks = 0; ks < KS / 16; ++ks) {
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
        load_rows(0, R0);
#pragma unroll
        for (int j = 0; j < 4; ++j) split_tile(R0, j, ah[j], al[j]);
      }
#pragma unroll
      for (int ks = 0; ks < KS / 16; ++ks) {
        const int kx = 16 * ks + 8 * kh;
        const vec8 bh = *reinterpret_cast<const vec8*>(&L.bh[st][brow][kx]);
        const vec8 bl = *reinterpret_cast<const vec8*>(&L.bl[st][brow][kx]);
        Rows Rn;
        if (ks + 1 < KS / 16) load_rows(ks + 1, Rn);
        // tile by tile: its three products, then the next substep's split of the same tile
        // into the registers they have just read (issued among the following MFMAs)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cha[j] = mfma32<PREC>(al[j], bh, cha[j]);
          cha[j] = mfma32<PREC>(ah[j], bl, cha[j]);
          cha[j] = mfma32<PREC>(ah[j], bh, cha[j]);
          if (ks + 1 < KS / 16) split_tile(Rn, j, ah[j], al[j]);
        }
      }
      }
      if (++link == CHAIN || !more) {   // wave-uniform
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
  if (!wave_on) return;

  // partial sums: acc[j][r] = E[pair j of block wfirst + 8 (r/4) + 4 kh + r % 4][mode P - 64 + brow]
  const int t = P - 64 + brow;
  double* dst = part + ((size_t)s * nchunk + chunk) * npairs * P;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ob = wfirst + 8 * (r >> 2) + 4 * kh + (r & 3);
    if (ob >= nblk) continue;
    const int2 bb = blocks[ob];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = bb.x + (j >> 1), b = bb.y + (j & 1);
      if (a >= P || b >= P || a > b || t < b) continue;   // needed modes only: t >= b (>= 0)
      double v = (double)acc[j][r];
      if (F16) v *= 1.0 / ((double)mscale[a] * (double)mscale[b] * (double)mscale[t] * (double)wscale);   // powers of two
      dst[(size_t)pair_of[a * P + b] * P + t] = v;
    }
  }
}

}  // namespace

// 2 x 2 pair blocks (a0, b0 even, a0 <= b0) sorted by b0, then a0, and the work items
// (first block of a group of 32, mode tile).
void make_pair_blocks22(int P, std::vector<int2>& blocks, std::vector<int2>& items) {
  blocks.clear();
  items.clear();
  for (int b = 0; b < P; b += 2)
    for (int a = 0; a <= b; a += 2) blocks.push_back(make_int2(a, b));
  for (int g = 0; g < (int)blocks.size(); g += BPW) {
    items.push_back(make_int2(g, 1));
    if (P - blocks[g].y > 32) items.push_back(make_int2(g, 0));
  }
}

size_t cubic_split_lds() { return sizeof(Lds); }

hipError_t cubic_split_set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)k_cubic_split<MODAL_BF16X3>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_cubic_split<MODAL_F16X3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

hipError_t launch_cubic_split(const modal_ctx* c, const void* maps, int S, int nchunk, int chunk_px, double* part,
                              hipStream_t st) {
  if (c->P > kMaxP || chunk_px % KS != 0 || (long long)nchunk * chunk_px < c->npix) return hipErrorInvalidValue;
  const int ngroups = (c->t.nitems + NW - 1) / NW;
  const int nslots = 8 * ((nchunk + 7) / 8);
  const size_t grid = (size_t)nslots * ngroups * S;
  const size_t lds = sizeof(Lds);
#define LAUNCH(PR)                                                                                              \
  hipLaunchKernelGGL((k_cubic_split<PR>), dim3(grid), dim3(NT), lds, st, c->P, c->npairs, c->npix, S, nchunk,     \
                     chunk_px, c->t.nblk, c->t.nitems, ngroups, c->t.blk, c->t.items, c->t.pair_of,               \
                     (const float*)maps, c->t.w32, c->t.mscale, c->wscale, c->npix % 4 == 0 ? 1 : 0, part)
  if (c->prec == MODAL_F16X3) LAUNCH(MODAL_F16X3);
  else LAUNCH(MODAL_BF16X3);
#undef LAUNCH
  return hipGetLastError();
}

}  // namespace modal
