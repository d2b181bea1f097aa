// Adjoint of the cubic reduction with respect to the filtered maps.
//
// For L = sum_n c_n beta^hat_n, beta^hat_prs = sum_x w (M_p M_r M_s - V_pr M_s - V_ps M_r - V_rs M_p),
//   dL/dM_u(x) = w(x) sum_{(ab)} K_{u,(ab)} (M_a M_b - V_ab)(x),
// where K_{u,(ab)} = c_{sort(u,a,b)} times the number of legs of that triple equal
// to u (each leg of the product differentiates to the other two).  The pair-mean part
// - w sum K V is linear in the state, and its image in harmonic space is a contraction
// of the state's Z with K folded by the filters (k_lin_harm.hip); so the kernels here
// form only the cubic part
//   G_u(x) = w(x) sum_{(ab)} K_{u,(ab)} M_a(x) M_b(x)
// per pixel.  G then goes through the r2c ring FFT and the adjoint Legendre
// contraction (k_fft.hip, k_fisher.hip).
#include "common.h"

namespace modal {
namespace {

__global__ void k_slot(int P, int npairs, int nmax, int S, const int* __restrict__ tri_of,
                       const int* __restrict__ tri_mult, const double* __restrict__ cot, double* __restrict__ K) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)P * npairs;
  if (i >= per * S) return;
  const size_t s = i / per, k = i - s * per;
  K[i] = cot[s * nmax + tri_of[k]] * (double)tri_mult[k];
}

constexpr int kPx = 64;
constexpr int kPc = 16;

// One workgroup: 64 pixels of SK skies (SK = 2 for float maps, 1 for double); the slot
// coefficients of each 16-pair chunk are staged in LDS once for the SK skies, so the inner
// loop reads LDS only.  Thread (px, ug) accumulates the modes u = ug + 4 i.
template <typename T, int SK>
__global__ __launch_bounds__(256) void k_pair_adjoint(int P, int npairs, int npix, int S,
                                                      const int* __restrict__ pair_a, const int* __restrict__ pair_b,
                                                      const T* __restrict__ maps, const T* __restrict__ w,
                                                      const double* __restrict__ K,
                                                      T* __restrict__ G) {
  const int s0 = blockIdx.y * SK;
  const int x0 = blockIdx.x * kPx;
  const int px = threadIdx.x & 63, ug = threadIdx.x >> 6;
  const int x = x0 + px;
  __shared__ T Mt[SK][kMaxP][kPx];
  __shared__ double Ks[SK][kMaxP][kPc];
  __shared__ int sa[kPc], sb[kPc];
  for (int e = threadIdx.x; e < SK * P * kPx; e += 256) {
    const int sk = e / (P * kPx), rem = e - sk * P * kPx, p = rem / kPx, xx = rem - p * kPx;
    const int s = s0 + sk;
    Mt[sk][p][xx] = (s < S && x0 + xx < npix) ? maps[((size_t)s * P + p) * npix + x0 + xx] : T(0);
  }
  double acc[SK][16];
#pragma unroll
  for (int sk = 0; sk < SK; ++sk)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[sk][i] = 0.0;
  for (int c0 = 0; c0 < npairs; c0 += kPc) {
    const int nc = min(kPc, npairs - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < SK * P * kPc; e += 256) {
      const int sk = e / (P * kPc), rem = e - sk * P * kPc, u = rem / kPc, pc = rem - u * kPc;
      const int s = s0 + sk;
      Ks[sk][u][pc] = (s < S && pc < nc) ? K[((size_t)s * P + u) * npairs + c0 + pc] : 0.0;
    }
    if (threadIdx.x < kPc) {
      sa[threadIdx.x] = threadIdx.x < nc ? pair_a[c0 + threadIdx.x] : 0;
      sb[threadIdx.x] = threadIdx.x < nc ? pair_b[c0 + threadIdx.x] : 0;
    }
    __syncthreads();
    if (x < npix) {
      for (int pc = 0; pc < nc; ++pc) {
        const int a = sa[pc], b = sb[pc];
#pragma unroll
        for (int sk = 0; sk < SK; ++sk) {
          const double A = (double)Mt[sk][a][px] * (double)Mt[sk][b][px];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int u = ug + 4 * i;
            if (u < P) acc[sk][i] += Ks[sk][u][pc] * A;
          }
        }
      }
    }
  }
  if (x >= npix) return;
  const double wx = (double)w[x];
#pragma unroll
  for (int sk = 0; sk < SK; ++sk) {
    const int s = s0 + sk;
    if (s >= S) break;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int u = ug + 4 * i;
      if (u < P) G[((size_t)s * P + u) * npix + x] = T(wx * acc[sk][i]);
    }
  }
}

// Float maps, P <= 48: the same contraction on the matrix cores in FP32,
//   G[u][x] = w(x) sum_pairs K[u][pair] M_a(x) M_b(x),
// a GEMM with rows = modes u (three 16-row tiles), columns = pixels, inner index = pairs,
// on v_mfma_f32_16x16x4_f32 (lane l holds A[l % 16][l / 16], B[l / 16][l % 16], and
// accumulator register r is D[4 (l / 16) + r][l % 16]).  A = K of a 64-pair chunk (FP32,
// in LDS), B = the pair product of the lane's pixel and pair, formed on the fly.  Each
// chunk is a chain of 16 MFMAs from zero, added to the running sums with a vector add.
// The S skies of one pixel block are consecutive workgroups on one XCD (workgroups are
// dealt to the 8 XCDs round-robin).
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
constexpr int kMx = 128;  // pixels per workgroup (32 per wave: two 16-column tiles)
constexpr int kMc = 64;   // pairs per staged chunk (16 MFMA steps of 4)
constexpr int kMt = 3;    // 16-mode tiles (P <= 48)

__global__ __launch_bounds__(256) void k_pair_adjoint_mfma(int P, int npairs, int npix,
                                                           const int* __restrict__ pair_a,
                                                           const int* __restrict__ pair_b,
                                                           const float* __restrict__ maps, const float* __restrict__ w,
                                                           const double* __restrict__ K, float* __restrict__ G,
                                                           int S, int nblk) {
  const int i8 = blockIdx.x >> 3;
  const int blk = (blockIdx.x & 7) + 8 * (i8 / S);
  if (blk >= nblk) return;   // whole workgroup, before any barrier
  const int s = i8 % S, x0 = blk * kMx;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int xl0 = wv * 32 + l16, xl1 = xl0 + 16;   // this lane's pixels within the block
  __shared__ float Mt[kMaxP][kMx];
  __shared__ float Ks[kMt * 16][kMc + 1];
  __shared__ int sab[kMc];        // a | b << 8 of each pair of the chunk
  const float* Ms = maps + (size_t)s * P * npix;
  for (int e = tid; e < P * kMx; e += 256) {
    const int p = e / kMx, xx = e - p * kMx;
    Mt[p][xx] = x0 + xx < npix ? Ms[(size_t)p * npix + x0 + xx] : 0.f;
  }
  f32x4 acc[2][kMt];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int t = 0; t < kMt; ++t) acc[c][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const double* Kslab = K + (size_t)s * P * npairs;
  // the next chunk's K and pair modes are loaded into registers before this chunk's
  // MFMAs, so that their latency is hidden behind them
  constexpr int NK = kMt * 16 * kMc / 256;
  double pk[NK];
  int pab = 0;
  auto load_chunk = [&](int c0) {
    const int nc = min(kMc, npairs - c0);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const int e = tid + 256 * i, u = e / kMc, pc = e - u * kMc;
      pk[i] = (u < P && pc < nc) ? Kslab[(size_t)u * npairs + c0 + pc] : 0.0;
    }
    if (tid < kMc) pab = tid < nc ? (pair_a[c0 + tid] | (pair_b[c0 + tid] << 8)) : 0;
  };
  load_chunk(0);
  for (int c0 = 0; c0 < npairs; c0 += kMc) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const int e = tid + 256 * i, u = e / kMc, pc = e - u * kMc;
      Ks[u][pc] = (float)pk[i];
    }
    if (tid < kMc) sab[tid] = pab;
    __syncthreads();
    if (c0 + kMc < npairs) load_chunk(c0 + kMc);
    // pairs past nc have zero K columns: whatever their product is contributes nothing
    f32x4 ch[2][kMt];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int t = 0; t < kMt; ++t) ch[c][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int ks = 0; ks < kMc / 4; ++ks) {
      const int pc = 4 * ks + kq;
      const int ab = sab[pc], a = ab & 0xff, b2 = (ab >> 8) & 0xff;
      const float b0 = Mt[a][xl0] * Mt[b2][xl0], b1 = Mt[a][xl1] * Mt[b2][xl1];
#pragma unroll
      for (int t = 0; t < kMt; ++t) {
        const float av = Ks[16 * t + l16][pc];
        ch[0][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b0, ch[0][t], 0, 0, 0);
        ch[1][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b1, ch[1][t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int t = 0; t < kMt; ++t) acc[c][t] += ch[c][t];
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int x = x0 + (c ? xl1 : xl0);
    if (x >= npix) continue;
    const float wx = w[x];
#pragma unroll
    for (int t = 0; t < kMt; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int u = 16 * t + 4 * kq + r;
        if (u < P) G[((size_t)s * P + u) * npix + x] = wx * acc[c][t][r];
      }
  }
}

// Split-precision contexts, P <= 48: the cubic part on the fp16 matrix cores with split
// operands,
//   G[u][x] = w(x) 2^E sum_k A[u][k] B[k][x],  A = 2^-E K[u][(ab)] / (s_a s_b),  B = (s_a M_a)(s_b M_b),
// with s_p the context's power-of-two map scales (~ 1/sigma_p) and 2^-E a power of two per sky
// that puts max |A| near 2^14, so both operands sit well inside the fp16 range and every
// scaling is exact.  On v_mfma_f32_32x32x16_f16 (lane l holds A[l % 32][8 (l / 32) + i],
// B[8 (l / 32) + i][l % 32]; accumulator register j is D[8 (j / 4) + 4 (l / 32) + j % 4][l % 32]):
// rows = modes (one or two 32-row tiles), columns = pixels, inner index = pairs.
//   A = Ah + Al: fp16 hi and lo of the FP32 value, split once per sky;
//   the scaled maps are held as fp16 pairs m = h + l (h = f16(m), l = f16(m - h)), and a pair
//   product is formed with packed fp16 arithmetic, two pairs per instruction:
//     H = h_a h_b (rounded), r = fma(h_a, h_b, -H) (exact: the residual of a 22-bit product fits
//     in fp16), L = fma(l_a, h_b, fma(h_a, l_b, r)),
//   so B = H + L carries about 21 bits (the l_a l_b term, 2^-22, is dropped);
//   each product is Ah H + Ah L + Al H.
// The inner index runs over 8-pair groups (a, b = B0 .. B0 + 7), B0 a multiple of 8 with
// B0 >= 8 floor(a / 8): a lane reads h_a, l_a and the eight h_b, l_b of its pixel from the map
// row in LDS (two 2-byte and two 16-byte reads), and the slots with b < a or b >= P carry A = 0
// (for P = 40: 960 slots for 820 pairs).  An MFMA K step of 16 takes groups 2t (lanes 0-31)
// and 2t + 1 (lanes 32-63); the map reads and products of step t + 1 are issued among the
// MFMAs of step t (software pipeline).  The A operands of SG_KC steps are staged in LDS, double
// buffered; the MFMAs of SG_CH staged chunks accumulate from zero into a chain that is then
// added to the running FP32 sums (the matrix core truncates the addend of a long accumulation).
// A workgroup is 4 waves and 256 pixels of one sky (70 KB of LDS: two workgroups per CU).
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(2 * sizeof(_Float16)))) _Float16 f16x2;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
constexpr int SG_NW = 4;               // waves per workgroup (two workgroups per CU)
constexpr int SG_PX = 64 * SG_NW;      // pixels per workgroup: two 32-column tiles per wave
constexpr int SG_PP = 48;              // modes held per map row (P <= 48; rows zero past P)
constexpr int SG_MS = 2 * SG_PP + 8;   // map row stride in halves: hi words, lo words, pad (208 B)
constexpr int SG_KC = 2;               // K steps per staged chunk
constexpr int SG_CH = 4;               // staged chunks per accumulation chain
constexpr int SG_GC = 2 * SG_KC;       // 8-pair groups per chunk
constexpr int SG_MAXG = 176;           // groups for P = 48 (168), padded to a whole chunk
constexpr int SG_EMAX = 14;            // max |A| is scaled to about 2^SG_EMAX

// number of 8-pair groups of P modes (before padding to whole chunks)
__host__ __device__ inline int sg_groups(int P) {
  int n = 0;
  for (int a = 0; a < P; ++a) n += (P + 7) / 8 - a / 8;
  return n;
}

// fp16 hi/lo words of two values (packed low half first); each split starts from one
// rounded FP32 value
__device__ inline void sg_split2(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  asm("" : "+v"(v0), "+v"(v1));
  const _Float16 h0 = (_Float16)v0, h1 = (_Float16)v1;
  const _Float16 r0 = (_Float16)(v0 - (float)h0), r1 = (_Float16)(v1 - (float)h1);
  hi = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
  lo = (uint32_t)__builtin_bit_cast(uint16_t, r0) | ((uint32_t)__builtin_bit_cast(uint16_t, r1) << 16);
}

// Per sky: the power of two 2^-E with max_{u, (ab)} |K[u][(ab)]| / (s_a s_b) * 2^-E in
// [2^(SG_EMAX - 1), 2^SG_EMAX) (1 when K is zero).  sc[s] = {2^-E, 2^E}.
__global__ __launch_bounds__(256) void k_adj_kscale(int P, int npairs, const int* __restrict__ pair_a,
                                                    const int* __restrict__ pair_b, const float* __restrict__ mscale,
                                                    const double* __restrict__ K, float2* __restrict__ sc) {
  const int s = blockIdx.x;
  __shared__ double red[256];
  double mx = 0.0;
  for (int e = threadIdx.x; e < P * npairs; e += 256) {
    const int k = e % npairs;
    mx = fmax(mx, fabs(K[(size_t)s * P * npairs + e]) / ((double)mscale[pair_a[k]] * (double)mscale[pair_b[k]]));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e = 0;
    if (red[0] > 0.0) {
      frexp(red[0], &e);   // red[0] in [2^(e-1), 2^e)
      e = min(max(e - SG_EMAX, -120), 120);   // both scales stay finite floats
    }
    sc[s] = make_float2(ldexpf(1.f, -e), ldexpf(1.f, e));
  }
}

// A operands: Ks[s][g][0 = hi, 1 = lo][mode 0..63][8 fp16] for the padded groups, and the
// group table grp[g] = a | B0 << 8.  One thread per (s, g, mode).
__global__ __launch_bounds__(64) void k_adj_ksplit(int P, int npairs, int ng, const int* __restrict__ pair_of,
                                                   const float* __restrict__ mscale, const float2* __restrict__ sc,
                                                   const double* __restrict__ K, u32x4* __restrict__ Ks,
                                                   int* __restrict__ grp) {
  const int u = threadIdx.x, g = blockIdx.x, s = blockIdx.y;
  int a = 0, r = g, B0 = 0;
  const int nb8 = (P + 7) / 8;
  if (g < ng) {
    while (r >= nb8 - a / 8) r -= nb8 - a / 8, ++a;
    B0 = 8 * (a / 8 + r);
  }
  if (s == 0 && u == 0) grp[g] = a | (B0 << 8);
  const double f = (double)sc[s].x / (double)mscale[a];
  float v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int b = B0 + i;
    v[i] = (g < ng && u < P && b >= a && b < P)
               ? (float)(K[((size_t)s * P + u) * npairs + pair_of[a * P + b]] * f / (double)mscale[b])
               : 0.f;
  }
  u32x4 hi, lo;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t h, l;
    sg_split2(v[2 * k], v[2 * k + 1], h, l);
    hi[k] = h;
    lo[k] = l;
  }
  u32x4* o = Ks + ((size_t)s * gridDim.x + g) * 2 * 64;
  o[u] = hi;
  o[64 + u] = lo;
}

struct SgLds {
  uint16_t ms[SG_PX][SG_MS];   // per pixel: fp16 hi of the scaled maps [0, 48), lo [48, 96)
  u32x4 a[2][SG_GC][2][64];    // [buffer][group][hi, lo][mode]
  int grp[SG_MAXG];
  float msc[SG_PP];            // map scales, zero past P
};

template <int MT>
__global__ __launch_bounds__(64 * SG_NW) void k_pair_adjoint_split(int P, int npix, int ngp,
                                                                     const int* __restrict__ grp,
                                                                     const float* __restrict__ maps,
                                                                     const float* __restrict__ w,
                                                                     const float* __restrict__ mscale,
                                                                     const float2* __restrict__ sc,
                                                                     const u32x4* __restrict__ Ks,
                                                                     float* __restrict__ G) {
  __shared__ SgLds L;
  const int s = blockIdx.y, x0 = blockIdx.x * SG_PX;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int c = lane & 31, h = lane >> 5;
  const float* Ms = maps + (size_t)s * P * npix;
  // the scaled maps as fp16 pairs: thread (xx = tid, modes 2i, 2i + 1), coalesced along pixels.
  // All loads are issued before the first is used: one round trip instead of 24.
  {
    constexpr int NS = SG_PP / 2;
    const int xx = tid;
    const bool in = x0 + xx < npix;
    const float* col = Ms + x0 + min(xx, npix - 1 - x0);
    float m[2 * NS];
#pragma unroll
    for (int i = 0; i < 2 * NS; ++i) m[i] = col[(size_t)min(i, P - 1) * npix];   // valid for every i and lane
    if (tid < SG_PP) L.msc[tid] = tid < P ? mscale[tid] : 0.f;
    for (int e = tid; e < ngp; e += 64 * SG_NW) L.grp[e] = grp[e];
    __syncthreads();
    // the scale (zero past P and past the last pixel) multiplies: a select of the loaded
    // value would let the compiler branch around each load
#pragma unroll
    for (int i = 0; i < 2 * NS; ++i) m[i] *= in ? L.msc[i] : 0.f;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int p = 2 * i;
      uint32_t hw, lw;
      sg_split2(m[p], m[p + 1], hw, lw);
      *reinterpret_cast<uint32_t*>(&L.ms[xx][p]) = hw;
      *reinterpret_cast<uint32_t*>(&L.ms[xx][SG_PP + p]) = lw;
    }
  }
  const u32x4* Kslab = Ks + (size_t)s * ngp * 2 * 64;
  constexpr int NL = SG_GC * 2 * 64 / (64 * SG_NW);   // 16-byte operand words per thread per chunk
  const int nch = ngp / SG_GC;
  u32x4 pre[NL];
  auto load_chunk = [&](int ch) {   // a valid chunk for every ch (clamped); used only when ch < nch
#pragma unroll
    for (int i = 0; i < NL; ++i) pre[i] = Kslab[(size_t)min(ch, nch - 1) * SG_GC * 2 * 64 + tid + 64 * SG_NW * i];
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = tid + 64 * SG_NW * i;
      L.a[buf][e >> 7][(e >> 6) & 1][e & 63] = pre[i];
    }
  };
  f32x16 acc[MT][2], cc[MT][2];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[mt][ct][j] = cc[mt][ct][j] = 0.f;
  const uint16_t* row[2] = {L.ms[wv * 64 + c], L.ms[wv * 64 + 32 + c]};   // this lane's pixel of each tile
  // The lane's map words of K step t (group 2t + h: a, B0) for both pixel tiles, and the
  // fp16 hi/lo pair products formed from them.
  struct Maps {
    uint32_t ha[2], la[2];
    u32x4 hb[2], lb[2];
  };
  const int nk = ngp / 2;
  auto read_maps = [&](int t, Maps& R) {
    const int gv = L.grp[2 * t + h];
    const int a = gv & 0xff, B0 = gv >> 8;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      R.ha[ct] = row[ct][a];
      R.la[ct] = row[ct][SG_PP + a];
      R.hb[ct] = *reinterpret_cast<const u32x4*>(row[ct] + B0);
      R.lb[ct] = *reinterpret_cast<const u32x4*>(row[ct] + SG_PP + B0);
    }
  };
  auto make_b = [&](const Maps& R, int ct, f16x8& bh, f16x8& bl) {
    const uint32_t ha = R.ha[ct], la = R.la[ct];
    const f16x2 xa = __builtin_bit_cast(f16x2, ha | (ha << 16)), ya = __builtin_bit_cast(f16x2, la | (la << 16));
    u32x4 H4, L4;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // vector elements go through scalars first: a bit_cast of the element itself is
      // dropped by the compiler
      const uint32_t wb = R.hb[ct][k], vb = R.lb[ct][k];
      const f16x2 xb = __builtin_bit_cast(f16x2, wb), yb = __builtin_bit_cast(f16x2, vb);
      f16x2 Hh = xa * xb;
      uint32_t Hb = __builtin_bit_cast(uint32_t, Hh);
      asm("" : "+v"(Hb));   // H is one rounded product, used as is below
      Hh = __builtin_bit_cast(f16x2, Hb);
      f16x2 r = __builtin_elementwise_fma(xa, xb, -Hh);
      r = __builtin_elementwise_fma(xa, yb, r);
      r = __builtin_elementwise_fma(ya, xb, r);
      H4[k] = Hb;
      L4[k] = __builtin_bit_cast(uint32_t, r);
    }
    bh = __builtin_bit_cast(f16x8, H4);
    bl = __builtin_bit_cast(f16x8, L4);
  };
  auto read_a = [&](int t, f16x8* ah, f16x8* al) {
    const int buf = (t / SG_KC) & 1, gl = 2 * (t % SG_KC) + h;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      ah[mt] = __builtin_bit_cast(f16x8, L.a[buf][gl][0][32 * mt + c]);
      al[mt] = __builtin_bit_cast(f16x8, L.a[buf][gl][1][32 * mt + c]);
    }
  };
  // Software pipeline: the A operands, map words and pair products of step t + 1 are read
  // and formed among the MFMAs of step t (for the last step, those of the last step again,
  // unused).  A chunks: chunks 0 and 1 are staged before the loop; in chunk ch, a barrier
  // before its last step (all waves are then past their reads of chunk ch's operands, and
  // chunk ch + 1 is visible) is followed by the store of chunk ch + 2 into chunk ch's buffer.
  load_chunk(0);
  store_chunk(0);
  load_chunk(1);
  store_chunk(1);
  load_chunk(2);
  __syncthreads();   // maps, group table, chunks 0 and 1
  f16x8 bh[2], bl[2], ah[MT], al[MT];
  {
    Maps R0;
    read_maps(0, R0);
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) make_b(R0, ct, bh[ct], bl[ct]);
    read_a(0, ah, al);
  }
  auto chunk = [&](int ch) {
#pragma unroll
    for (int kk = 0; kk < SG_KC; ++kk) {
      const int t = ch * SG_KC + kk;
      const int tn = min(t + 1, nk - 1);
      if (kk == SG_KC - 1) {
        __syncthreads();
        if (ch + 2 < nch) store_chunk(ch & 1);
        load_chunk(ch + 3);
      }
      Maps Rn;
      read_maps(tn, Rn);
      f16x8 ahn[MT], aln[MT];
      read_a(tn, ahn, aln);
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          cc[mt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[mt], bh[ct], cc[mt][ct], 0, 0, 0);
          cc[mt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[mt], bl[ct], cc[mt][ct], 0, 0, 0);
          cc[mt][ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[mt], bh[ct], cc[mt][ct], 0, 0, 0);
        }
        make_b(Rn, ct, bh[ct], bl[ct]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        ah[mt] = ahn[mt];
        al[mt] = aln[mt];
      }
    }
  };
  // chains of SG_CH staged chunks join the running sums
  for (int ch0 = 0; ch0 < nch; ch0 += SG_CH) {
#pragma unroll
    for (int j = 0; j < SG_CH; ++j)
      if (ch0 + j < nch) chunk(ch0 + j);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        acc[mt][ct] += cc[mt][ct];
#pragma unroll
        for (int j = 0; j < 16; ++j) cc[mt][ct][j] = 0.f;
      }
  }
  const float up = sc[s].y;   // 2^E
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    const int x = x0 + wv * 64 + 32 * ct + c;
    if (x >= npix) continue;
    const float wx = w[x];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int u = 32 * mt + 8 * (j / 4) + 4 * h + j % 4;
        if (u < P) G[((size_t)s * P + u) * npix + x] = (wx * acc[mt][ct][j]) * up;
      }
  }
}

}  // namespace

hipError_t launch_slot_matrix(const modal_ctx* c, const double* cot, int S, void* K, hipStream_t st) {
  const size_t tot = (size_t)c->P * c->npairs * S;
  hipLaunchKernelGGL(k_slot, dim3((tot + 255) / 256), dim3(256), 0, st, c->P, c->npairs, c->nmax, S, c->t.tri_of,
                     c->t.tri_mult, cot, (double*)K);
  return hipGetLastError();
}

static bool split_adjoint(const modal_ctx* c) {
  return (c->prec == MODAL_BF16X3 || c->prec == MODAL_F16X3) && c->P <= SG_PP;
}

size_t pair_adjoint_ws_bytes(const modal_ctx* c, int S) {
  return split_adjoint(c) ? (size_t)S * SG_MAXG * 2 * 64 * 16 + SG_MAXG * 4 + (size_t)S * 8 : 0;
}

hipError_t launch_pair_adjoint(const modal_ctx* c, const void* maps, const void* K, int S, void* G, void* ws,
                               hipStream_t st) {
  if (split_adjoint(c)) {
    const int ng = sg_groups(c->P), ngp = (ng + SG_GC - 1) / SG_GC * SG_GC;
    u32x4* Ks = (u32x4*)ws;
    int* grp = (int*)((char*)ws + (size_t)S * SG_MAXG * 2 * 64 * 16);
    float2* sc = (float2*)(grp + SG_MAXG);
    hipLaunchKernelGGL(k_adj_kscale, dim3(S), dim3(256), 0, st, c->P, c->npairs, c->t.pair_a, c->t.pair_b,
                       c->t.mscale, (const double*)K, sc);
    hipLaunchKernelGGL(k_adj_ksplit, dim3(ngp, S), dim3(64), 0, st, c->P, c->npairs, ng, c->t.pair_of, c->t.mscale,
                       sc, (const double*)K, Ks, grp);
    const dim3 grid((c->npix + SG_PX - 1) / SG_PX, S);
    if (c->P <= 32)
      hipLaunchKernelGGL(k_pair_adjoint_split<1>, grid, dim3(64 * SG_NW), 0, st, c->P, c->npix, ngp, grp,
                         (const float*)maps, c->t.w32, c->t.mscale, sc, Ks, (float*)G);
    else
      hipLaunchKernelGGL(k_pair_adjoint_split<2>, grid, dim3(64 * SG_NW), 0, st, c->P, c->npix, ngp, grp,
                         (const float*)maps, c->t.w32, c->t.mscale, sc, Ks, (float*)G);
    return hipGetLastError();
  }
  if (is_f64(c)) {
    hipLaunchKernelGGL((k_pair_adjoint<double, 1>), dim3((c->npix + kPx - 1) / kPx, S), dim3(256), 0, st, c->P,
                       c->npairs, c->npix, S, c->t.pair_a, c->t.pair_b, (const double*)maps, c->t.w64,
                       (const double*)K, (double*)G);
  } else if (c->P <= kMt * 16) {
    const int nblk = (c->npix + kMx - 1) / kMx;
    hipLaunchKernelGGL(k_pair_adjoint_mfma, dim3(8 * ((nblk + 7) / 8) * S), dim3(256), 0, st, c->P, c->npairs,
                       c->npix, c->t.pair_a, c->t.pair_b, (const float*)maps, c->t.w32, (const double*)K, (float*)G,
                       S, nblk);
  } else {
    hipLaunchKernelGGL((k_pair_adjoint<float, 2>), dim3((c->npix + kPx - 1) / kPx, (S + 1) / 2), dim3(256), 0, st,
                       c->P, c->npairs, c->npix, S, c->t.pair_a, c->t.pair_b, (const float*)maps, c->t.w32,
                       (const double*)K, (float*)G);
  }
  return hipGetLastError();
}

}  // namespace modal
