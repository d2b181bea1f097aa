// Modal trispectrum (Sec. IV): for separable modes q_p q_r q_s q_u, p <= r <= s <= u,
//   tau_prsu = sum_x w [M_p M_r M_s M_u - (6 pairs) V_ab M_c M_d + (3 pairings) V_ab V_cd].
// Rearranged exactly as a symmetric rank-npix update over the pairs:
//   K_(ab),(cd) = sum_x w A_ab A_cd - 6 sum_x w V_ab V_cd,   A_ab = M_a M_b - 3 V_ab,
//   tau_prsu = (K_(pr),(su) + K_(ps),(ru) + K_(pu),(rs)) / 3,
// since the three pairings of A A expand to 3 MMMM - 3 (6 pairs) V M M + 9 (3 pairings) V V.
// Without a linear-term state V = 0.  The V V term is sky-independent and computed once
// per call by the same kernels with A = V.
//
// The update is a pairs x pairs SYRK with K = pixels.  Operands sqrt(w) A are formed on
// the fly (w >= 0 splits evenly over both sides), never stored in HBM:
//   * float maps (bf16x3 / f16x3 / f32 contexts): split-bf16 MFMA 32x32x16 with three
//     products, 128 x 128 output tiles, two skies per workgroup (one per half, 64 x 64
//     per wave), operands of a 32-pixel step formed once per half into LDS (each thread
//     4 pixels of 8 operand rows), maps and pair means read from pixel-block-major copies
//     (k_quad_vtile), FP32 chains of CH steps joined in FP32, FP32 partial sums per pixel
//     chunk reduced in FP64;
//   * double maps (f64 contexts): FP64 on the vector ALUs, 64 x 64 tiles, 4 x 4 per thread.
#include "common.h"

#include <algorithm>

namespace modal {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;

constexpr int TT = 128;      // output tile of the MFMA kernel (rows = cols)
constexpr int PXS = 32;      // pixels per staged step (two MFMA K = 16 steps)
constexpr int OPS = PXS;     // operand row stride in LDS (bf16; 16-byte fragments stay aligned)
constexpr int MPS = PXS + 4; // map row stride in LDS (floats; rows stay 16-byte aligned)
constexpr int CH = 16;       // staged steps per MFMA accumulation chain (96 MFMAs per tile)
constexpr int GPR = PXS / 4; // 4-pixel groups per row
constexpr int RPT = 2 * TT * GPR / 256;   // operand rows per thread (8)
constexpr int SKW = 2;       // skies per workgroup, one per half: the pair means are loaded once
constexpr int NTQ = 256 * SKW;

struct TriLds {
  float ms[SKW][kMaxP][MPS];
  float4 vs[RPT][256];     // pair means of thread t's rows and pixels (read by t of both halves)
  float4 sw[256];          // sqrt(w) of thread t's 4 pixels
  uint16_t oh[SKW][2 * TT][OPS];
  uint16_t ol[SKW][2 * TT][OPS];
};

__device__ inline uint32_t bf16_pair(float a, float b) {
  typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
  bf16x2 h;
  h[0] = (__bf16)a;
  h[1] = (__bf16)b;
  return __builtin_bit_cast(uint32_t, h);
}

// hi = RNE bf16(v), lo = RNE bf16(v - hi) of two values, packed
__device__ inline void split2(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  asm("" : "+v"(v0), "+v"(v1));
  hi = bf16_pair(v0, v1);
  lo = bf16_pair(v0 - __builtin_bit_cast(float, hi << 16), v1 - __builtin_bit_cast(float, hi & 0xffff0000u));
}

// Tile pair (ti, tj), ti <= tj, of the R x R result, pixel chunk c, skies SKW z + h for the
// two halves h of the workgroup (vmode: operands are the pair means themselves, one
// "sky").  part[s][c][tp][TT][TT] FP32 sums of the chunk.
// Thread t of a half forms the operands of the 4 pixels 4 (t % 8) .. + 3 of the rows
// t / 8 + 32 j, j < 8 (rows 0..127 of tile ti, then 128..255 of tile tj): its pair-mean and
// weight loads are float4 and coalesced along each row, its map reads and operand writes
// are 16- and 8-byte LDS accesses.  The pair means of a step are the same for both skies:
// half h loads the rows j = 4 h .. 4 h + 3 and both halves read all eight, so each pair
// mean is read from HBM once per two skies.  V and the maps are pixel-block-major copies
// made by k_quad_vtile, so the rows of a step are contiguous runs.
__global__ __launch_bounds__(NTQ) __attribute__((amdgpu_waves_per_eu(2))) void k_quad_syrk(int P, int R, int npix, int S, int nchunk, int chunk_px, int ntp,
                                                   const int2* __restrict__ tpairs, const int* __restrict__ pair_a,
                                                   const int* __restrict__ pair_b, const float* __restrict__ maps,
                                                   const float* __restrict__ V, const float* __restrict__ w,
                                                   int vmode, int vec, float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char traw[];
  TriLds& L = *reinterpret_cast<TriLds*>(traw);
  const int tp = blockIdx.x, chunk = blockIdx.y;
  const int2 tt = tpairs[tp];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int h = tid >> 8, t = tid & 255;           // sky half, thread within the half
  const int s = SKW * blockIdx.z + h;
  const bool skyok = s < S;                        // uniform over the half's four waves
  const int wq = wv & 3, wi = wq >> 1, wj = wq & 1;
  const int g = t & (GPR - 1), rsub = t / GPR;
  // this thread's operand rows r = rsub + 32 j (j < 4 in tile ti, j >= 4 in tile tj):
  // pair index rowp(j); its two modes, 8 bits each, packed two rows to a word
  const int rb0 = tt.x * TT + rsub, rb1 = tt.y * TT + rsub - TT;
  auto rowp = [&](int j) { return (j < RPT / 2 ? rb0 : rb1) + 32 * j; };
  uint32_t pab[RPT / 2] = {};
  unsigned rokm = 0;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int orow = rowp(j);
    const bool ok = orow < R;
    const uint32_t ab = ok ? (uint32_t)(pair_a[orow] | (pair_b[orow] << 8)) : 0u;
    pab[j >> 1] |= ab << (16 * (j & 1));
    rokm |= ok ? (1u << j) : 0u;
  }
  const bool hasV = V != nullptr;   // no state: V = 0 (never read); vmode always has V
  const int nblk = (npix + PXS - 1) / PXS;
  const float* Msky = maps + (size_t)min(s, S - 1) * nblk * P * PXS;   // block-major copy of the maps
  const int x0 = chunk * chunk_px, x1 = min(npix, x0 + chunk_px);

  f32x16 acc[2][2], cha[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = cha[a][b][r] = 0.f;
  int link = 0;
  // Staging in 4-pixel groups (float4; npix % 4 == 0 and 32-pixel chunk starts keep a
  // group wholly inside or wholly past the chunk end).  The next step's loads are issued
  // into registers before this step's operand formation and MFMAs, so their latency is
  // hidden behind that work.
  constexpr int NML = (kMaxP * GPR + 255) / 256;        // map groups per thread (2)
  constexpr int RPH = RPT / SKW;                        // pair-mean rows loaded per thread (4)
  float4 pv[RPH], pm[NML], pw;
  auto load_step = [&](int xs) {
#pragma unroll
    for (int k = 0; k < NML; ++k) {
      const int e = t + 256 * k, r = e / GPR, gg = e - r * GPR, x = xs + 4 * gg;
      pm[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (!vmode && skyok && r < P && x < x1)
        pm[k] = *reinterpret_cast<const float4*>(Msky + ((size_t)(x >> 5) * P + r) * PXS + (x & 31));
    }
    const int x = xs + 4 * g;
#pragma unroll
    for (int jj = 0; jj < RPH; ++jj) {
      const int j = RPH * h + jj;
      pv[jj] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (hasV && x < x1 && ((rokm >> j) & 1u))
        pv[jj] = *reinterpret_cast<const float4*>(V + ((size_t)(x >> 5) * R + rowp(j)) * PXS + (x & 31));
    }
    pw = make_float4(0.f, 0.f, 0.f, 0.f);
    if (h == 0 && x < x1) pw = *reinterpret_cast<const float4*>(w + x);
  };
  auto store_step = [&]() {
#pragma unroll
    for (int k = 0; k < NML; ++k) {
      const int e = t + 256 * k, r = e / GPR, gg = e - r * GPR;
      if (r < kMaxP) *reinterpret_cast<float4*>(&L.ms[h][r][4 * gg]) = pm[k];
    }
#pragma unroll
    for (int jj = 0; jj < RPH; ++jj) L.vs[RPH * h + jj][t] = pv[jj];
    if (h == 0) L.sw[t] = make_float4(sqrtf(pw.x), sqrtf(pw.y), sqrtf(pw.z), sqrtf(pw.w));
  };
  // element-wise staging (npix % 4 != 0): the same layout, scalar loads
  auto stage_scalar = [&](int xs) {
    if (!vmode)
      for (int e = t; e < P * PXS; e += 256) {
        const int r = e / PXS, i = e - r * PXS, x = xs + i;
        L.ms[h][r][i] = (skyok && x < x1) ? Msky[((size_t)(x >> 5) * P + r) * PXS + (x & 31)] : 0.f;
      }
    float q[4], sq[4];
#pragma unroll
    for (int jj = 0; jj < RPH; ++jj) {
      const int j = RPH * h + jj;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int x = xs + 4 * g + k;
        q[k] = (hasV && x < x1 && ((rokm >> j) & 1u)) ? V[((size_t)(x >> 5) * R + rowp(j)) * PXS + (x & 31)] : 0.f;
      }
      L.vs[j][t] = make_float4(q[0], q[1], q[2], q[3]);
    }
    if (h == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int x = xs + 4 * g + k;
        sq[k] = x < x1 ? sqrtf(w[x]) : 0.f;
      }
      L.sw[t] = make_float4(sq[0], sq[1], sq[2], sq[3]);
    }
  };
  if (vec) load_step(x0);
  for (int xs = x0; xs < x1; xs += PXS) {
    __syncthreads();
    if (vec) store_step();
    else stage_scalar(xs);
    __syncthreads();
    if (vec && xs + PXS < x1) load_step(xs + PXS);
    // operands sqrt(w) (M_a M_b - 3 V_ab), or sqrt(w) V_ab, split hi/lo, 4 pixels x 8 rows
    if (skyok) {
      const float4 sq = L.sw[t];
#pragma unroll
      for (int j = 0; j < RPT; ++j) {
        const int r = rsub + 32 * j;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if ((rokm >> j) & 1u) {
          const float4 vv = hasV ? L.vs[j][t] : make_float4(0.f, 0.f, 0.f, 0.f);
          if (vmode) {
            v = vv;
          } else {
            const uint32_t ab = pab[j >> 1] >> (16 * (j & 1));
            const float4 ma = *reinterpret_cast<const float4*>(&L.ms[h][ab & 0xff][4 * g]);
            const float4 mb = *reinterpret_cast<const float4*>(&L.ms[h][(ab >> 8) & 0xff][4 * g]);
            v.x = fmaf(ma.x, mb.x, -3.f * vv.x);
            v.y = fmaf(ma.y, mb.y, -3.f * vv.y);
            v.z = fmaf(ma.z, mb.z, -3.f * vv.z);
            v.w = fmaf(ma.w, mb.w, -3.f * vv.w);
          }
          v.x *= sq.x;
          v.y *= sq.y;
          v.z *= sq.z;
          v.w *= sq.w;
        }
        uint32_t h0, l0, h1, l1;
        split2(v.x, v.y, h0, l0);
        split2(v.z, v.w, h1, l1);
        *reinterpret_cast<uint2*>(&L.oh[h][r][4 * g]) = make_uint2(h0, h1);
        *reinterpret_cast<uint2*>(&L.ol[h][r][4 * g]) = make_uint2(l0, l1);
        if (j & 1) __builtin_amdgcn_sched_barrier(0);   // two rows in flight at a time (registers)
      }
    }
    __syncthreads();
    if (skyok) {
#pragma unroll
      for (int ks = 0; ks < PXS / 16; ++ks) {
        const int kx = 16 * ks + 8 * (lane >> 5);
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int ra = 64 * wi + 32 * u + (lane & 31);
          const int rb = TT + 64 * wj + 32 * u + (lane & 31);
          ah[u] = *reinterpret_cast<const bf16x8*>(&L.oh[h][ra][kx]);
          al[u] = *reinterpret_cast<const bf16x8*>(&L.ol[h][ra][kx]);
          bh[u] = *reinterpret_cast<const bf16x8*>(&L.oh[h][rb][kx]);
          bl[u] = *reinterpret_cast<const bf16x8*>(&L.ol[h][rb][kx]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) cha[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], cha[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) cha[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], cha[a][b], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) cha[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], cha[a][b], 0, 0, 0);
      }
      if (++link == CH || xs + PXS >= x1) {   // uniform
        link = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acc[a][b] += cha[a][b];
#pragma unroll
            for (int r = 0; r < 16; ++r) cha[a][b][r] = 0.f;
          }
      }
    }
  }
  if (!skyok) return;
  // acc[a][b][r] = D[64 wi + 32 a + 8 (r / 4) + 4 (lane / 32) + r % 4][64 wj + 32 b + lane % 32]
  float* dst = part + (((size_t)s * nchunk + chunk) * ntp + tp) * TT * TT;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 64 * wi + 32 * a + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int j = 64 * wj + 32 * b + (lane & 31);
        dst[i * TT + j] = acc[a][b][r];
      }
}

// Pixel-block-major copy of the pair means: Vt[b][pair][i] = V[pair][32 b + i] (zero past
// npix).  The update reads, per 32-pixel step, 256 rows of one block: contiguous here,
// 256 separate 128-byte pieces of the pair-major planes otherwise.  A workgroup copies
// 32 rows x 8 blocks; each row is read as 1 KB runs, each block written as 4 KB runs.
__global__ __launch_bounds__(256) void k_quad_vtile(int R, int npix, int nblk, int vec, const float* __restrict__ V,
                                                    float* __restrict__ Vt) {
  const int row = blockIdx.y * 32 + (threadIdx.x >> 3), g = threadIdx.x & 7;
  if (row >= R) return;
  V += (size_t)blockIdx.z * R * npix;   // batch z: R rows of npix -> nblk blocks of R x 32
  Vt += (size_t)blockIdx.z * nblk * R * PXS;
  const float* src = V + (size_t)row * npix;
#pragma unroll
  for (int b8 = 0; b8 < 8; ++b8) {
    const int blk = blockIdx.x * 8 + b8;
    if (blk >= nblk) break;
    const int x = blk * PXS + 4 * g;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (vec && x < npix) {
      v = *reinterpret_cast<const float4*>(src + x);   // npix % 4 == 0: the group is inside
    } else if (!vec) {
      v.x = x < npix ? src[x] : 0.f;
      v.y = x + 1 < npix ? src[x + 1] : 0.f;
      v.z = x + 2 < npix ? src[x + 2] : 0.f;
      v.w = x + 3 < npix ? src[x + 3] : 0.f;
    }
    *reinterpret_cast<float4*>(Vt + ((size_t)blk * R + row) * PXS + 4 * g) = v;
  }
}

// K[s][i][j] (i, j < R, FP64, both triangles) = sum over chunks of the tile partials.
__global__ __launch_bounds__(256) void k_quad_reduce(int R, int nchunk, int ntp, int ntile, const float* __restrict__ part,
                                                     double* __restrict__ K) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  if (e >= (size_t)R * R) return;
  const int i = (int)(e / R), j = (int)(e - (size_t)i * R);
  int ti = i / TT, tj = j / TT, ii = i - ti * TT, jj = j - tj * TT;
  if (ti > tj) {   // the lower tiles are the transposes of the upper ones
    const int t = ti; ti = tj; tj = t;
    const int u = ii; ii = jj; jj = u;
  }
  const int tp = ti * ntile - ti * (ti - 1) / 2 + (tj - ti);
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += (double)part[(((size_t)s * nchunk + c) * ntp + tp) * TT * TT + ii * TT + jj];
  K[(size_t)s * R * R + e] = acc;
}

// FP64 path: K[s][i][j] for a 64 x 64 tile (bi, bj), bj <= bi, mirrored; whole pixel range.
__global__ __launch_bounds__(256) void k_quad_syrk64(int P, int R, int npix, const int* __restrict__ pair_a,
                                                     const int* __restrict__ pair_b, const double* __restrict__ maps,
                                                     const double* __restrict__ V, const double* __restrict__ w,
                                                     int vmode, double* __restrict__ K) {
  constexpr int KC = 16;
  __shared__ double Ai[KC][65], Aj[KC][65];
  const int bi = blockIdx.y, bj = blockIdx.x, s = blockIdx.z;
  if (bj > bi) return;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const double* Msky = maps + (size_t)s * P * npix;
  double acc[4][4] = {};
  for (int x0 = 0; x0 < npix; x0 += KC) {
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * KC * 64; e += 256) {
      const int side = e / (KC * 64), rem = e - side * KC * 64, r = rem / KC, k = rem - r * KC;
      const int row = (side ? bj : bi) * 64 + r, x = x0 + k;
      double v = 0.0;
      if (row < R && x < npix) {
        const double vv = V ? V[(size_t)row * npix + x] : 0.0;
        v = vmode ? vv : Msky[(size_t)pair_a[row] * npix + x] * Msky[(size_t)pair_b[row] * npix + x] - 3.0 * vv;
        v *= sqrt(w[x]);
      }
      (side ? Aj : Ai)[k][r] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Ai[k][ty * 4 + u];
        b[u] = Aj[k][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
  }
  double* Ks = K + (size_t)s * R * R;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = bi * 64 + ty * 4 + u, j = bj * 64 + tx * 4 + v;
      if (i < R && j < R && (bi != bj || j <= i)) {
        Ks[(size_t)i * R + j] = acc[u][v];
        Ks[(size_t)j * R + i] = acc[u][v];
      }
    }
}

// tau[s][n] = (1/3) sum over the three pairings of (K[s] - 6 KVV)
__global__ __launch_bounds__(256) void k_quad_gather(int R, int nquad, int S, const int* __restrict__ quad,
                                                     const double* __restrict__ K, const double* __restrict__ KVV,
                                                     double* __restrict__ tau) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= S * nquad) return;
  const int s = e / nquad, n = e - s * nquad;
  const int* qd = quad + 6 * n;
  const double* Ks = K + (size_t)s * R * R;
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const size_t o = (size_t)qd[2 * j] * R + qd[2 * j + 1];
    acc += Ks[o] - (KVV ? 6.0 * KVV[o] : 0.0);
  }
  tau[e] = acc * (1.0 / 3.0);
}

}  // namespace

int quad_chunks(int npix) { return std::max(1, std::min(16, npix / 4096)); }
int quad_ntile(int R) { return (R + TT - 1) / TT; }
size_t quad_lds() { return sizeof(TriLds); }

hipError_t quad_set_lds() {
  return hipFuncSetAttribute((const void*)k_quad_syrk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(TriLds));
}

// K [S][R][R] FP64 for the S skies' maps (vmode 0) or for V itself (vmode 1, S = 1).  For
// the float contexts the maps and V are pixel-block-major copies (launch_quad_vtile), for
// FP64 the maps and the pair-major planes of the state.
hipError_t launch_quad_syrk(const modal_ctx* c, const void* maps, const void* V, int S, int vmode, const int2* tpairs,
                            float* part, double* K, hipStream_t st) {
  const int R = c->npairs;
  if (c->prec == MODAL_F64) {
    const int nb = (R + 63) / 64;
    hipLaunchKernelGGL(k_quad_syrk64, dim3(nb, nb, S), dim3(256), 0, st, c->P, R, c->npix, c->t.pair_a, c->t.pair_b,
                       (const double*)maps, (const double*)V, c->t.w64, vmode, K);
    return hipGetLastError();
  }
  const int ntile = quad_ntile(R), ntp = ntile * (ntile + 1) / 2;
  const int nchunk = quad_chunks(c->npix);
  const int chunk_px = ((c->npix + nchunk - 1) / nchunk + PXS - 1) / PXS * PXS;
  hipError_t e = quad_set_lds();
  if (e != hipSuccess) return e;
  const int vec = c->npix % 4 == 0 ? 1 : 0;
  hipLaunchKernelGGL(k_quad_syrk, dim3(ntp, nchunk, (S + SKW - 1) / SKW), dim3(NTQ), sizeof(TriLds), st, c->P, R,
                     c->npix, S, nchunk, chunk_px, ntp, tpairs, c->t.pair_a, c->t.pair_b, (const float*)maps, (const float*)V, c->t.w32,
                     vmode, vec, part);
  const size_t tot = (size_t)R * R;
  hipLaunchKernelGGL(k_quad_reduce, dim3((tot + 255) / 256, S), dim3(256), 0, st, R, nchunk, ntp, ntile, part, K);
  return hipGetLastError();
}

hipError_t launch_quad_gather(const modal_ctx* c, int nquad, int S, const int* quad, const double* K, const double* KVV,
                              double* tau, hipStream_t st) {
  hipLaunchKernelGGL(k_quad_gather, dim3((S * nquad + 255) / 256), dim3(256), 0, st, c->npairs, nquad, S, quad, K, KVV,
                     tau);
  return hipGetLastError();
}

size_t quad_vtile_bytes(const modal_ctx* c) {
  if (c->prec == MODAL_F64) return 0;
  return (size_t)((c->npix + PXS - 1) / PXS) * c->npairs * PXS * 4;
}

hipError_t launch_quad_vtile(const modal_ctx* c, const void* V, int rows, int batch, float* Vt, hipStream_t st) {
  const int nblk = (c->npix + PXS - 1) / PXS;
  hipLaunchKernelGGL(k_quad_vtile, dim3((nblk + 7) / 8, (rows + 31) / 32, batch), dim3(256), 0, st, rows, c->npix,
                     nblk, c->npix % 4 == 0 ? 1 : 0, (const float*)V, Vt);
  return hipGetLastError();
}

size_t quad_mtile_bytes(const modal_ctx* c, int S) {
  if (c->prec == MODAL_F64) return 0;
  return (size_t)S * ((c->npix + PXS - 1) / PXS) * c->P * PXS * 4;
}

size_t quad_part_bytes(const modal_ctx* c, int S) {
  if (c->prec == MODAL_F64) return 0;
  const int ntile = quad_ntile(c->npairs), ntp = ntile * (ntile + 1) / 2;
  return (size_t)S * quad_chunks(c->npix) * ntp * TT * TT * 4;
}

}  // namespace modal
