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

}  // namespace

hipError_t launch_slot_matrix(const modal_ctx* c, const double* cot, int S, void* K, hipStream_t st) {
  const size_t tot = (size_t)c->P * c->npairs * S;
  hipLaunchKernelGGL(k_slot, dim3((tot + 255) / 256), dim3(256), 0, st, c->P, c->npairs, c->nmax, S, c->t.tri_of,
                     c->t.tri_mult, cot, (double*)K);
  return hipGetLastError();
}

hipError_t launch_pair_adjoint(const modal_ctx* c, const void* maps, const void* K, int S, void* G, hipStream_t st) {
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
