// Cubic pixel reduction as a pair x mode contraction over pixels (VALU path).
//
//   E_{(ab),t} = sum_x w(x) M_a(x) M_b(x) M_t(x)
//   out_prs = scale (E_{(pr),s} + E_{(ps),r} + E_{(rs),p}) + scale2 (L_{(pr),s} + L_{(ps),r} + L_{(rs),p})
//
// With scale = 1/3 the first term is beta_prs (the three pairings are equal); with
// L the linear-term sums of k_lin_harm.hip and scale2 = -1 the second subtracts
// lin_prs (eq. bbispect with the three pairings of the "3 C a" linear term of
// eq. bispectrumest).
//
// This kernel is the FP64 path: one
// workgroup per (pixel chunk, block of 64 pairs, map) accumulating in FP64.
// The matrix-core path (FP32 and the splits) lives in k_cubic_split.hip and uses the
// reduction k_reduce_single below.
#include "common.h"

namespace modal {
namespace {

constexpr int kChunk = 65536;  // pixels per split-K chunk
constexpr int kTile = 64;      // pixels staged in LDS per step

template <typename T>
__global__ __launch_bounds__(256) void k_cubic_valu(int P, int npairs, int npix, int nchunk,
                                                    const int* __restrict__ pair_a, const int* __restrict__ pair_b,
                                                    const T* __restrict__ maps, const T* __restrict__ w,
                                                    double* __restrict__ part) {
  const int chunk = blockIdx.x;
  const int s = blockIdx.z;
  const int pl = threadIdx.x & 63;
  const int tg = threadIdx.x >> 6;
  const int pair = blockIdx.y * 64 + pl;
  const bool pv = pair < npairs;
  const int a = pv ? pair_a[pair] : 0;
  const int b = pv ? pair_b[pair] : 0;
  __shared__ T Mt[kMaxP][kTile];
  __shared__ T wt[kTile];
  double acc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.0;
  const T* Ms = maps + (size_t)s * P * npix;
  const int x0c = chunk * kChunk;
  const int x1c = min(npix, x0c + kChunk);
  for (int x0 = x0c; x0 < x1c; x0 += kTile) {
    const int nt = min(kTile, x1c - x0);
    for (int i = threadIdx.x; i < P * kTile; i += 256) {
      const int p = i / kTile, xx = i - p * kTile;
      Mt[p][xx] = xx < nt ? Ms[(size_t)p * npix + x0 + xx] : T(0);
    }
    if (threadIdx.x < kTile) wt[threadIdx.x] = threadIdx.x < nt ? w[x0 + threadIdx.x] : T(0);
    __syncthreads();
    if (pv) {
      for (int xx = 0; xx < nt; ++xx) {
        const double A = (double)Mt[a][xx] * (double)Mt[b][xx] * (double)wt[xx];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int t = tg + 4 * i;
          if (t < P) acc[i] += A * (double)Mt[t][xx];
        }
      }
    }
    __syncthreads();
  }
  if (!pv) return;
  double* dst = part + (((size_t)s * nchunk + chunk) * npairs + pair) * P;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int t = tg + 4 * i;
    if (t < P) dst[t] = acc[i];
  }
}

__global__ void k_reduce_chunks(int nchunk, size_t per, int S, const double* __restrict__ part, double* __restrict__ E) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per * S) return;
  const size_t s = i / per, k = i - s * per;
  const double* src = part + s * nchunk * per + k;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += src[(size_t)c * per];
  E[i] = acc;
}

// out_n = scale * (three pairings of E) + scale2 * (three pairings of E2); either may be absent
__global__ void k_symm(int nmax, int npairs, int P, int S, double scale, const int* __restrict__ tri,
                       const double* __restrict__ E, double scale2, const double* __restrict__ E2,
                       double* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (n >= nmax) return;
  const int* tr = tri + 6 * n;  // p, r, s, pair(pr), pair(ps), pair(rs)
  const size_t o = (size_t)s * npairs * P;
  const size_t i1 = (size_t)tr[3] * P + tr[2], i2 = (size_t)tr[4] * P + tr[1], i3 = (size_t)tr[5] * P + tr[0];
  double v = 0.0;
  if (E) v = scale * (E[o + i1] + E[o + i2] + E[o + i3]);
  if (E2) v += scale2 * (E2[o + i1] + E2[o + i2] + E2[o + i3]);
  out[(size_t)s * nmax + n] = v;
}

// out_n = scale * sum_c part[s][c][cell_n] + scale2 * (three pairings of E2): beta_prs is
// the one cell (pair, mode) of the split contraction that holds it (any of the three
// pairings of the triple; the table of cells comes with the contraction's plan).  Thread i
// takes triple n = order[i], the triples sorted by cell, so that a wave reads runs of
// neighbouring cells of each chunk's partial sums.
__global__ void k_reduce_single(int nmax, int npairs, int P, int nchunk, const int* __restrict__ tri,
                                const int* __restrict__ cell, const int* __restrict__ order,
                                const double* __restrict__ part, double scale, double scale2,
                                const double* __restrict__ E2, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (i >= nmax) return;
  const int n = order[i];
  const int* tr = tri + 6 * n;
  const size_t per = (size_t)npairs * P;
  const size_t i1 = (size_t)cell[n];
  const double* src = part + (size_t)s * nchunk * per + i1;
  double v = 0.0;
  for (int c = 0; c < nchunk; ++c) v += src[(size_t)c * per];
  v *= scale;
  if (E2) {
    const size_t o = (size_t)s * per;
    v += scale2 * (E2[o + (size_t)tr[3] * P + tr[2]] + E2[o + (size_t)tr[4] * P + tr[1]] +
                   E2[o + (size_t)tr[5] * P + tr[0]]);
  }
  out[(size_t)s * nmax + n] = v;
}

}  // namespace

hipError_t launch_reduce_single(const modal_ctx* c, const double* part, int S, int nchunk, double scale,
                                const double* E2, double scale2, double* out, hipStream_t st) {
  if (!c->t.cell || !c->t.cell_order) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_single, dim3((c->nmax + 255) / 256, S), dim3(256), 0, st, c->nmax, c->npairs, c->P,
                     nchunk, c->t.tri, c->t.cell, c->t.cell_order, part, scale, scale2, E2, out);
  return hipGetLastError();
}

int cubic_nchunk(const modal_ctx* c) { return (c->npix + kChunk - 1) / kChunk; }

hipError_t launch_cubic_valu(const modal_ctx* c, const void* maps, int S, double* part, hipStream_t st) {
  // FP64 contexts only: the others contract on the matrix cores (k_cubic_split.hip)
  if (!is_f64(c)) return hipErrorInvalidValue;
  const int nchunk = cubic_nchunk(c);
  dim3 grid(nchunk, (c->npairs + 63) / 64, S);
  hipLaunchKernelGGL(k_cubic_valu<double>, grid, dim3(256), 0, st, c->P, c->npairs, c->npix, nchunk, c->t.pair_a,
                     c->t.pair_b, (const double*)maps, c->t.w64, part);
  return hipGetLastError();
}

// out = scale (three pairings of the chunk-reduced part) + scale2 (three pairings of E2);
// part == nullptr leaves only the E2 term, E2 == nullptr only the first.
hipError_t launch_reduce_symm(const modal_ctx* c, const double* part, int S, int nchunk, double scale, double* E,
                              const double* E2, double scale2, double* out, hipStream_t st) {
  if (part) {
    const size_t per = (size_t)c->npairs * c->P;
    const size_t tot = per * S;
    hipLaunchKernelGGL(k_reduce_chunks, dim3((tot + 255) / 256), dim3(256), 0, st, nchunk, per, S, part, E);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_symm, dim3((c->nmax + 255) / 256, S), dim3(256), 0, st, c->nmax, c->npairs, c->P, S, scale,
                     c->t.tri, part ? E : nullptr, scale2, E2, out);
  return hipGetLastError();
}

}  // namespace modal
