// Monte-Carlo linear-term accumulator: U_pr(x) += sum_s M^s_p(x) M^s_r(x).
//
// The linear term of eq. (bispectrumest) pairs two legs of the cubic with their
// Gaussian expectation; Sec. II takes that expectation from Monte-Carlo
// simulations with the experimental effects included.  The accumulator holds one
// pixel plane per mode pair; FINALIZE scales it by 1/N to give V_pr(x).
// Memory-bound: one read-modify-write of U per batch of S maps (bytes: npairs npix
// 2 sizeof(T) + S P npix sizeof(T)).
#include "common.h"

namespace modal {
namespace {

// Pairs in 5 x 5 tiles (a in [5 ta, 5 ta + 5), b in [5 tb, 5 tb + 5), ta <= tb) of the
// upper triangle of the P x P mode grid: a tile needs 10 map rows per sky (5 on the
// diagonal) for its 25 products.  A thread owns PX consecutive pixels (one vector load per
// row); a workgroup owns one tile of 256 PX pixels.  The batch sum is formed in registers
// in T and added to U once, so each U plane segment is read and written once per batch;
// U is streamed with non-temporal loads and stores, which keeps the L2 for the maps.  The
// tiles of one pixel block are consecutive workgroups on one XCD (workgroups are dealt to
// the 8 XCDs round-robin), so they run together and the block's map rows, needed by
// every tile, come from HBM once and from that XCD's L2 afterwards.  (Measured at l_max
// 1000, P 40, S 8: 5 x 5 tiles of 4 pixels 7.9 ms; 4 x 4 8.5 ms; 8 x 8 tiles of one pixel
// 12.5 ms, of two 10.5 ms; 56 ms with a pair block per workgroup re-reading the maps.)
constexpr int kTile = 5;
constexpr int kThreads = 256;

template <typename T, int N>
struct Vec { typedef T type __attribute__((ext_vector_type(N))); };
template <typename T>
struct Vec<T, 1> { typedef T type; };

template <typename V>
__device__ inline auto lane(const V& v, int k) { return v[k]; }
__device__ inline float lane(const float& v, int) { return v; }
__device__ inline double lane(const double& v, int) { return v; }

template <typename T, int PX>
__global__ __launch_bounds__(kThreads) void k_lin_acc(int P, int npix, int S, int nblk, int ntiles,
                                                      const int* __restrict__ pair_of, const T* __restrict__ maps,
                                                      T* __restrict__ U) {
  typedef typename Vec<T, PX>::type V;
  const int bid = blockIdx.x;
  const int i8 = bid >> 3;
  const int blk = (bid & 7) + 8 * (i8 / ntiles);
  if (blk >= nblk) return;
  int tile = i8 % ntiles, ta = 0;
  const int nt = (P + kTile - 1) / kTile;
  while (tile >= nt - ta) {   // row ta of the tile triangle holds nt - ta tiles
    tile -= nt - ta;
    ++ta;
  }
  const int tb = ta + tile;
  const int x = (blk * kThreads + threadIdx.x) * PX;   // npix % PX == 0 (host)
  if (x >= npix) return;   // no barriers below
  const int a0 = ta * kTile, b0 = tb * kTile;
  T acc[kTile][kTile][PX];
#pragma unroll
  for (int i = 0; i < kTile; ++i)
#pragma unroll
    for (int j = 0; j < kTile; ++j)
#pragma unroll
      for (int k = 0; k < PX; ++k) acc[i][j][k] = T(0);
  for (int s = 0; s < S; ++s) {
    const T* Ms = maps + (size_t)s * P * npix + x;
    V va[kTile], vb[kTile];
#pragma unroll
    for (int i = 0; i < kTile; ++i) {   // rows past P are loaded clamped, never stored
      va[i] = *reinterpret_cast<const V*>(Ms + (size_t)min(a0 + i, P - 1) * npix);
      vb[i] = *reinterpret_cast<const V*>(Ms + (size_t)min(b0 + i, P - 1) * npix);
    }
#pragma unroll
    for (int i = 0; i < kTile; ++i)
#pragma unroll
      for (int j = 0; j < kTile; ++j)
#pragma unroll
        for (int k = 0; k < PX; ++k) acc[i][j][k] += lane(va[i], k) * lane(vb[j], k);
  }
#pragma unroll
  for (int i = 0; i < kTile; ++i) {
    const int a = a0 + i;
#pragma unroll
    for (int j = 0; j < kTile; ++j) {
      const int b = b0 + j;
      if (a < P && b < P && a <= b) {
        V* u = reinterpret_cast<V*>(U + (size_t)pair_of[a * P + b] * npix + x);
        V v = __builtin_nontemporal_load(u);
        if constexpr (PX == 1) {
          v += acc[i][j][0];
        } else {
#pragma unroll
          for (int k = 0; k < PX; ++k) v[k] += acc[i][j][k];
        }
        __builtin_nontemporal_store(v, u);
      }
    }
  }
}

template <typename T, int PX>
void lin_acc_launch(const modal_ctx* c, const void* maps, int S, void* U, hipStream_t st) {
  const int nblk = (c->npix / PX + kThreads - 1) / kThreads, nt = (c->P + kTile - 1) / kTile;
  const int ntiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL((k_lin_acc<T, PX>), dim3(8 * ((nblk + 7) / 8) * ntiles), dim3(kThreads), 0, st, c->P, c->npix, S,
                     nblk, ntiles, c->t.pair_of, (const T*)maps, (T*)U);
}

// Element-wise kernels over whole state buffers loop with the grid's stride: one dispatch
// holds fewer than 2^32 work-items per dimension, and the pair planes of a state exceed
// that (4.7e9 words at l_max 1000, P 40; 6.0e9 elements at P 50).
constexpr size_t kStrideBlocks = 65536;
inline unsigned stride_blocks(size_t n) { return (unsigned)std::min((n + 255) / 256, kStrideBlocks); }

template <typename T>
__global__ void k_scale(size_t n, T* __restrict__ U, double s) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) U[i] = T((double)U[i] * s);
}

__global__ void k_zero(size_t n, uint32_t* __restrict__ p) {
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) p[i] = 0u;
}

}  // namespace

hipError_t launch_lin_accumulate(const modal_ctx* c, const void* maps, int S, void* U, hipStream_t st) {
  // vector loads need rows (npix elements apart) aligned to the vector width
  if (is_f64(c)) {
    if (c->npix % 2 == 0) lin_acc_launch<double, 2>(c, maps, S, U, st);
    else lin_acc_launch<double, 1>(c, maps, S, U, st);
  } else {
    if (c->npix % 4 == 0) lin_acc_launch<float, 4>(c, maps, S, U, st);
    else lin_acc_launch<float, 1>(c, maps, S, U, st);
  }
  return hipGetLastError();
}

hipError_t launch_lin_scale(const modal_ctx* c, void* U, double s, hipStream_t st) {
  const size_t n = (size_t)c->npairs * c->npix;
  if (n == 0) return hipSuccess;
  if (is_f64(c))
    hipLaunchKernelGGL(k_scale<double>, dim3(stride_blocks(n)), dim3(256), 0, st, n, (double*)U, s);
  else
    hipLaunchKernelGGL(k_scale<float>, dim3(stride_blocks(n)), dim3(256), 0, st, n, (float*)U, s);
  return hipGetLastError();
}

// Zero fill by kernel (graph-capture safe, unlike a memset node).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(stride_blocks(n)), dim3(256), 0, st, n, (uint32_t*)p);
  return hipGetLastError();
}

}  // namespace modal
