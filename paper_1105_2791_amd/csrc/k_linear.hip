// Monte-Carlo linear-term accumulator: U_pr(x) += sum_s M^s_p(x) M^s_r(x).
//
// The linear term of eq. (bispectrumest) pairs two legs of the cubic with their
// Gaussian expectation; Sec. II takes that expectation from Monte-Carlo
// simulations with the experimental effects included.  The accumulator holds one
// pixel plane per mode pair; FINALIZE scales it by 1/N to give V_pr(x).
// Memory-bound: one read-modify-write of U per batch of S maps.
#include "common.h"

namespace modal {
namespace {

constexpr int kPairBlk = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_lin_acc(int P, int npairs, int npix, int S, const int* __restrict__ pair_a,
                                                 const int* __restrict__ pair_b, const T* __restrict__ maps,
                                                 T* __restrict__ U) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int p0 = blockIdx.y * kPairBlk;
  __shared__ int sa[kPairBlk], sb[kPairBlk];
  if (threadIdx.x < kPairBlk) {
    const int pr = p0 + threadIdx.x;
    sa[threadIdx.x] = pr < npairs ? pair_a[pr] : 0;
    sb[threadIdx.x] = pr < npairs ? pair_b[pr] : 0;
  }
  __syncthreads();
  if (x >= npix) return;
  double acc[kPairBlk];
#pragma unroll
  for (int k = 0; k < kPairBlk; ++k) acc[k] = 0.0;
  for (int s = 0; s < S; ++s) {
    const T* Ms = maps + (size_t)s * P * npix + x;
#pragma unroll
    for (int k = 0; k < kPairBlk; ++k) acc[k] += (double)Ms[(size_t)sa[k] * npix] * (double)Ms[(size_t)sb[k] * npix];
  }
#pragma unroll
  for (int k = 0; k < kPairBlk; ++k) {
    const int pr = p0 + k;
    if (pr < npairs) {
      T* u = U + (size_t)pr * npix + x;
      *u = T((double)*u + acc[k]);
    }
  }
}

template <typename T>
__global__ void k_scale(size_t n, T* __restrict__ U, double s) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) U[i] = T((double)U[i] * s);
}

__global__ void k_zero(size_t n, uint32_t* __restrict__ p) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

hipError_t launch_lin_accumulate(const modal_ctx* c, const void* maps, int S, void* U, hipStream_t st) {
  dim3 grid((c->npix + 255) / 256, (c->npairs + kPairBlk - 1) / kPairBlk);
  if (is_f64(c))
    hipLaunchKernelGGL(k_lin_acc<double>, grid, dim3(256), 0, st, c->P, c->npairs, c->npix, S, c->t.pair_a,
                       c->t.pair_b, (const double*)maps, (double*)U);
  else
    hipLaunchKernelGGL(k_lin_acc<float>, grid, dim3(256), 0, st, c->P, c->npairs, c->npix, S, c->t.pair_a,
                       c->t.pair_b, (const float*)maps, (float*)U);
  return hipGetLastError();
}

hipError_t launch_lin_scale(const modal_ctx* c, void* U, double s, hipStream_t st) {
  const size_t n = (size_t)c->npairs * c->npix;
  if (is_f64(c))
    hipLaunchKernelGGL(k_scale<double>, dim3((n + 255) / 256), dim3(256), 0, st, n, (double*)U, s);
  else
    hipLaunchKernelGGL(k_scale<float>, dim3((n + 255) / 256), dim3(256), 0, st, n, (float*)U, s);
  return hipGetLastError();
}

// Zero fill by kernel (graph-capture safe, unlike a memset node).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, st, n, (uint32_t*)p);
  return hipGetLastError();
}

}  // namespace modal
