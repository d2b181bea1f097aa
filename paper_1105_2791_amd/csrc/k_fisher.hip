// Fisher estimate of the modal covariance from gradients.
//
// For Gaussian maps with exact pairing expectation in the linear term,
// E[J C J^T] = 18 zeta (J = d beta^hat / d a over the real dof of a, C their
// covariance), which follows from eq. (linearterm): beta^hat = T(aaa) - 3 T(C a)
// so J = 3 T(aa - C, .) and the expectation counts 18 of the Wick pairings that
// give 6 zeta in <beta^hat beta^hat^T>.  Hence zeta_F = (1/(18N)) sum_i J_i C J_i^T.
//
// J never needs forming: with qw = q / sqrt(C_l),
//   J_{prs,lm} = qw_p(l) Z_{rs,lm} + qw_r(l) Z_{ps,lm} + qw_s(l) Z_{pr,lm},
//   Z_{ab,lm}  = c_m sum_j lambda_lm(theta_j) sum_k w (M_a M_b - V_ab)(theta_j, phi_k) e^{-i m phi_k}
// (c_m = 2 - delta_m0; Re/Im of Z are the derivatives with respect to Re/Im a_lm),
// so J C J^T only needs, per l, the cross spectra of the pair adjoints
//   X_l[a][b] = C_l [Re Z_a(l,0) Re Z_b(l,0) + 1/2 sum_{m>=1} (Re Z_a Re Z_b + Im Z_a Im Z_b)],
// accumulated over maps, and the assembly
//   F_{nn'} = (1/(18N)) sum over the 3 x 3 leg choices of sum_l qw_u(l) qw_u'(l) X_l[pair][pair'].
#include "common.h"

namespace modal {
namespace {

template <typename T> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

// G[pair][x] = w(x) (M_a M_b - V_ab)(x) for one map.
template <typename T, bool LIN>
__global__ __launch_bounds__(256) void k_pair_maps(int npairs, int npix, const int* __restrict__ pa,
                                                   const int* __restrict__ pb, const T* __restrict__ maps,
                                                   const T* __restrict__ V, const T* __restrict__ w,
                                                   T* __restrict__ G) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int pair = blockIdx.y;
  if (x >= npix) return;
  const int a = pa[pair], b = pb[pair];
  double v = (double)maps[(size_t)a * npix + x] * (double)maps[(size_t)b * npix + x];
  if (LIN) v -= (double)V[(size_t)pair * npix + x];
  G[(size_t)pair * npix + x] = T(v * (double)w[x]);
}

// Z[col][lm] = c_m sum_j lambda_lm(theta_j) (Gh_N +- Gh_S)(col, m), one thread per l,
// NC columns per thread; the ring values are staged in LDS already folded, Gh_N + Gh_S
// and Gh_N - Gh_S in FP64, so that each thread reads the one its parity of l - m needs.
constexpr int NC = 16;
constexpr int RCH = 32;

template <typename T>
__global__ __launch_bounds__(64) void k_adj_legendre_cols(int lmax, int ntheta, int nrp, int ncol, int nalm,
                                                          const T* __restrict__ lam,
                                                          const typename vec2<T>::type* __restrict__ Gh,
                                                          typename vec2<T>::type* __restrict__ Z) {
  using T2 = typename vec2<T>::type;
  const int m = blockIdx.y;
  const int L = lmax + 1 - m;
  const int li = blockIdx.x * 64 + threadIdx.x;
  const int c0 = blockIdx.z * NC;
  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;
  const T* lrow = lam + off * nrp;
  __shared__ double2 hp[RCH][NC];   // Gh_N + Gh_S (even l - m)
  __shared__ double2 hm[RCH][NC];   // Gh_N - Gh_S (odd l - m)
  double ar[NC], ai[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) ar[q] = ai[q] = 0.0;
  const bool odd = (li & 1);
  for (int j0 = 0; j0 < nrp; j0 += RCH) {
    const int nj = min(RCH, nrp - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < RCH * NC; e += 64) {
      const int jj = e / NC, q = e - jj * NC;
      T2 vn, vs;
      vn.x = vn.y = vs.x = vs.y = T(0);
      const int col = c0 + q, j = j0 + jj;
      if (jj < nj && col < ncol) {
        const T2* g = Gh + ((size_t)col * (lmax + 1) + m) * ntheta;   // Gh[col][m][ring]
        vn = g[j];
        const int js = ntheta - 1 - j;
        if (js != j) vs = g[js];
      }
      hp[jj][q] = make_double2((double)vn.x + (double)vs.x, (double)vn.y + (double)vs.y);
      hm[jj][q] = make_double2((double)vn.x - (double)vs.x, (double)vn.y - (double)vs.y);
    }
    __syncthreads();
    if (li < L) {
      const double2(*h)[NC] = odd ? hm : hp;
      for (int jj = 0; jj < nj; ++jj) {
        const double lv = (double)lrow[(size_t)(j0 + jj) * L + li];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          const double2 v = h[jj][q];
          ar[q] += lv * v.x;
          ai[q] += lv * v.y;
        }
      }
    }
  }
  if (li >= L) return;
  const double cm = (m == 0) ? 1.0 : 2.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int col = c0 + q;
    if (col >= ncol) break;
    T2 z;
    z.x = T(cm * ar[q]);
    z.y = T(m == 0 ? 0.0 : cm * ai[q]);
    Z[(size_t)col * nalm + off + li] = z;
  }
}

// The same sums on the matrix cores for the split-precision contexts: per m a GEMM
//   Z[l][c] = sum_j lambda[m][j][l] H_{(l - m) mod 2}[j][c],  H_0 = Gh_N + Gh_S, H_1 = Gh_N - Gh_S,
// with K = the northern rings and the real and imaginary parts of the columns as
// separate GEMM columns.  v_mfma_f32_32x32x2f32 (lane l holds A[l % 32][l / 32],
// B[l / 32][l % 32]; accumulator register r is D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]).
// A workgroup owns 64 consecutive l - m (32 even and 32 odd: one tile each) of one m and
// 64 complex columns; wave w owns the columns [16 w, 16 w + 16) as 32 GEMM columns.  A
// lane reads the even and odd lambda of its row from the table row of its ring; the
// folded ring values of 32 rings are staged in LDS for all four waves.  The MFMAs of a
// staged chunk accumulate from zero and the chunk joins the running FP32 sum with a
// round-to-nearest add.  The matrix core's FP32 accumulation raised the FP32-context
// linear term's error against the oracle from 2.7e-6 to 6.5e-6 of rms (its bound is
// 1e-5; a running FP64 sum did not lower it and cost 25 %), so FP32 contexts keep the
// FP64 vector sums above; f16x3 contexts, whose operands carry 2^-22, take this kernel, and
// bf16x3 contexts the split-operand kernel below.
constexpr int AL_RC = 32;   // rings per staged chunk
constexpr int AL_NC = 64;   // complex columns per workgroup

__global__ __launch_bounds__(256) void k_adj_legendre_mfma(int lmax, int ntheta, int nrp, int ncol, int nalm,
                                                           const float* __restrict__ lam, const float2* __restrict__ Gh,
                                                           float* __restrict__ Z) {
  typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
  const int m = blockIdx.y;
  const int L = lmax + 1 - m;
  const int ib = blockIdx.x * 32;   // row i of a tile is l - m = 2 (ib + i) + parity
  if (2 * ib >= L) return;          // whole workgroup: no barrier reached
  const int c0 = blockIdx.z * AL_NC;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int row = lane & 31, kh = lane >> 5;
  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;
  const float* lrow = lam + off * nrp;
  __shared__ float2 hp[AL_RC][AL_NC + 1], hm[AL_RC][AL_NC + 1];
  f32x16 acc[2], cha[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = cha[t][r] = 0.f;
  const int li = 2 * (ib + row);             // this lane's even A row; the odd one is li + 1
  const bool ok0 = li < L, ok1 = li + 1 < L;
  const int bc = 16 * wv + (row >> 1);       // this lane's B (and D) column: complex column, part
  const int part = row & 1;
  // software pipeline: the next chunk's lambda values and folded ring values are loaded
  // into registers (unconditionally, indices clamped) while this chunk's MFMAs run
  constexpr int NE = AL_RC * AL_NC / 256;   // staged ring values per thread
  float la0[AL_RC / 2], la1[AL_RC / 2];     // this lane's A values of one chunk
  float2 gn[NE], gs[NE];
  auto load_chunk = [&](int j0) {
#pragma unroll
    for (int k2 = 0; k2 < AL_RC / 2; ++k2) {
      const int j = min(j0 + 2 * k2 + kh, nrp - 1);
      const float* lp = lrow + (size_t)j * L + min(li, L - 1);
      la0[k2] = lp[0];
      la1[k2] = lp[ok1 ? 1 : 0];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {   // consecutive threads: consecutive rings of one column
      const int e = tid + 256 * u, jj = e % AL_RC, q = e / AL_RC;
      const int col = min(c0 + q, ncol - 1), j = min(j0 + jj, nrp - 1);
      const float2* g = Gh + ((size_t)col * (lmax + 1) + m) * ntheta;   // Gh[col][m][ring]
      gn[u] = g[j];
      gs[u] = g[ntheta - 1 - j];
    }
  };
  auto store_chunk = [&](int j0) {
    const int nj = min(AL_RC, nrp - j0);
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int e = tid + 256 * u, jj = e % AL_RC, q = e / AL_RC;
      const int j = j0 + jj;
      const bool in = jj < nj && c0 + q < ncol;
      const float2 vn = in ? gn[u] : make_float2(0.f, 0.f);
      const float2 vs = (in && ntheta - 1 - j != j) ? gs[u] : make_float2(0.f, 0.f);   // the equator ring once
      hp[jj][q] = make_float2(vn.x + vs.x, vn.y + vs.y);
      hm[jj][q] = make_float2(vn.x - vs.x, vn.y - vs.y);
    }
  };
  load_chunk(0);
  store_chunk(0);
  for (int j0 = 0; j0 < nrp; j0 += AL_RC) {
    const int nj = min(AL_RC, nrp - j0);
    float a0c[AL_RC / 2], a1c[AL_RC / 2];
#pragma unroll
    for (int k2 = 0; k2 < AL_RC / 2; ++k2) {
      const bool in = 2 * k2 + kh < nj;
      a0c[k2] = (in && ok0) ? la0[k2] : 0.f;
      a1c[k2] = (in && ok1) ? la1[k2] : 0.f;
    }
    __syncthreads();   // hp, hm of this chunk are in LDS
    const bool more = j0 + AL_RC < nrp;
    if (more) load_chunk(j0 + AL_RC);
#pragma unroll
    for (int k2 = 0; k2 < AL_RC / 2; ++k2) {
      const int jj = 2 * k2 + kh;
      const float2 he = hp[jj][bc], ho = hm[jj][bc];
      cha[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0c[k2], part ? he.y : he.x, cha[0], 0, 0, 0);
      cha[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1c[k2], part ? ho.y : ho.x, cha[1], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      acc[t] += cha[t];
#pragma unroll
      for (int r = 0; r < 16; ++r) cha[t][r] = 0.f;
    }
    __syncthreads();   // every wave is done with this chunk's hp, hm
    if (more) store_chunk(j0 + AL_RC);
  }
  const int col = c0 + bc;
  if (col >= ncol) return;
  const float cm = (m == 0) ? 1.f : 2.f;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int lr = 2 * (ib + 8 * (r >> 2) + 4 * kh + (r & 3)) + t;
      if (lr < L) Z[((size_t)col * nalm + off + lr) * 2 + part] = (m == 0 && part) ? 0.f : cm * acc[t][r];
    }
}

// bf16x3 contexts: the same sums on the bf16 matrix cores with split operands.  Per m,
//   Z^T[c][l] = sum_j H_{(l - m) mod 2}^T[c][j] lambda[m][j][l]   (K = the northern rings),
// on v_mfma_f32_32x32x16_bf16: A = H^T (rows = 32 real columns, K = 16 rings), B = lambda
// (K = 16 rings, N = 32 l of one parity); lane l holds A[l % 32][8 (l / 32) + i] and
// B[8 (l / 32) + i][l % 32]; accumulator register r is D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
// Both operands are split into bf16 hi + lo and each product is Ah Bh + Ah Bl + Al Bh.
// Workgroup: 4 waves, one m, 128 consecutive l - m (wave w: the 32 l of parity w / 2 in
// the half w % 2), 64 complex columns (4 tiles of 32 real columns).  The folded ring values
// of a 32-ring chunk are split and staged in LDS, double buffered; each lane loads the
// lambda of its l at the 16 rings of its two K steps from the FP32 table one chunk ahead
// and splits them in registers.  The workgroups of one m (l blocks x column blocks) run
// back to back on one XCD, so lambda[m] and the ring values of m come from HBM about once.  An output takes
// 3 nrp / 16 accumulations (144 at 768 rings); the truncation of the matrix core's
// accumulation stays below the operand split error.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
constexpr int AS_L = 128;         // l per workgroup (32 of one parity per wave)
constexpr int AS_NC = 64;         // complex columns per workgroup
constexpr int AS_RC = 32;         // rings per staged chunk (two K steps)
constexpr int AS_RS = AS_RC + 8;  // LDS row stride of a staged column (16-bit words): 16-byte reads of 16 lanes on distinct banks

struct AsLds {
  uint16_t h[2][2][2 * AS_NC][AS_RS];   // [buffer][parity][real column][ring of the chunk]
  uint16_t l[2][2][2 * AS_NC][AS_RS];
};

__device__ inline uint32_t as_bf16x2(float a, float b) {
  typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
  bf16x2 v;
  v[0] = (__bf16)a;
  v[1] = (__bf16)b;
  return __builtin_bit_cast(uint32_t, v);
}

// bf16 hi/lo words of two values (RNE each; the split starts from the rounded FP32 value)
__device__ inline void as_split2(float v0, float v1, uint32_t& hi, uint32_t& lo) {
  asm("" : "+v"(v0), "+v"(v1));
  uint32_t hb = as_bf16x2(v0, v1);
  asm("" : "+v"(hb));
  hi = hb;
  lo = as_bf16x2(v0 - __builtin_bit_cast(float, hb << 16), v1 - __builtin_bit_cast(float, hb & 0xffff0000u));
}

__global__ __launch_bounds__(256) void k_adj_legendre_split(int lmax, int ntheta, int nrp, int ncol, int nalm, int nlb,
                                                            int ncb, const float* __restrict__ lam,
                                                            const float2* __restrict__ Gh, float* __restrict__ Z) {
  typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
  const int xcd = blockIdx.x & 7, i8 = blockIdx.x >> 3, per = nlb * ncb;
  const int m = xcd + 8 * (i8 / per);
  const int lb = (i8 % per) / ncb, cb = (i8 % per) % ncb;
  const int L = lmax + 1 - m;
  if (m > lmax || lb * AS_L >= L) return;   // whole workgroup, before any barrier
  const int c0 = cb * AS_NC;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, n = lane & 31, h = lane >> 5;
  const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;
  const float* lrow = lam + off * nrp;
  __shared__ AsLds S;
  const int par = wv >> 1;                        // the parity of l - m of this wave's rows
  const int li = lb * AS_L + 64 * (wv & 1) + 2 * n + par;   // this lane's B column (l - m)
  const int lcl = min(li, L - 1);
  // lambda at rings 32 c + 16 kk + 8 h + i of the lane's l for the two K steps kk of chunk c
  // (valid addresses for every c), loaded one chunk ahead
  float lv[2][8], lvn[2][8];
  auto load_lam = [&](int c, float (&dst)[2][8]) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int i = 0; i < 8; ++i) dst[kk][i] = lrow[(size_t)min(AS_RC * c + 16 * kk + 8 * h + i, nrp - 1) * L + lcl];
  };
  // ring values of a chunk: thread (column q, ring pair jp) for four (q, jp), north and south
  constexpr int NU = AS_NC * AS_RC / 2 / 256;
  float2 gn[NU][2], gs[NU][2];
  auto load_g = [&](int r0) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + 256 * u, jp = e % (AS_RC / 2), q = e / (AS_RC / 2);
      const float2* g = Gh + ((size_t)min(c0 + q, ncol - 1) * (lmax + 1) + m) * ntheta;   // Gh[col][m][ring]
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int j = min(r0 + 2 * jp + k, nrp - 1);
        gn[u][k] = g[j];
        gs[u][k] = g[ntheta - 1 - j];
      }
    }
  };
  auto store_g = [&](int r0, int buf) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = tid + 256 * u, jp = e % (AS_RC / 2), q = e / (AS_RC / 2);
      float hp[2][2], hm[2][2];   // [part][ring of the pair]
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int j = r0 + 2 * jp + k;
        const bool in = j < nrp && c0 + q < ncol;
        const float2 vn = in ? gn[u][k] : make_float2(0.f, 0.f);
        const float2 vs = (in && ntheta - 1 - j != j) ? gs[u][k] : make_float2(0.f, 0.f);   // the equator ring once
        hp[0][k] = vn.x + vs.x;
        hp[1][k] = vn.y + vs.y;
        hm[0][k] = vn.x - vs.x;
        hm[1][k] = vn.y - vs.y;
      }
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        uint32_t hi, lo;
        as_split2(hp[part][0], hp[part][1], hi, lo);
        *reinterpret_cast<uint32_t*>(&S.h[buf][0][2 * q + part][2 * jp]) = hi;
        *reinterpret_cast<uint32_t*>(&S.l[buf][0][2 * q + part][2 * jp]) = lo;
        as_split2(hm[part][0], hm[part][1], hi, lo);
        *reinterpret_cast<uint32_t*>(&S.h[buf][1][2 * q + part][2 * jp]) = hi;
        *reinterpret_cast<uint32_t*>(&S.l[buf][1][2 * q + part][2 * jp]) = lo;
      }
    }
  };
  f32x16 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[ct][r] = 0.f;
  const int nch = (nrp + AS_RC - 1) / AS_RC;
  load_g(0);
  store_g(0, 0);
  load_g(AS_RC);
  load_lam(0, lv);
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    // chunk ch + 1 into the other buffer (last read in chunk ch - 1, before the barrier
    // that ended it), then the loads of chunk ch + 2
    if (ch + 1 < nch) {
      store_g((ch + 1) * AS_RC, buf ^ 1);
      load_g((ch + 2) * AS_RC);
    }
    load_lam(ch + 1, lvn);   // the next chunk's lambda (clamped past the last ring: unused)
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      bf16x8 bh, bl;
      {
        u32x4 hv, lo4;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          uint32_t hw, lw2;
          as_split2(lv[kk][2 * k], lv[kk][2 * k + 1], hw, lw2);
          hv[k] = hw;
          lo4[k] = lw2;
        }
        bh = __builtin_bit_cast(bf16x8, hv);
        bl = __builtin_bit_cast(bf16x8, lo4);
      }
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&S.h[buf][par][32 * ct + n][16 * kk + 8 * h]));
        const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(&S.l[buf][par][32 * ct + n][16 * kk + 8 * h]));
        acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[ct], 0, 0, 0);
        acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[ct], 0, 0, 0);
        acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int i = 0; i < 8; ++i) lv[kk][i] = lvn[kk][i];
    __syncthreads();   // chunk ch read by all waves; chunk ch + 1 visible
  }
  if (li >= L) return;
  const float cm = (m == 0) ? 1.f : 2.f;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int rc = 32 * ct + 8 * (r >> 2) + 4 * h + (r & 3);
      const int col = c0 + (rc >> 1), part = rc & 1;
      if (col < ncol) Z[((size_t)col * nalm + off + li) * 2 + part] = (m == 0 && part) ? 0.f : cm * acc[ct][r];
    }
}

// X[l][a][b] += C_l [Re Za Re Zb (m=0) + 1/2 sum_{m>=1} (Re Za Re Zb + Im Za Im Zb)], 64x64 tiles, lower tiles only.
constexpr int XT = 64;
constexpr int MC = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_cross_spectra(int lmax, int npairs, int nalm,
                                                       const typename vec2<T>::type* __restrict__ Z,
                                                       const double* __restrict__ cvar, double* __restrict__ X) {
  using T2 = typename vec2<T>::type;
  const int l = blockIdx.z;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  const int i0 = bi * XT, j0 = bj * XT;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ double Zi[2 * MC][XT + 1];
  __shared__ double Zj[2 * MC][XT + 1];
  double acc[4][4] = {};
  for (int m0 = 0; m0 <= l; m0 += MC) {
    __syncthreads();
    for (int e = threadIdx.x; e < MC * XT; e += 256) {
      const int mm = e / XT, r = e - mm * XT;
      const int m = m0 + mm;
      double ir = 0, ii = 0, jr = 0, jim = 0;
      if (m <= l) {
        const size_t idx = (size_t)m * (2 * lmax + 3 - m) / 2 + (l - m);
        const double wgt = (m == 0) ? 1.0 : 0.7071067811865476;  // sqrt(1/2) per factor
        if (i0 + r < npairs) {
          const T2 z = Z[(size_t)(i0 + r) * nalm + idx];
          ir = wgt * (double)z.x;
          ii = (m == 0) ? 0.0 : wgt * (double)z.y;
        }
        if (j0 + r < npairs) {
          const T2 z = Z[(size_t)(j0 + r) * nalm + idx];
          jr = wgt * (double)z.x;
          jim = (m == 0) ? 0.0 : wgt * (double)z.y;
        }
      }
      Zi[2 * mm][r] = ir;
      Zi[2 * mm + 1][r] = ii;
      Zj[2 * mm][r] = jr;
      Zj[2 * mm + 1][r] = jim;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < 2 * MC; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Zi[k][ty * 4 + u];
        b[u] = Zj[k][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
  }
  const double cl = cvar[l];
  double* Xl = X + (size_t)l * npairs * npairs;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
      if (i < npairs && j < npairs && j <= i) {
        const double d = cl * acc[u][v];
        Xl[(size_t)i * npairs + j] += d;
        if (i != j) Xl[(size_t)j * npairs + i] += d;
      }
    }
}

// F[n][n'] = scale sum_{legs} sum_l qw_u(l) qw_u'(l) X_l[pair][pair'] (n <= n', mirrored).
__global__ __launch_bounds__(256) void k_fisher_assemble(int nmax, int npairs, int lmax, const int* __restrict__ tri,
                                                         const double* __restrict__ qw, const double* __restrict__ X,
                                                         double scale, double* __restrict__ F) {
  const int n = blockIdx.y;
  const int np = blockIdx.x * 256 + threadIdx.x;
  if (np >= nmax || np < n) return;
  const int* t1 = tri + 6 * n;
  const int* t2 = tri + 6 * np;
  // legs: (u, complementary pair): (p, rs), (r, ps), (s, pr)
  const int u1[3] = {t1[0], t1[1], t1[2]}, c1[3] = {t1[5], t1[4], t1[3]};
  const int u2[3] = {t2[0], t2[1], t2[2]}, c2[3] = {t2[5], t2[4], t2[3]};
  const size_t pp = (size_t)npairs * npairs;
  double acc = 0.0;
  for (int l = 0; l <= lmax; ++l) {
    const double* Xl = X + l * pp;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double qa = qw[(size_t)u1[a] * (lmax + 1) + l];
#pragma unroll
      for (int b = 0; b < 3; ++b)
        acc += qa * qw[(size_t)u2[b] * (lmax + 1) + l] * Xl[(size_t)c1[a] * npairs + c2[b]];
    }
  }
  F[(size_t)n * nmax + np] = scale * acc;
  F[(size_t)np * nmax + n] = scale * acc;
}

}  // namespace

hipError_t launch_pair_maps(const modal_ctx* c, const void* maps, const void* V, void* G, hipStream_t st) {
  dim3 grid((c->npix + 255) / 256, c->npairs);
#define LAUNCH(T, L, W)                                                                                     \
  hipLaunchKernelGGL((k_pair_maps<T, L>), grid, dim3(256), 0, st, c->npairs, c->npix, c->t.pair_a,         \
                     c->t.pair_b, (const T*)maps, (const T*)V, (const T*)W, (T*)G)
  if (is_f64(c)) {
    if (V) LAUNCH(double, true, c->t.w64);
    else LAUNCH(double, false, c->t.w64);
  } else {
    if (V) LAUNCH(float, true, c->t.w32);
    else LAUNCH(float, false, c->t.w32);
  }
#undef LAUNCH
  return hipGetLastError();
}

hipError_t launch_adj_legendre_cols(const modal_ctx* c, const void* lam, const void* Gh, int ncol, void* Z,
                                    hipStream_t st) {
  if (is_f64(c)) {
    dim3 grid((c->lmax + 1 + 63) / 64, c->lmax + 1, (ncol + NC - 1) / NC);
    hipLaunchKernelGGL(k_adj_legendre_cols<double>, grid, dim3(64), 0, st, c->lmax, c->ntheta, c->nrp, ncol, c->nalm,
                       (const double*)lam, (const double2*)Gh, (double2*)Z);
  } else if (c->prec == MODAL_F32) {
    dim3 grid((c->lmax + 1 + 63) / 64, c->lmax + 1, (ncol + NC - 1) / NC);
    hipLaunchKernelGGL(k_adj_legendre_cols<float>, grid, dim3(64), 0, st, c->lmax, c->ntheta, c->nrp, ncol, c->nalm,
                       (const float*)lam, (const float2*)Gh, (float2*)Z);
  } else if (c->prec == MODAL_BF16X3) {
    const int nlb = (c->lmax + AS_L) / AS_L, ncb = (ncol + AS_NC - 1) / AS_NC;
    const dim3 grid(8 * ((c->lmax + 8) / 8) * nlb * ncb);
    hipLaunchKernelGGL(k_adj_legendre_split, grid, dim3(256), 0, st, c->lmax, c->ntheta, c->nrp, ncol, c->nalm, nlb,
                       ncb, (const float*)lam, (const float2*)Gh, (float*)Z);
  } else {
    dim3 grid((c->lmax + 1 + 63) / 64, c->lmax + 1, (ncol + AL_NC - 1) / AL_NC);
    hipLaunchKernelGGL(k_adj_legendre_mfma, grid, dim3(256), 0, st, c->lmax, c->ntheta, c->nrp, ncol, c->nalm,
                       (const float*)lam, (const float2*)Gh, (float*)Z);
  }
  return hipGetLastError();
}

hipError_t launch_cross_spectra(const modal_ctx* c, const void* Z, const double* cvar, double* X, hipStream_t st) {
  const int nb = (c->npairs + XT - 1) / XT;
  dim3 grid(nb, nb, c->lmax + 1);
  if (is_f64(c))
    hipLaunchKernelGGL(k_cross_spectra<double>, grid, dim3(256), 0, st, c->lmax, c->npairs, c->nalm,
                       (const double2*)Z, cvar, X);
  else
    hipLaunchKernelGGL(k_cross_spectra<float>, grid, dim3(256), 0, st, c->lmax, c->npairs, c->nalm,
                       (const float2*)Z, cvar, X);
  return hipGetLastError();
}

hipError_t launch_fisher_assemble(const modal_ctx* c, const double* X, double scale, double* F, hipStream_t st) {
  dim3 grid((c->nmax + 255) / 256, c->nmax);
  hipLaunchKernelGGL(k_fisher_assemble, grid, dim3(256), 0, st, c->nmax, c->npairs, c->lmax, c->t.tri, c->t.qw64, X,
                     scale, F);
  return hipGetLastError();
}

}  // namespace modal
