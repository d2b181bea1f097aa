// Internal declarations shared by the host code and the HIP kernels of
// libmodal.  Not part of the public ABI (include/modal.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/modal.h"

namespace modal {

constexpr int kMaxP = 64;          // largest number of mode functions supported
constexpr int kMaxFactors = 16;    // FFT radix plan length
constexpr int kRecPad = 64;       // zero recurrence entries after the last (l, m)
constexpr double kLogSeedFloor = -62.383246250395075;  // ln(2^-90): smaller lambda are dropped

struct FftPlan {
  int N;                 // ring length nphi (even)
  int K;                 // N / 2, length of the complex transform
  int nf;                // number of radix stages
  int radix[kMaxFactors];
};

// Device tables owned by a context (all allocated in modal_create).
struct Tables {
  double* x = nullptr;         // [ntheta] cos theta_j, north to south
  double* ringw = nullptr;     // [ntheta] w_GL(theta_j) * 2 pi / nphi
  double* w64 = nullptr;       // [ntheta*nphi] pixel weights (ringw * mask)
  float* w32 = nullptr;        // same, float
  double* rec = nullptr;       // [nalm + kRecPad][2] recurrence coefficients (A_lm, B_lm)
  double* seed = nullptr;      // [lmax+1][nrp][2] lambda at l_start and l_start + 1
  int* lstart = nullptr;       // [lmax+1][nrp] first significant l per (m, ring)
  int* lstart_blk = nullptr;   // [lmax+1][nrp/64 rounded up] block minimum of lstart
  double* qw64 = nullptr;      // [P][lmax+1] q_p(l) / sqrt(C_l)
  float* qw32 = nullptr;
  double* tw64 = nullptr;      // [nphi][2] exp(2 pi i t / nphi)
  float* tw32 = nullptr;
  float* twp32 = nullptr;      // [K - 1][2] per-pass twiddles of the register-pass ring FFT
  int* pair_a = nullptr;       // [npairs] first mode of each pair
  int* pair_b = nullptr;       // [npairs] second mode
  int* tri = nullptr;          // [nmax][6] p, r, s, pair(pr), pair(ps), pair(rs)
  int* quad = nullptr;         // [nquad][6] pair indices of the three pairings (pr|su), (ps|ru), (pu|rs)
  int nquad = 0;
  int2* qtiles = nullptr;      // tile pairs (ti <= tj) of the pairs x pairs update
  int4* zrows = nullptr;       // [nzrows] ideal-covariance rows: (p, r, s, mode), runs of equal (p, r)
  int nzrows = 0;              //   padded to multiples of 4 with (p, r, r, -1)
  int* pair_of = nullptr;      // [P][P] pair index of (min, max)
  int* tri_of = nullptr;       // [P][npairs] triple index of sort(u, a, b)
  int* tri_mult = nullptr;     // [P][npairs] multiplicity of u in that triple
  int* flag = nullptr;         // [4] device status words (Cholesky pivot)
  int2* items = nullptr;       // [nitems] (first slot, window base s0) work items of the split contraction
  int nitems = 0;
  int4* cslot = nullptr;       // [ncslot] (a0, b0, zlo, zhi) blocks of the split contraction's items, 32 per item
  int ncslot = 0;
  int cmult = 1;               // waves per item of the split contraction (1, 2, 4 or 8)
  int* cell = nullptr;         // [nmax] pair * P + mode of the partial-sum cell holding beta_n (split contraction)
  int* cell_order = nullptr;   // [nmax] the triples sorted by their cell
  float* mscale = nullptr;     // [P] exact powers of two ~ 1/sigma_p (split-fp16 contraction)
  uint4* lamtab = nullptr;     // split synthesis: lambda operand words per (m, wave of rings, chunk)
  long long* lamtab_off = nullptr;   // [lmax+1] first record of each m
};

}  // namespace modal

struct modal_ctx {
  int lmax = 0, ntheta = 0, nphi = 0, P = 0, prec = 0;
  int nalm = 0, npairs = 0, nmax = 0, nrp = 0, npix = 0;
  int device = 0;
  size_t max_lds = 65536;
  bool legendre_mfma = false;   // MFMA synthesis enabled (F32 / BF16X3 when the LDS fits)
  // tuned launch parameters (modal_autotune); 0 = default
  int tune_chunk_px = 0;        // pixels per split-K chunk of the MFMA contraction target
  int tune_fft_rings = 0;       // rings per FFT workgroup
  float wscale = 1.f;           // power of two ~ npix / 4pi (split-fp16 contraction)
  modal::FftPlan fft{};
  bool fft_rg = false;          // register-pass ring FFTs (float maps, radices 24/8/4/2/3/5; 47 x 8 x 8 at K 3008)
  modal::FftPlan fft_rg_plan{};
  modal::Tables t{};
  std::vector<double> x_host, wgl_host;
  std::vector<double> q_host, cl_host;   // the mode functions and filter spectrum given at creation
  std::vector<double> mu_host, wmu_host; // Gauss-Legendre rule of the 1-D Legendre integrals (on first use)
  std::string last_error;
  // per-stage timing (modal_profile_enable)
  bool profile = false;
  struct Mark { int stage; hipEvent_t a, b; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> event_pool;
  // second stream and events of the Cholesky's look-ahead (created on first use)
  hipStream_t side = nullptr;
  hipEvent_t ev_a = nullptr, ev_p = nullptr;
  double stage_ms[MODAL_NSTAGES] = {};
  long long stage_n[MODAL_NSTAGES] = {};
  // linear-term state bookkeeping (the device state holds the pair planes)
  const void* lin_state = nullptr;
  long long lin_count = 0;
  bool lin_final = false;
};

namespace modal {

// Layout of the synthesis output F (complex per (sequence, ring, m)): rings are
// grouped by eight, [seq][ring / 8][m][ring % 8], so that the ring FFT of a group
// reads one contiguous block and the synthesis writes 64-byte runs of rings.
__host__ __device__ inline int f_ring_blocks(int ntheta) { return (ntheta + 7) / 8; }
__host__ __device__ inline size_t f_index(int seq, int ring, int m, int lmax, int nrb8) {
  return (((size_t)seq * nrb8 + (ring >> 3)) * (size_t)(lmax + 1) + m) * 8 + (ring & 7);
}

// Workgroup barrier that orders LDS only: this wave's LDS operations complete, then all
// waves meet.  Unlike __syncthreads() it does not wait for outstanding global stores,
// for loops whose workgroup never reads back what it stored.  The memory clobber keeps
// the compiler from moving memory operations across it.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ---- launchers (defined in the .hip files); all return hipSuccess or the error
hipError_t launch_seeds(const modal_ctx* c, const double* logpref, hipStream_t st);

// Legendre synthesis: F (f_index layout) complex, double2 for F64, float2 otherwise
hipError_t launch_legendre(const modal_ctx* c, const void* alm, int S, void* F, hipStream_t st);
hipError_t launch_legendre_mfma(const modal_ctx* c, const void* alm, int S, void* F, hipStream_t st);
// split bf16/fp16 synthesis on 32x32 tiles, lambda in registers (k_legendre_split.hip)
hipError_t launch_legendre_split(const modal_ctx* c, const void* alm, int S, void* F, hipStream_t st);
size_t legendre_split_lds();
hipError_t legendre_split_set_lds(size_t bytes);
// the split synthesis's lambda table (built once per context when it fits)
size_t lambda_table_records(const modal_ctx* c, std::vector<long long>* off);
size_t lambda_table_bytes(const modal_ctx* c);
hipError_t build_lambda_table(modal_ctx* c, hipStream_t st);
size_t legendre_mfma_lds(const modal_ctx* c);
hipError_t legendre_mfma_set_lds(size_t bytes);
// ring c2r FFT: maps[S][P][ntheta][nphi] from F
hipError_t launch_fft_c2r(const modal_ctx* c, const void* F, int S, void* maps, hipStream_t st);
// ring r2c FFT: Gh[S][P][lmax+1][ntheta] complex from G[S][P][ntheta][nphi]
hipError_t launch_fft_r2c(const modal_ctx* c, const void* G, int S, void* Gh, hipStream_t st);
hipError_t launch_fft_r2c_rows(const modal_ctx* c, const void* G, size_t nseq, void* Gh, hipStream_t st);
int fft_rings_per_block(const modal_ctx* c);
bool fft_plan_rg(int N, FftPlan& p);
std::vector<float> fft_rg_twiddles(const FftPlan& p);
size_t fft_rg_lds(const modal_ctx* c);
hipError_t fft_rg_set_lds(size_t bytes);
int fft_rings_max(const modal_ctx* c);
int chunk_target_default(const modal_ctx* c);
int chunk_target_min(const modal_ctx* c);

// Fisher covariance from pair adjoints
hipError_t launch_pair_maps(const modal_ctx* c, const void* maps, const void* V, void* G, hipStream_t st);
hipError_t launch_adj_legendre_cols(const modal_ctx* c, const void* lam, const void* Gh, int ncol, void* Z,
                                    hipStream_t st);
hipError_t launch_cross_spectra(const modal_ctx* c, const void* Z, const double* cvar, double* X, hipStream_t st);
hipError_t launch_fisher_assemble(const modal_ctx* c, const double* X, double scale, double* F, hipStream_t st);

// cubic pixel reduction E_(ab),t = sum_x w M_a M_b M_t into
// partials[S][nchunk][npairs][P] float64 (VALU FP64 path / matrix-core paths)
int cubic_nchunk(const modal_ctx* c);
hipError_t launch_cubic_valu(const modal_ctx* c, const void* maps, int S, double* partials, hipStream_t st);
bool cubic_mfma_available(const modal_ctx* c);
int cubic_mfma_nchunk(const modal_ctx* c);
int cubic_mfma_nchunk_max(const modal_ctx* c);
// out[S][nmax] = scale (three pairings of the chunk sum of partials) + scale2 (three
// pairings of E2[S][npairs][P]); partials or E2 may be null
hipError_t launch_reduce_symm(const modal_ctx* c, const double* partials, int S, int nchunk, double scale,
                              double* E, const double* E2, double scale2, double* out, hipStream_t st);
// matrix-core contraction on 32x32 tiles (k_cubic_split.hip; FP32 and split contexts): work
// items of 32 blocks of 2 x 2 pairs against a 32-mode window, over a cover of the triples by
// (block, window) cells; make_cubic_cover builds it (false if the plan fails)
bool make_cubic_cover(int P, const std::vector<int>& pair_of, std::vector<int4>& slots, std::vector<int2>& items,
                      std::vector<int>& cell, int* mult);
size_t cubic_split_lds();
hipError_t cubic_split_set_lds(size_t bytes);
hipError_t launch_cubic_split(const modal_ctx* c, const void* maps, int S, int nchunk, int chunk_px, double* part,
                              hipStream_t st);
int cubic_chunk_px(const modal_ctx* c);
// out[S][nmax] = sum over chunks of part at (pair(pr), s) + scale2 (three pairings of E2)
hipError_t launch_reduce_single(const modal_ctx* c, const double* part, int S, int nchunk, double scale,
                                const double* E2, double scale2, double* out, hipStream_t st);
// linear term from the harmonic pair means Z[npairs][nalm] (k_lin_harm.hip):
// X[S][npairs][lmax+1] scratch, L[S][npairs][P] = sum_x w V_ab M^s_t
hipError_t launch_weight_planes(const modal_ctx* c, const void* V, int nk, void* G, hipStream_t st);
hipError_t launch_lin_harmonic(const modal_ctx* c, const void* Z, const void* alm, int S, double* X, double* L,
                               hipStream_t st);

// linear term accumulator
hipError_t launch_lin_accumulate(const modal_ctx* c, const void* maps, int S, void* U, hipStream_t st);
hipError_t launch_lin_scale(const modal_ctx* c, void* U, double s, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// adjoint
hipError_t launch_slot_matrix(const modal_ctx* c, const double* cot, int S, void* K, hipStream_t st);
// workspace of launch_pair_adjoint (the split operands of the slot coefficients; 0 when unused)
size_t pair_adjoint_ws_bytes(const modal_ctx* c, int S);
hipError_t launch_pair_adjoint(const modal_ctx* c, const void* maps, const void* K, int S, void* G, void* ws,
                               hipStream_t st);
hipError_t launch_lin_vjp(const modal_ctx* c, const double* K, const void* Z, int S, void* H, void* grad,
                          hipStream_t st);
hipError_t launch_lambda_table(const modal_ctx* c, void* lam, hipStream_t st);
hipError_t launch_adj_combine(const modal_ctx* c, const void* Z, int S, void* grad, hipStream_t st);

// FP64 dense linear algebra
hipError_t launch_syrk(int n, int N, const double* B, double scale, double* Z, hipStream_t st);
hipError_t launch_center_rows(int n, int N, const double* B, double* C, hipStream_t st);
hipError_t launch_copy_lower(int n, const double* src, double* dst, hipStream_t st);
// in-place Cholesky of the lower triangle of A (row-major, n x n); flag[0] = 1 + first bad pivot
// blocked right-looking Cholesky with look-ahead: the next diagonal block and panel run on
// side while the rest of the trailing update runs on st (ev_a, ev_p order them); st is
// joined with side when it returns.  With nrhs > 0 the solves L Y = B of nrhs right-hand
// sides stored as rows of B [nrhs][n] run too, each block's step right after the block is
// factored (the inverted diagonal block and its panel); Y gets the solution, B is
// overwritten below the blocks
hipError_t launch_cholesky_lookahead(int n, double* A, int* flag, hipStream_t st, hipStream_t side, hipEvent_t ev_a,
                                     hipEvent_t ev_p, int nrhs = 0, double* B = nullptr, double* Y = nullptr);
// solve L Y = B in place for nrhs right-hand sides stored as rows of B [nrhs][n]
hipError_t launch_trsm_rows(int n, const double* L, int nrhs, double* B, hipStream_t st);
hipError_t launch_estimator(int n, const double* y, const double* Z, int S, double* out, hipStream_t st);

// low-rank covariance I + sum b b^T: noise vectors, Woodbury estimator, closed-form rotation
size_t noise_ws_bytes(int N);
int noise_block_max();
hipError_t launch_noise_vectors(int N, int n, int k, int iters, const double* B, double* bt, double* ws,
                                double* mu_dev, hipStream_t st);
size_t lowrank_ws_bytes(int S);
hipError_t launch_fnl_lowrank(int n, int k, const double* bt, const double* alpha, const double* beta, int S,
                              double* ws, double* out, hipStream_t st);
hipError_t launch_bivector_rotate(int n, const double* b, const double* x, int R, double* y, hipStream_t st);

// theory mode coefficients of separable shapes and the ideal covariance (1-D Legendre integrals)
int shapes_nmu(int lmax);
hipError_t launch_legendre_series(int L, int nmu, int P, int nf, const double* U, const double* B, const double* mu,
                                  double* F, hipStream_t st);
hipError_t launch_alpha_modes(int nmax, int P, int T, int nmu, const int* tri, const double* F, const double* wmu,
                              double* alpha, hipStream_t st);
hipError_t launch_ideal_cov(int nmax, int P, int nmu, int nrows, const int4* zrows, const double* F,
                            const double* wmu, double* Z, hipStream_t st);

// truncated orthonormal frame: pivoted, truncated Cholesky (k_frame.hip)
size_t frame_ws_bytes(int n);
hipError_t launch_frame(int n, const double* Z, double tol, int* perm, double* L11, int* k_host, void* ws,
                        hipStream_t st);
hipError_t launch_gather_cols(int n, int k, int R, const double* x, const int* perm, double* y, hipStream_t st);
hipError_t launch_gather_sym(int n, int k, const double* Z, const int* perm, double* Zk, hipStream_t st);

// modal trispectrum (pairs x pairs update over pixels)
int quad_chunks(int npix);
int quad_ntile(int R);
size_t quad_part_bytes(const modal_ctx* c, int S);
size_t quad_vtile_bytes(const modal_ctx* c);
hipError_t launch_quad_vtile(const modal_ctx* c, const void* V, int rows, int batch, float* Vt, hipStream_t st);
size_t quad_mtile_bytes(const modal_ctx* c, int S);
hipError_t launch_quad_syrk(const modal_ctx* c, const void* maps, const void* V, int S, int vmode, const int2* tpairs,
                            float* part, double* K, hipStream_t st);
hipError_t launch_quad_gather(const modal_ctx* c, int nquad, int S, const int* quad, const double* K, const double* KVV,
                              double* tau, hipStream_t st);

// modal power spectrum (quadratic pixel reduction)
int power_chunk_px();
size_t power_part_bytes(int P, int npix, int S);
size_t power_lds(int P, bool f64);
hipError_t power_set_lds();
hipError_t launch_power_beta(const modal_ctx* c, const void* maps, int S, const void* zstate, double* part,
                             double* beta, hipStream_t st);
hipError_t launch_power_alpha(const modal_ctx* c, const double* dcl, double* alpha, hipStream_t st);
hipError_t launch_power_rows(const modal_ctx* c, const double* q, const double* cw, double* X, hipStream_t st);

// helpers
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
inline bool is_f64(const modal_ctx* c) { return c->prec == MODAL_F64; }
inline size_t real_bytes(const modal_ctx* c) { return is_f64(c) ? 8 : 4; }

}  // namespace modal
