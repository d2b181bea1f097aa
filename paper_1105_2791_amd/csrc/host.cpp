// Host side of libmodal: context construction (FP64 tables), validation,
// workspace carving and the extern "C" entry points declared in include/modal.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"

namespace modal {
hipError_t fft_set_lds_limit(size_t bytes);
}  // namespace modal

// Workspace of modal_beta_noalloc: a fixed device array (one copy per GPU, alive until
// the process ends).  In host code the symbol is only a stand-in, never a device
// address: its address on each device comes from hipGetSymbolAddress, resolved once
// per device with that device current (modal_create), and only that address is used.
static __device__ __align__(256) unsigned char scratch[MODAL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of the scratch array (resolved on first use).
hipError_t scratch_resolve(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = p;
  return hipSuccess;
}

void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}
}  // namespace

using namespace modal;

namespace {

const double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes (descending) and weights by Newton iteration on P_n, carried out
// in x87 extended precision: the weights 2 / ((1 - z^2) P_n'(z)^2) near the poles lose
// about n^2 ulps when P_n' is evaluated at a node rounded to double (3.7e-11 relative
// at n = 1501 in double, below the double rounding in extended precision).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  typedef long double R;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const R pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    R z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
    R pp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      R p1 = 1.0L, p2 = 0.0L;
      for (int j = 1; j <= n; ++j) {
        const R p3 = p2;
        p2 = p1;
        p1 = ((2.0L * j - 1.0L) * z * p2 - (j - 1.0L) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0L);
      const R z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-19L) {
        // one more evaluation of the derivative at the converged node
        p1 = 1.0L;
        p2 = 0.0L;
        for (int j = 1; j <= n; ++j) {
          const R p3 = p2;
          p2 = p1;
          p1 = ((2.0L * j - 1.0L) * z * p2 - (j - 1.0L) * p3) / j;
        }
        pp = n * (z * p1 - p2) / (z * z - 1.0L);
        break;
      }
    }
    x[i] = (double)z;
    x[n - 1 - i] = -(double)z;
    w[i] = w[n - 1 - i] = (double)(2.0L / ((1.0L - z * z) * pp * pp));
  }
  if (n & 1) x[n / 2] = 0.0;
}

bool fft_plan(int N, FftPlan& p) {
  p.N = N;
  p.K = N / 2;
  p.nf = 0;
  int K = p.K;
  auto push = [&](int r) {
    if (p.nf >= kMaxFactors) return false;
    p.radix[p.nf++] = r;
    return true;
  };
  while (K % 4 == 0) { if (!push(4)) return false; K /= 4; }
  while (K % 2 == 0) { if (!push(2)) return false; K /= 2; }
  for (int r = 3; K > 1; r += 2) {
    while (K % r == 0) { if (!push(r)) return false; K /= r; }
    if (r > 4096) return false;
  }
  return true;
}

struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    void* p = base ? base + used : nullptr;
    used += align256(bytes);
    return p;
  }
};

modal_status fail(modal_ctx* c, modal_status s, const std::string& msg) {
  if (c) c->last_error = msg;
  return s;
}

#define HIPTRY(expr)                                                                         \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(c, MODAL_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));      \
  } while (0)

size_t alm_bytes(const modal_ctx* c) { return (size_t)c->nalm * 2 * real_bytes(c); }
// synthesis output (f_index layout; also large enough for the adjoint's [S][P][lmax+1][ntheta])
size_t F_bytes(const modal_ctx* c, int S) {
  return (size_t)S * c->P * f_ring_blocks(c->ntheta) * 8 * (c->lmax + 1) * 2 * real_bytes(c);
}
size_t maps_bytes(const modal_ctx* c, int S) { return (size_t)S * c->P * c->npix * real_bytes(c); }
int nchunk_for(const modal_ctx* c) { return cubic_mfma_available(c) ? cubic_mfma_nchunk(c) : cubic_nchunk(c); }
// sized for the smallest chunk the autotuner may choose, so a workspace stays valid after tuning
size_t part_bytes(const modal_ctx* c, int S) {
  const int nc = cubic_mfma_available(c) ? cubic_mfma_nchunk_max(c) : cubic_nchunk(c);
  return (size_t)S * nc * c->npairs * c->P * 8;
}
size_t E_bytes(const modal_ctx* c, int S) { return (size_t)S * c->npairs * c->P * 8; }
size_t X_bytes(const modal_ctx* c, int S) { return (size_t)S * c->npairs * (c->lmax + 1) * 8; }
size_t lam_bytes(const modal_ctx* c) { return (size_t)c->nalm * c->nrp * real_bytes(c); }
// linear-term state: pixel pair means V[npairs][npix], then their weighted adjoint
// transforms Z[npairs][nalm] (complex, alm dtype)
size_t lin_V_bytes(const modal_ctx* c) { return align256((size_t)c->npairs * c->npix * real_bytes(c)); }
size_t lin_Z_bytes(const modal_ctx* c) { return align256((size_t)c->npairs * c->nalm * 2 * real_bytes(c)); }
const void* lin_Z(const modal_ctx* c, const void* state) { return (const char*)state + lin_V_bytes(c); }
// pair planes transformed per pass when a state is finalised
int fin_chunk(const modal_ctx* c) { return std::min(c->npairs, 64); }

size_t ws_size(const modal_ctx* c, int op, int S) {
  Carver cv(nullptr);
  switch (op) {
    case MODAL_OP_FILTER_MAPS: cv.take(F_bytes(c, S)); break;
    case MODAL_OP_BETA:
    case MODAL_OP_BETA_LOO:
      cv.take(F_bytes(c, S)); cv.take(maps_bytes(c, S)); cv.take(part_bytes(c, S)); cv.take(E_bytes(c, S));
      cv.take(X_bytes(c, S)); cv.take(E_bytes(c, S));
      break;
    case MODAL_OP_LINEAR_APPLY: cv.take(X_bytes(c, S)); cv.take(E_bytes(c, S)); break;
    case MODAL_OP_LINEAR_FINALIZE:
      cv.take(lam_bytes(c)); cv.take((size_t)fin_chunk(c) * c->npix * real_bytes(c));
      cv.take((size_t)fin_chunk(c) * c->ntheta * (c->lmax + 1) * 2 * real_bytes(c));
      break;
    case MODAL_OP_LINEAR_ACCUMULATE: cv.take(F_bytes(c, S)); cv.take(maps_bytes(c, S)); break;
    case MODAL_OP_BETA_VJP:
      cv.take(F_bytes(c, S)); cv.take(maps_bytes(c, S)); cv.take((size_t)S * c->P * c->npairs * 8);
      cv.take(maps_bytes(c, S)); cv.take(F_bytes(c, S)); cv.take(lam_bytes(c));
      cv.take((size_t)S * c->P * alm_bytes(c)); cv.take((size_t)S * c->npairs * (c->lmax + 1) * real_bytes(c));
      cv.take(pair_adjoint_ws_bytes(c, S));
      break;
    case MODAL_OP_COVARIANCE_SAMPLE: cv.take(256); break;
    case MODAL_OP_COVARIANCE_CENTERED: cv.take((size_t)S * c->nmax * 8); break;
    case MODAL_OP_COVARIANCE_FISHER:
      cv.take(F_bytes(c, 1)); cv.take(maps_bytes(c, 1)); cv.take((size_t)c->npairs * c->npix * real_bytes(c));
      cv.take((size_t)c->npairs * c->ntheta * (c->lmax + 1) * 2 * real_bytes(c)); cv.take(lam_bytes(c));
      cv.take((size_t)c->npairs * c->nalm * 2 * real_bytes(c));
      cv.take((size_t)(c->lmax + 1) * c->npairs * c->npairs * 8); cv.take((size_t)(c->lmax + 1) * 8);
      break;
    case MODAL_OP_FNL:
      cv.take((size_t)c->nmax * c->nmax * 8); cv.take((size_t)(S + 1) * c->nmax * 8); cv.take((size_t)(S + 1) * 8);
      cv.take(16); cv.take((size_t)(S + 1) * c->nmax * 8);
      break;
    case MODAL_OP_NOISE_VECTORS: cv.take(noise_ws_bytes(S)); break;
    case MODAL_OP_FNL_LOWRANK: cv.take(lowrank_ws_bytes(S)); break;
    case MODAL_OP_ALPHA_SEPARABLE: {
      const size_t nmu = shapes_nmu(c->lmax), L = c->lmax + 1;
      cv.take(nmu * 8); cv.take(nmu * 8); cv.take(3 * (size_t)S * L * 8); cv.take(3 * (size_t)S * nmu * c->P * 8);
      break;
    }
    case MODAL_OP_POWER_BETA:
      cv.take(F_bytes(c, S)); cv.take(maps_bytes(c, S)); cv.take(power_part_bytes(c->P, c->npix, S));
      break;
    case MODAL_OP_POWER_ALPHA: cv.take((size_t)(c->lmax + 1) * 8); break;
    case MODAL_OP_TRISPECTRUM:
      cv.take(F_bytes(c, S)); cv.take(maps_bytes(c, S)); cv.take(quad_part_bytes(c, S > 0 ? S : 1));
      cv.take((size_t)S * c->npairs * c->npairs * 8); cv.take((size_t)c->npairs * c->npairs * 8);
      cv.take(quad_vtile_bytes(c)); cv.take(quad_mtile_bytes(c, S));
      break;
    case MODAL_OP_POWER_COVARIANCE:
      cv.take((size_t)c->P * (c->lmax + 1) * 8); cv.take((size_t)(c->lmax + 1) * 8);
      cv.take((size_t)(c->lmax + 1) * c->P * 8);
      break;
    case MODAL_OP_POWER_FNL:
      cv.take((size_t)c->P * c->P * 8); cv.take((size_t)(S + 1) * c->P * 8); cv.take((size_t)(S + 1) * 8);
      cv.take(16); cv.take((size_t)(S + 1) * c->P * 8);
      break;
    case MODAL_OP_FRAME: cv.take(frame_ws_bytes(c->nmax)); break;
    case MODAL_OP_FNL_FRAME:
      cv.take((size_t)c->nmax * c->nmax * 8); cv.take((size_t)(S + 1) * c->nmax * 8);
      cv.take((size_t)c->nmax * c->nmax * 8); cv.take((size_t)(S + 1) * c->nmax * 8); cv.take((size_t)(S + 1) * 8);
      cv.take(16); cv.take((size_t)(S + 1) * c->nmax * 8);
      break;
    case MODAL_OP_IDEAL_COVARIANCE: {
      const size_t nmu = shapes_nmu(c->lmax), L = c->lmax + 1;
      cv.take(nmu * 8); cv.take(nmu * 8); cv.take((size_t)c->P * L * 8); cv.take((size_t)c->P * L * 8);
      cv.take((size_t)c->P * nmu * c->P * 8);
      break;
    }
    default: return 0;
  }
  return cv.used;
}

modal_status check_ws(modal_ctx* c, int op, int S, void* ws, size_t ws_bytes) {
  const size_t need = ws_size(c, op, S);
  if (need > 0 && !ws) return fail(c, MODAL_EINVAL, "workspace pointer is NULL");
  if (ws_bytes < need)
    return fail(c, MODAL_ENOSPACE, "workspace too small: need " + std::to_string(need) + " bytes, got " +
                                       std::to_string(ws_bytes));
  return MODAL_OK;
}

modal_status set_device(modal_ctx* c) {
  int cur = -1;
  HIPTRY(hipGetDevice(&cur));
  if (cur != c->device) HIPTRY(hipSetDevice(c->device));
  return MODAL_OK;
}

// Brackets one stage with HIP events when profiling is enabled.
struct StageTimer {
  modal_ctx* c;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  static hipEvent_t get(modal_ctx* c) {
    if (!c->event_pool.empty()) {
      hipEvent_t e = c->event_pool.back();
      c->event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  StageTimer(modal_ctx* c_, int stage_, hipStream_t st_) : c(c_), stage(stage_), st(st_) {
    if (!c->profile) return;
    a = get(c);
    if (a && hipEventRecord(a, st) != hipSuccess) {
      c->event_pool.push_back(a);
      a = nullptr;
    }
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = get(c);
    if (b && hipEventRecord(b, st) == hipSuccess) {
      c->marks.push_back({stage, a, b});
    } else {
      c->event_pool.push_back(a);
      if (b) c->event_pool.push_back(b);
    }
  }
};

#define STAGE(id, expr)                      \
  do {                                       \
    StageTimer _t(c, (id), st);              \
    HIPTRY(expr);                            \
  } while (0)

// Filter maps for S maps into 'maps' using F as scratch.
modal_status run_maps(modal_ctx* c, const void* alm, int S, void* F, void* maps, hipStream_t st) {
  if (c->prec == MODAL_BF16X3 || c->prec == MODAL_F16X3)
    STAGE(MODAL_STAGE_LEGENDRE, launch_legendre_split(c, alm, S, F, st));
  else if (c->legendre_mfma) STAGE(MODAL_STAGE_LEGENDRE, launch_legendre_mfma(c, alm, S, F, st));
  else STAGE(MODAL_STAGE_LEGENDRE, launch_legendre(c, alm, S, F, st));
  STAGE(MODAL_STAGE_FFT, launch_fft_c2r(c, F, S, maps, st));
  return MODAL_OK;
}

// beta (state == nullptr) or beta - lin for S maps: the cubic contraction over
// pixels, and the linear term from the state's harmonic pair means.
// out = sb beta + sl lin (lin from the state; sl = -1, sb = 1 gives beta^hat)
modal_status run_beta(modal_ctx* c, const void* maps, const void* alm, const void* state, int S, double* part,
                      double* E, double* X, double* L, double* out, hipStream_t st, double sb = 1.0,
                      double sl = -1.0) {
  // the matrix cores over the triple cover (split and FP32 contexts), the vector ALUs in FP64
  const bool split = cubic_mfma_available(c);
  if (split) STAGE(MODAL_STAGE_CUBIC, launch_cubic_split(c, maps, S, nchunk_for(c), cubic_chunk_px(c), part, st));
  else STAGE(MODAL_STAGE_CUBIC, launch_cubic_valu(c, maps, S, part, st));
  if (state) STAGE(MODAL_STAGE_LINEAR, launch_lin_harmonic(c, lin_Z(c, state), alm, S, X, L, st));
  if (split)
    STAGE(MODAL_STAGE_REDUCE, launch_reduce_single(c, part, S, nchunk_for(c), sb, state ? L : nullptr, sl, out, st));
  else
    STAGE(MODAL_STAGE_REDUCE,
          launch_reduce_symm(c, part, S, nchunk_for(c), sb / 3.0, E, state ? L : nullptr, sl, out, st));
  return MODAL_OK;
}

modal_status check_state(modal_ctx* c, const void* state) {
  if (state && (state != c->lin_state || !c->lin_final))
    return fail(c, MODAL_ENOTREADY, "linear-term state not finalised on this context");
  return MODAL_OK;
}

// Places every constant table of a context in the caller's device buffer (live) or only
// adds up its aligned size (dry: no HIP call at all).  Both modes run the same code, so the
// size query and the placement cannot disagree.
struct Placer {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool dry = true;
  template <typename V>
  hipError_t put(V** dst, const std::vector<V>& src) {   // device copy of a host vector
    const size_t bytes = align256(std::max<size_t>(1, src.size()) * sizeof(V));
    if (!dry) {
      if (used + bytes > cap) return hipErrorOutOfMemory;
      *dst = reinterpret_cast<V*>(base + used);
      if (!src.empty()) {
        const hipError_t e = hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice);
        if (e != hipSuccess) return e;
      }
    }
    used += bytes;
    return hipSuccess;
  }
  template <typename V>
  hipError_t take(V** dst, size_t count) {   // uninitialised region
    const size_t bytes = align256(std::max<size_t>(1, count) * sizeof(V));
    if (!dry) {
      if (used + bytes > cap) return hipErrorOutOfMemory;
      *dst = reinterpret_cast<V*>(base + used);
    }
    used += bytes;
    return hipSuccess;
  }
};

// LDS per workgroup assumed by the size query (gfx950); a live context uses the device's value.
constexpr size_t kGfx950Lds = 163840;

bool valid_shape_args(int lmax, int ntheta, int nphi, int P, int prec, modal_status* st) {
  if (lmax < 0 || P < 1 || P > kMaxP || prec < MODAL_F64 || prec > MODAL_F16X3) {
    *st = MODAL_EINVAL;
    return false;
  }
  if (ntheta <= lmax || nphi <= 2 * lmax || (nphi & 1) || ntheta < 1) {
    *st = MODAL_ESHAPE;
    return false;
  }
  return true;
}

void init_shapes(modal_ctx* c, int lmax, int ntheta, int nphi, int P, int prec) {
  c->lmax = lmax;
  c->ntheta = ntheta;
  c->nphi = nphi;
  c->P = P;
  c->prec = prec;
  c->nalm = (lmax + 1) * (lmax + 2) / 2;
  c->npairs = P * (P + 1) / 2;
  c->nmax = P * (P + 1) * (P + 2) / 6;
  c->nrp = (ntheta + 1) / 2;
  c->npix = ntheta * nphi;
}

// Kernel variants the context's shapes allow (host decisions from the LDS size); live also
// raises the kernels' dynamic-LDS limits.
modal_status choose_kernels(modal_ctx* c, bool live) {
  const int prec = c->prec;
  if ((prec == MODAL_BF16X3 || prec == MODAL_F16X3) && !cubic_mfma_available(c)) return MODAL_EUNSUPPORTED;
  if (!fft_plan(c->nphi, c->fft)) return MODAL_ESHAPE;
  const size_t fft_lds = (size_t)fft_rings_per_block(c) * 2 * c->fft.K * 2 * real_bytes(c);
  if (fft_lds > c->max_lds) return MODAL_EUNSUPPORTED;
  if (live && fft_lds > 65536 && fft_set_lds_limit(fft_lds) != hipSuccess) return MODAL_EDEVICE;
  c->fft_rg = false;
  if (prec != MODAL_F64 && fft_plan_rg(c->nphi, c->fft_rg_plan)) {
    const size_t rg = fft_rg_lds(c);
    if (rg <= c->max_lds) {
      if (live && rg > 65536 && fft_rg_set_lds(rg) != hipSuccess) return MODAL_EDEVICE;
      c->fft_rg = true;
    }
  }
  c->legendre_mfma = false;
  if (prec == MODAL_F32 || prec == MODAL_BF16X3 || prec == MODAL_F16X3) {
    if (prec != MODAL_F32) {
      const size_t lneed = legendre_split_lds();
      if (lneed + 1024 > c->max_lds) return MODAL_EUNSUPPORTED;
      if (live && lneed > 65536 && legendre_split_set_lds(lneed) != hipSuccess) return MODAL_EDEVICE;
      const size_t cneed = cubic_split_lds();
      if (cneed + 1024 > c->max_lds) return MODAL_EUNSUPPORTED;
      if (live && cneed > 65536 && cubic_split_set_lds(cneed) != hipSuccess) return MODAL_EDEVICE;
    }
    const size_t need = legendre_mfma_lds(c);
    if (need <= c->max_lds) {
      if (live && need > 65536 && legendre_mfma_set_lds(need) != hipSuccess) return MODAL_EDEVICE;
      c->legendre_mfma = true;
    }
  }
  return MODAL_OK;
}

// Host construction of every table and its placement (dry: sizes only).  Live, it also
// computes the recurrence seeds and, with MODAL_CTX_LAMBDA_TABLE, the lambda table.
modal_status place_tables(modal_ctx* c, const double* q_host, const double* cl_host, const double* mask_host,
                          unsigned flags, Placer& pl) {
  const int lmax = c->lmax, ntheta = c->ntheta, nphi = c->nphi, P = c->P, prec = c->prec;
  const bool live = !pl.dry;
  auto ok = [](hipError_t e) { return e == hipSuccess; };
  // --- grid
  gauss_legendre(ntheta, c->x_host, c->wgl_host);
  std::vector<double> ringw(ntheta), w64((size_t)ntheta * nphi);
  std::vector<float> w32((size_t)ntheta * nphi);
  for (int j = 0; j < ntheta; ++j) {
    ringw[j] = c->wgl_host[j] * 2.0 * kPi / nphi;
    for (int k = 0; k < nphi; ++k) {
      const size_t i = (size_t)j * nphi + k;
      w64[i] = ringw[j] * (mask_host ? mask_host[i] : 1.0);
      w32[i] = (float)w64[i];
    }
  }
  // --- recurrence coefficients and seed prefactors
  // zero entries past the last m let a 64-step chunk read past l = lmax without a clamp
  std::vector<double> rec(2 * ((size_t)c->nalm + kRecPad), 0.0), logpref(lmax + 1);
  double cum = 0.0;
  for (int m = 0; m <= lmax; ++m) {
    if (m > 0) cum += std::log((2.0 * m - 1.0) / (2.0 * m));
    logpref[m] = 0.5 * (std::log((2.0 * m + 1.0) / (4.0 * kPi)) + cum);
    const size_t off = (size_t)m * (2 * lmax + 3 - m) / 2;
    for (int l = m + 1; l <= lmax; ++l) {
      double A, B;
      if (l == m + 1) {
        A = std::sqrt(2.0 * m + 3.0);
        B = 0.0;
      } else {
        const double ll = l, mm = m;
        A = std::sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
        B = A * std::sqrt(((ll - 1.0) * (ll - 1.0) - mm * mm) / (4.0 * (ll - 1.0) * (ll - 1.0) - 1.0));
      }
      rec[2 * (off + (l - m))] = A;
      rec[2 * (off + (l - m)) + 1] = B;
    }
  }
  // --- whitened mode functions
  c->q_host.assign(q_host, q_host + (size_t)P * (lmax + 1));
  c->cl_host.assign(cl_host, cl_host + lmax + 1);
  std::vector<double> qw64((size_t)P * (lmax + 1));
  std::vector<float> qw32(qw64.size());
  for (int p = 0; p < P; ++p)
    for (int l = 0; l <= lmax; ++l) {
      const double cl = cl_host[l];
      const double v = cl > 0.0 ? q_host[(size_t)p * (lmax + 1) + l] / std::sqrt(cl) : 0.0;
      qw64[(size_t)p * (lmax + 1) + l] = v;
      qw32[(size_t)p * (lmax + 1) + l] = (float)v;
    }
  // --- twiddles
  std::vector<double> tw64(2 * (size_t)nphi);
  std::vector<float> tw32(2 * (size_t)nphi);
  for (int t = 0; t < nphi; ++t) {
    const double a = 2.0 * kPi * (double)t / (double)nphi;
    tw64[2 * t] = std::cos(a);
    tw64[2 * t + 1] = std::sin(a);
    tw32[2 * t] = (float)tw64[2 * t];
    tw32[2 * t + 1] = (float)tw64[2 * t + 1];
  }
  // --- pair / triple index tables
  std::vector<int> pa, pb, pair_of((size_t)P * P, -1), tri, tri_of((size_t)P * c->npairs), tri_mult((size_t)P * c->npairs);
  for (int p = 0; p < P; ++p)
    for (int r = p; r < P; ++r) {
      pair_of[(size_t)p * P + r] = pair_of[(size_t)r * P + p] = (int)pa.size();
      pa.push_back(p);
      pb.push_back(r);
    }
  std::vector<int> tri_index((size_t)P * P * P, -1);
  for (int p = 0; p < P; ++p)
    for (int r = p; r < P; ++r)
      for (int s = r; s < P; ++s) {
        tri_index[((size_t)p * P + r) * P + s] = (int)(tri.size() / 6);
        tri.insert(tri.end(), {p, r, s, pair_of[(size_t)p * P + r], pair_of[(size_t)p * P + s], pair_of[(size_t)r * P + s]});
      }
  for (int u = 0; u < P; ++u)
    for (int k = 0; k < c->npairs; ++k) {
      int v[3] = {u, pa[k], pb[k]};
      std::sort(v, v + 3);
      tri_of[(size_t)u * c->npairs + k] = tri_index[((size_t)v[0] * P + v[1]) * P + v[2]];
      tri_mult[(size_t)u * c->npairs + k] = (v[0] == u) + (v[1] == u) + (v[2] == u);
    }

  // trispectrum: quadruples p <= r <= s <= u with the pair indices of their three pairings,
  // and the tile pairs of the pairs x pairs update
  std::vector<int> quad;
  for (int p = 0; p < P; ++p)
    for (int r = p; r < P; ++r)
      for (int s2 = r; s2 < P; ++s2)
        for (int u = s2; u < P; ++u) {
          auto pr = [&](int a, int b) { return pair_of[(size_t)std::min(a, b) * P + std::max(a, b)]; };
          quad.insert(quad.end(), {pr(p, r), pr(s2, u), pr(p, s2), pr(r, u), pr(p, u), pr(r, s2)});
        }
  c->t.nquad = (int)(quad.size() / 6);
  // ideal-covariance rows: the modes in their order, each run of equal (p, r) padded to a
  // multiple of 4, so that every aligned group of four rows shares (p, r)
  std::vector<int4> zrows;
  for (int p = 0; p < P; ++p)
    for (int r = p; r < P; ++r) {
      for (int s = r; s < P; ++s) zrows.push_back(make_int4(p, r, s, tri_index[((size_t)p * P + r) * P + s]));
      while (zrows.size() % 4) zrows.push_back(make_int4(p, r, r, -1));
    }
  c->t.nzrows = (int)zrows.size();
  std::vector<int2> qtiles;
  {
    const int nt = quad_ntile(c->npairs);
    for (int ti = 0; ti < nt; ++ti)
      for (int tj = ti; tj < nt; ++tj) qtiles.push_back(make_int2(ti, tj));
  }

  // exact power-of-two scales for the split-fp16 contraction: whitened maps have
  // variance sigma_p^2 = sum_{C_l > 0} (2l+1)/(4 pi) q_p(l)^2
  std::vector<float> mscale(P, 1.f);
  for (int p = 0; p < P; ++p) {
    double v = 0.0;
    for (int l = 0; l <= lmax; ++l)
      if (cl_host[l] > 0.0) v += (2.0 * l + 1.0) / (4.0 * kPi) * q_host[(size_t)p * (lmax + 1) + l] * q_host[(size_t)p * (lmax + 1) + l];
    const int e = v > 0.0 ? (int)std::lround(0.5 * std::log2(v)) : 0;
    mscale[p] = (float)std::ldexp(1.0, -e);
  }
  c->wscale = (float)std::ldexp(1.0, (int)std::lround(std::log2((double)c->npix / (4.0 * kPi))));
  Tables& t = c->t;
  if (!ok(pl.put(&t.mscale, mscale))) return MODAL_EDEVICE;
  std::vector<int2> items;
  std::vector<int4> cslots;
  std::vector<int> cell;
  if (prec == MODAL_BF16X3 || prec == MODAL_F16X3 || prec == MODAL_F32) {
    if (!make_cubic_cover(P, pair_of, cslots, items, cell, &t.cmult))
      return fail(c, MODAL_EINVAL, "no cover of the triples by the contraction's items");
  }
  t.nitems = (int)items.size();
  t.ncslot = (int)cslots.size();
  std::vector<int> cell_order(cell.size());
  for (size_t n = 0; n < cell.size(); ++n) cell_order[n] = (int)n;
  std::sort(cell_order.begin(), cell_order.end(), [&](int x, int y) { return cell[x] < cell[y]; });
  if (!ok(pl.put(&t.items, items)) || !ok(pl.put(&t.cslot, cslots)) ||
      !ok(pl.put(&t.cell, cell)) || !ok(pl.put(&t.cell_order, cell_order)))
    return MODAL_EDEVICE;
  if (c->fft_rg && !ok(pl.put(&t.twp32, fft_rg_twiddles(c->fft_rg_plan)))) return MODAL_EDEVICE;
  std::vector<double> xs(c->x_host);
  if (!ok(pl.put(&t.x, xs)) || !ok(pl.put(&t.ringw, ringw)) || !ok(pl.put(&t.w64, w64)) || !ok(pl.put(&t.w32, w32)) ||
      !ok(pl.put(&t.rec, rec)) || !ok(pl.put(&t.qw64, qw64)) || !ok(pl.put(&t.qw32, qw32)) ||
      !ok(pl.put(&t.tw64, tw64)) || !ok(pl.put(&t.tw32, tw32)) || !ok(pl.put(&t.pair_a, pa)) ||
      !ok(pl.put(&t.pair_b, pb)) || !ok(pl.put(&t.tri, tri)) || !ok(pl.put(&t.pair_of, pair_of)) ||
      !ok(pl.put(&t.tri_of, tri_of)) || !ok(pl.put(&t.tri_mult, tri_mult)) || !ok(pl.put(&t.quad, quad)) ||
      !ok(pl.put(&t.qtiles, qtiles)) || !ok(pl.put(&t.zrows, zrows)))
    return MODAL_EDEVICE;
  if (!ok(pl.take(&t.seed, 2 * (size_t)(lmax + 1) * c->nrp)) || !ok(pl.take(&t.lstart, (size_t)(lmax + 1) * c->nrp)) ||
      !ok(pl.take(&t.flag, 4)))
    return MODAL_EDEVICE;
  double* d_logpref = nullptr;
  if (!ok(pl.put(&d_logpref, logpref))) return MODAL_EDEVICE;
  if (live) {
    hipError_t e = launch_seeds(c, d_logpref, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return MODAL_EDEVICE;
  }
  // split precisions: with MODAL_CTX_LAMBDA_TABLE the synthesis reads lambda from a table
  // computed here once, instead of running the recurrence for every block of columns
  if ((prec == MODAL_BF16X3 || prec == MODAL_F16X3) && (flags & MODAL_CTX_LAMBDA_TABLE)) {
    std::vector<long long> off;
    lambda_table_records(c, &off);
    if (!ok(pl.put(&t.lamtab_off, off)) || !ok(pl.take(&t.lamtab, lambda_table_bytes(c) / sizeof(uint4))))
      return MODAL_EDEVICE;
    if (live) {
      hipError_t e = build_lambda_table(c, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
      if (e != hipSuccess) return MODAL_EDEVICE;
    }
  }
  return MODAL_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char* modal_version(void) { return "libmodal 0.2 (gfx950)"; }

size_t modal_ctx_bytes(int lmax, int ntheta, int nphi, int P, int prec, unsigned flags) {
  modal_status st = MODAL_OK;
  if (!valid_shape_args(lmax, ntheta, nphi, P, prec, &st)) return 0;
  modal_ctx c;
  init_shapes(&c, lmax, ntheta, nphi, P, prec);
  c.max_lds = kGfx950Lds;
  if (choose_kernels(&c, false) != MODAL_OK) return 0;
  std::vector<double> q((size_t)P * (lmax + 1), 1.0), cl(lmax + 1, 1.0);
  Placer pl;
  if (place_tables(&c, q.data(), cl.data(), nullptr, flags, pl) != MODAL_OK) return 0;
  return pl.used;
}

modal_status modal_create(modal_ctx** out, int lmax, int ntheta, int nphi, int P, int prec, unsigned flags,
                          const double* q_host, const double* cl_host, const double* mask_host, void* tables_dev,
                          size_t table_bytes) {
  if (!out) return MODAL_EINVAL;
  *out = nullptr;
  modal_status st = MODAL_OK;
  if (!q_host || !cl_host) return MODAL_EINVAL;
  if (!valid_shape_args(lmax, ntheta, nphi, P, prec, &st)) return st;
  if (flags & ~(unsigned)MODAL_CTX_LAMBDA_TABLE) return MODAL_EINVAL;
  // the size the query reports for these arguments, checked before any device call
  const size_t need = modal_ctx_bytes(lmax, ntheta, nphi, P, prec, flags);
  if (need == 0) return MODAL_EUNSUPPORTED;
  if (!tables_dev) return MODAL_EINVAL;
  if (table_bytes < need) return MODAL_ENOSPACE;
  if (reinterpret_cast<uintptr_t>(tables_dev) % 256 != 0) return MODAL_EINVAL;
  modal_ctx* c = new (std::nothrow) modal_ctx();
  if (!c) return MODAL_EDEVICE;
  init_shapes(c, lmax, ntheta, nphi, P, prec);
  auto bail = [&](modal_status s) {
    modal_destroy(c);
    return s;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(MODAL_EDEVICE);
  if (scratch_resolve(c->device) != hipSuccess) return bail(MODAL_EDEVICE);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess && lds > 0)
    c->max_lds = (size_t)lds;
  if ((st = choose_kernels(c, true)) != MODAL_OK) return bail(st);
  Placer pl;
  pl.dry = false;
  pl.base = static_cast<char*>(tables_dev);
  pl.cap = table_bytes;
  if ((st = place_tables(c, q_host, cl_host, mask_host, flags, pl)) != MODAL_OK) return bail(st);
  *out = c;
  return MODAL_OK;
}

void modal_destroy(modal_ctx* c) {
  if (!c) return;
  for (auto& mk : c->marks) {
    (void)hipEventDestroy(mk.a);
    (void)hipEventDestroy(mk.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
    (void)hipEventDestroy(c->ev_a);
    (void)hipEventDestroy(c->ev_p);
  }
  delete c;   // the tables live in the caller's buffer
}

const char* modal_last_error(const modal_ctx* c) { return c ? c->last_error.c_str() : "null context"; }
int modal_nalm(const modal_ctx* c) { return c ? c->nalm : -1; }
int modal_nmax(const modal_ctx* c) { return c ? c->nmax : -1; }
int modal_nquad(const modal_ctx* c) { return c ? c->t.nquad : -1; }
int modal_npairs(const modal_ctx* c) { return c ? c->npairs : -1; }
int modal_cubic_path(const modal_ctx* c) {
  if (!c) return -1;
  if (!cubic_mfma_available(c)) return 0;
  return c->prec == MODAL_F32 ? 1 : 2;
}

int modal_cubic_plan(int P, int max_items, int* items_out, int* slots_out, int* cell_out, int* mult_out) {
  if (P < 1 || P > kMaxP) return -MODAL_EINVAL;
  std::vector<int> pair_of((size_t)P * P, -1);
  int np = 0;
  for (int p = 0; p < P; ++p)
    for (int r = p; r < P; ++r) pair_of[(size_t)p * P + r] = pair_of[(size_t)r * P + p] = np++;
  std::vector<int4> slots;
  std::vector<int2> items;
  std::vector<int> cell;
  int mult = 1;
  if (!make_cubic_cover(P, pair_of, slots, items, cell, &mult)) return -MODAL_EINVAL;
  const int n = (int)items.size();
  if (n > max_items) return -MODAL_EINVAL;
  for (int i = 0; i < n && items_out; ++i) {
    items_out[2 * i] = items[i].x;
    items_out[2 * i + 1] = items[i].y;
  }
  for (size_t i = 0; i < slots.size() && slots_out; ++i) {
    slots_out[4 * i] = slots[i].x;
    slots_out[4 * i + 1] = slots[i].y;
    slots_out[4 * i + 2] = slots[i].z;
    slots_out[4 * i + 3] = slots[i].w;
  }
  if (cell_out) std::copy(cell.begin(), cell.end(), cell_out);
  if (mult_out) *mult_out = mult;
  return n;
}

double modal_cubic_issued_macs(const modal_ctx* c) {
  if (!c) return 0.0;
  if (c->prec == MODAL_BF16X3 || c->prec == MODAL_F16X3) return (double)c->t.nitems * 32 * 4 * 32 * 3;
  if (c->prec == MODAL_F32 && cubic_mfma_available(c)) return (double)c->t.nitems * 32 * 4 * 32;
  return (double)c->npairs * c->P;
}

modal_status modal_grid(const modal_ctx* c, double* x_host, double* w_host) {
  if (!c) return MODAL_EINVAL;
  if (x_host) std::memcpy(x_host, c->x_host.data(), sizeof(double) * c->ntheta);
  if (w_host) std::memcpy(w_host, c->wgl_host.data(), sizeof(double) * c->ntheta);
  return MODAL_OK;
}

modal_status modal_workspace_size(const modal_ctx* c, int op, int S, size_t* bytes) {
  if (!c || !bytes || S < 0 || op < MODAL_OP_FILTER_MAPS || op > MODAL_OP_BETA_LOO) return MODAL_EINVAL;
  *bytes = ws_size(c, op, S);
  return MODAL_OK;
}

size_t modal_linear_state_size(const modal_ctx* c) { return c ? lin_V_bytes(c) + lin_Z_bytes(c) : 0; }

modal_status modal_filter_maps(modal_ctx* c, const void* alm, int S, void* maps, void* ws, size_t ws_bytes,
                               modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alm || !maps || S <= 0) return fail(c, MODAL_EINVAL, "filter_maps: null pointer or S <= 0");
  modal_status s = check_ws(c, MODAL_OP_FILTER_MAPS, S, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  Carver cv(ws);
  void* F = cv.take(F_bytes(c, S));
  return run_maps(c, alm, S, F, maps, (hipStream_t)stream);
}

modal_status modal_beta(modal_ctx* c, const void* alm, int S, const void* state, double* beta, void* ws,
                        size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alm || !beta || S <= 0) return fail(c, MODAL_EINVAL, "beta: null pointer or S <= 0");
  modal_status s = check_state(c, state);
  if (s != MODAL_OK) return s;
  if ((s = check_ws(c, MODAL_OP_BETA, S, ws, ws_bytes)) != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  Carver cv(ws);
  void* F = cv.take(F_bytes(c, S));
  void* maps = cv.take(maps_bytes(c, S));
  double* part = (double*)cv.take(part_bytes(c, S));
  double* E = (double*)cv.take(E_bytes(c, S));
  double* X = (double*)cv.take(X_bytes(c, S));
  double* L = (double*)cv.take(E_bytes(c, S));
  if ((s = run_maps(c, alm, S, F, maps, st)) != MODAL_OK) return s;
  return run_beta(c, maps, alm, state, S, part, E, X, L, beta, st);
}

modal_status modal_beta_loo(modal_ctx* c, const void* alm, int S, const void* state, double* beta, void* ws,
                            size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alm || !beta || S <= 0) return fail(c, MODAL_EINVAL, "beta_loo: null pointer or S <= 0");
  if (!state) return fail(c, MODAL_EINVAL, "beta_loo: needs the linear-term state");
  modal_status s = check_state(c, state);
  if (s != MODAL_OK) return s;
  const double N = (double)c->lin_count;
  if (c->lin_count < 2) return fail(c, MODAL_ENOTREADY, "beta_loo: the state holds fewer than 2 skies");
  if ((s = check_ws(c, MODAL_OP_BETA_LOO, S, ws, ws_bytes)) != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  Carver cv(ws);
  void* F = cv.take(F_bytes(c, S));
  void* maps = cv.take(maps_bytes(c, S));
  double* part = (double*)cv.take(part_bytes(c, S));
  double* E = (double*)cv.take(E_bytes(c, S));
  double* X = (double*)cv.take(X_bytes(c, S));
  double* L = (double*)cv.take(E_bytes(c, S));
  if ((s = run_maps(c, alm, S, F, maps, st)) != MODAL_OK) return s;
  // beta - (N lin - 3 beta) / (N - 1): the sky's own pair products removed from the mean
  return run_beta(c, maps, alm, state, S, part, E, X, L, beta, st, (N + 2.0) / (N - 1.0), -N / (N - 1.0));
}

modal_status modal_beta_noalloc(modal_ctx* c, const void* alm, int S, const void* state, double* beta,
                                modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alm || !beta || S <= 0) return fail(c, MODAL_EINVAL, "beta_noalloc: null pointer or S <= 0");
  modal_status s = check_state(c, state);
  if (s != MODAL_OK) return s;
  const size_t need = ws_size(c, MODAL_OP_BETA, S);
  if (need > (size_t)MODAL_NOALLOC_SCRATCH_BYTES)
    return fail(c, MODAL_ENOSPACE, "beta_noalloc: these shapes need " + std::to_string(need) +
                                       " bytes of workspace, the fixed scratch holds " +
                                       std::to_string((size_t)MODAL_NOALLOC_SCRATCH_BYTES) +
                                       " (call modal_beta with a caller workspace)");
  if ((s = set_device(c)) != MODAL_OK) return s;
  void* ws = scratch_ptr(c->device);
  if (!ws) return fail(c, MODAL_EDEVICE, "beta_noalloc: scratch address not resolved on this device");
  // stage timing would create events; it stays off for this call
  const bool prof = c->profile;
  c->profile = false;
  s = modal_beta(c, alm, S, state, beta, ws, (size_t)MODAL_NOALLOC_SCRATCH_BYTES, stream);
  c->profile = prof;
  return s;
}

modal_status modal_linear_term(modal_ctx* c, int mode, const void* alm, int S, void* state, double* lin, void* ws,
                               size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!state) return fail(c, MODAL_EINVAL, "linear_term: null state");
  modal_status s = set_device(c);
  if (s != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  switch (mode) {
    case MODAL_LIN_RESET:
      HIPTRY(launch_zero(state, modal_linear_state_size(c), st));
      c->lin_state = state;
      c->lin_count = 0;
      c->lin_final = false;
      return MODAL_OK;
    case MODAL_LIN_ACCUMULATE: {
      if (!alm || S <= 0) return fail(c, MODAL_EINVAL, "linear_term: null alm or S <= 0");
      if (state != c->lin_state || c->lin_final)
        return fail(c, MODAL_ENOTREADY, "linear_term: ACCUMULATE needs a state RESET on this context and not finalised");
      if ((s = check_ws(c, MODAL_OP_LINEAR_ACCUMULATE, S, ws, ws_bytes)) != MODAL_OK) return s;
      Carver cv(ws);
      void* F = cv.take(F_bytes(c, S));
      void* maps = cv.take(maps_bytes(c, S));
      if ((s = run_maps(c, alm, S, F, maps, st)) != MODAL_OK) return s;
      STAGE(MODAL_STAGE_LINACC, launch_lin_accumulate(c, maps, S, state, st));
      c->lin_count += S;
      return MODAL_OK;
    }
    case MODAL_LIN_FINALIZE: {
      if (state != c->lin_state || c->lin_final || c->lin_count <= 0)
        return fail(c, MODAL_ENOTREADY, "linear_term: FINALIZE needs an accumulated, unfinalised state");
      if ((s = check_ws(c, MODAL_OP_LINEAR_FINALIZE, 1, ws, ws_bytes)) != MODAL_OK) return s;
      HIPTRY(launch_lin_scale(c, state, 1.0 / (double)c->lin_count, st));
      // Z = c_m sum_j lambda_lm sum_k w V e^{-i m phi_k} for every pair plane
      Carver cv(ws);
      void* lam = cv.take(lam_bytes(c));
      const int nch = fin_chunk(c);
      void* G = cv.take((size_t)nch * c->npix * real_bytes(c));
      void* Gh = cv.take((size_t)nch * c->ntheta * (c->lmax + 1) * 2 * real_bytes(c));
      STAGE(MODAL_STAGE_ADJ_LEGENDRE, launch_lambda_table(c, lam, st));
      char* Z = (char*)state + lin_V_bytes(c);
      for (int p0 = 0; p0 < c->npairs; p0 += nch) {
        const int nk = std::min(nch, c->npairs - p0);
        const void* Vp = (const char*)state + (size_t)p0 * c->npix * real_bytes(c);
        STAGE(MODAL_STAGE_ADJ_PAIR, launch_weight_planes(c, Vp, nk, G, st));
        STAGE(MODAL_STAGE_ADJ_FFT, launch_fft_r2c_rows(c, G, (size_t)nk, Gh, st));
        STAGE(MODAL_STAGE_ADJ_LEGENDRE,
              launch_adj_legendre_cols(c, lam, Gh, nk, Z + (size_t)p0 * c->nalm * 2 * real_bytes(c), st));
      }
      c->lin_final = true;
      return MODAL_OK;
    }
    case MODAL_LIN_APPLY: {
      if (!alm || !lin || S <= 0) return fail(c, MODAL_EINVAL, "linear_term: APPLY needs alm, lin and S > 0");
      if ((s = check_state(c, state)) != MODAL_OK) return s;
      if ((s = check_ws(c, MODAL_OP_LINEAR_APPLY, S, ws, ws_bytes)) != MODAL_OK) return s;
      Carver cv(ws);
      double* X = (double*)cv.take(X_bytes(c, S));
      double* L = (double*)cv.take(E_bytes(c, S));
      STAGE(MODAL_STAGE_LINEAR, launch_lin_harmonic(c, lin_Z(c, state), alm, S, X, L, st));
      STAGE(MODAL_STAGE_REDUCE, launch_reduce_symm(c, nullptr, S, 0, 0.0, nullptr, L, 1.0, lin, st));
      return MODAL_OK;
    }
    default:
      return fail(c, MODAL_EINVAL, "linear_term: bad mode");
  }
}

modal_status modal_beta_vjp(modal_ctx* c, const void* alm, int S, const void* state, const double* cot, void* grad,
                            void* ws, size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alm || !cot || !grad || S <= 0) return fail(c, MODAL_EINVAL, "beta_vjp: null pointer or S <= 0");
  modal_status s = check_state(c, state);
  if (s != MODAL_OK) return s;
  if ((s = check_ws(c, MODAL_OP_BETA_VJP, S, ws, ws_bytes)) != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  Carver cv(ws);
  void* F = cv.take(F_bytes(c, S));
  void* maps = cv.take(maps_bytes(c, S));
  void* K = cv.take((size_t)S * c->P * c->npairs * 8);
  void* G = cv.take(maps_bytes(c, S));
  void* Gh = cv.take(F_bytes(c, S));
  void* lam = cv.take(lam_bytes(c));
  void* Zc = cv.take((size_t)S * c->P * alm_bytes(c));   // per (sky, mode) column
  void* H = cv.take((size_t)S * c->npairs * (c->lmax + 1) * real_bytes(c));
  void* Kw = cv.take(pair_adjoint_ws_bytes(c, S));
  if ((s = run_maps(c, alm, S, F, maps, st)) != MODAL_OK) return s;
  STAGE(MODAL_STAGE_ADJ_PAIR, launch_slot_matrix(c, cot, S, K, st));
  // the cubic part in pixel space; the pair-mean part is added in harmonic space below
  STAGE(MODAL_STAGE_ADJ_PAIR, launch_pair_adjoint(c, maps, K, S, G, Kw, st));
  STAGE(MODAL_STAGE_ADJ_FFT, launch_fft_r2c(c, G, S, Gh, st));
  STAGE(MODAL_STAGE_ADJ_LEGENDRE, launch_lambda_table(c, lam, st));
  STAGE(MODAL_STAGE_ADJ_LEGENDRE, launch_adj_legendre_cols(c, lam, Gh, S * c->P, Zc, st));
  STAGE(MODAL_STAGE_ADJ_LEGENDRE, launch_adj_combine(c, Zc, S, grad, st));
  if (state) STAGE(MODAL_STAGE_LINEAR, launch_lin_vjp(c, (const double*)K, lin_Z(c, state), S, H, grad, st));
  return MODAL_OK;
}

modal_status modal_covariance(modal_ctx* c, int method, const double* beta, const void* alm, const void* state,
                              const double* cvar_host, int N, double* zeta, void* ws, size_t ws_bytes,
                              modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!zeta || N <= 0) return fail(c, MODAL_EINVAL, "covariance: null zeta or N <= 0");
  modal_status s = set_device(c);
  if (s != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  if (method == MODAL_COV_SAMPLE) {
    if (!beta) return fail(c, MODAL_EINVAL, "covariance: SAMPLE needs beta");
    STAGE(MODAL_STAGE_COVARIANCE, launch_syrk(c->nmax, N, beta, 1.0 / (6.0 * N), zeta, st));
    return MODAL_OK;
  }
  if (method == MODAL_COV_SAMPLE_CENTERED) {
    if (!beta) return fail(c, MODAL_EINVAL, "covariance: SAMPLE_CENTERED needs beta");
    if (N < 2) return fail(c, MODAL_EINVAL, "covariance: SAMPLE_CENTERED needs N >= 2");
    if ((s = check_ws(c, MODAL_OP_COVARIANCE_CENTERED, N, ws, ws_bytes)) != MODAL_OK) return s;
    double* B = (double*)ws;
    STAGE(MODAL_STAGE_COVARIANCE, launch_center_rows(c->nmax, N, beta, B, st));
    STAGE(MODAL_STAGE_COVARIANCE, launch_syrk(c->nmax, N, B, 1.0 / (6.0 * (N - 1)), zeta, st));
    return MODAL_OK;
  }
  if (method == MODAL_COV_FISHER) {
    if (!alm || !cvar_host) return fail(c, MODAL_EINVAL, "covariance: FISHER needs alm and cvar");
    if ((s = check_state(c, state)) != MODAL_OK) return s;
    if ((s = check_ws(c, MODAL_OP_COVARIANCE_FISHER, N, ws, ws_bytes)) != MODAL_OK) return s;
    Carver cv(ws);
    void* F = cv.take(F_bytes(c, 1));
    void* maps = cv.take(maps_bytes(c, 1));
    void* G = cv.take((size_t)c->npairs * c->npix * real_bytes(c));
    void* Gh = cv.take((size_t)c->npairs * c->ntheta * (c->lmax + 1) * 2 * real_bytes(c));
    void* lam = cv.take(lam_bytes(c));
    void* Z = cv.take((size_t)c->npairs * c->nalm * 2 * real_bytes(c));
    const size_t xbytes = (size_t)(c->lmax + 1) * c->npairs * c->npairs * 8;
    double* X = (double*)cv.take(xbytes);
    double* cvar = (double*)cv.take((size_t)(c->lmax + 1) * 8);
    HIPTRY(hipMemcpyAsync(cvar, cvar_host, (size_t)(c->lmax + 1) * 8, hipMemcpyHostToDevice, st));
    HIPTRY(hipStreamSynchronize(st));   // cvar_host may be released on return
    HIPTRY(launch_zero(X, xbytes, st));
    STAGE(MODAL_STAGE_ADJ_LEGENDRE, launch_lambda_table(c, lam, st));
    const size_t abytes = alm_bytes(c);
    for (int i = 0; i < N; ++i) {
      const void* ai = (const char*)alm + (size_t)i * abytes;
      if ((s = run_maps(c, ai, 1, F, maps, st)) != MODAL_OK) return s;
      STAGE(MODAL_STAGE_ADJ_PAIR, launch_pair_maps(c, maps, state, G, st));
      STAGE(MODAL_STAGE_ADJ_FFT, launch_fft_r2c_rows(c, G, (size_t)c->npairs, Gh, st));
      STAGE(MODAL_STAGE_ADJ_LEGENDRE, launch_adj_legendre_cols(c, lam, Gh, c->npairs, Z, st));
      STAGE(MODAL_STAGE_COVARIANCE, launch_cross_spectra(c, Z, cvar, X, st));
    }
    STAGE(MODAL_STAGE_COVARIANCE, launch_fisher_assemble(c, X, 1.0 / (18.0 * N), zeta, st));
    return MODAL_OK;
  }
  return fail(c, MODAL_EINVAL, "covariance: bad method");
}

// Cholesky estimator for n modes: E_s = y.z_s / y.y, sigma^2 = factor / y.y (factor = 3! or 2!,
// the number of cross pairings of the legs).
modal_status estimate(modal_ctx* c, int op, int n, double factor, const double* zeta, const double* alpha,
                      const double* beta, int beta_stride, int S, double* E_host, double* sigma2_host, double* L_dev,
                      void* ws, size_t ws_bytes, hipStream_t st) {
  if (!zeta || !alpha || !sigma2_host || S < 0 || (S > 0 && (!beta || !E_host)))
    return fail(c, MODAL_EINVAL, "fnl: null pointer or S < 0");
  modal_status s = check_ws(c, op, S, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  Carver cv(ws);
  double* L = (double*)cv.take((size_t)n * n * 8);
  double* rows = (double*)cv.take((size_t)(S + 1) * n * 8);
  double* dots = (double*)cv.take((size_t)(S + 1) * 8);
  int* flag = (int*)cv.take(16);
  double* sol = (double*)cv.take((size_t)(S + 1) * n * 8);
  HIPTRY(launch_zero(flag, 16, st));
  HIPTRY(hipMemcpyAsync(L, zeta, (size_t)n * n * 8, hipMemcpyDeviceToDevice, st));
  HIPTRY(hipMemcpyAsync(rows, alpha, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
  if (S > 0)
    HIPTRY(hipMemcpy2DAsync(rows + n, (size_t)n * 8, beta, (size_t)beta_stride * 8, (size_t)n * 8, S,
                            hipMemcpyDeviceToDevice, st));
  {
    StageTimer _t(c, MODAL_STAGE_CHOLESKY, st);
    if (!c->side) {
      HIPTRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
      HIPTRY(hipEventCreateWithFlags(&c->ev_a, hipEventDisableTiming));
      HIPTRY(hipEventCreateWithFlags(&c->ev_p, hipEventDisableTiming));
    }
    // the factorization with the solves of the S + 1 right-hand sides folded in
    HIPTRY(launch_cholesky_lookahead(n, L, flag, st, c->side, c->ev_a, c->ev_p, S + 1, rows, sol));
    HIPTRY(launch_estimator(n, sol, nullptr, S, dots, st));
  }
  if (L_dev) HIPTRY(launch_copy_lower(n, L, L_dev, st));
  std::vector<double> h(S + 1);
  int hflag[4] = {0, 0, 0, 0};
  HIPTRY(hipMemcpyAsync(h.data(), dots, (size_t)(S + 1) * 8, hipMemcpyDeviceToHost, st));
  HIPTRY(hipMemcpyAsync(hflag, flag, 16, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  if (hflag[0] != 0)
    return fail(c, MODAL_ENOTPD, "fnl: zeta is not positive definite at pivot " + std::to_string(hflag[0] - 1));
  const double yy = h[0];
  *sigma2_host = factor / yy;
  for (int i = 0; i < S; ++i) E_host[i] = h[1 + i] / yy;
  return MODAL_OK;
}

modal_status modal_fnl(modal_ctx* c, const double* zeta, const double* alpha, const double* beta, int S,
                       double* E_host, double* sigma2_host, double* L_dev, void* ws, size_t ws_bytes,
                       modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  return estimate(c, MODAL_OP_FNL, c->nmax, 6.0, zeta, alpha, beta, c->nmax, S, E_host, sigma2_host, L_dev, ws,
                  ws_bytes, (hipStream_t)stream);
}

modal_status modal_power_beta(modal_ctx* c, const void* alm, int S, const void* state, double* beta, void* ws,
                              size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alm || !beta || S <= 0) return fail(c, MODAL_EINVAL, "power_beta: null pointer or S <= 0");
  modal_status s = check_state(c, state);
  if (s != MODAL_OK) return s;
  if ((s = check_ws(c, MODAL_OP_POWER_BETA, S, ws, ws_bytes)) != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  if (power_lds(c->P, is_f64(c)) > c->max_lds) return fail(c, MODAL_EUNSUPPORTED, "power_beta: LDS too small");
  HIPTRY(power_set_lds());
  hipStream_t st = (hipStream_t)stream;
  Carver cv(ws);
  void* F = cv.take(F_bytes(c, S));
  void* maps = cv.take(maps_bytes(c, S));
  double* part = (double*)cv.take(power_part_bytes(c->P, c->npix, S));
  if ((s = run_maps(c, alm, S, F, maps, st)) != MODAL_OK) return s;
  {
    StageTimer _t(c, MODAL_STAGE_CUBIC, st);
    HIPTRY(launch_power_beta(c, maps, S, state ? lin_Z(c, state) : nullptr, part, beta, st));
  }
  return MODAL_OK;
}

modal_status modal_trispectrum(modal_ctx* c, const void* alm, int S, const void* state, double* tau, void* ws,
                               size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alm || !tau || S <= 0) return fail(c, MODAL_EINVAL, "trispectrum: null pointer or S <= 0");
  if (c->prec == MODAL_F32)
    return fail(c, MODAL_EUNSUPPORTED,
                "trispectrum: no FP32 update (the float update is split-bf16 or split-fp16); use a MODAL_F64, "
                "MODAL_BF16X3 or MODAL_F16X3 context");
  modal_status s = check_state(c, state);
  if (s != MODAL_OK) return s;
  if ((s = check_ws(c, MODAL_OP_TRISPECTRUM, S, ws, ws_bytes)) != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const size_t R2 = (size_t)c->npairs * c->npairs;
  Carver cv(ws);
  void* F = cv.take(F_bytes(c, S));
  void* maps = cv.take(maps_bytes(c, S));
  float* part = (float*)cv.take(quad_part_bytes(c, S));
  double* K = (double*)cv.take((size_t)S * R2 * 8);
  double* KVV = (double*)cv.take(R2 * 8);
  float* Vt = (float*)cv.take(quad_vtile_bytes(c));
  float* Mt = (float*)cv.take(quad_mtile_bytes(c, S));
  if ((s = run_maps(c, alm, S, F, maps, st)) != MODAL_OK) return s;
  {
    StageTimer _t(c, MODAL_STAGE_CUBIC, st);
    // the V planes lead the state; float contexts read them and the maps through
    // pixel-block-major copies
    const void* V = state;
    const void* M = maps;
    if (c->prec != MODAL_F64) {
      if (state) {
        HIPTRY(launch_quad_vtile(c, state, c->npairs, 1, Vt, st));
        V = Vt;
      }
      HIPTRY(launch_quad_vtile(c, maps, c->P, S, Mt, st));
      M = Mt;
    }
    HIPTRY(launch_quad_syrk(c, M, V, S, 0, c->t.qtiles, part, K, st));
    if (state) HIPTRY(launch_quad_syrk(c, nullptr, V, 1, 1, c->t.qtiles, part, KVV, st));
  }
  {
    StageTimer _t(c, MODAL_STAGE_REDUCE, st);
    HIPTRY(launch_quad_gather(c, c->t.nquad, S, c->t.quad, K, state ? KVV : nullptr, tau, st));
  }
  return MODAL_OK;
}

modal_status modal_power_alpha(modal_ctx* c, const double* dcl, double* alpha, void* ws, size_t ws_bytes,
                               modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!dcl || !alpha) return fail(c, MODAL_EINVAL, "power_alpha: null pointer");
  modal_status s = check_ws(c, MODAL_OP_POWER_ALPHA, 0, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  double* d = (double*)ws;
  HIPTRY(hipMemcpyAsync(d, dcl, (size_t)(c->lmax + 1) * 8, hipMemcpyHostToDevice, st));
  HIPTRY(launch_power_alpha(c, d, alpha, st));
  HIPTRY(hipStreamSynchronize(st));
  return MODAL_OK;
}

modal_status modal_power_ideal_covariance(modal_ctx* c, const double* c_host, double* zeta, void* ws, size_t ws_bytes,
                                          modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!zeta) return fail(c, MODAL_EINVAL, "power_ideal_covariance: null pointer");
  modal_status s = check_ws(c, MODAL_OP_POWER_COVARIANCE, 0, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int L = c->lmax + 1;
  std::vector<double> cw(L);
  for (int l = 0; l < L; ++l) cw[l] = c_host ? c_host[l] : (c->cl_host[l] > 0.0 ? 1.0 : 0.0);
  Carver cv(ws);
  double* q = (double*)cv.take((size_t)c->P * L * 8);
  double* dc = (double*)cv.take((size_t)L * 8);
  double* X = (double*)cv.take((size_t)L * c->P * 8);
  HIPTRY(hipMemcpyAsync(q, c->q_host.data(), (size_t)c->P * L * 8, hipMemcpyHostToDevice, st));
  HIPTRY(hipMemcpyAsync(dc, cw.data(), (size_t)L * 8, hipMemcpyHostToDevice, st));
  {
    StageTimer _t(c, MODAL_STAGE_COVARIANCE, st);
    HIPTRY(launch_power_rows(c, q, dc, X, st));
    HIPTRY(launch_syrk(c->P, L, X, 1.0, zeta, st));
  }
  HIPTRY(hipStreamSynchronize(st));
  return MODAL_OK;
}

modal_status modal_power_fnl(modal_ctx* c, const double* zeta, const double* alpha, const double* beta, int S,
                             double* E_host, double* sigma2_host, void* ws, size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  return estimate(c, MODAL_OP_POWER_FNL, c->P, 2.0, zeta, alpha, beta, c->npairs, S, E_host, sigma2_host, nullptr,
                  ws, ws_bytes, (hipStream_t)stream);
}

modal_status modal_noise_vectors(modal_ctx* c, const double* beta, int N, int k, int iters, double* bt,
                                 double* mu_host, void* ws, size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!beta || !bt || !mu_host) return fail(c, MODAL_EINVAL, "noise_vectors: null pointer");
  const int n = c->nmax;
  if (N < 1 || iters < 1 || k < 1 || k > noise_block_max() || k > N || k > n)
    return fail(c, MODAL_EINVAL, "noise_vectors: need N >= 1, iters >= 1 and 1 <= k <= min(16, N, nmax)");
  modal_status s = check_ws(c, MODAL_OP_NOISE_VECTORS, N, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  double* mu_dev = (double*)((char*)ws + noise_ws_bytes(N) - align256((size_t)noise_block_max() * 8));
  {
    StageTimer _t(c, MODAL_STAGE_COVARIANCE, st);
    HIPTRY(launch_noise_vectors(N, n, k, iters, beta, bt, (double*)ws, mu_dev, st));
  }
  HIPTRY(hipMemcpyAsync(mu_host, mu_dev, (size_t)k * 8, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  return MODAL_OK;
}

modal_status modal_fnl_lowrank(modal_ctx* c, const double* bt, int k, const double* alpha, const double* beta, int S,
                               double* E_host, double* sigma2_host, void* ws, size_t ws_bytes,
                               modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!alpha || !sigma2_host || S < 0 || (S > 0 && (!beta || !E_host)) || (k > 0 && !bt))
    return fail(c, MODAL_EINVAL, "fnl_lowrank: null pointer or S < 0");
  if (k < 0 || k > noise_block_max()) return fail(c, MODAL_EINVAL, "fnl_lowrank: need 0 <= k <= 16");
  modal_status s = check_ws(c, MODAL_OP_FNL_LOWRANK, S, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  double* out = (double*)((char*)ws + align256((size_t)(S + 1 + noise_block_max()) * (noise_block_max() + 1) * 8));
  {
    StageTimer _t(c, MODAL_STAGE_CHOLESKY, st);
    HIPTRY(launch_fnl_lowrank(c->nmax, k, bt, alpha, beta, S, (double*)ws, out, st));
  }
  std::vector<double> h(S + 1);
  HIPTRY(hipMemcpyAsync(h.data(), out, (size_t)(S + 1) * 8, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  const double yy = h[0];
  if (!(yy > 0.0)) return fail(c, MODAL_EINVAL, "fnl_lowrank: alpha^T zeta^-1 alpha is not positive");
  *sigma2_host = 6.0 / yy;
  for (int i = 0; i < S; ++i) E_host[i] = h[1 + i] / yy;
  return MODAL_OK;
}

modal_status modal_bivector_rotate(modal_ctx* c, const double* b, const double* x, int R, double* y,
                                   modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (R < 0 || (R > 0 && (!b || !x || !y))) return fail(c, MODAL_EINVAL, "bivector_rotate: null pointer or R < 0");
  if (R == 0) return MODAL_OK;
  modal_status s = set_device(c);
  if (s != MODAL_OK) return s;
  HIPTRY(launch_bivector_rotate(c->nmax, b, x, R, y, (hipStream_t)stream));
  return MODAL_OK;
}

modal_status modal_alpha_separable(modal_ctx* c, const double* terms, int T, double* alpha, void* ws, size_t ws_bytes,
                                   modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!terms || !alpha || T < 1 || T > 64) return fail(c, MODAL_EINVAL, "alpha_separable: null pointer or T not in 1..64");
  modal_status s = check_ws(c, MODAL_OP_ALPHA_SEPARABLE, T, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int L = c->lmax + 1, nmu = shapes_nmu(c->lmax);
  if ((int)c->mu_host.size() != nmu) gauss_legendre(nmu, c->mu_host, c->wmu_host);
  const std::vector<double>& mu = c->mu_host;
  const std::vector<double>& wmu = c->wmu_host;
  Carver cv(ws);
  double* dmu = (double*)cv.take((size_t)nmu * 8);
  double* dw = (double*)cv.take((size_t)nmu * 8);
  double* U = (double*)cv.take(3 * (size_t)T * L * 8);
  double* F = (double*)cv.take(3 * (size_t)T * nmu * c->P * 8);
  HIPTRY(hipMemcpyAsync(dmu, mu.data(), (size_t)nmu * 8, hipMemcpyHostToDevice, st));
  HIPTRY(hipMemcpyAsync(dw, wmu.data(), (size_t)nmu * 8, hipMemcpyHostToDevice, st));
  HIPTRY(hipMemcpyAsync(U, terms, 3 * (size_t)T * L * 8, hipMemcpyHostToDevice, st));
  {
    StageTimer _t(c, MODAL_STAGE_COVARIANCE, st);
    HIPTRY(launch_legendre_series(L, nmu, c->P, 3 * T, U, c->t.qw64, dmu, F, st));
    HIPTRY(launch_alpha_modes(c->nmax, c->P, T, nmu, c->t.tri, F, dw, alpha, st));
  }
  HIPTRY(hipStreamSynchronize(st));
  return MODAL_OK;
}

modal_status modal_ideal_covariance(modal_ctx* c, const double* c_host, double* zeta, void* ws, size_t ws_bytes,
                                    modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!zeta) return fail(c, MODAL_EINVAL, "ideal_covariance: null pointer");
  modal_status s = check_ws(c, MODAL_OP_IDEAL_COVARIANCE, 0, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int L = c->lmax + 1, nmu = shapes_nmu(c->lmax), P = c->P;
  if ((int)c->mu_host.size() != nmu) gauss_legendre(nmu, c->mu_host, c->wmu_host);
  const std::vector<double>& mu = c->mu_host;
  const std::vector<double>& wmu = c->wmu_host;
  // U_b(l) = c_l q_b(l), B_a(l) = q_a(l): F[b][k][a] = Q_ab(mu_k)
  std::vector<double> u((size_t)P * L);
  for (int b = 0; b < P; ++b)
    for (int l = 0; l < L; ++l) {
      const double cw = c_host ? c_host[l] : (c->cl_host[l] > 0.0 ? 1.0 : 0.0);
      u[(size_t)b * L + l] = cw * c->q_host[(size_t)b * L + l];
    }
  Carver cv(ws);
  double* dmu = (double*)cv.take((size_t)nmu * 8);
  double* dw = (double*)cv.take((size_t)nmu * 8);
  double* U = (double*)cv.take((size_t)P * L * 8);
  double* Bq = (double*)cv.take((size_t)P * L * 8);
  double* F = (double*)cv.take((size_t)P * nmu * P * 8);
  HIPTRY(hipMemcpyAsync(dmu, mu.data(), (size_t)nmu * 8, hipMemcpyHostToDevice, st));
  HIPTRY(hipMemcpyAsync(dw, wmu.data(), (size_t)nmu * 8, hipMemcpyHostToDevice, st));
  HIPTRY(hipMemcpyAsync(U, u.data(), (size_t)P * L * 8, hipMemcpyHostToDevice, st));
  HIPTRY(hipMemcpyAsync(Bq, c->q_host.data(), (size_t)P * L * 8, hipMemcpyHostToDevice, st));
  {
    StageTimer _t(c, MODAL_STAGE_COVARIANCE, st);
    HIPTRY(launch_legendre_series(L, nmu, P, P, U, Bq, dmu, F, st));
    HIPTRY(launch_ideal_cov(c->nmax, P, nmu, c->t.nzrows, c->t.zrows, F, dw, zeta, st));
  }
  HIPTRY(hipStreamSynchronize(st));
  return MODAL_OK;
}

modal_status modal_frame(modal_ctx* c, const double* zeta0, double tol, int* k_host, int* perm, double* L11, void* ws,
                         size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!zeta0 || !k_host || !perm || !L11) return fail(c, MODAL_EINVAL, "frame: null pointer");
  if (!(tol >= 0.0 && tol < 1.0)) return fail(c, MODAL_EINVAL, "frame: tol outside [0, 1)");
  modal_status s = check_ws(c, MODAL_OP_FRAME, 0, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  int k = 0;
  {
    StageTimer _t(c, MODAL_STAGE_CHOLESKY, (hipStream_t)stream);
    HIPTRY(launch_frame(c->nmax, zeta0, tol, perm, L11, &k, ws, (hipStream_t)stream));
  }
  *k_host = k;
  if (k == 0) return fail(c, MODAL_ENOTPD, "frame: no positive pivot");
  return MODAL_OK;
}

modal_status modal_frame_rotate(modal_ctx* c, int k, const int* perm, const double* L11, const double* x, int R,
                                double* y, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (R < 0 || (R > 0 && (!perm || !L11 || !x || !y))) return fail(c, MODAL_EINVAL, "frame_rotate: null pointer or R < 0");
  if (k < 1 || k > c->nmax) return fail(c, MODAL_EINVAL, "frame_rotate: k outside 1..nmax");
  if (R == 0) return MODAL_OK;
  modal_status s = set_device(c);
  if (s != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  HIPTRY(launch_gather_cols(c->nmax, k, R, x, perm, y, st));
  HIPTRY(launch_trsm_rows(k, L11, R, y, st));
  return MODAL_OK;
}

modal_status modal_fnl_frame(modal_ctx* c, const double* zeta, int k, const int* perm, const double* alpha,
                             const double* beta, int S, double* E_host, double* sigma2_host, void* ws,
                             size_t ws_bytes, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (!zeta || !perm || !alpha || !sigma2_host || S < 0 || (S > 0 && (!beta || !E_host)))
    return fail(c, MODAL_EINVAL, "fnl_frame: null pointer or S < 0");
  if (k < 1 || k > c->nmax) return fail(c, MODAL_EINVAL, "fnl_frame: k outside 1..nmax");
  modal_status s = check_ws(c, MODAL_OP_FNL_FRAME, S, ws, ws_bytes);
  if (s != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int n = c->nmax;
  Carver cv(ws);
  double* Zk = (double*)cv.take((size_t)n * n * 8);
  double* rows = (double*)cv.take((size_t)(S + 1) * n * 8);
  HIPTRY(launch_gather_sym(n, k, zeta, perm, Zk, st));
  HIPTRY(launch_gather_cols(n, k, 1, alpha, perm, rows, st));
  if (S > 0) HIPTRY(launch_gather_cols(n, k, S, beta, perm, rows + k, st));
  // the estimator on k modes, its own workspace after the gathered arrays
  void* ws2 = (char*)ws + cv.used;
  return estimate(c, MODAL_OP_FNL, k, 6.0, Zk, rows, rows + k, k, S, E_host, sigma2_host, nullptr, ws2,
                  ws_bytes - cv.used, st);
}

modal_status modal_whiten(modal_ctx* c, const double* L, const double* x, int R, double* y, modal_stream_t stream) {
  if (!c) return MODAL_EINVAL;
  if (R < 0 || (R > 0 && (!L || !x || !y))) return fail(c, MODAL_EINVAL, "whiten: null pointer or R < 0");
  if (R == 0) return MODAL_OK;
  modal_status s = set_device(c);
  if (s != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int n = c->nmax;
  if (y != x) HIPTRY(hipMemcpyAsync(y, x, (size_t)R * n * 8, hipMemcpyDeviceToDevice, st));
  HIPTRY(launch_trsm_rows(n, L, R, y, st));
  return MODAL_OK;
}

}  // extern "C"

struct modal_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

extern "C" {

modal_status modal_beta_graph_create(int n, modal_ctx* const* ctxs, const void* const* alms, const int* S,
                                     const void* const* states, double* const* betas, void* const* ws,
                                     const size_t* ws_bytes, modal_graph** out) {
  if (!out) return MODAL_EINVAL;
  *out = nullptr;
  if (n <= 0 || !ctxs || !alms || !S || !betas || !ws || !ws_bytes) return MODAL_EINVAL;
  const int dev = ctxs[0] ? ctxs[0]->device : -1;
  // validate everything before capturing
  for (int i = 0; i < n; ++i) {
    modal_ctx* c = ctxs[i];
    if (!c || c->device != dev) return MODAL_EINVAL;
    const std::string tag = "graph call " + std::to_string(i) + ": ";
    if (!alms[i] || !betas[i] || S[i] <= 0) return fail(c, MODAL_EINVAL, tag + "null pointer or S <= 0");
    modal_status s = check_state(c, states ? states[i] : nullptr);
    if (s == MODAL_OK) s = check_ws(c, MODAL_OP_BETA, S[i], ws[i], ws_bytes[i]);
    if (s != MODAL_OK) return fail(c, s, tag + c->last_error);
  }
  modal_ctx* c = ctxs[0];
  modal_status s = set_device(c);
  if (s != MODAL_OK) return s;
  hipStream_t cap = nullptr;
  HIPTRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  std::vector<bool> prof(n);
  for (int i = 0; i < n; ++i) {
    prof[i] = ctxs[i]->profile;
    ctxs[i]->profile = false;
  }
  modal_status rs = MODAL_OK;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int i = 0; i < n && rs == MODAL_OK; ++i) {
      rs = modal_beta(ctxs[i], alms[i], S[i], states ? states[i] : nullptr, betas[i], ws[i], ws_bytes[i], cap);
      if (rs != MODAL_OK) ctxs[i]->last_error = "graph call " + std::to_string(i) + ": " + ctxs[i]->last_error;
    }
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess) e = e2;
  }
  for (int i = 0; i < n; ++i) ctxs[i]->profile = prof[i];
  (void)hipStreamDestroy(cap);
  if (rs != MODAL_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rs;
  }
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(c, MODAL_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  modal_graph* g = new (std::nothrow) modal_graph();
  if (!g) {
    (void)hipGraphDestroy(graph);
    return MODAL_EDEVICE;
  }
  g->graph = graph;
  g->device = dev;
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    modal_graph_destroy(g);
    return fail(c, MODAL_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  *out = g;
  return MODAL_OK;
}

modal_status modal_graph_launch(modal_graph* g, modal_stream_t stream) {
  if (!g || !g->exec) return MODAL_EINVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? MODAL_OK : MODAL_EDEVICE;
}

void modal_graph_destroy(modal_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

modal_status modal_autotune(modal_ctx* c, const void* alm, int S, const void* state, double* beta, void* ws,
                            size_t ws_bytes, modal_stream_t stream, int* chunk_px, int* fft_rings) {
  if (!c) return MODAL_EINVAL;
  modal_status s = check_state(c, state);
  if (s != MODAL_OK) return s;
  if (!alm || !beta || S <= 0) return fail(c, MODAL_EINVAL, "autotune: null pointer or S <= 0");
  if ((s = check_ws(c, MODAL_OP_BETA, S, ws, ws_bytes)) != MODAL_OK) return s;
  if ((s = set_device(c)) != MODAL_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  HIPTRY(hipEventCreate(&a));
  HIPTRY(hipEventCreate(&b));
  const bool prof = c->profile;
  c->profile = false;
  auto time_beta = [&](float* ms) -> modal_status {
    modal_status r = modal_beta(c, alm, S, state, beta, ws, ws_bytes, st);   // warm-up
    if (r != MODAL_OK) return r;
    if (hipEventRecord(a, st) != hipSuccess) return MODAL_EDEVICE;
    for (int i = 0; i < 2 && r == MODAL_OK; ++i) r = modal_beta(c, alm, S, state, beta, ws, ws_bytes, st);
    if (r != MODAL_OK) return r;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(ms, a, b) != hipSuccess)
      return MODAL_EDEVICE;
    return MODAL_OK;
  };
  float best = 1e30f;
  int best_chunk = 65536, best_r = fft_rings_max(c);
  const int lo = chunk_target_min(c);
  const int chunks[] = {lo, 2 * lo, 4 * lo, 8 * lo};
  int best_chunk_init = chunk_target_default(c);
  best_chunk = best_chunk_init;
  // rings per FFT workgroup only matter for the LDS ping-pong FFT kernel
  for (int r = c->fft_rg ? 1 : fft_rings_max(c); r >= 1 && s == MODAL_OK; r >>= 1)
    for (int ch : chunks) {
      if (c->prec == MODAL_F32 && ch > chunk_target_default(c)) continue;   // FP32 keeps short chunks
      c->tune_chunk_px = ch;
      c->tune_fft_rings = r;
      float ms = 0.f;
      if ((s = time_beta(&ms)) != MODAL_OK) break;
      if (ms < best) {
        best = ms;
        best_chunk = ch;
        best_r = r;
      }
      if (!cubic_mfma_available(c)) break;   // the chunk only matters for the MFMA contraction
    }
  c->tune_chunk_px = best_chunk;
  c->tune_fft_rings = best_r;
  c->profile = prof;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (s != MODAL_OK) return s;
  if (chunk_px) *chunk_px = best_chunk;
  if (fft_rings) *fft_rings = best_r;
  return MODAL_OK;
}

modal_status modal_profile_enable(modal_ctx* c, int enable) {
  if (!c) return MODAL_EINVAL;
  c->profile = enable != 0;
  return MODAL_OK;
}

modal_status modal_profile_read(modal_ctx* c, double* ms, long long* count, int reset) {
  if (!c) return MODAL_EINVAL;
  for (auto& mk : c->marks) {
    float t = 0.f;
    HIPTRY(hipEventSynchronize(mk.b));
    HIPTRY(hipEventElapsedTime(&t, mk.a, mk.b));
    c->stage_ms[mk.stage] += t;
    c->stage_n[mk.stage] += 1;
    c->event_pool.push_back(mk.a);
    c->event_pool.push_back(mk.b);
  }
  c->marks.clear();
  for (int i = 0; i < MODAL_NSTAGES; ++i) {
    if (ms) ms[i] = c->stage_ms[i];
    if (count) count[i] = c->stage_n[i];
    if (reset) {
      c->stage_ms[i] = 0.0;
      c->stage_n[i] = 0;
    }
  }
  return MODAL_OK;
}

}  // extern "C"
