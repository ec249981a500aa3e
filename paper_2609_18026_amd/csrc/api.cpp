// extern "C" entry points of include/mlg.h: argument validation and the kernel sequence of
// each operation.  Every step of the computation runs in the library's own HIP kernels.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "mlg_internal.h"

namespace mlg {
mlg_status build_plan(mlg_plan_s* p);
void destroy_plan(mlg_plan_s* p);
extern thread_local std::string g_last_error;

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool factorable(int n) {
  int r[16];
  return n >= 1 && n <= 1024 && factor_radices(n, r) >= 0;
}

// Workspace partition for FP64 plans: 7 mixed arrays, 5 triangular arrays.
struct Ws {
  double* X[7];
  double* T[5];
};

Ws partition(const mlg_plan_s* p, void* ws) {
  Ws w{};
  char* b = static_cast<char*>(ws);
  size_t o = 0;
  for (int i = 0; i < 7; ++i) {
    w.X[i] = reinterpret_cast<double*>(b + o);
    o += p->mixed_elems * 2 * sizeof(double);
  }
  for (int i = 0; i < 5; ++i) {
    w.T[i] = reinterpret_cast<double*>(b + o);
    o += p->tri_elems * 2 * sizeof(double);
  }
  return w;
}

mlg_status check_plan(mlg_plan p) {
  if (!p) return fail(MLG_E_ARG, "plan is NULL");
  return MLG_OK;
}

// entry points that work on FP64 data only
mlg_status check_fp64(mlg_plan p, const char* what) {
  if (!p) return fail(MLG_E_ARG, "plan is NULL");
  if (p->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, std::string(what) + " needs an MLG_FP64 plan");
  return MLG_OK;
}

// Device-resident workspace of mlg_rhs_tp_noalloc: one copy per GPU, held from the first use of the
// library on that GPU until the process ends.  Host code never uses the array's name as an
// address: the device address of each GPU's copy comes from hipGetSymbolAddress.
constexpr size_t kScratchBytes = size_t(192) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// With 'device' current: look up (once) the address of that GPU's copy of the array.
mlg_status scratch_setup(int device) {
  if (device < 0 || device >= kScratchDevices) return fail(MLG_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return MLG_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(MLG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return MLG_OK;
}

void* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kScratchDevices) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace
}  // namespace mlg

using namespace mlg;

extern "C" {

const char* mlg_last_error(void) { return g_last_error.c_str(); }

mlg_status mlg_plan_create(const mlg_grid* grid, mlg_precision prec, int device, mlg_plan* out) {
  if (!out) return fail(MLG_E_ARG, "out is NULL");
  *out = nullptr;
  if (!grid) return fail(MLG_E_ARG, "grid is NULL");
  mlg_grid g = *grid;
  if (!std::isfinite(g.ell) || !std::isfinite(g.lz)) return fail(MLG_E_NONFINITE, "ell and L_z must be finite");
  if (!(g.ell > 0)) return fail(MLG_E_ARG, "ell must be positive");
  if (!(g.lz > 0)) return fail(MLG_E_ARG, "L_z must be positive");
  if (g.nr < 2) return fail(MLG_E_ARG, "N_r must be at least 2");
  if (g.nphi < 2 || g.nz < 1) return fail(MLG_E_ARG, "N_phi must be >= 2 and N_z >= 1");
  if (g.nrc < 0 || g.nphic < 0 || g.nzc < 0) return fail(MLG_E_ARG, "chops must be non-negative");
  if (g.nrc == 0) g.nrc = g.nr;
  if (g.nphic == 0) g.nphic = g.nphi / 2;
  if (g.nzc == 0) g.nzc = g.nz / 2 > 0 ? g.nz / 2 : 1;
  if (g.nrc > g.nr) return fail(MLG_E_ARG, "N_r^c exceeds N_r");
  if (g.nphic > g.nphi / 2 + 1) return fail(MLG_E_ARG, "N_phi^c exceeds N_phi/2 + 1");
  if (g.nzc > g.nz / 2 + 1) return fail(MLG_E_ARG, "N_z^c exceeds N_z/2 + 1");
  if (g.dealias != 0 && g.dealias != 1) return fail(MLG_E_ARG, "dealias must be 0 or 1");
  if (g.nr > 4096) return fail(MLG_E_UNSUPPORTED, "N_r above 4096");
  if (!factorable(g.nphi) || !factorable(g.nz))
    return fail(MLG_E_UNSUPPORTED, "N_phi and N_z must be <= 1024 with prime factors 2, 3, 5 only");
  if (prec != MLG_FP64 && prec != MLG_FP32 && prec != MLG_SPLIT_BF16)
    return fail(MLG_E_UNSUPPORTED, "unknown precision");
  if (prec != MLG_FP64) {
    // reduced-precision plans: float data, the register-resident 256-point FFTs and the folded products
    if (g.nphi != 256 || g.nz != 256)
      return fail(MLG_E_UNSUPPORTED, "MLG_FP32 and MLG_SPLIT_BF16 plans need N_phi = N_z = 256");
    if (g.nr % 2 != 0) return fail(MLG_E_UNSUPPORTED, "MLG_FP32 and MLG_SPLIT_BF16 plans need an even N_r");
    if ((int64_t)g.nr * g.nz > (int64_t(1) << 23) || g.nrc > 512)
      return fail(MLG_E_UNSUPPORTED, "MLG_FP32 and MLG_SPLIT_BF16 plans need N_r <= 32768 and N_r^c <= 512");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(MLG_E_ARG, "device index out of range or no HIP device");
  DeviceGuard guard(device);
  if (!guard.ok) return fail(MLG_E_DEVICE, "hipSetDevice failed");
  // the no-allocation entry point's workspace on this GPU (a failure here is reported by that
  // entry point, which retries the lookup; plans themselves do not need it)
  if (scratch_setup(device) != MLG_OK) set_error("");
  mlg_plan_s* p = new (std::nothrow) mlg_plan_s();
  if (!p) return fail(MLG_E_ALLOC, "host allocation failed");
  p->g = g;
  p->prec = prec;
  p->device = device;
  p->nr = g.nr;
  p->nphi = g.nphi;
  p->nz = g.nz;
  p->nrc = g.nrc;
  p->M = g.nphic;
  p->nzc = g.nzc;
  p->dealias_m = (g.nphi - 1) / 3;
  p->dealias_k = (g.nz - 1) / 3;
  p->phi_nrad = factor_radices(g.nphi, p->phi_rad);
  p->z_nrad = factor_radices(g.nz, p->z_rad);
  if (const char* e = std::getenv("MLG_RADIAL_FOLD")) p->use_fold = std::strcmp(e, "0") != 0;
  if (prec != MLG_FP64) p->use_fold = true;  // the reduced-precision paths are the folded ones
  mlg_status st = build_plan(p);
  if (st != MLG_OK) {
    std::string msg = g_last_error;
    destroy_plan(p);
    return fail(st, msg);
  }
  *out = p;
  return MLG_OK;
}

mlg_status mlg_plan_destroy(mlg_plan plan) {
  if (!plan) return MLG_OK;
  DeviceGuard guard(plan->device);
  destroy_plan(plan);
  return MLG_OK;
}

mlg_status mlg_plan_query(mlg_plan p, mlg_layout* out) {
  if (mlg_status st = check_plan(p)) return st;
  if (!out) return fail(MLG_E_ARG, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->phys_elems = (int64_t)p->nz * p->nr * p->nphi;
  out->spec_rows = p->tau;
  out->spec_elems = p->tau * p->nz;
  out->workspace_bytes = (int64_t)p->ws_bytes;
  out->M = p->M;
  out->nrc = p->nrc;
  out->nzc = p->nzc;
  out->real_bytes = p->prec == MLG_FP64 ? 8 : 4;
  out->dealias_m = p->dealias_m;
  out->dealias_k = p->dealias_k;
  return MLG_OK;
}

mlg_status mlg_plan_nodes(mlg_plan p, double* x, double* w, double* r) {
  if (mlg_status st = check_plan(p)) return st;
  for (int i = 0; i < p->nr; ++i) {
    if (x) x[i] = p->x[i];
    if (w) w[i] = p->w[i];
    if (r) r[i] = p->r[i];
  }
  return MLG_OK;
}

// Radial products of one scalar field: folded over the node symmetry for even N_r (unless the plan
// was created with MLG_RADIAL_FOLD=0), the generic batched GEMM otherwise.
static mlg_status scalar_radial(const mlg_plan_s* p, int dir, const double* B, double* C, hipStream_t s) {
  if (p->prec == MLG_SPLIT_BF16) return launch_split_scalar(p, dir, B, C, s);
  if (p->prec == MLG_FP32) return launch_scalar_fold(p, dir, B, C, s);
  if (p->use_fold && p->nr % 2 == 0) return launch_scalar_fold(p, dir, B, C, s);
  GemmProds pr{};
  pr.nprod = 1;
  pr.A[0] = dir > 0 ? p->d_Pb : p->d_Pf;
  pr.B[0] = B;
  pr.C[0] = C;
  return dir > 0 ? launch_gemm(p, pr, p->d_desc_bwd, p->max_rows_bwd, 2 * p->nz, s)
                 : launch_gemm(p, pr, p->d_desc_fwd, p->max_rows_fwd, 2 * p->nz, s);
}

mlg_status mlg_forward(mlg_plan p, const void* phys, void* spec, void* ws, void* stream) {
  if (mlg_status st = check_plan(p)) return st;
  if (!phys || !spec || !ws) return fail(MLG_E_ARG, "null buffer");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = partition(p, ws);
  mlg_status st;
  if ((st = launch_phi_forward(p, static_cast<const double*>(phys), w.X[0], s))) return st;
  if ((st = scalar_radial(p, -1, w.X[0], static_cast<double*>(spec), s))) return st;
  return launch_zfft(p, static_cast<double*>(spec), static_cast<double*>(spec), p->tau, -1, nullptr, 0, -1, s);
}

mlg_status mlg_backward(mlg_plan p, const void* spec, void* phys, void* ws, void* stream) {
  if (mlg_status st = check_plan(p)) return st;
  if (!phys || !spec || !ws) return fail(MLG_E_ARG, "null buffer");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = partition(p, ws);
  mlg_status st;
  if ((st = launch_zfft(p, static_cast<const double*>(spec), w.T[0], p->tau, +1, nullptr, 0, -1, s))) return st;
  if ((st = scalar_radial(p, +1, w.T[0], w.X[0], s))) return st;
  return launch_phi_backward(p, w.X[0], static_cast<double*>(phys), s);
}

mlg_status mlg_rhs_scalar(mlg_plan p, int kind, double gamma, const void* spec_u, void* spec_out, void* ws,
                          void* stream) {
  if (mlg_status st = check_plan(p)) return st;
  if (!spec_u || !spec_out || !ws) return fail(MLG_E_ARG, "null buffer");
  if (spec_u == spec_out) return fail(MLG_E_ARG, "spec_u and spec_out must not alias");
  if (kind != MLG_RHS_U2 && kind != MLG_RHS_KPP) return fail(MLG_E_ARG, "unknown RHS kind");
  if (!std::isfinite(gamma)) return fail(MLG_E_ARG, "gamma must be finite");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = partition(p, ws);
  mlg_status st;
  // the two-thirds mask applies to the field entering the product (read as zero outside it by the
  // inverse z transform) and to the product
  const bool mask = p->g.dealias != 0;
  const int32_t* row_m = mask ? p->d_row_m : nullptr;
  const int mask_k = mask ? p->dealias_k : -1;
  if ((st = launch_zfft(p, static_cast<const double*>(spec_u), w.T[0], p->tau, +1, row_m, p->dealias_m, mask_k, s)))
    return st;
  if ((st = scalar_radial(p, +1, w.T[0], w.X[0], s))) return st;
  if ((st = launch_phi_scalar_rhs(p, kind, gamma, w.X[0], s))) return st;
  if ((st = scalar_radial(p, -1, w.X[0], static_cast<double*>(spec_out), s))) return st;
  return launch_zfft(p, static_cast<double*>(spec_out), static_cast<double*>(spec_out), p->tau, -1, row_m,
                     p->dealias_m, mask_k, s);
}

}  // extern "C"

// Whether mlg_rhs_tp skips the orders and axial blocks the two-thirds mask removes: the folded
// FP64 / FP32 or the split synthesis followed by the 256-point z (or split z DFT) and phi stages
// (the kernels that leave them unread, or discard what they read there); otherwise the synthesis
// writes them as zeros.
static bool rhs_skips_masked(const mlg_plan_s* p) {
  const bool synth_ok = p->prec == MLG_SPLIT_BF16 || (p->use_fold && p->nr % 2 == 0);
  return p->g.dealias != 0 && synth_ok && p->nz == 256 && p->nphi == 256 && p->use_fast_fft &&
         (int64_t)p->nr * p->nz <= (int64_t(1) << 23);
}

// The kernel sequence of mlg_rhs_tp on the workspace 'ws' (caller-provided, or the per-GPU array of
// mlg_rhs_tp_noalloc).
static mlg_status rhs_tp_run(mlg_plan p, const double* U, const void* psi, const void* chi, void* psi_n, void* chi_n,
                             void* taps, void* ws, void* stream) {
  if (mlg_status st = check_plan(p)) return st;
  if (!psi || !chi || !psi_n || !chi_n || !ws) return fail(MLG_E_ARG, "null buffer");
  if (psi_n == chi_n || psi_n == psi || psi_n == chi || chi_n == psi || chi_n == chi)
    return fail(MLG_E_ARG, "outputs must not alias each other or the inputs");
  if (p->nrc > 512) return fail(MLG_E_UNSUPPORTED, "mlg_rhs_tp supports N_r^c up to 512");
  double Uh[3] = {0.0, 0.0, 0.0};
  if (U) {
    for (int i = 0; i < 3; ++i) {
      if (!std::isfinite(U[i])) return fail(MLG_E_ARG, "background U must be finite");
      Uh[i] = U[i];
    }
  }
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = partition(p, ws);
  mlg_status st;
  // 1. radial synthesis: the six velocity / vorticity harmonics (k spectral), fused.  Under the
  // two-thirds mask the potentials enter through it (Sec. 3.3: the fields of a product hold no mode
  // in the dealiasing margin); with the 256-point z and phi stages the masked orders and column
  // blocks are not synthesized at all, and the stages after it do not read them
  const bool dealias = p->g.dealias != 0;
  SynthMask smask;
  if (dealias) {
    int mm, km;
    active_columns(p, &mm, &km);
    smask.mkeep = p->dealias_m;
    smask.kmax = km;
    smask.skip = rhs_skips_masked(p);
  }
  if (p->prec == MLG_SPLIT_BF16)
    st = launch_split_synth(p, static_cast<const double*>(psi), static_cast<const double*>(chi), w.X, s, smask);
  else
    st = launch_synth_gemm(p, static_cast<const double*>(psi), static_cast<const double*>(chi), w.X, s, smask);
  if (st) return st;
  // the logarithmic proxy parts of the potentials, when they carry amplitudes (Eq. logproxy)
  if ((st = launch_proxy_fields(p, w.X, s))) return st;
  // 2. inverse z transforms of the six fields (under the mask: the kept orders, the kept slots read)
  const int64_t mrows = (int64_t)(dealias ? std::min(p->M, p->dealias_m + 1) : p->M) * p->nr;
  if ((st = launch_zfft_fields(p, w.X, w.X, 6, mrows, +1, nullptr, 0, dealias ? smask.kmax : -1, s))) return st;
  // 3. phi stage: nodal u, w -> N = (U + u) x w -> harmonics of N_r/r, N_phi/r, N_z
  double* tp = static_cast<double*>(taps);
  if ((st = launch_phi_vec_rhs(p, Uh, w.X, tp, s))) return st;
  // 4. forward z transforms of the orders the projection uses.  From here on every plan computes in
  // FP64: the solves of step 6 are ill-conditioned along the far-field directions of the Gram
  // matrices (cond(Dbar_1) ~ 1e9 at N_r = 256), and the curl-type sources are a small residual of
  // N for flows near a steady state, so reduced-precision source products would be amplified there
  const int fp64_only = 1;
  int mmax, kmax;
  active_columns(p, &mmax, &kmax);
  const int64_t frows = (int64_t)mmax * p->nr;
  // the projection products read only the slots |k| <= kmax: the others need not be written
  if ((st = launch_zfft_fields(p, w.X, w.X, 3, frows, -1, nullptr, 0, kmax, s, fp64_only, true))) return st;
  // 5. Galerkin projections onto Pbar and Q = T - 2(1+x) Pbar with the C, K', Zhat epilogue
  double* src3[3] = {w.T[0], w.T[1], w.T[2]};
  if ((st = launch_proj_gemm(p, w.X, src3, mmax, kmax, s))) return st;
  // 6. elliptic solves per (m, k)
  const double* csrc[3] = {w.T[0], w.T[1], w.T[2]};
  double* tsrc = tp ? tp + (size_t)9 * p->nz * p->nr * p->nphi : nullptr;
  return launch_projection(p, csrc, static_cast<double*>(psi_n), static_cast<double*>(chi_n), tsrc, s);
}

extern "C" {

mlg_status mlg_rhs_tp(mlg_plan p, const double* U, const void* psi, const void* chi, void* psi_n, void* chi_n,
                      void* taps, void* ws, void* stream) {
  return rhs_tp_run(p, U, psi, chi, psi_n, chi_n, taps, ws, stream);
}

mlg_status mlg_rhs_tp_noalloc(mlg_plan p, const double* U, const void* psi, const void* chi, void* psi_n,
                              void* chi_n, void* taps, void* stream) {
  if (mlg_status st = check_plan(p)) return st;
  if (p->ws_bytes > kScratchBytes)
    return fail(MLG_E_UNSUPPORTED, "mlg_rhs_tp_noalloc: the plan needs " + std::to_string(p->ws_bytes) +
                                       " workspace bytes, above the fixed " + std::to_string(kScratchBytes));
  if (p->timing.enabled) return fail(MLG_E_ARG, "mlg_rhs_tp_noalloc: timing hooks are enabled (they create events)");
  DeviceGuard guard(p->device);
  if (!guard.ok) return fail(MLG_E_DEVICE, "hipSetDevice failed");
  void* ws = scratch_address(p->device);
  if (!ws) {
    if (mlg_status st = scratch_setup(p->device)) return st;
    ws = scratch_address(p->device);
  }
  return rhs_tp_run(p, U, psi, chi, psi_n, chi_n, taps, ws, stream);
}

mlg_status mlg_step_setup(mlg_plan p, const mlg_dissip* d) {
  if (mlg_status st = check_fp64(p, "mlg_step_setup")) return st;
  if (!d) return fail(MLG_E_ARG, "dissip is NULL");
  if (!std::isfinite(d->nu) || !std::isfinite(d->nu_h) || !std::isfinite(d->dt))
    return fail(MLG_E_NONFINITE, "non-finite step parameters");
  if (d->nu < 0 || d->nu_h < 0 || !(d->dt > 0)) return fail(MLG_E_ARG, "need nu >= 0, nu_h >= 0, dt > 0");
  if (d->p != 4 && d->p != 6 && d->p != 8) return fail(MLG_E_ARG, "p must be 4, 6 or 8");
  DeviceGuard guard(p->device);
  return step_setup(p, d);
}

mlg_status mlg_step_febe(mlg_plan p, int half, const void* s, const void* A, void* out, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_step_febe")) return st;
  if (!p->step_ready) return fail(MLG_E_ARG, "mlg_step_setup has not been called");
  if (!s || !A || !out) return fail(MLG_E_ARG, "null buffer");
  if (out == s || out == A) return fail(MLG_E_ARG, "out must not alias the inputs");
  DeviceGuard guard(p->device);
  return launch_step(p, 0, half ? 0 : 1, static_cast<const double*>(s), static_cast<const double*>(A), nullptr,
                     static_cast<double*>(out), static_cast<hipStream_t>(stream));
}

mlg_status mlg_step_abcn(mlg_plan p, const void* s, const void* A_now, const void* A_prev, void* out, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_step_abcn")) return st;
  if (!p->step_ready) return fail(MLG_E_ARG, "mlg_step_setup has not been called");
  if (!s || !A_now || !A_prev || !out) return fail(MLG_E_ARG, "null buffer");
  if (out == s || out == A_now || out == A_prev) return fail(MLG_E_ARG, "out must not alias the inputs");
  DeviceGuard guard(p->device);
  return launch_step(p, 1, 0, static_cast<const double*>(s), static_cast<const double*>(A_now),
                     static_cast<const double*>(A_prev), static_cast<double*>(out), static_cast<hipStream_t>(stream));
}

mlg_status mlg_eval_harmonic(mlg_plan p, const void* spec, int32_t m, int32_t kk, const double* r, int64_t npts,
                             void* out, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_eval_harmonic")) return st;
  if (!spec || !out || (npts > 0 && !r)) return fail(MLG_E_ARG, "null buffer");
  if (m < 0 || m >= p->M || kk < 0 || kk >= p->nz) return fail(MLG_E_ARG, "harmonic (m, kk) out of range");
  if (npts < 0) return fail(MLG_E_ARG, "npts must be >= 0");
  DeviceGuard guard(p->device);
  return launch_eval_harmonic(p, static_cast<const double*>(spec), m, kk, r, npts, static_cast<double*>(out),
                              static_cast<hipStream_t>(stream));
}

mlg_status mlg_filter_setup(mlg_plan p, const mlg_filter_cfg* cfg) {
  if (mlg_status st = check_fp64(p, "mlg_filter_setup")) return st;
  if (!cfg) {
    p->filter_on = false;
    return MLG_OK;
  }
  const double v[4] = {cfg->zeta_c, cfg->tau, cfg->eps_max, cfg->relax};
  for (double x : v)
    if (!std::isfinite(x)) return fail(MLG_E_ARG, "filter parameters must be finite");
  if (cfg->zeta_c < 0.0 || cfg->zeta_c >= 1.0) return fail(MLG_E_ARG, "filter: 0 <= zeta_c < 1");
  if (cfg->tau <= 0.0) return fail(MLG_E_ARG, "filter: tau must be > 0");
  if (cfg->eps_max < 0.0) return fail(MLG_E_ARG, "filter: eps_max must be >= 0");
  if (cfg->relax <= 0.0 || cfg->relax > 1.0) return fail(MLG_E_ARG, "filter: 0 < relax <= 1");
  DeviceGuard guard(p->device);
  const size_t bytes = (size_t)(4 + 2 * FILTER_BLOCKS) * sizeof(double);
  if (!p->d_filter) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->d_filter), bytes);
    if (e != hipSuccess) {
      p->d_filter = nullptr;
      return fail(MLG_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
  }
  const double zero[4] = {0.0, 0.0, 0.0, 0.0};
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(p->d_filter, zero, sizeof(zero), hipMemcpyHostToDevice));
  p->filter_zc = cfg->zeta_c;
  p->filter_tau = cfg->tau;
  p->filter_epsmax = cfg->eps_max;
  p->filter_relax = cfg->relax;
  p->filter_on = true;
  return MLG_OK;
}

mlg_status mlg_filter_apply(mlg_plan p, int32_t slot, void* spec, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_filter_apply")) return st;
  if (!p->filter_on) return fail(MLG_E_ARG, "mlg_filter_setup has not enabled the filter");
  if (slot != 0 && slot != 1) return fail(MLG_E_ARG, "filter slot must be 0 or 1");
  if (!spec) return fail(MLG_E_ARG, "null buffer");
  DeviceGuard guard(p->device);
  return launch_filter(p, slot, static_cast<double*>(spec), static_cast<hipStream_t>(stream));
}

mlg_status mlg_filter_state(mlg_plan p, double* out4) {
  if (mlg_status st = check_plan(p)) return st;
  if (!out4) return fail(MLG_E_ARG, "null buffer");
  if (!p->d_filter) return fail(MLG_E_ARG, "mlg_filter_setup has never been called");
  DeviceGuard guard(p->device);
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(out4, p->d_filter, 4 * sizeof(double), hipMemcpyDeviceToHost));
  return MLG_OK;
}

mlg_status mlg_tp_advance(mlg_plan p, const double* U, void* psi, void* chi, void* hist_psi, void* hist_chi,
                          int32_t nsteps, int32_t start, mlg_closure closure, void* tmp, void* ws, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_tp_advance")) return st;
  if (!p->step_ready) return fail(MLG_E_ARG, "mlg_step_setup has not been called");
  if (!psi || !chi || !hist_psi || !hist_chi || !tmp || !ws) return fail(MLG_E_ARG, "null buffer");
  if (nsteps < 0) return fail(MLG_E_ARG, "nsteps must be >= 0");
  if (closure && closure_plan(closure) != p) return fail(MLG_E_ARG, "the closure belongs to another plan");
  if (nsteps == 0) return MLG_OK;
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)p->tau * p->nz * 2;  // doubles per spectral array
  double* t[6];
  for (int i = 0; i < 6; ++i) t[i] = static_cast<double*>(tmp) + i * n;
  double* sp = static_cast<double*>(psi);
  double* sc = static_cast<double*>(chi);
  double* hp = static_cast<double*>(hist_psi);
  double* hc = static_cast<double*>(hist_chi);
  mlg_status st;
  auto rhs = [&](const double* a, const double* b, double* ra, double* rb) -> mlg_status {
    if (mlg_status e = mlg_rhs_tp(p, U, a, b, ra, rb, nullptr, ws, stream)) return e;
    if (mlg_status e = launch_proxy_force(p, ra, rb, s)) return e;   // dissipation of the proxy parts
    return closure ? closure_correct(closure, a, b, ra, rb, s) : MLG_OK;
  };
  // the adaptive modal filter between steps (Sec. 3.3), when enabled
  auto filter = [&]() -> mlg_status {
    if (!p->filter_on) return MLG_OK;
    if (mlg_status e = launch_filter(p, 0, sp, s)) return e;
    return launch_filter(p, 1, sc, s);
  };
  int done = 0;
  if (start) {
    // s1 = 2 S_{dt/2}(S_{dt/2}(s0)) - S_dt(s0), S_h(s) = (I - h L)^{-1} (s + h A(s))
    if ((st = rhs(sp, sc, hp, hc))) return st;
    if ((st = launch_step(p, 0, 1, sp, hp, nullptr, t[2], s)) || (st = launch_step(p, 0, 1, sc, hc, nullptr, t[3], s)))
      return st;
    if ((st = launch_step(p, 0, 0, sp, hp, nullptr, t[4], s)) || (st = launch_step(p, 0, 0, sc, hc, nullptr, t[5], s)))
      return st;
    if ((st = rhs(t[4], t[5], t[0], t[1]))) return st;
    if ((st = launch_step(p, 0, 0, t[4], t[0], nullptr, t[4], s)) ||
        (st = launch_step(p, 0, 0, t[5], t[1], nullptr, t[5], s)))
      return st;
    if ((st = launch_richardson(p, t[4], t[2], sp, s)) || (st = launch_richardson(p, t[5], t[3], sc, s))) return st;
    if ((st = filter())) return st;
    done = 1;
  }
  // AB-CN: the nonlinear terms alternate between (hist) and (t0, t1); the step runs in place
  double* prev[2] = {hp, hc};
  for (; done < nsteps; ++done) {
    double* now[2] = {prev[0] == hp ? t[0] : hp, prev[0] == hp ? t[1] : hc};
    if ((st = rhs(sp, sc, now[0], now[1]))) return st;
    if ((st = launch_step(p, 1, 0, sp, now[0], prev[0], sp, s)) || (st = launch_step(p, 1, 0, sc, now[1], prev[1], sc, s)))
      return st;
    if ((st = filter())) return st;
    prev[0] = now[0];
    prev[1] = now[1];
  }
  if (prev[0] != hp) {
    MLG_HIP_TRY(hipMemcpyAsync(hp, prev[0], n * sizeof(double), hipMemcpyDeviceToDevice, s));
    MLG_HIP_TRY(hipMemcpyAsync(hc, prev[1], n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return MLG_OK;
}

mlg_status mlg_scalar_advance(mlg_plan p, int32_t kind, double gamma, void* state, void* hist, int32_t nsteps,
                              int32_t start, void* tmp, void* ws, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_scalar_advance")) return st;
  if (!p->step_ready) return fail(MLG_E_ARG, "mlg_step_setup has not been called");
  if (!state || !hist || !tmp || !ws) return fail(MLG_E_ARG, "null buffer");
  if (kind != MLG_RHS_U2 && kind != MLG_RHS_KPP) return fail(MLG_E_ARG, "kind must be MLG_RHS_U2 or MLG_RHS_KPP");
  if (!std::isfinite(gamma)) return fail(MLG_E_ARG, "gamma must be finite");
  if (nsteps < 0) return fail(MLG_E_ARG, "nsteps must be >= 0");
  if (nsteps == 0) return MLG_OK;
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t n = (size_t)p->tau * p->nz * 2;  // doubles per spectral array
  double* t[3];
  for (int i = 0; i < 3; ++i) t[i] = static_cast<double*>(tmp) + i * n;
  double* sp = static_cast<double*>(state);
  double* hp = static_cast<double*>(hist);
  mlg_status st;
  auto rhs = [&](const double* a, double* ra) { return mlg_rhs_scalar(p, kind, gamma, a, ra, ws, stream); };
  auto filter = [&]() -> mlg_status { return p->filter_on ? launch_filter(p, 0, sp, s) : MLG_OK; };
  int done = 0;
  if (start) {
    // s1 = 2 S_{dt/2}(S_{dt/2}(s0)) - S_dt(s0), S_h(s) = (I - h L)^{-1} (s + h A(s))
    if ((st = rhs(sp, hp))) return st;
    if ((st = launch_step(p, 0, 1, sp, hp, nullptr, t[1], s))) return st;
    if ((st = launch_step(p, 0, 0, sp, hp, nullptr, t[2], s))) return st;
    if ((st = rhs(t[2], t[0]))) return st;
    if ((st = launch_step(p, 0, 0, t[2], t[0], nullptr, t[2], s))) return st;
    if ((st = launch_richardson(p, t[2], t[1], sp, s))) return st;
    if ((st = filter())) return st;
    done = 1;
  }
  // AB-CN: the nonlinear term alternates between hist and t0; the step runs in place
  double* prev = hp;
  for (; done < nsteps; ++done) {
    double* now = prev == hp ? t[0] : hp;
    if ((st = rhs(sp, now))) return st;
    if ((st = launch_step(p, 1, 0, sp, now, prev, sp, s))) return st;
    if ((st = filter())) return st;
    prev = now;
  }
  if (prev != hp) MLG_HIP_TRY(hipMemcpyAsync(hp, prev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return MLG_OK;
}

mlg_status mlg_synthesize(mlg_plan p, const void* psi, const void* chi, void* uw, void* ws, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_synthesize")) return st;
  if (!psi || !chi || !uw || !ws) return fail(MLG_E_ARG, "null buffer");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = partition(p, ws);
  mlg_status st;
  if ((st = launch_synth_gemm(p, static_cast<const double*>(psi), static_cast<const double*>(chi), w.X, s))) return st;
  if ((st = launch_proxy_fields(p, w.X, s))) return st;
  const int64_t mrows = (int64_t)p->M * p->nr;
  const size_t pe = (size_t)p->nz * p->nr * p->nphi;
  for (int i = 0; i < 6; ++i) {
    if ((st = launch_zfft(p, w.X[i], w.X[i], mrows, +1, nullptr, 0, -1, s))) return st;
    if ((st = launch_phi_backward(p, w.X[i], static_cast<double*>(uw) + i * pe, s))) return st;
  }
  return MLG_OK;
}

mlg_status mlg_tp_energy(mlg_plan p, const void* psi, const void* chi, double* energy, void* ws, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_tp_energy")) return st;
  if (!psi || !chi || !energy || !ws) return fail(MLG_E_ARG, "null buffer");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = partition(p, ws);
  if (mlg_status st = launch_synth_gemm(p, static_cast<const double*>(psi), static_cast<const double*>(chi), w.X, s))
    return st;
  if (mlg_status st = launch_proxy_fields(p, w.X, s)) return st;
  return launch_energy(p, w.X, energy, w.T[0], s);
}

mlg_status mlg_tp_enstrophy(mlg_plan p, const void* psi, const void* chi, double* enstrophy, void* ws, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_tp_enstrophy")) return st;
  if (!psi || !chi || !enstrophy || !ws) return fail(MLG_E_ARG, "null buffer");
  DeviceGuard guard(p->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = partition(p, ws);
  if (mlg_status st = launch_synth_gemm(p, static_cast<const double*>(psi), static_cast<const double*>(chi), w.X, s))
    return st;
  if (mlg_status st = launch_proxy_fields(p, w.X, s)) return st;
  return launch_energy(p, w.X + 3, enstrophy, w.T[0], s);   // the same quadrature on the vorticity
}

mlg_status mlg_laplacian_solve(mlg_plan p, int variant, const void* f, void* s, double* c, void* ws, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_laplacian_solve")) return st;
  if (!f || !s || !ws || !c) return fail(MLG_E_ARG, "null buffer");
  if (f == s) return fail(MLG_E_ARG, "f and s must not alias");
  if (variant != MLG_LOG_PRESCRIBE && variant != MLG_LOG_SOLVE) return fail(MLG_E_ARG, "unknown variant");
  DeviceGuard guard(p->device);
  Ws w = partition(p, ws);
  double* c_in = variant == MLG_LOG_PRESCRIBE ? c : nullptr;
  double* c_out = variant == MLG_LOG_SOLVE ? c : nullptr;
  return launch_poisson(p, variant, static_cast<const double*>(f), static_cast<double*>(s), c_in, c_out, w.T[0],
                        w.T[1], static_cast<hipStream_t>(stream));
}

mlg_status mlg_remove_far_field(mlg_plan p, void* spec, void* stream) {
  if (mlg_status st = check_fp64(p, "mlg_remove_far_field")) return st;
  if (!spec) return fail(MLG_E_ARG, "null buffer");
  DeviceGuard guard(p->device);
  return launch_far_field(p, static_cast<double*>(spec), static_cast<hipStream_t>(stream));
}

mlg_status mlg_set_log_proxy(mlg_plan p, double c_psi, double c_chi) {
  if (mlg_status st = check_plan(p)) return st;
  if (!std::isfinite(c_psi) || !std::isfinite(c_chi)) return fail(MLG_E_ARG, "proxy amplitudes must be finite");
  if (p->prec != MLG_FP64 && (c_psi != 0.0 || c_chi != 0.0))
    return fail(MLG_E_UNSUPPORTED, "logarithmic proxy amplitudes need an MLG_FP64 plan");
  p->log_cpsi = c_psi;
  p->log_cchi = c_chi;
  return MLG_OK;
}

mlg_status mlg_timing_enable(mlg_plan p, int enable) {
  if (mlg_status st = check_plan(p)) return st;
  p->timing.enabled = enable != 0;
  return MLG_OK;
}

mlg_status mlg_timing_read(mlg_plan p, const char* kernel, double* total_ms, int64_t* launches) {
  if (mlg_status st = check_plan(p)) return st;
  if (!kernel || !total_ms || !launches) return fail(MLG_E_ARG, "null argument");
  DeviceGuard guard(p->device);
  double ms = 0;
  int64_t n = 0;
  auto& recs = p->timing.recs;
  std::vector<mlg::Timing::Rec> keep;
  for (auto& r : recs) {
    if (r.name != kernel) {
      keep.push_back(r);
      continue;
    }
    MLG_HIP_TRY(hipEventSynchronize(r.b));
    float t = 0;
    MLG_HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    ++n;
    p->timing.pool.push_back(r.a);
    p->timing.pool.push_back(r.b);
  }
  recs.swap(keep);
  *total_ms = ms;
  *launches = n;
  return MLG_OK;
}

}  // extern "C"
