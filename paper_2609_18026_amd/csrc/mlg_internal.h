// Internal declarations of the mlg library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mlg.h"

namespace mlg {

// Thread-local error message plus a helper that records it and returns a status.
void set_error(const std::string& msg);
mlg_status fail(mlg_status st, const std::string& msg);

#define MLG_HIP_TRY(expr)                                                               \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::mlg::fail(MLG_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// One radial product of the batched GEMM, per azimuthal order m:
//   C[rows x ncol] = A^T B with A stored k-major (K x rows, leading dim lda) and
//   B stored k-major (K x ncol, leading dim ncol).  Offsets are in elements.
struct GemmDesc {
  int64_t a_off, b_off, c_off;
  int32_t rows, K, lda, m;
};

constexpr int kMaxProds = 8;
struct GemmProds {
  const double* A[kMaxProds];
  const double* B[kMaxProds];
  double* C[kMaxProds];
  int32_t lscale[kMaxProds];  // 1: scale B row (degree n = k + m) by n(n+1)
  int32_t nprod;
};

// Pentadiagonal SPD Gram matrix G_m = <Pbar_n, (1-x)^2 Pbar_j> factored as L D L^T.
// Per m, entries for n = n0(m) .. nrc-1 where n0 = max(m, 1); stored at goff[m] + (n - n0).
struct GramFactors {
  std::vector<double> g0, g1, g2;  // G_{n,n}, G_{n,n+1}, G_{n,n+2}
  std::vector<double> d, l1, l2;   // D_n, L_{n,n-1}, L_{n,n-2}
  std::vector<int64_t> goff;       // size M + 1
};

}  // namespace mlg

namespace mlg {
// Event-pair recorder used when timing is enabled on a plan.
struct Timing {
  bool enabled = false;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void begin(const char* name, hipStream_t s);
  void end(hipStream_t s);
  ~Timing();
};
}  // namespace mlg

struct mlg_plan_s {
  mutable mlg::Timing timing;
  mlg_grid g{};
  mlg_precision prec = MLG_FP64;
  int device = 0;
  int nr = 0, nphi = 0, nz = 0, nrc = 0, M = 0, nzc = 0;
  int dealias_m = 0, dealias_k = 0;
  int64_t tau = 0;
  std::vector<int64_t> off;  // M + 1 triangular row offsets
  // host FP64 grid (ascending x)
  std::vector<double> x, w, r, theta, one_minus_x, one_plus_x, q, rinv;
  // device tables (FP64)
  double* d_Pb = nullptr;   // backward Pbar, per m [n-m][i]
  double* d_Pf = nullptr;   // forward w*Pbar, per m [i][n-m]
  double* d_Tb = nullptr;   // backward Tbar = (1-x^2) dPbar/dx, per m [n-m][i]
  double* d_Qf = nullptr;   // forward w*(Tbar - 2(1+x)Pbar), per m [i][n-m]
  // MLG_FP32 plans: the backward Pbar, Tbar and forward w Pbar tables rounded to float (same layouts)
  float* d_Pb32 = nullptr;
  float* d_Tb32 = nullptr;
  float* d_Pf32 = nullptr;
  double* d_node = nullptr; // nodal vectors: rinv[nr], q[nr], opx[nr], area weight w ell^2/(1-x)^2 [nr]
  double* d_tw_phi = nullptr;  // exp(-2 pi i t / N_phi), interleaved
  double* d_tw_z = nullptr;    // exp(-2 pi i t / N_z), interleaved
  int32_t* d_row_m = nullptr;  // azimuthal order of every triangular row
  mlg::GemmDesc* d_desc_fwd = nullptr;
  mlg::GemmDesc* d_desc_bwd = nullptr;
  double* d_gram = nullptr;    // packed g0,g1,g2 | LDL^T 1/d,l1,l2 | UDU^T 1/d,u1,u2 (9 * ngram)
  int64_t* d_goff = nullptr;
  int64_t ngram = 0;
  // L D L^T factors of G + kap^2 ell^2 L^-1 for every active (m, k) column of the projection:
  // (l1, l2) and 1 / pivot at [m][n - m][padded column of the aligned blocks, see col_blocks],
  // nrc + 2 rows per order (rows past the column and padding columns are zero); the identity for k = 0
  double2* d_qfl = nullptr;
  double* d_qfr = nullptr;
  int max_rows_fwd = 0, max_rows_bwd = 0;
  // inverse Laplacian of the m = k = 0 block (Eq. logproxy): [0] = g_0 - Dbar_{0,1:} shat^g and
  // [n] = shat^g_n for n >= 1, the response of the solved degrees to the image g of grad_h^2 Lambda
  double* d_poisson = nullptr;
  // split-bfloat16 tables (MLG_SPLIT_BF16 plans): hi / lo parts, rows padded to 32 entries
  unsigned short* d_split_syn[4] = {nullptr, nullptr, nullptr, nullptr};  // Pbar^T hi/lo, Tbar^T hi/lo [i][kpad]
  int64_t* d_split_syn_off = nullptr;
  int32_t* d_split_syn_kpad = nullptr;
  unsigned short* d_split_prj[2] = {nullptr, nullptr};  // W Pbar hi/lo [n-m][ipad] (scalar forward products)
  int64_t* d_split_prj_off = nullptr;
  int split_ipad = 0;
  uint32_t* d_split_zdft = nullptr;  // N_z = 256 split plans: DFT-product constants [dir][lane][40 words]
  // semi-implicit step operators (mlg_step_setup): per m, X_m = G_m L / ell^2 restricted to
  // n >= max(m, 1) is L^{-1/2} Q diag(lam) Q^T L^{1/2}; the step applies scalar functions of
  // lam + kappa^2 between the two products
  double* d_step_fwd = nullptr;   // per m [n][j] = Q[n][j] sqrt(L_n)     (V^{-1} as a k-major A operand)
  double* d_step_bwd = nullptr;   // per m [j][n] = Q[n][j] / sqrt(L_n)   (V as a k-major A operand)
  double* d_step_lam = nullptr;   // per m eigenvalues
  double* d_step_u = nullptr;     // m = 0: u_j = sum_n X_{0 n} V[n][j]
  int64_t* d_step_qoff = nullptr; // per m offsets into fwd / bwd (M + 1)
  int64_t* d_step_loff = nullptr; // per m offsets into lam (M + 1)
  double* d_step_w = nullptr;     // scratch: tau * nz complex + (nrc - 1) * nz complex
  int step_maxk = 0;
  double step_dt = 0, step_nu = 0, step_nuh = 0;
  int step_q = 1;                 // p / 2 (hyperviscosity power of grad^2), 1 when nu_h = 0
  bool step_ready = false;
  // adaptive modal filter (mlg_filter_setup): d_filter holds [eps_psi, eps_chi, f_psi, f_chi] and
  // then 2 * FILTER_BLOCKS partial sums
  double* d_filter = nullptr;
  bool filter_on = false;
  double filter_zc = 0, filter_tau = 0, filter_epsmax = 0, filter_relax = 0;
  // logarithmic proxy amplitudes of the potentials (mlg_set_log_proxy) and, once the step is set
  // up, the forcing L Lambda of the regular parts on the m = 0, k = 0 column (N_r^c reals)
  double log_cpsi = 0, log_cchi = 0;
  double* d_logf = nullptr;
  bool use_fast_fft = true;   // register-resident 256-point kernels when a length is 256
  bool use_fold = true;       // parity-folded radial products when N_r is even (MLG_RADIAL_FOLD=0 disables)
  int phi_rad[12] = {0};
  int phi_nrad = 0;
  int z_rad[12] = {0};
  int z_nrad = 0;
  // workspace partition (bytes)
  size_t ws_bytes = 0;
  size_t mixed_elems = 0;   // M * nr * nz complex
  size_t tri_elems = 0;     // tau * nz complex
};

namespace mlg {
// plan.cpp
int factor_radices(int n, int* rad);
// Gauss-Legendre nodes as angles theta_i (ascending x = cos theta) and weights, long double
void gl_theta(int N, std::vector<long double>& theta, std::vector<long double>& w);
// Pbar_n^m(cos t) for n = m .. nmax into out[n - m]
void pbar_col(int m, int nmax, long double t, long double* out);
// kernels.hip launchers (all enqueue on 'stream')
mlg_status launch_gemm(const mlg_plan_s* p, const GemmProds& prods, const GemmDesc* d_desc,
                       int max_rows, int ncol, hipStream_t stream);
mlg_status launch_phi_forward(const mlg_plan_s* p, const double* phys, double* mixed, hipStream_t s);
mlg_status launch_phi_backward(const mlg_plan_s* p, const double* mixed, double* phys, hipStream_t s);
mlg_status launch_phi_scalar_rhs(const mlg_plan_s* p, int kind, double gamma, double* mixed, hipStream_t s);
mlg_status launch_phi_vec_rhs(const mlg_plan_s* p, const double* U, double* const* f6, double* taps,
                              hipStream_t s);
// z-FFT over 'rows' contiguous lines of N_z complex values.  dir = -1 forward (scaled by 1/N_z),
// +1 backward.  The spectral side (the input of the backward transform, the output of the forward
// one) is zero outside the axial chop, at |k| > mask_k when mask_k >= 0, and on the rows whose
// order row_m[row] exceeds mask_m when row_m is given (the two-thirds mask).
mlg_status launch_zfft(const mlg_plan_s* p, const double* in, double* out, int64_t rows, int dir,
                       const int32_t* row_m, int mask_m, int mask_k, hipStream_t s);
// the same transform of nf fields (1..6) of `rows` lines each, in one launch where the kernel allows
// axial modal kinetic energy from the velocity harmonics u_r, u_phi, u_z (mixed layout)
mlg_status launch_energy(const mlg_plan_s* p, double* const* u3, double* energy, double* scratch, hipStream_t s);
// (fp64_only: the FP64 transforms also on a split-bfloat16 plan; kept_only: the forward transform
// may leave the slots outside the chop and masks unwritten, where the 256-point kernel runs)
mlg_status launch_zfft_fields(const mlg_plan_s* p, const double* const* in, double* const* out, int nf, int64_t rows,
                              int dir, const int32_t* row_m, int mask_m, int mask_k, hipStream_t s,
                              bool fp64_only = false, bool kept_only = false);
// Elliptic solves from the projection sources (C, K', Zhat); taps_src receives C, K, Zhat.
mlg_status launch_projection(const mlg_plan_s* p, const double* const* src3, double* psi_n, double* chi_n,
                             double* taps_src, hipStream_t s);
// gemm_fused.hip: synthesis of the six velocity / vorticity harmonics from (psi, chi), and the five
// projection products with the C, K', Zhat epilogue on the active (m < mmax, |k| <= kmax) columns.
// The two-thirds mask on the potentials that enter the RHS: orders above mkeep and axial slots with
// |k| > kmax are read as zero.  skip (folded and split synthesis): launch only the kept orders and
// the aligned column blocks of the kept slots; the harmonics of the other orders and blocks are
// then not written, and the z and phi stages after it must not use them.
struct SynthMask {
  int mkeep = 1 << 29, kmax = 1 << 29;
  bool skip = false;
};
mlg_status launch_synth_gemm(const mlg_plan_s* p, const double* psi, const double* chi, double* const* out6,
                             hipStream_t s, const SynthMask& mask = SynthMask());
mlg_status launch_proj_gemm(const mlg_plan_s* p, double* const* in3, double* const* out3, int mmax, int kmax,
                            hipStream_t s);
// gemm_fold.hip: the same two products folded over the node symmetry x -> -x (even N_r)
mlg_status launch_synth_fold(const mlg_plan_s* p, const double* psi, const double* chi, double* const* out6,
                             hipStream_t s, const SynthMask& mask);
// parity-folded radial products of one scalar field: dir > 0 backward (spectral rows -> harmonics
// at the nodes), dir < 0 forward; even N_r only
mlg_status launch_scalar_fold(const mlg_plan_s* p, int dir, const double* B, double* C, hipStream_t s);
mlg_status launch_proj_fold(const mlg_plan_s* p, double* const* in3, double* const* out3, int mmax, int kmax,
                            hipStream_t s);
// gemm_split.hip: the same two products with split-bfloat16 operands and FP32 accumulation
mlg_status launch_split_synth(const mlg_plan_s* p, const double* psi, const double* chi, double* const* out6,
                              hipStream_t s, const SynthMask& mask);
// split-bfloat16 radial products of the scalar transform pair: dir > 0 backward, dir < 0 forward
mlg_status launch_split_scalar(const mlg_plan_s* p, int dir, const double* in, double* out, hipStream_t s);
// split-bfloat16 z transforms of N_z = 256 as two radix-16 DFT products on MFMA (same arguments
// and masks as launch_zfft256)
mlg_status launch_split_zdft(const mlg_plan_s* p, const double* const* in, double* const* out, int nf, int64_t rows,
                             int dir, const int32_t* row_m, int mask_m, int mask_k, hipStream_t s);
// step.hip: semi-implicit operators and the step kernel (mode 0 FE-BE, 1 AB-CN; which 0: h = dt/2, 1: h = dt)
mlg_status step_setup(mlg_plan_s* p, const mlg_dissip* d);
mlg_status launch_step(const mlg_plan_s* p, int mode, int which, const double* s, const double* a1, const double* a0,
                       double* out, hipStream_t st);
// s1 = 2 half - full over all spectral elements (the Richardson start-up of Sec. 3.3)
mlg_status launch_richardson(const mlg_plan_s* p, const double* half, const double* full, double* out,
                             hipStream_t st);
// adaptive modal filter of Sec. 3.3 on one packed spectral field with state slot 'slot' (0, 1)
constexpr int FILTER_BLOCKS = 256;
mlg_status launch_filter(const mlg_plan_s* p, int slot, double* spec, hipStream_t s);
// plan.cpp: L Lambda = nu g + nu_h (-Dbar_0)^{q-1} g on the m = 0 degrees (g: the image of
// grad_h^2 Lambda, Eq. logproxy), in long double
void proxy_forcing(const mlg_plan_s* p, double nu, double nuh, int q, std::vector<double>& out);
// kernels.hip: the proxy parts of u_phi, u_z, w_phi, w_z added to the m = 0, k = 0 harmonics of the
// six synthesised fields (mixed layout), and the forcing added to the m = 0, k = 0 column of the RHS
mlg_status launch_proxy_fields(const mlg_plan_s* p, double* const* f6, hipStream_t s);
mlg_status launch_proxy_force(const mlg_plan_s* p, double* psi_n, double* chi_n, hipStream_t s);
// kernels.hip: one (m, kk) column of a packed spectral field evaluated at npts radii (complex out)
mlg_status launch_eval_harmonic(const mlg_plan_s* p, const double* spec, int m, int kk, const double* r, int64_t npts,
                                double* out, hipStream_t s);
// closure.hip: features -> network -> judge -> corrected (rpsi, rchi), all on 'st'
mlg_status closure_correct(mlg_closure_s* c, const double* psi, const double* chi, double* rpsi, double* rchi,
                           hipStream_t st);
const mlg_plan_s* closure_plan(const mlg_closure_s* c);
// active column bounds of the projection: m < mmax, |k| <= kmax
void active_columns(const mlg_plan_s* p, int* mmax, int* kmax);

// The projection's active axial slots (|k| <= kmax) in blocks of 8 consecutive FFT slots aligned
// to 8, so that the 8 complex values of a row a block touches form one aligned 128-byte segment:
// blocks 0 .. nbpos-1 cover slots 0 .. 8 nbpos - 1 (active where kk <= kmax), blocks nbpos ..
// nblk-1 cover slots nstart .. (active where kk >= nz - kmax).  A padded column index
// idx = 8 b + c (0 <= idx < 8 nblk) names one slot; the positive and negative ranges never share
// an active slot because kmax < nz / 2 (or nz = 1 and kmax = 0).
struct ColBlocks {
  int nbpos, nstart, nblk;
};
__host__ __device__ inline ColBlocks col_blocks(int kmax, int nz) {
  ColBlocks b;
  b.nbpos = (kmax + 8) / 8;
  b.nstart = ((nz - kmax) / 8) * 8;
  b.nblk = b.nbpos + (kmax >= 1 ? (nz - b.nstart + 7) / 8 : 0);
  return b;
}
__host__ __device__ inline int colblk_kk(const ColBlocks& b, int idx, int kmax, int nz, bool& active) {
  if (idx < 8 * b.nbpos) {
    active = idx <= kmax && idx < nz;
    return idx;
  }
  const int kk = b.nstart + idx - 8 * b.nbpos;
  active = kmax >= 1 && kk >= nz - kmax && kk < nz;
  return kk;
}
mlg_status launch_mask_tri(const mlg_plan_s* p, double* spec, hipStream_t s);
// poisson.hip: inverse Laplacian of a scalar (variant 0: prescribed amplitude *c_in, 1: solved into
// *c_out; ws0: tau * nz complex, ws1: tau * nz reals), and the far-field level removal of m = 0
mlg_status launch_poisson(const mlg_plan_s* p, int variant, const double* f, double* s, const double* c_in,
                          double* c_out, double* ws0, double* ws1, hipStream_t st);
mlg_status launch_far_field(const mlg_plan_s* p, double* spec, hipStream_t st);
// fft256.hip: register-resident 256-point transforms (used when N_z or N_phi equals 256)
mlg_status launch_zfft256(const mlg_plan_s* p, const double* const* in, double* const* out, int nf, int64_t rows,
                          int dir, const int32_t* row_m, int mask_m, int mask_k, hipStream_t s,
                          bool kept_only = false);
mlg_status launch_phi256_forward(const mlg_plan_s* p, const double* phys, double* mixed, hipStream_t s);
mlg_status launch_phi256_backward(const mlg_plan_s* p, const double* mixed, double* phys, hipStream_t s);
mlg_status launch_phi256_scalar(const mlg_plan_s* p, int kind, double gamma, double* mixed, hipStream_t s);
mlg_status launch_phi256_vec(const mlg_plan_s* p, const double* U, double* const* f6, double* taps, hipStream_t s);
}  // namespace mlg
