/*
 * mlg.h -- C ABI of an MI355X (gfx950) library for the mapped associated-Legendre /
 * Fourier spectral method of Lee & Wang, "MLegS: A modern mapped Legendre spectral
 * method solver for unbounded domains with parallelization".
 *
 * The library computes, on one GPU, the physical <-> spectral transform pair of
 * Eq. expansion (Sec. 3.1; the transform order of Sec. 4.1), the pseudospectral
 * scalar products of Sec. 3.3 and Sec. 5.2, and the toroidal-poloidal nonlinear term
 * P[(U + u) x omega] of Sec. 3.2 / Sec. 5.3 (Eq. tp, Eq. tp-poisson, Eq. tp-evolution).
 *
 * Conventions shared by every entry point
 *  - Every call returns mlg_status; 0 (MLG_OK) is success.  No exception crosses the
 *    ABI.  mlg_last_error() returns a thread-local message for the last failure.
 *  - Device buffers (phys, spec, ws, ...) are owned by the caller: plain device
 *    pointers allocated with hipMalloc (or any allocator of the same device).  The
 *    plan owns its own device tables and frees them in mlg_plan_destroy.
 *  - 'stream' is a hipStream_t passed as void* (NULL = the default stream).  Work is
 *    enqueued asynchronously; argument errors are reported synchronously; device
 *    errors surface as MLG_E_DEVICE on the call that detects them.
 *  - One plan may be used from one stream at a time; concurrent streams need their
 *    own workspace buffers.
 *
 * Data layouts (MLG_FP64 plans: real = double, complex = interleaved double pair; MLG_FP32
 * and MLG_SPLIT_BF16 plans and FP32 batches: float / interleaved float pair; real_bytes of
 * mlg_plan_query says which)
 *  - physical field: real [N_z][N_r][N_phi], element (l, i, j) = s(r_i, phi_j, z_l),
 *    r_i ascending (x_i the Gauss-Legendre nodes, r = ell sqrt((1+x)/(1-x)), Eq. map),
 *    phi_j = 2 pi j / N_phi, z_l = L_z l / N_z.
 *  - spectral field: complex, packed triangular [tau][N_z]; row off(m) + (n - m) holds
 *    shat_{n m k} for m = 0 .. M-1, n = m .. N_r^c-1, off(m) = sum_{m'<m} (N_r^c - m'),
 *    tau = off(M).  Column kk is the FFT slot of k (kk = k mod N_z).  Slots with
 *    |k| >= N_z^c and the Nyquist slot are written as zero and never read.
 *    Only m >= 0 is stored; shat_{n,-m,-k} = conj(shat_{n,m,k}) (Sec. 3.1).  The m = 0
 *    harmonic enters the backward transform through its real part; a real field has a
 *    Hermitian m = 0 column, which the library does not enforce.
 *  - normalisation: forward = (1/(N_phi N_z)) sum over phi and z, then Gauss-Legendre
 *    projection sum_i w_i Pbar_n^m(x_i); backward = the plain sum of Eq. expansion.
 *    Pbar_n^m = N_n^m P_n^m (Eq. norm) without the Condon-Shortley phase.
 */
#ifndef MLG_H
#define MLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLG_OK = 0,
  MLG_E_ARG = 1,          /* invalid argument (null pointer, size, chop, unsupported value) */
  MLG_E_ALLOC = 2,        /* device or host allocation failed                               */
  MLG_E_DEVICE = 3,       /* a HIP call or kernel launch failed                             */
  MLG_E_UNSUPPORTED = 4,  /* valid request the library does not implement (e.g. FFT length) */
  MLG_E_NONFINITE = 5     /* non-finite input to plan creation                              */
} mlg_status;

typedef enum {
  MLG_FP64 = 0,        /* double data, FP64 arithmetic (MFMA f64 for the radial products)    */
  MLG_FP32 = 1,        /* float data.  Batches: streamed tables (built in FP64), FP32        */
                       /* arithmetic.  Plans: the radial products of the transform pair, the */
                       /* scalar RHS and the vector synthesis on FP32 MFMA with FP32 tables   */
                       /* (built in FP64); the FFTs and pointwise products in FP64 arithmetic */
                       /* on float-stored intermediates; the projection's source products    */
                       /* and solves in FP64 (they read the float-stored N and are ill-      */
                       /* conditioned along far-field directions, so reduced-precision       */
                       /* products there would be amplified)                                 */
  MLG_SPLIT_BF16 = 2   /* plans only, float data: the radial products of the transform pair,  */
                       /* the scalar RHS and the vector synthesis, and their z transforms as  */
                       /* two radix-16 DFT products, on MFMA with hi/lo bfloat16 operands and */
                       /* FP32 accumulation (a_hi b_hi + a_hi b_lo + a_lo b_hi); the phi FFTs, */
                       /* pointwise products, the projection's forward z transforms, source   */
                       /* products and solves as for MLG_FP32                                 */
} mlg_precision;

/* Reduced-precision plans (MLG_FP32, MLG_SPLIT_BF16) need N_phi = N_z = 256, an even N_r,
 * N_r <= 32768 and N_r^c <= 512; they serve mlg_forward, mlg_backward, mlg_rhs_scalar,
 * mlg_rhs_tp and mlg_rhs_tp_noalloc (the taps stay double).  Every other plan entry point,
 * the closure and truncation need MLG_FP64 plans and return MLG_E_UNSUPPORTED otherwise. */

enum { MLG_RHS_U2 = 0, MLG_RHS_KPP = 1 };

/* Grid and chops of one field (Sec. 3.1).  Chops: 0 selects the default
 * N_r^c = N_r, N_phi^c = N_phi/2 (orders m < N_phi/2), N_z^c = max(1, N_z/2).
 * Bounds enforced: 2 <= N_r, N_r^c <= N_r, N_phi^c <= N_phi/2 + 1, N_z^c <= N_z/2 + 1,
 * ell > 0, L_z > 0, all finite.  'dealias' = 1 applies the two-thirds mask (keep
 * m <= floor((N_phi-1)/3) and |k| <= floor((N_z-1)/3)) to the fields entering the RHS products
 * and to the RHS outputs (Sec. 3.3: the dealiasing margin between chop and collocation count,
 * in which the fields of a product hold no mode): input modes outside the mask are read as zero. */
typedef struct {
  int32_t nr, nphi, nz;
  int32_t nrc, nphic, nzc;
  double ell, lz;
  int32_t dealias;
} mlg_grid;

/* Sizes of the arrays a plan reads and writes. */
typedef struct {
  int64_t phys_elems;       /* N_z * N_r * N_phi reals                                   */
  int64_t spec_rows;        /* tau                                                       */
  int64_t spec_elems;       /* tau * N_z complex values                                  */
  int64_t workspace_bytes;  /* bytes of device workspace every call of this plan needs  */
  int32_t M;                /* stored azimuthal orders                                   */
  int32_t nrc, nzc;         /* resolved radial and axial chops                           */
  int32_t real_bytes;       /* bytes of one real of the data arrays (8 for MLG_FP64 plans, */
                            /* 4 for MLG_FP32 and MLG_SPLIT_BF16 plans)                    */
  int32_t dealias_m, dealias_k;  /* largest kept m and |k| under the two-thirds mask     */
} mlg_layout;

typedef struct mlg_plan_s* mlg_plan;

/* Create a plan: validates the grid, builds on the host in FP64 the Gauss-Legendre nodes
 * and weights, the tables Pbar_n^m(x_i) (Eq. norm, normalised recurrence, no factorials),
 * r d/dr Pbar, the horizontal-Laplacian Gram factors of Eq. del2h-entries and the FFT
 * twiddles, then copies them to 'device'.  Errors: MLG_E_ARG for bad sizes/chops/ell,
 * MLG_E_NONFINITE for non-finite ell or L_z, MLG_E_UNSUPPORTED for N_phi or N_z whose
 * factors are not all 2, 3 or 5, or N_phi, N_z above 1024, or a reduced-precision plan off its
 * sizes (see above); MLG_E_ALLOC/DEVICE on HIP failure.
 * On failure *out is NULL and nothing is leaked.  For even N_r the FP64 radial products of the
 * vector RHS use the node symmetry x -> -x and the parity of Pbar_n^m (half the flops); the
 * environment variable MLG_RADIAL_FOLD=0, read at creation, selects the unfolded products. */
mlg_status mlg_plan_create(const mlg_grid* grid, mlg_precision prec, int device, mlg_plan* out);

/* Free the plan's device tables.  NULL is accepted. */
mlg_status mlg_plan_destroy(mlg_plan plan);

/* Fill *out with the plan's array sizes. */
mlg_status mlg_plan_query(mlg_plan plan, mlg_layout* out);

/* Host copies (length N_r, any may be NULL) of the nodes x_i, weights w_i and radii r_i. */
mlg_status mlg_plan_nodes(mlg_plan plan, double* x, double* w, double* r);

/* Forward transform (Sec. 4.1 order: phi FFT, radial projection per m, z FFT):
 * phys (device, physical layout) -> spec (device, spectral layout).  ws: device
 * workspace of mlg_layout.workspace_bytes.  phys is not modified. */
mlg_status mlg_forward(mlg_plan plan, const void* phys, void* spec, void* ws, void* stream);

/* Backward transform, Eq. expansion: spec -> phys.  spec is not modified. */
mlg_status mlg_backward(mlg_plan plan, const void* spec, void* phys, void* ws, void* stream);

/* Pseudospectral scalar term (Sec. 3.3; Eq. kpp): out = Mask(F(g(B(Mask(u))))) with
 * g(u) = u^2 (kind MLG_RHS_U2) or gamma u (1 - u) (kind MLG_RHS_KPP); the mask is applied
 * (on the way in and on the way out) when the plan's grid has dealias = 1.  spec_u and spec_out
 * may not alias. */
mlg_status mlg_rhs_scalar(mlg_plan plan, int kind, double gamma, const void* spec_u,
                          void* spec_out, void* ws, void* stream);

/* Toroidal-poloidal nonlinear term (Sec. 3.2, Sec. 5.3, Eq. tp-evolution):
 * (psi_n, chi_n) = Mask(P[(U + u) x omega]) with u = curl(psi z) + curl curl(chi z),
 * omega = curl u and U = (U[0], U[1], U[2]) a uniform Cartesian background (host array;
 * NULL = 0); with dealias = 1, u and omega are those of the masked potentials (Mask(psi),
 * Mask(chi)): the orders and axial modes outside the mask are not read.  P takes the gradient-free part through the axial curl and curl-curl
 * (Eq. tp-poisson); the m = 0 blocks use the decay gauge psi, chi -> 0 as r -> infinity.
 * psi and chi are the regular parts of the potentials: a net circulation or axial volume flux
 * is carried by the logarithmic proxy amplitudes of mlg_set_log_proxy (Eq. logproxy), whose
 * velocity and vorticity enter u and omega here.  'taps' may be NULL; otherwise a device buffer of
 * 9 * phys_elems + 3 * spec_elems values (reals, then complex) receiving nodal
 * u_r, u_phi, u_z, w_r, w_phi, w_z, N_r, N_phi, N_z and the sources C, K, Zhat.
 * A radial margin N_r^c < N_r (Sec. 3.3) is allowed: the products are formed on the N_r nodes and
 * projected onto the degrees below N_r^c.  Requires N_r^c <= 512 (MLG_E_UNSUPPORTED otherwise). */
mlg_status mlg_rhs_tp(mlg_plan plan, const double* U, const void* psi, const void* chi,
                      void* psi_n, void* chi_n, void* taps, void* ws, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mlg_rhs_tp without the 'ws' argument.  The workspace is a
 * fixed array of 192 MiB (201326592 bytes) in the library's device memory, one copy per GPU, which
 * each GPU holds from the library's first use there until the process ends; the call allocates
 * nothing and launches the same kernels as mlg_rhs_tp, so the outputs are identical.  Plans whose
 * mlg_layout.workspace_bytes exceed the array get MLG_E_UNSUPPORTED (128^3 at the default chops fits);
 * a plan with timing hooks enabled gets MLG_E_ARG (they create events).  The array keeps the last
 * call's contents; no kernel relies on it starting at zero.  All calls on one GPU share the array:
 * calls that overlap in time on the same GPU (other streams, other threads) race and must be
 * serialised by the caller. */
mlg_status mlg_rhs_tp_noalloc(mlg_plan plan, const double* U, const void* psi, const void* chi,
                              void* psi_n, void* chi_n, void* taps, void* stream);

/* ---------------------------------------------------------------- semi-implicit time stepping
 * ds/dt = A(s) + L s (Sec. 3.3, Eq. split) with L = nu grad^2 - nu_h (-grad^2)^{p/2}
 * (Eq. dissipation), composed per (m, k) from the truncated horizontal Laplacian of
 * Eq. del2h-entries (grad^2 = Dbar_m - kappa^2). */
typedef struct {
  double nu, nu_h;  /* nu >= 0, nu_h >= 0 */
  int32_t p;        /* 4, 6 or 8 (used when nu_h > 0) */
  double dt;        /* > 0 */
} mlg_dissip;

/* Prepare the step operators for every m: -grad^2 = X_m + kappa^2 with X_m = G_m diag(n(n+1)) / ell^2
 * is diagonalised on the host in FP64 (X_m = V diag(lam) V^{-1}, V = L^{-1/2} Q with Q the
 * orthogonal eigenvectors of L^{1/2} G_m L^{1/2} / ell^2; the n = 0 row of m = 0 is treated
 * exactly as the block-triangular part it is), and V, V^{-1}, lam are uploaded.  A step then
 * applies the scalar functions of Eq. abcn / FE-BE to lam + kappa^2 between two products per m,
 * the same operator as a banded factorisation of I - h L per (m, k).  Replaces earlier step
 * operators; synchronises the device.  Errors: MLG_E_ARG, MLG_E_NONFINITE, MLG_E_ALLOC. */
mlg_status mlg_step_setup(mlg_plan plan, const mlg_dissip* d);
/* FE-BE step: out = (I - h L)^{-1} (s + h A) with h = dt/2 (half = 1) or h = dt (half = 0); the
 * Richardson start-up of Sec. 3.3 is s1 = 2 S_{dt/2}(S_{dt/2}(s0)) - S_dt(s0). */
mlg_status mlg_step_febe(mlg_plan plan, int half, const void* s, const void* A, void* out, void* stream);
/* AB-CN step, Eq. abcn: out = (I - dt/2 L)^{-1} [(I + dt/2 L) s + dt/2 (3 A_now - A_prev)].
 * All arrays spectral (packed triangular); out must not alias the inputs.  Calls on one plan
 * share its step scratch and must not overlap. */
mlg_status mlg_step_abcn(mlg_plan plan, const void* s, const void* A_now, const void* A_prev, void* out, void* stream);

/* Inverse Laplacian of a scalar (Sec. 3.1, Eq. laplacian, Eq. logproxy): s = (grad^2)^{-1} f per
 * harmonic, (Dbar_m - kappa_k^2) shat = fhat with the truncated Dbar_m of Eq. del2h-entries, for
 * every stored (m, k) other than m = k = 0 (slots outside the axial chop are written as zero).  The
 * m = k = 0 block is singular (Dbar_0 annihilates the constant Pbar_0^0); the potential carries one
 * extra real amplitude c of Lambda = ln(r^2 + ell^2), s = c Lambda + sum shat_n Pbar_n^0, and the
 * paper's two variants differ only in that block:
 *  MLG_LOG_PRESCRIBE: c is read from *c; Dbar_0 shat = fhat - c g with its first row replaced by
 *    the decay gauge sum_n Pbar_n^0(1) shat_n = 0 (g: the coefficients of grad_h^2 Lambda);
 *  MLG_LOG_SOLVE: the first column of Dbar_0 is replaced by g, so that the unknown of Pbar_0^0
 *    becomes c: [g | Dbar_0[:, 1:]] (c, shat_1, ...) = fhat; c is written to *c, and the constant
 *    shat_0, which the Laplacian does not see, is fixed by the same decay gauge.
 * The m = k = 0 column is that of a real field: the real part of fhat is used and the column of s
 * is real.  f, s: packed spectral arrays (no aliasing); c: device pointer to one double; ws: the
 * plan workspace.  Each (m, k) column is one thread's L D L^T sweep of the SPD system
 * (G_m + kappa^2 ell^2 L^-1) y = -ell^2 fhat, y = diag(n(n+1)) shat (Dbar_m = -G_m L / ell^2 with G_m the
 * pentadiagonal Gram matrix).  Errors: MLG_E_ARG (null or aliased buffers, unknown variant). */
enum { MLG_LOG_PRESCRIBE = 0, MLG_LOG_SOLVE = 1 };
mlg_status mlg_laplacian_solve(mlg_plan plan, int variant, const void* f, void* s, double* c, void* ws, void* stream);

/* Removal of the free far-field level of the axisymmetric components (Sec. 3.1): Pbar_n^0 tends to
 * Pbar_n^0(1) = sqrt((2n + 1)/2) as r -> infinity, so every m = 0 harmonic has the level
 * sum_n Pbar_n^0(1) shat_{n,0,k} at infinity.  For every axial slot it is removed through the
 * constant basis function: shat_{0,0,k} -= level / Pbar_0^0(1), i.e. the constant at infinity is
 * subtracted from the component everywhere and every derivative is unchanged.  In place on a
 * packed spectral array. */
mlg_status mlg_remove_far_field(mlg_plan plan, void* spec, void* stream);

/* Logarithmic proxies (Sec. 3.1, Eq. logproxy): the potentials are psi~ + c_psi Lambda and
 * chi~ + c_chi Lambda with Lambda(r) = ln(r^2 + ell^2), the spectral arrays holding the regular parts
 * psi~, chi~.  The proxy parts add u_phi = -2 c_psi r / (r^2 + ell^2), u_z = -c_chi grad_h^2 Lambda,
 * w_phi = c_chi d(grad_h^2 Lambda)/dr and w_z = -c_psi grad_h^2 Lambda (grad_h^2 Lambda =
 * 4 ell^2 / (r^2 + ell^2)^2) to the velocity and vorticity of mlg_rhs_tp, mlg_synthesize,
 * mlg_tp_energy and mlg_tp_enstrophy: a circulation -4 pi c_psi and an axial volume flux
 * -4 pi c_chi at infinity.  Both are constants of the motion, so mlg_tp_advance keeps them and adds
 * the dissipation of the proxy parts, c L Lambda (a fixed vector on the m = 0, k = 0 degrees, built
 * by mlg_step_setup), to the nonlinear terms of the regular parts.  Default 0 and 0.
 * Errors: MLG_E_ARG (non-finite amplitude). */
mlg_status mlg_set_log_proxy(mlg_plan plan, double c_psi, double c_chi);

/* Enstrophy per axial slot: the quadrature of mlg_tp_energy applied to the vorticity,
 *   enstrophy[kk] = (L_z / 2) int_0^{2 pi} int_0^inf |omega_k|^2 r dr dphi,
 * so that the sum over the slots is (1/2) int |omega|^2 dV over one axial period.  Same buffers
 * and errors as mlg_tp_energy (FP64 plans). */
mlg_status mlg_tp_enstrophy(mlg_plan plan, const void* psi, const void* chi, double* enstrophy, void* ws,
                            void* stream);

/* Value of one harmonic of a packed spectral field at arbitrary radii (Eq. expansion, Eq. map):
 *   out[j] = sum_{n=m}^{N_r^c-1} s_{n m kk} Pbar_n^m(x(r_j)),  x(r) = (r^2 - ell^2) / (r^2 + ell^2),
 * for 0 <= m < N_phi^c and axial slot 0 <= kk < N_z.  r: device array of npts radii (>= 0); out:
 * device array of npts complex values (2 npts doubles).  Pbar follows the normalised recurrence of the
 * plan's tables in FP64.  For m = 0, kk = 0 the value is the azimuthal and axial mean of the field at
 * radius r (the quantity whose level sets give a front radius).  Errors: MLG_E_ARG. */
mlg_status mlg_eval_harmonic(mlg_plan plan, const void* spec, int32_t m, int32_t kk, const double* r, int64_t npts,
                             void* out, void* stream);

/* Adaptive modal filter (Sec. 3.3, the paragraph on aliasing and dissipation), applied between
 * steps.  Every stored coefficient s_{n m k} of a field whose normalised index
 *   zeta = max(n / N_r^c, m / N_phi^c, |k| / N_z^c)
 * exceeds zeta_c is multiplied by exp(-eps ((zeta - zeta_c) / (1 - zeta_c))^8).  The amplitude eps
 * follows the fraction f of the field's coefficient energy (sum of |s|^2 over the stored
 * coefficients) held above zeta_c: each application measures f, moves eps towards
 * eps_max * clip((f - tau) / tau, 0, 1) by the fraction 'relax', then filters with the new eps.
 * eps starts at 0, so the filter stays inactive while f < tau; it is bounded by eps_max and each
 * field (slot 0: psi, slot 1: chi) keeps its own state on the device. */
typedef struct {
  double zeta_c;   /* cutoff, 0 <= zeta_c < 1 (2/3 is the value this library's driver uses)     */
  double tau;      /* target tail fraction, > 0 (the paper's default 2e-2)                      */
  double eps_max;  /* saturation amplitude, >= 0 (36: exp(-36) ~ 2e-16 at the last index)      */
  double relax;    /* relaxation per application, 0 < relax <= 1                               */
} mlg_filter_cfg;

/* Enable the filter with 'cfg' and reset both states to eps = 0, f = 0 (cfg NULL disables it).
 * While enabled, mlg_tp_advance filters psi (slot 0) and chi (slot 1) after every step.
 * Allocates the state on the first call; synchronises the device.  Errors: MLG_E_ARG for a
 * parameter out of range or non-finite, MLG_E_ALLOC. */
mlg_status mlg_filter_setup(mlg_plan plan, const mlg_filter_cfg* cfg);
/* One application to the packed spectral field 'spec' (device, modified in place) with state
 * slot 0 or 1; asynchronous on 'stream'.  Errors: MLG_E_ARG (filter not enabled, bad slot, NULL). */
mlg_status mlg_filter_apply(mlg_plan plan, int32_t slot, void* spec, void* stream);
/* Host copy of the state {eps_0, eps_1, f_0, f_1} (f: the tail fraction the last application
 * measured).  Synchronises the device.  Errors: MLG_E_ARG (filter never enabled), MLG_E_DEVICE. */
mlg_status mlg_filter_state(mlg_plan plan, double* out4);

/* Nodal velocity and vorticity of a toroidal-poloidal pair (Sec. 3.2, Eq. tp):
 * u = curl(psi z) + curl curl(chi z), omega = curl u.  'uw' is a device buffer of
 * 6 * phys_elems reals receiving u_r, u_phi, u_z, w_r, w_phi, w_z (physical layout each).
 * The radial products use the plan's precision. */
mlg_status mlg_synthesize(mlg_plan plan, const void* psi, const void* chi, void* uw, void* ws, void* stream);

/* Axial modal kinetic energy of a toroidal-poloidal pair: the diagnostic from which Sec. 5.3
 * (Results and validation) reads the growth rate of the Crow instability, alpha =
 * (pi b^2 / Gamma) d ln E_1 / dt.  For every axial FFT slot kk (signed k = kk for 2 kk < N_z,
 * else kk - N_z):
 *   energy[kk] = (L_z / 2) int_0^{2 pi} int_0^inf |u_k|^2 r dr dphi,
 * u_k the axial Fourier coefficient of the velocity of (psi, chi) (Eq. tp), the area integral
 * taken by the Gauss-Legendre rule in the mapped variable (r dr = ell^2/(1-x)^2 dx) and by
 * Parseval in phi; the sum over kk is the kinetic energy of one axial period.  psi, chi: device,
 * packed triangular spectra; energy: device array of N_z doubles (written); ws: the plan's
 * workspace.  FP64 plans only (MLG_E_UNSUPPORTED otherwise); null buffers: MLG_E_ARG.
 * Partial sums are added in a fixed order, so the result is deterministic. */
mlg_status mlg_tp_energy(mlg_plan plan, const void* psi, const void* chi, double* energy, void* ws, void* stream);

/* Optional per-kernel timing, for benchmarks and profiling (not needed for computation).
 * While enabled, every kernel launch of the plan is bracketed by two HIP events recorded on
 * the launch's stream.  mlg_timing_read waits for the recorded events, returns the summed
 * elapsed milliseconds and the launch count for kernel family 'kernel' ("radial_gemm",
 * "synth_gemm", "proj_gemm", "phi_fft", "z_fft", "projection", "mask"), and clears that family's
 * records.  Reading an unknown family returns 0 ms and 0 launches. */
mlg_status mlg_timing_enable(mlg_plan plan, int enable);
mlg_status mlg_timing_read(mlg_plan plan, const char* kernel, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------- batched 2D instances
 * Many independent 2D fields (N_z = 1) of uneven sizes, each with its own grid, advanced by three
 * persistent launches (backward transforms, azimuthal stage, forward projections, each block walking
 * its share of the phase's cost-sorted work list): the pseudospectral KPP term
 * R_b = Mask(F(gamma u (1 - u))), u = B(Mask(u_hat_b)), of Sec. 3.3 and Sec. 5.2 (Eq. kpp), for
 * every instance b with dealias = 1 in its grid (orders above the two-thirds mask are read as zero).  Spectra of all instances are packed in one device buffer: instance b occupies the
 * complex elements [spec_offsets[b], spec_offsets[b+1]) in the packed triangular layout of a
 * single 2D plan.  Data are complex128 (MLG_FP64) or complex64 (MLG_FP32); tables and the in-kernel
 * Legendre recurrence are built in FP64. */
typedef struct mlg_batch_s* mlg_batch;

/* Launch shape of the persistent kernels: regenerate Pbar by its recurrence in the backward
 * phase (1) or stream tables (0); threads per block (64, 128, 256); blocks per compute unit
 * (1..8, capped by occupancy); azimuthal lines per work item (even, 2..32). */
typedef struct {
  int32_t recurrence, threads, blocks_per_cu, lines;
} mlg_batch_config;

/* Build per-instance nodes, tables and work lists on the host (FP64) and copy them to 'device'.
 * Each grid needs N_z = 1, 2 <= N_r <= 256, 2 <= N_phi <= 256 with prime factors 2, 3, 5, ell > 0.
 * Errors: MLG_E_ARG, MLG_E_UNSUPPORTED, MLG_E_ALLOC, MLG_E_DEVICE; *out is NULL on failure. */
mlg_status mlg_batch_create(int count, const mlg_grid* grids, mlg_precision prec, int device, mlg_batch* out);
mlg_status mlg_batch_destroy(mlg_batch batch);
/* spec_offsets: host array of count + 1 entries (may be NULL); workspace_bytes may be NULL. */
mlg_status mlg_batch_query(mlg_batch batch, int64_t* spec_offsets, int64_t* workspace_bytes);
/* The three launches over all instances, in stream order.  spec_in and spec_out must not alias. */
mlg_status mlg_batch_rhs_scalar(mlg_batch batch, double gamma, const void* spec_in, void* spec_out, void* ws,
                                void* stream);
mlg_status mlg_batch_set_config(mlg_batch batch, const mlg_batch_config* config);
mlg_status mlg_batch_get_config(mlg_batch batch, mlg_batch_config* config);
/* Autotuner: times every candidate launch shape (recurrence or tables x 128/256 threads x 1, 2, 4, 8
 * blocks per CU x 4, 8, 16 lines per item) on the given buffers with HIP events, keeps the fastest
 * for later calls and returns it (chosen, best_ms may be NULL).  Overwrites spec_out. */
mlg_status mlg_batch_autotune(mlg_batch batch, double gamma, const void* spec_in, void* spec_out, void* ws,
                              void* stream, mlg_batch_config* chosen, double* best_ms);

/* ---------------------------------------------------------------- spectral truncation
 * Coefficients of the mapped Legendre-Fourier expansion (Sec. 3.1, Eq. expansion) do not depend
 * on the grid size, since Pbar_n^m is independent of N_r; moving a state between two plans is
 * therefore a copy: dst(m, n, k) = src(m, n, k) where the source stores (m, n, k) and the
 * destination's axial chop keeps k, else 0.  Both plans FP64 with equal ell and L_z
 * (MLG_E_ARG otherwise); src and dst are packed spectral arrays of their plans; no aliasing. */
mlg_status mlg_truncate(mlg_plan from, mlg_plan to, const void* src, void* dst, void* stream);

/* ---------------------------------------------------------------- learned coarse-grid closure
 * An addition to the paper's method (no passage defines it).  For a coarse FP64 plan with
 * N_r^c <= 64, a network corrects every (m, k) column of the toroidal-poloidal nonlinear term:
 * (psi_n, chi_n) <- (psi_n, chi_n) + C(psi, chi).  Columns: m = 0 .. M-1 times the axial slots
 * kept by the chop, in FFT order (k = 0, 1, .., k_max, -k_max, .., -1); column index
 * m * n_k + j.  Features of a column (MLG_CLOSURE_NIN = 258): Re psi_n, Im psi_n, Re chi_n,
 * Im chi_n for n = 0 .. 63 at offsets 0, 64, 128, 192 (zero for n < m or n >= N_r^c), then
 * m / M and k / k_max.  Outputs (MLG_CLOSURE_NOUT = 256) use the same four blocks of 64.
 * Network: tanh(W1 x' + b1) -> tanh(W2 h1 + b2) -> W3 h2 + b3 with x' = x * x_scale
 * (per feature); correction = output * y_scale (per output).  Hidden width 256; products in
 * bfloat16 on MFMA with FP32 accumulation; FP32 master weights, trained with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the mean squared error in the
 * normalised output space.  m = 0 corrections are made Hermitian in k.
 * The plain solver is the judge: a correction is dropped (fallback: the plain coarse term is
 * kept) when ||C|| or ||RHS|| is non-finite or ||C|| > beta ||RHS||, norms over both fields, and,
 * with a reference plan (mlg_closure_set_reference), when it moves the coarse term away from the
 * plain term evaluated on the finer grid. */
#define MLG_CLOSURE_NIN 258
#define MLG_CLOSURE_NOUT 256
#define MLG_CLOSURE_HIDDEN 256
typedef struct mlg_closure_s* mlg_closure;
typedef struct {
  int32_t max_batch;  /* largest training batch (rows), 1 .. 2^20 */
  double beta;        /* judge threshold, >= 0 */
} mlg_closure_cfg;

/* Parameters in host order W1 [256][258], b1 [256], W2 [256][256], b2, W3 [256][256], b3. */
int32_t mlg_closure_param_count(void);
/* The closure keeps a pointer to 'coarse', which must outlive it.  Weights start at zero and
 * scales at one.  Errors: MLG_E_ARG, MLG_E_UNSUPPORTED (non-FP64 plan or N_r^c > 64), MLG_E_ALLOC. */
mlg_status mlg_closure_create(const mlg_closure_cfg* cfg, mlg_plan coarse, mlg_closure* out);
mlg_status mlg_closure_destroy(mlg_closure closure);
mlg_status mlg_closure_columns(mlg_closure closure, int32_t* ncols);
/* Host arrays of mlg_closure_param_count() floats.  set_params also clears the Adam moments and
 * step count; get_grads returns the gradient of the last training step.  These synchronise. */
mlg_status mlg_closure_set_params(mlg_closure closure, const float* params);
mlg_status mlg_closure_get_params(mlg_closure closure, float* params);
mlg_status mlg_closure_get_grads(mlg_closure closure, float* grads);
/* Host arrays: x_scale [258] (finite), y_scale [256] (finite, non-zero). */
mlg_status mlg_closure_set_scales(mlg_closure closure, const float* x_scale, const float* y_scale);
mlg_status mlg_closure_get_scales(mlg_closure closure, float* x_scale, float* y_scale);
/* Raw (unscaled) features of every column of the coarse state (psi, chi): device float
 * [ncols][258]. */
mlg_status mlg_closure_features(mlg_closure closure, const void* psi, const void* chi, float* x_out, void* stream);
/* Raw targets: y_out [ncols][256] (device float) = (ref - coarse term) at the output positions,
 * with ref the truncated fine term and (psi_n, chi_n) the coarse term, all coarse-plan arrays. */
mlg_status mlg_closure_targets(mlg_closure closure, const void* ref_psi, const void* ref_chi, const void* psi_n,
                               const void* chi_n, float* y_out, void* stream);
/* Network on nb raw feature rows x [nb][258] -> raw outputs y [nb][256] (device floats);
 * 1 <= nb <= max(max_batch, ncols). */
mlg_status mlg_closure_forward(mlg_closure closure, const float* x, int32_t nb, float* y, void* stream);
/* One Adam step on nb rows of the raw data set (data_x [count][258], data_y [count][256], device
 * floats): rows idx[0 .. nb-1] (device int32, NULL = rows 0 .. nb-1), 1 <= nb <= max_batch.
 * loss_out (host, may be NULL) receives the batch loss before the update; the call then
 * synchronises the stream and reports MLG_E_ARG if an index was outside [0, count) (such rows
 * count as zero rows). */
mlg_status mlg_closure_train_step(mlg_closure closure, const float* data_x, const float* data_y,
                                  const int32_t* idx, int64_t count, int32_t nb, float lr, float* loss_out,
                                  void* stream);
/* Correct the coarse term (rhs_psi, rhs_chi) of the coarse state (psi, chi) in place, subject to
 * the judge.  used_fallback (host, may be NULL; non-NULL synchronises the stream) receives 1 when
 * the correction was dropped.  Calls that overlap on one closure race (shared buffers). */
mlg_status mlg_closure_infer(mlg_closure closure, const void* psi, const void* chi, void* rhs_psi, void* rhs_chi,
                             int32_t* used_fallback, void* stream);
/* Judge decisions so far (synchronises the device). */
mlg_status mlg_closure_stats(mlg_closure closure, int64_t* calls, int64_t* fallbacks);
/* The plain solver on a finer grid as judge of the closure's error: with a reference plan set, every
 * correction C of the coarse term A_c(s) is also compared with Ar = T A_ref(E s), the same
 * toroidal-poloidal term (mlg_rhs_tp with the background U, host array, NULL = 0) of the coarse
 * state zero-extended (E) to 'ref' and truncated back (T), and is dropped unless
 * ||A_c + C - Ar|| <= ||A_c - Ar|| (norms over both fields), besides the beta rule.  'ref' must be
 * FP64, on the same device, with equal ell and L_z, keep every coefficient of the coarse plan
 * (M, N_r^c and N_z^c at least the coarse values) and N_r^c <= 512, and outlive the closure; more
 * nodes than degrees (N_r > N_r^c, N_phi, N_z above the coarse ones) make Ar the over-resolved term
 * of the coarse state.  Its logarithmic-proxy amplitudes must match the coarse plan's.  NULL removes
 * the reference.  Allocates the reference workspace; synchronises.  Errors: MLG_E_ARG,
 * MLG_E_UNSUPPORTED, MLG_E_ALLOC. */
mlg_status mlg_closure_set_reference(mlg_closure closure, mlg_plan ref, const double* U);

/* ---------------------------------------------------------------- time integration of (psi, chi)
 * nsteps steps of Eq. abcn for both potentials (the operators of mlg_step_setup, which must have
 * been called), with A = mlg_rhs_tp(U, psi, chi), corrected by 'closure' when non-NULL (its
 * plan must be 'plan').  start = 1: the first step is the Richardson start-up of Sec. 3.3 and
 * (hist_psi, hist_chi) are outputs; start = 0: they hold A^{j-1} from the previous call.  On
 * return they hold A of the last state a step started from.  psi, chi are advanced in place and,
 * when mlg_filter_setup has enabled the filter, filtered after every step.
 * tmp: device buffer of 6 * spec_elems complex128; ws: the plan workspace. */
mlg_status mlg_tp_advance(mlg_plan plan, const double* U, void* psi, void* chi, void* hist_psi, void* hist_chi,
                          int32_t nsteps, int32_t start, mlg_closure closure, void* tmp, void* ws, void* stream);

/* Semi-implicit integration of one scalar, ds/dt = A(s) + L s (Sec. 3.3) with A = mlg_rhs_scalar(kind,
 * gamma) (Eq. kpp for MLG_RHS_KPP) and L the operator of mlg_step_setup: nsteps steps of Eq. abcn;
 * start = 1: the first is the Richardson start-up of Sec. 3.3 and 'hist' is an output; start = 0:
 * 'hist' holds A^{j-1} from the previous call.  On return 'hist' holds A of the last state a step
 * started from; 'state' is advanced in place and, when mlg_filter_setup has enabled the filter,
 * filtered after every step with state slot 0.  tmp: device buffer of 3 * spec_elems complex128;
 * ws: the plan workspace.  Errors: MLG_E_ARG (no step setup, NULL buffer, bad kind, nsteps < 0). */
mlg_status mlg_scalar_advance(mlg_plan plan, int32_t kind, double gamma, void* state, void* hist, int32_t nsteps,
                              int32_t start, void* tmp, void* ws, void* stream);

/* Message for the last error on this thread ("" if none). */
const char* mlg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLG_H */
