// Inverse Laplacian of a scalar with the logarithmic proxy, and removal of the far-field level of
// axisymmetric components (Sec. 3.1: Eq. laplacian, Eq. logproxy and the far-field paragraph).
//
// Per harmonic (m, k) the Laplacian is Dbar_m - kappa^2 with Dbar_m = -G_m L / ell^2, G_m the SPD
// pentadiagonal Gram matrix <Pbar_n, (1-x)^2 Pbar_j> and L = diag(n (n + 1)) (the nodal identity
// behind Eq. del2h-entries).  On the degrees n >= n0 = max(m, 1) the system for y = L shat is
// (G_m + kappa^2 ell^2 L^-1) y = -ell^2 fhat, symmetric positive definite: one thread per column
// factors it as L D L^T while it sweeps the degrees upwards, keeping the factors in the workspace,
// and substitutes back downwards.  The degree n = 0 of m = 0 (the constant, which the horizontal
// Laplacian annihilates) follows from the first row for k != 0; for k = 0 the paper's two variants:
// the prescribed amplitude c (first row replaced by the decay gauge) or the amplitude solved for
// (first column replaced by the image g of grad_h^2 Lambda).  The second is the first with c chosen
// so that the first row holds: shat = shat^f - c shat^g, shat^g the plan constant response to g.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

using namespace ::mlg::dev;

mlg_status check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MLG_OK;
}

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }

struct PoissonArgs {
  const double2* f;
  double2* s;
  double2* fac;        // workspace: (l1, l2) per packed element
  double* rdiag;       // workspace: 1 / pivot per packed element
  const double* gram;  // plan Gram entries: g0 | g1 | g2 packed like the spectrum's rows
  const int64_t* off;  // packed row offset of every order
  const double* logsg; // [0] = g_0 - Dbar_{0,1:} shat^g, [n] = shat^g_n (n >= 1)
  const double* c_in;  // prescribed amplitude (variant 0)
  double* c_out;       // solved amplitude (variant 1)
  int64_t ngram;
  int M, nrc, nz, nzc, variant;
  double ell2, kap0, g0, g1, g2;  // g0..g2: the image of grad_h^2 Lambda on Pbar_0^0 .. Pbar_2^0
};

__device__ __forceinline__ bool kept_slot(int kk, int nz, int nzc) {
  const int k = kval(kk, nz);
  if (nz > 1 && 2 * kk == nz) return false;  // Nyquist
  return (k < 0 ? -k : k) < nzc;
}

// One thread per (m, kk) column; threads of a block share m and take consecutive slots.
__global__ __launch_bounds__(64) void poisson_kernel(PoissonArgs a) {
  const int m = blockIdx.y;
  const int kk = blockIdx.x * 64 + threadIdx.x;
  if (m >= a.M || kk >= a.nz) return;
  const int nz = a.nz, nrc = a.nrc;
  if (m >= nrc) return;
  const int64_t row0 = a.off[m];
  const double2* __restrict__ f = a.f + row0 * nz + kk;
  double2* __restrict__ s = a.s + row0 * nz + kk;
  const int cnt = nrc - m;
  if (!kept_slot(kk, nz, a.nzc)) {
    for (int t = 0; t < cnt; ++t) s[(int64_t)t * nz] = make_double2(0.0, 0.0);
    return;
  }
  double2* __restrict__ fac = a.fac + row0 * nz + kk;
  double* __restrict__ rd = a.rdiag + row0 * nz + kk;
  const double* __restrict__ G0 = a.gram + row0;
  const double* __restrict__ G1 = a.gram + a.ngram + row0;
  const double* __restrict__ G2 = a.gram + 2 * a.ngram + row0;
  const double kap = a.kap0 * kval(kk, nz);
  const double shift = kap * kap * a.ell2;
  const bool block00 = (m == 0 && kap == 0.0);
  const double cpre = (block00 && a.variant == 0) ? a.c_in[0] : 0.0;
  const int n0 = m > 0 ? m : 1;
  const int t0 = n0 - m;  // first solved row of the column
  // forward sweep: L D L^T of G + shift L^-1 on n >= n0, z = L^-1 b stored in s
  double d1 = 0.0, d2 = 0.0, l1p = 0.0;  // pivots of n-1, n-2 and l1 of n-1
  double2 z1 = make_double2(0.0, 0.0), z2 = z1;
  for (int t = t0; t < cnt; ++t) {
    const int n = m + t;
    const double Ln = (double)n * (n + 1.0);
    double2 b = f[(int64_t)t * nz];
    if (block00) {
      b.y = 0.0;
      const double gn = n == 1 ? a.g1 : (n == 2 ? a.g2 : 0.0);
      b.x -= cpre * gn;
    }
    b = cscale(b, -a.ell2);
    double l2 = 0.0, l1 = 0.0;
    if (t - 2 >= t0) l2 = G2[t - 2] / d2;
    if (t - 1 >= t0) {
      double g = G1[t - 1];
      if (t - 2 >= t0) g -= l2 * d2 * l1p;
      l1 = g / d1;
    }
    double d = G0[t] + shift / Ln;
    if (t - 1 >= t0) d -= l1 * l1 * d1;
    if (t - 2 >= t0) d -= l2 * l2 * d2;
    const double2 z = make_double2(b.x - l1 * z1.x - l2 * z2.x, b.y - l1 * z1.y - l2 * z2.y);
    fac[(int64_t)t * nz] = make_double2(l1, l2);
    rd[(int64_t)t * nz] = 1.0 / d;
    s[(int64_t)t * nz] = z;
    z2 = z1;
    z1 = z;
    d2 = d1;
    d1 = d;
    l1p = l1;
  }
  // backward sweep: y_n = z_n / d_n - l1_{n+1} y_{n+1} - l2_{n+2} y_{n+2}; shat_n = y_n / L_n
  double2 y1 = make_double2(0.0, 0.0), y2 = y1;   // y of n+1, n+2
  double l1n = 0.0, l2n = 0.0, l2nn = 0.0;        // l1 of n+1, l2 of n+1, l2 of n+2
  double2 ylo1 = y1, ylo2 = y1;                   // y of n0, n0 + 1 (for the first row of m = 0)
  for (int t = cnt - 1; t >= t0; --t) {
    const int n = m + t;
    const double2 z = s[(int64_t)t * nz];
    const double r = rd[(int64_t)t * nz];
    const double2 y = make_double2(z.x * r - l1n * y1.x - l2nn * y2.x, z.y * r - l1n * y1.y - l2nn * y2.y);
    const double2 fl = fac[(int64_t)t * nz];
    s[(int64_t)t * nz] = cscale(y, 1.0 / ((double)n * (n + 1.0)));
    y2 = y1;
    y1 = y;
    l2nn = l2n;
    l1n = fl.x;
    l2n = fl.y;
    if (t == t0) ylo1 = y;
    if (t == t0 + 1) ylo2 = y;
  }
  if (m != 0) return;
  // m = 0: the constant (degree 0)
  if (!block00) {
    // first row: sum_{j=1,2} Dbar_{0j} shat_j - kappa^2 shat_0 = f_0, Dbar_{0j} = -G_{0j} L_j / ell^2
    const double2 f0 = f[0];
    const double2 acc = make_double2(G1[0] * ylo1.x + (cnt > 2 ? G2[0] * ylo2.x : 0.0),
                                     G1[0] * ylo1.y + (cnt > 2 ? G2[0] * ylo2.y : 0.0));
    const double ik = 1.0 / (kap * kap);
    s[0] = make_double2((-acc.x / a.ell2 - f0.x) * ik, (-acc.y / a.ell2 - f0.y) * ik);
    return;
  }
  double c = cpre;
  if (a.variant == 1) {
    // c (g_0 - Dbar_{0,1:} shat^g) = f_0 - Dbar_{0,1:} shat^f, then shat = shat^f - c shat^g
    const double rowf = -(G1[0] * ylo1.x + (cnt > 2 ? G2[0] * ylo2.x : 0.0)) / a.ell2;
    c = (f[0].x - rowf) / a.logsg[0];
    for (int t = 1; t < cnt; ++t) {
      double2 v = s[(int64_t)t * nz];
      v.x -= c * a.logsg[t];
      s[(int64_t)t * nz] = v;
    }
    a.c_out[0] = c;
  }
  // decay gauge: sum_n Pbar_n^0(1) shat_n = 0 with Pbar_n^0(1) = sqrt((2n + 1) / 2)
  double lev = 0.0;
  for (int t = 1; t < cnt; ++t) lev += sqrt((2.0 * t + 1.0) * 0.5) * s[(int64_t)t * nz].x;
  s[0] = make_double2(-lev / sqrt(0.5), 0.0);
  for (int t = 1; t < cnt; ++t) s[(int64_t)t * nz].y = 0.0;
}

// shat_{0,0,k} -= (sum_n Pbar_n^0(1) shat_{n,0,k}) / Pbar_0^0(1), one thread per axial slot.
__global__ __launch_bounds__(64) void far_field_kernel(double2* spec, int nrc, int nz) {
  const int kk = blockIdx.x * 64 + threadIdx.x;
  if (kk >= nz) return;
  double2 lev = make_double2(0.0, 0.0);
  for (int n = 0; n < nrc; ++n) {
    const double v = sqrt((2.0 * n + 1.0) * 0.5);
    const double2 x = spec[(int64_t)n * nz + kk];
    lev.x += v * x.x;
    lev.y += v * x.y;
  }
  const double r = 1.0 / sqrt(0.5);
  double2 x0 = spec[kk];
  x0.x -= lev.x * r;
  x0.y -= lev.y * r;
  spec[kk] = x0;
}

}  // namespace

mlg_status launch_poisson(const mlg_plan_s* p, int variant, const double* f, double* s, const double* c_in,
                          double* c_out, double* ws0, double* ws1, hipStream_t st) {
  PoissonArgs a{};
  a.f = reinterpret_cast<const double2*>(f);
  a.s = reinterpret_cast<double2*>(s);
  a.fac = reinterpret_cast<double2*>(ws0);
  a.rdiag = ws1;
  a.gram = p->d_gram;
  a.off = p->d_goff;
  a.logsg = p->d_poisson;
  a.c_in = c_in;
  a.c_out = c_out;
  a.ngram = p->ngram;
  a.M = p->M;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.nzc = p->nzc;
  a.variant = variant;
  a.ell2 = p->g.ell * p->g.ell;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  // Eq. logproxy on the normalised basis: (4/3, -2, 2/3) / (sqrt((2n + 1)/2) ell^2)
  a.g0 = 4.0 / 3.0 / std::sqrt(0.5) / a.ell2;
  a.g1 = -2.0 / std::sqrt(1.5) / a.ell2;
  a.g2 = 2.0 / 3.0 / std::sqrt(2.5) / a.ell2;
  dim3 grid((unsigned)((p->nz + 63) / 64), (unsigned)p->M);
  poisson_kernel<<<grid, 64, 0, st>>>(a);
  return check("poisson_kernel");
}

mlg_status launch_far_field(const mlg_plan_s* p, double* spec, hipStream_t st) {
  far_field_kernel<<<(unsigned)((p->nz + 63) / 64), 64, 0, st>>>(reinterpret_cast<double2*>(spec), p->nrc, p->nz);
  return check("far_field_kernel");
}

}  // namespace mlg
