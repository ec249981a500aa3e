// Semi-implicit time stepping of ds/dt = A(s) + L s (Sec. 3.3) on the GPU.
//
// L = nu grad^2 - nu_h (-grad^2)^{p/2} (Eq. dissipation) acts per (m, k) harmonic as a banded
// matrix composed from the truncated horizontal Laplacian: grad^2 = Dbar_m - kappa^2 with
// Dbar_m = -G_m diag(n(n+1)) / ell^2 (G_m the exact Gram matrix <Pbar_n, (1-x)^2 Pbar_j>).  Its
// half-bandwidth is b = p with hyperviscosity, else 2.  At setup the host forms, per (m, |k|),
// the band of L and banded LU factors with partial pivoting of I - h L for h = dt/2 (AB-CN,
// Eq. abcn, and the half FE-BE sub-step) and h = dt (the full FE-BE sub-step of the Richardson
// start-up).  A step kernel runs one thread per (m, k) column: it forms the right-hand side
// (applying L with a register window of 2b + 1 coefficients), then forward elimination with
// the recorded row interchanges and back substitution with U (upper bandwidth 2b).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

using namespace ::mlg::dev;
using ld = long double;

constexpr int BMAX = 8;

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }

struct StepArgs {
  const double2* s;
  const double2* a1;   // A^j (or A for FE-BE)
  const double2* a0;   // A^{j-1} (AB-CN only)
  double2* out;
  const double* band;  // L band: per (row, c = 0..2b) x nkabs
  const double* fac;   // LU: per (row, c) x nkabs, c = 0..b-1 multipliers, b pivot offset, b+1.. U (1/U_nn first)
  const int64_t* off;
  int M, nrc, nz, nzc, b, nkabs, ncoef_band, ncoef_fac, mode;  // mode 0 FE-BE, 1 AB-CN
  double h;
};

__global__ __launch_bounds__(64) void step_kernel(StepArgs a) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= (int64_t)a.M * a.nz) return;
  const int m = (int)(col / a.nz);
  const int kk = (int)(col - (int64_t)m * a.nz);
  if (m >= a.nrc) return;
  const int nz = a.nz;
  const int K = a.nrc - m;
  const int64_t base = a.off[m];
  const int k = kval(kk, nz);
  const int ka = k < 0 ? -k : k;
  const bool nyq = (nz % 2 == 0 && nz > 1 && k == -(nz / 2));
  double2* out = a.out + base * nz + kk;
  const double2 z0 = make_double2(0.0, 0.0);
  if (nyq || ka >= a.nzc) {
    for (int t = 0; t < K; ++t) out[(int64_t)t * nz] = z0;
    return;
  }
  const double2* s = a.s + base * nz + kk;
  const double2* a1 = a.a1 + base * nz + kk;
  const double2* a0 = a.a0 ? a.a0 + base * nz + kk : nullptr;
  const int b = a.b;
  const int nk = a.nkabs;
  auto bandv = [&](int t, int c) { return a.band[((base + t) * a.ncoef_band + c) * nk + ka]; };
  auto facv = [&](int t, int c) { return a.fac[((base + t) * a.ncoef_fac + c) * nk + ka]; };
  // ---- right-hand side
  double2 win[2 * BMAX + 1];  // s_{t-b} .. s_{t+b}
#pragma unroll
  for (int j = 0; j < 2 * BMAX + 1; ++j) {
    const int t = j - b;
    win[j] = (j <= 2 * b && t >= 0 && t < K) ? s[(int64_t)t * nz] : z0;
  }
  for (int t = 0; t < K; ++t) {
    double2 r;
    if (a.mode == 1) {
      double2 Ls = z0;
#pragma unroll
      for (int j = 0; j < 2 * BMAX + 1; ++j)
        if (j <= 2 * b) Ls = cadd(Ls, cscale(win[j], bandv(t, j)));
      const double2 A1 = a1[(int64_t)t * nz], A0 = a0[(int64_t)t * nz];
      r = make_double2(win[b].x + a.h * Ls.x + a.h * (3.0 * A1.x - A0.x),
                       win[b].y + a.h * Ls.y + a.h * (3.0 * A1.y - A0.y));
    } else {
      const double2 A1 = a1[(int64_t)t * nz];
      r = make_double2(win[b].x + a.h * A1.x, win[b].y + a.h * A1.y);
    }
    out[(int64_t)t * nz] = r;
#pragma unroll
    for (int j = 0; j < 2 * BMAX; ++j) win[j] = win[j + 1];
    const int tn = t + b + 1;
    win[2 * BMAX] = z0;
#pragma unroll
    for (int j = 0; j < 2 * BMAX + 1; ++j)
      if (j == 2 * b) win[j] = tn < K ? s[(int64_t)tn * nz] : z0;
  }
  // ---- forward elimination with row interchanges: window v[0..b] = rows t .. t+b
  double2 v[BMAX + 1];
#pragma unroll
  for (int j = 0; j < BMAX + 1; ++j) v[j] = (j <= b && j < K) ? out[(int64_t)j * nz] : z0;
  for (int t = 0; t < K; ++t) {
    const int pv = (int)facv(t, b);
    double2 vp = v[0];
#pragma unroll
    for (int j = 1; j < BMAX + 1; ++j)
      if (j == pv) vp = v[j];
#pragma unroll
    for (int j = 1; j < BMAX + 1; ++j)
      if (j == pv) v[j] = v[0];
    v[0] = vp;
#pragma unroll
    for (int j = 1; j < BMAX + 1; ++j)
      if (j <= b) v[j] = csub(v[j], cscale(v[0], facv(t, j - 1)));
    out[(int64_t)t * nz] = v[0];
#pragma unroll
    for (int j = 0; j < BMAX; ++j) v[j] = v[j + 1];
    v[BMAX] = z0;
    const int tn = t + b + 1;
#pragma unroll
    for (int j = 0; j < BMAX + 1; ++j)
      if (j == b) v[j] = tn < K ? out[(int64_t)tn * nz] : z0;
  }
  // ---- back substitution with U (diagonal stored as its reciprocal, then 2b superdiagonals)
  double2 x[2 * BMAX];  // x_{t+1} .. x_{t+2b}
#pragma unroll
  for (int j = 0; j < 2 * BMAX; ++j) x[j] = z0;
  for (int t = K - 1; t >= 0; --t) {
    double2 r = out[(int64_t)t * nz];
#pragma unroll
    for (int j = 0; j < 2 * BMAX; ++j)
      if (j < 2 * b) r = csub(r, cscale(x[j], facv(t, b + 2 + j)));
    const double2 xt = cscale(r, facv(t, b + 1));
    out[(int64_t)t * nz] = xt;
#pragma unroll
    for (int j = 2 * BMAX - 1; j > 0; --j) x[j] = x[j - 1];
    x[0] = xt;
  }
}

// Banded helpers on the host (long double).  A band matrix of half-bandwidth w over n rows is
// stored row-major as n x (2w + 1), entry (i, j) at [i][j - i + w].
struct Band {
  int n = 0, w = 0;
  std::vector<ld> a;
  Band(int n_, int w_) : n(n_), w(w_), a((size_t)n_ * (2 * w_ + 1), 0) {}
  ld get(int i, int j) const {
    if (j < i - w || j > i + w || j < 0 || j >= n) return 0;
    return a[(size_t)i * (2 * w + 1) + (j - i + w)];
  }
  void set(int i, int j, ld v) { a[(size_t)i * (2 * w + 1) + (j - i + w)] = v; }
};

Band band_mul(const Band& A, const Band& B) {
  Band C(A.n, A.w + B.w);
  for (int i = 0; i < A.n; ++i)
    for (int j = std::max(0, i - C.w); j <= std::min(A.n - 1, i + C.w); ++j) {
      ld s = 0;
      for (int q = std::max({0, i - A.w, j - B.w}); q <= std::min({A.n - 1, i + A.w, j + B.w}); ++q)
        s += A.get(i, q) * B.get(q, j);
      C.set(i, j, s);
    }
  return C;
}

}  // namespace

mlg_status step_setup(mlg_plan_s* p, const mlg_dissip* d) {
  const int nrc = p->nrc, M = p->M, nz = p->nz;
  const int half = d->nu_h > 0 ? d->p / 2 : 1;
  const int b = 2 * half;
  const int kmax = std::max(0, std::min(p->nzc - 1, nz > 1 ? (nz - 1) / 2 : 0));
  const int nkabs = kmax + 1;
  const int ncb = 2 * b + 1, ncf = b + 2 + 2 * b;
  const ld ell2 = (ld)p->g.ell * (ld)p->g.ell;
  std::vector<double> band((size_t)p->tau * ncb * nkabs, 0.0);
  std::vector<double> fac[2];
  fac[0].assign((size_t)p->tau * ncf * nkabs, 0.0);
  fac[1].assign((size_t)p->tau * ncf * nkabs, 0.0);
  const ld hs[2] = {(ld)d->dt / 2, (ld)d->dt};
  for (int m = 0; m < M; ++m) {
    const int K = std::max(nrc - m, 0);
    if (K == 0) continue;
    // Gram entries of this order (the same exact construction as the projection's G)
    auto eps = [&](int n) -> ld { return (n <= m || n <= 0) ? 0 : sqrtl((ld)(n * n - m * m) / (ld)(4 * n * n - 1)); };
    for (int ka = 0; ka < nkabs; ++ka) {
      const ld kap = 2 * acosl(-1.0L) * ka / (ld)p->g.lz;
      Band X(K, 2);  // X = -(Dbar - kappa^2) = G L / ell^2 + kappa^2
      for (int i = 0; i < K; ++i) {
        const int n = m + i;
        for (int dj = -2; dj <= 2; ++dj) {
          const int j = i + dj;
          if (j < 0 || j >= K) continue;
          const int nj = m + j;
          ld g;
          const int lo = std::min(n, nj), hi = std::max(n, nj);
          if (hi == lo) g = 1 + eps(lo) * eps(lo) + eps(lo + 1) * eps(lo + 1);
          else if (hi == lo + 1) g = -2 * eps(hi);
          else g = eps(lo + 1) * eps(lo + 2);
          ld v = g * (ld)nj * (nj + 1) / ell2;
          if (dj == 0) v += kap * kap;
          X.set(i, j, v);
        }
      }
      // L = -nu X - nu_h X^{p/2}
      Band Lb(K, b);
      Band Xp = X;
      if (d->nu_h > 0)
        for (int q = 1; q < half; ++q) Xp = band_mul(Xp, X);
      for (int i = 0; i < K; ++i)
        for (int j = std::max(0, i - b); j <= std::min(K - 1, i + b); ++j) {
          ld v = -(ld)d->nu * X.get(i, j);
          if (d->nu_h > 0) v -= (ld)d->nu_h * Xp.get(i, j);
          Lb.set(i, j, v);
        }
      for (int i = 0; i < K; ++i)
        for (int c = 0; c < ncb; ++c) {
          const int j = i + c - b;
          band[((size_t)(p->off[m] + i) * ncb + c) * nkabs + ka] = (double)Lb.get(i, j);
        }
      // banded LU with partial pivoting of I - h L (upper bandwidth grows to 2b)
      for (int hi = 0; hi < 2; ++hi) {
        const int wu = 2 * b;
        std::vector<ld> A((size_t)K * (b + wu + 1), 0);  // row i holds columns i - b .. i + wu
        auto at = [&](int i, int j) -> ld& { return A[(size_t)i * (b + wu + 1) + (j - i + b)]; };
        for (int i = 0; i < K; ++i)
          for (int j = std::max(0, i - b); j <= std::min(K - 1, i + b); ++j)
            at(i, j) = (i == j ? 1 : 0) - hs[hi] * Lb.get(i, j);
        for (int t = 0; t < K; ++t) {
          int pr = t;
          ld best = fabsl(at(t, t));
          for (int r = t + 1; r <= std::min(K - 1, t + b); ++r)
            if (fabsl(at(r, t)) > best) { best = fabsl(at(r, t)); pr = r; }
          if (pr != t)
            for (int j = std::max(0, t - b); j <= std::min(K - 1, t + wu); ++j) {
              // rows t and pr both cover columns t .. t + wu after elimination of earlier columns
              if (j < pr - b || j > pr + wu || j < t - b || j > t + wu) continue;
              std::swap(at(t, j), at(pr, j));
            }
          const size_t fb = ((size_t)(p->off[m] + t) * ncf) * nkabs + ka;
          fac[hi][fb + (size_t)b * nkabs] = (double)(pr - t);
          const ld piv = at(t, t);
          for (int r = t + 1; r <= std::min(K - 1, t + b); ++r) {
            const ld l = at(r, t) / piv;
            at(r, t) = 0;
            fac[hi][fb + (size_t)(r - t - 1) * nkabs] = (double)l;
            if (l != 0)
              for (int j = t + 1; j <= std::min(K - 1, t + wu); ++j)
                if (j <= r + wu) at(r, j) -= l * at(t, j);
          }
          fac[hi][fb + (size_t)(b + 1) * nkabs] = (double)(1 / piv);
          for (int j = 1; j <= wu; ++j)
            fac[hi][fb + (size_t)(b + 1 + j) * nkabs] = (t + j < K) ? (double)at(t, t + j) : 0.0;
        }
      }
    }
  }
  for (double* q : {p->d_step_band, p->d_step_fac[0], p->d_step_fac[1]})
    if (q) (void)hipFree(q);
  p->d_step_band = p->d_step_fac[0] = p->d_step_fac[1] = nullptr;
  auto upl = [&](double** dst, const std::vector<double>& v) -> mlg_status {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(v.size(), 1) * sizeof(double));
    if (e != hipSuccess) { *dst = nullptr; return fail(MLG_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e)); }
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return fail(MLG_E_DEVICE, "hipMemcpy failed");
    return MLG_OK;
  };
  mlg_status st;
  if ((st = upl(&p->d_step_band, band)) || (st = upl(&p->d_step_fac[0], fac[0])) ||
      (st = upl(&p->d_step_fac[1], fac[1])))
    return st;
  p->step_b = b;
  p->step_nkabs = nkabs;
  p->step_dt = d->dt;
  p->step_ready = true;
  return MLG_OK;
}

mlg_status launch_step(const mlg_plan_s* p, int mode, int which, const double* s, const double* a1, const double* a0,
                       double* out, hipStream_t st) {
  StepArgs a{};
  a.s = reinterpret_cast<const double2*>(s);
  a.a1 = reinterpret_cast<const double2*>(a1);
  a.a0 = reinterpret_cast<const double2*>(a0);
  a.out = reinterpret_cast<double2*>(out);
  a.band = p->d_step_band;
  a.fac = p->d_step_fac[which];
  a.off = p->d_goff;
  a.M = p->M;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.nzc = p->nzc;
  a.b = p->step_b;
  a.nkabs = p->step_nkabs;
  a.ncoef_band = 2 * p->step_b + 1;
  a.ncoef_fac = p->step_b + 2 + 2 * p->step_b;
  a.mode = mode;
  a.h = which == 0 ? p->step_dt / 2 : p->step_dt;
  const int64_t cols = (int64_t)p->M * p->nz;
  dim3 grid((unsigned)((cols + 63) / 64));
  p->timing.begin("step", st);
  step_kernel<<<grid, 64, 0, st>>>(a);
  p->timing.end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string("step_kernel: ") + hipGetErrorString(e));
  return MLG_OK;
}

__global__ __launch_bounds__(256) void richardson_kernel(const double* half, const double* full, double* out,
                                                         int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 2.0 * half[i] - full[i];
}

mlg_status launch_richardson(const mlg_plan_s* p, const double* half, const double* full, double* out,
                             hipStream_t st) {
  const int64_t n = 2 * p->tau * p->nz;
  p->timing.begin("step", st);
  richardson_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(half, full, out, n);
  p->timing.end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string("richardson_kernel: ") + hipGetErrorString(e));
  return MLG_OK;
}

}  // namespace mlg
