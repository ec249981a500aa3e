// Semi-implicit time stepping of ds/dt = A(s) + L s (Sec. 3.3) on the GPU.
//
// L = nu grad^2 - nu_h (-grad^2)^{p/2} (Eq. dissipation) acts per (m, k) harmonic through the
// truncated horizontal Laplacian: -grad^2 = X_m + kappa^2 with X_m = G_m diag(n(n+1)) / ell^2
// (G_m the exact Gram matrix <Pbar_n, (1-x)^2 Pbar_j>, Eq. del2h-entries).  Every step operator
// is a rational function of -grad^2:
//   FE-BE  out = Phi s + Psi A,       Phi = 1 / (1 - h L),          Psi = h / (1 - h L);
//   AB-CN  out = Phi s + Psi (3 A1 - A0), Phi = (1 + h L) / (1 - h L), Psi = h / (1 - h L),  h = dt / 2
// (Eq. abcn).  The paper factors the banded matrices I - h L per (m, k); here X_m is
// diagonalised once per m on the host, X_m = V diag(lam) V^{-1} with V = L^{-1/2} Q and
// S = L^{1/2} G L^{1/2} / ell^2 = Q diag(lam) Q^T symmetric (n >= max(m, 1), where L > 0).
// The eigenvectors do not depend on kappa, so for all k at once
//   out = V [Phi(lam + kappa^2) (V^{-1} s) + Psi(lam + kappa^2) (V^{-1} a)],
// two FP64 MFMA products per m with the scalar functions applied in between.  For m = 0 the
// n = 0 row of X is (0, b^T) (its column is zero since L_0 = 0), so X is block upper triangular
// and the n = 0 output gains b^T V diag((f(mu) - f(alpha)) / lam) V^{-1} s' terms (divided
// differences, alpha = kappa^2), evaluated in closed form without cancellation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
bool sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& Q);

namespace {

using namespace ::mlg::dev;
using ld = long double;

constexpr int TM = 64;  // rows per block
constexpr int TC = 16;  // complex columns per block
constexpr int TK = 16;  // k depth per LDS stage

#define MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }

struct StepArgs {
  const double2* s;
  const double2* a1;
  const double2* a0;   // AB-CN: A^{j-1}; FE-BE: null
  double2* out;
  double2* W;          // packed like the spectra (rows n >= n0 of each m)
  double2* W0;         // m = 0 divided-difference products [j][kk]
  const double* fwd;
  const double* bwd;
  const double* lam;
  const double* u;
  const int64_t* qoff;
  const int64_t* loff;
  const int64_t* off;
  int M, nrc, nz, nzc, mode, q;   // mode 0 FE-BE, 1 AB-CN; q = p / 2 (1 without hyperviscosity)
  int gx, gy, gz;                 // tiles: axial column blocks, row blocks, orders
  double h, nu, nuh, kap0;
};

__device__ __forceinline__ bool active_slot(int kk, int nz, int nzc) {
  const int k = kval(kk, nz);
  const int ka = k < 0 ? -k : k;
  return ka < nzc && !(nz % 2 == 0 && nz > 1 && k == -(nz / 2));
}

// 1 - h L(mu) with L(mu) = -nu mu - nu_h mu^q
__device__ __forceinline__ double denom(const StepArgs& a, double mu) {
  double pw = mu;
  for (int i = 1; i < a.q; ++i) pw *= mu;
  return 1.0 + a.h * (a.nu * mu + a.nuh * pw);
}

// Z = V^{-1} [s | a] per m, then W = Phi Zs + Psi Za (and the m = 0 divided differences)
__global__ __launch_bounds__(256) void step_fwd_kernel(StepArgs a) {
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  if (m >= a.M || m >= a.nrc) return;
  const int n0 = m == 0 ? 1 : 0;
  const int K = a.nrc - m - n0;
  const int j0 = tl.y * TM, kk0 = tl.x * TC;
  if (j0 >= K || kk0 >= a.nz) return;
  const int nz = a.nz;
  const double* __restrict__ A = a.fwd + a.qoff[m];
  const int64_t rb = (a.off[m] + n0) * nz;
  const double2* __restrict__ s = a.s + rb;
  const double2* __restrict__ p1 = a.a1 + rb;
  const double2* __restrict__ p0 = a.a0 ? a.a0 + rb : nullptr;
  __shared__ double As[2][TK][TM];
  __shared__ double Bs[2][2][TK][2 * TC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double4_t acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p) acc[p][0] = acc[p][1] = double4_t{0.0, 0.0, 0.0, 0.0};
  // raw loads with indices clamped into the operands (no branch around a load); the AB-CN
  // combination 3 A1 - A0 and the zeros outside the operands are formed at the LDS store, so the
  // loads of the next stage stay in flight across this stage's MFMAs
  double ra[4];
  double2 rs, r1, r0v;
  const double2* __restrict__ q0 = p0 ? p0 : p1;
  const double c1 = p0 ? 3.0 : 1.0, c0 = p0 ? 1.0 : 0.0;
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kr = e >> 6, rr = e & 63;
      const int k = k0 + kr, j = j0 + rr;
      const int kc = k < K ? k : K - 1, jc = j < K ? j : K - 1;
      ra[t] = A[(int64_t)kc * K + jc];
    }
    const int kr = tid >> 4, cc = tid & 15;
    const int k = k0 + kr, kk = kk0 + cc;
    const int kc = k < K ? k : K - 1, kkc = kk < nz ? kk : nz - 1;
    const int64_t i = (int64_t)kc * nz + kkc;
    rs = s[i];
    r1 = p1[i];
    r0v = q0[i];
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const bool ok = k0 + (e >> 6) < K && j0 + (e & 63) < K;
      As[buf][e >> 6][e & 63] = ok ? ra[t] : 0.0;
    }
    const int kr = tid >> 4, cc = tid & 15;
    const bool ok = k0 + kr < K && kk0 + cc < nz;
    const double2 v = make_double2(c1 * r1.x - c0 * r0v.x, c1 * r1.y - c0 * r0v.y);
    Bs[buf][0][kr][cc] = ok ? rs.x : 0.0;
    Bs[buf][0][kr][TC + cc] = ok ? rs.y : 0.0;
    Bs[buf][1][kr][cc] = ok ? v.x : 0.0;
    Bs[buf][1][kr][TC + cc] = ok ? v.y : 0.0;
  };
  const int nk = (K + TK - 1) / TK;
  load(0);
  store(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      const double av = As[buf][kr][wave * 16 + (lane & 15)];
      acc[0][0] = MFMA(av, Bs[buf][0][kr][lane & 15], acc[0][0]);
      acc[0][1] = MFMA(av, Bs[buf][0][kr][TC + (lane & 15)], acc[0][1]);
      acc[1][0] = MFMA(av, Bs[buf][1][kr][lane & 15], acc[1][0]);
      acc[1][1] = MFMA(av, Bs[buf][1][kr][TC + (lane & 15)], acc[1][1]);
    }
    if (kt + 1 < nk) store(buf ^ 1, (kt + 1) * TK);
    __syncthreads();
  }
  const int kk = kk0 + (lane & 15);
  if (kk >= nz || !active_slot(kk, nz, a.nzc)) return;
  const double kap = a.kap0 * kval(kk, nz);
  const double alpha = kap * kap;
  const double* lam = a.lam + a.loff[m];
  const double Da = denom(a, alpha);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = j0 + wave * 16 + (lane >> 4) + 4 * v;
    if (j >= K) continue;
    const double lj = lam[j];
    const double mu = lj + alpha;
    const double D = denom(a, mu);
    const double psi = a.h / D;
    const double phi = a.mode == 1 ? 2.0 / D - 1.0 : 1.0 / D;
    const double zsr = acc[0][0][v], zsi = acc[0][1][v], zar = acc[1][0][v], zai = acc[1][1][v];
    a.W[rb + (int64_t)j * nz + kk] = make_double2(phi * zsr + psi * zar, phi * zsi + psi * zai);
    if (m == 0) {
      // (f(mu) - f(alpha)) / lam in closed form: L(mu) - L(alpha) = lam * dl
      double sum = 0.0, mp = 1.0;
      for (int i = 0; i < a.q; ++i) {
        double ap = 1.0;
        for (int t = 0; t < a.q - 1 - i; ++t) ap *= alpha;
        sum += mp * ap;
        mp *= mu;
      }
      const double dl = -a.nu - a.nuh * sum;
      const double inv = a.h * dl / (D * Da);
      const double dphi = (a.mode == 1 ? 2.0 : 1.0) * inv;
      const double dpsi = a.h * inv;
      a.W0[(int64_t)j * nz + kk] = make_double2(dphi * zsr + dpsi * zar, dphi * zsi + dpsi * zai);
    }
  }
}

// out rows n >= n0 = V W per m; inactive axial slots are zeroed
__global__ __launch_bounds__(256) void step_bwd_kernel(StepArgs a) {
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  if (m >= a.M || m >= a.nrc) return;
  const int n0 = m == 0 ? 1 : 0;
  const int K = a.nrc - m - n0;
  const int r0 = tl.y * TM, kk0 = tl.x * TC;
  if (r0 >= K || kk0 >= a.nz) return;
  const int nz = a.nz;
  const double* __restrict__ A = a.bwd + a.qoff[m];
  const int64_t rb = (a.off[m] + n0) * nz;
  const double2* __restrict__ Wm = a.W + rb;
  __shared__ double As[2][TK][TM];
  __shared__ double Bs[2][TK][2 * TC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double4_t acc[2];
  acc[0] = acc[1] = double4_t{0.0, 0.0, 0.0, 0.0};
  // raw loads with clamped indices, zeros applied at the LDS store (as in step_fwd_kernel)
  double ra[4];
  double2 rbv;
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kr = e >> 6, rr = e & 63;
      const int k = k0 + kr, r = r0 + rr;
      const int kc = k < K ? k : K - 1, rc = r < K ? r : K - 1;
      ra[t] = A[(int64_t)kc * K + rc];
    }
    const int kr = tid >> 4, cc = tid & 15;
    const int k = k0 + kr, kk = kk0 + cc;
    const int kc = k < K ? k : K - 1, kkc = kk < nz ? kk : nz - 1;
    rbv = Wm[(int64_t)kc * nz + kkc];
  };
  auto store = [&](int buf, int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const bool ok = k0 + (e >> 6) < K && r0 + (e & 63) < K;
      As[buf][e >> 6][e & 63] = ok ? ra[t] : 0.0;
    }
    const int kr = tid >> 4, cc = tid & 15;
    const bool ok = k0 + kr < K && kk0 + cc < nz;
    Bs[buf][kr][cc] = ok ? rbv.x : 0.0;
    Bs[buf][kr][TC + cc] = ok ? rbv.y : 0.0;
  };
  const int nk = (K + TK - 1) / TK;
  load(0);
  store(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      const double av = As[buf][kr][wave * 16 + (lane & 15)];
      acc[0] = MFMA(av, Bs[buf][kr][lane & 15], acc[0]);
      acc[1] = MFMA(av, Bs[buf][kr][TC + (lane & 15)], acc[1]);
    }
    if (kt + 1 < nk) store(buf ^ 1, (kt + 1) * TK);
    __syncthreads();
  }
  const int kk = kk0 + (lane & 15);
  if (kk >= nz) return;
  const bool act = active_slot(kk, nz, a.nzc);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = r0 + wave * 16 + (lane >> 4) + 4 * v;
    if (r >= K) continue;
    a.out[rb + (int64_t)r * nz + kk] = act ? make_double2(acc[0][v], acc[1][v]) : make_double2(0.0, 0.0);
  }
}

// m = 0, n = 0: out = Phi(alpha) s0 + Psi(alpha) a0 + sum_j u_j W0[j].  A block takes R0C axial
// columns; the R0S lanes of a column sum every R0S-th j (their loads all in flight at once) and
// the partial sums are added in LDS in a fixed order.
constexpr int R0C = 16;  // columns per block
constexpr int R0S = 16;  // partial sums per column

__global__ __launch_bounds__(R0C * R0S) void step_row0_kernel(StepArgs a) {
  __shared__ double2 part[R0S][R0C];
  const int c = threadIdx.x % R0C, sl = threadIdx.x / R0C;
  const int kk = blockIdx.x * R0C + c;
  const int K = a.nrc - 1;
  double re = 0.0, im = 0.0;
  if (kk < a.nz) {
#pragma unroll 8
    for (int j = sl; j < K; j += R0S) {
      const double2 w = a.W0[(int64_t)j * a.nz + kk];
      re += a.u[j] * w.x;
      im += a.u[j] * w.y;
    }
  }
  part[sl][c] = make_double2(re, im);
  __syncthreads();
  if (sl != 0 || kk >= a.nz) return;
  if (!active_slot(kk, a.nz, a.nzc)) {
    a.out[kk] = make_double2(0.0, 0.0);
    return;
  }
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int q = 0; q < R0S; ++q) {
    sr += part[q][c].x;
    si += part[q][c].y;
  }
  const double kap = a.kap0 * kval(kk, a.nz);
  const double alpha = kap * kap;
  const double D = denom(a, alpha);
  const double psi = a.h / D;
  const double phi = a.mode == 1 ? 2.0 / D - 1.0 : 1.0 / D;
  const double2 s0 = a.s[kk];
  double2 v = a.a1[kk];
  if (a.a0) v = make_double2(3.0 * v.x - a.a0[kk].x, 3.0 * v.y - a.a0[kk].y);
  a.out[kk] = make_double2(phi * s0.x + psi * v.x + sr, phi * s0.y + psi * v.y + si);
}


// ---------------------------------------------------------------- adaptive modal filter
// Sec. 3.3: every coefficient whose normalised index zeta = max(n / N_r^c, m / N_phi^c,
// |k| / N_z^c) exceeds zeta_c is multiplied by exp(-eps ((zeta - zeta_c) / (1 - zeta_c))^8); eps
// follows the fraction f of sum |s|^2 held above zeta_c: target eps_max clip((f - tau) / tau, 0, 1),
// relaxed as eps <- eps + r (target - eps), one state per field.  Three launches: partial sums over
// a fixed number of blocks (so the reduction order never depends on the device), the state update
// in one block, and the scaling.  The state stays on the device: a time loop never waits for it.
struct FilterArgs {
  double2* spec;
  const int32_t* row_m;
  const int64_t* off;
  int64_t rows;
  int nz, nzc, nrc, M;
  double zc, tau, eps_max, relax;
  double* state;  // [eps_0, eps_1, f_0, f_1]
  double* part;   // FILTER_BLOCKS x (tail, total)
  int slot;
};

__device__ __forceinline__ double filter_zeta(const FilterArgs& a, int64_t row, int kk) {
  const int m = a.row_m[row];
  const int n = m + (int)(row - a.off[m]);
  const int k = (2 * kk < a.nz) ? kk : kk - a.nz;
  const double zr = (double)n / a.nrc, zp = (double)m / a.M, zz = (double)(k < 0 ? -k : k) / a.nzc;
  return fmax(fmax(zr, zp), zz);
}

__global__ __launch_bounds__(256) void filter_sums_kernel(FilterArgs a) {
  __shared__ double st[256], sa[256];
  const int t = threadIdx.x;
  double tail = 0.0, total = 0.0;
  const int64_t n = a.rows * a.nz;
  for (int64_t e = (int64_t)blockIdx.x * 256 + t; e < n; e += (int64_t)FILTER_BLOCKS * 256) {
    const int64_t row = e / a.nz;
    const int kk = (int)(e - row * a.nz);
    const double2 v = a.spec[e];
    const double w = v.x * v.x + v.y * v.y;
    total += w;
    if (filter_zeta(a, row, kk) > a.zc) tail += w;
  }
  st[t] = tail;
  sa[t] = total;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      st[t] += st[t + h];
      sa[t] += sa[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    a.part[2 * blockIdx.x] = st[0];
    a.part[2 * blockIdx.x + 1] = sa[0];
  }
}

__global__ __launch_bounds__(FILTER_BLOCKS) void filter_update_kernel(FilterArgs a) {
  __shared__ double st[FILTER_BLOCKS], sa[FILTER_BLOCKS];
  const int t = threadIdx.x;
  st[t] = a.part[2 * t];
  sa[t] = a.part[2 * t + 1];
  __syncthreads();
  for (int h = FILTER_BLOCKS / 2; h > 0; h >>= 1) {
    if (t < h) {
      st[t] += st[t + h];
      sa[t] += sa[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double f = sa[0] > 0.0 ? st[0] / sa[0] : 0.0;
    const double target = a.eps_max * fmin(fmax((f - a.tau) / a.tau, 0.0), 1.0);
    const double e0 = a.state[a.slot];
    a.state[a.slot] = e0 + a.relax * (target - e0);
    a.state[2 + a.slot] = f;
  }
}

__global__ __launch_bounds__(256) void filter_apply_kernel(FilterArgs a) {
  const double eps = a.state[a.slot];
  const int64_t n = a.rows * a.nz;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / a.nz;
    const int kk = (int)(e - row * a.nz);
    const double zeta = filter_zeta(a, row, kk);
    if (zeta > a.zc) {
      const double x = (zeta - a.zc) / (1.0 - a.zc);
      const double x2 = x * x, x4 = x2 * x2;
      const double sg = exp(-eps * (x4 * x4));
      const double2 v = a.spec[e];
      a.spec[e] = make_double2(v.x * sg, v.y * sg);
    }
  }
}

}  // namespace

mlg_status step_setup(mlg_plan_s* p, const mlg_dissip* d) {
  const int nrc = p->nrc, M = p->M, nz = p->nz;
  const int Mm = std::min(M, nrc);
  const ld ell2 = (ld)p->g.ell * (ld)p->g.ell;
  std::vector<int64_t> qoff(M + 1, 0), loff(M + 1, 0);
  for (int m = 0; m < M; ++m) {
    const int Kp = m < Mm ? nrc - m - (m == 0 ? 1 : 0) : 0;
    qoff[m + 1] = qoff[m] + (int64_t)Kp * Kp;
    loff[m + 1] = loff[m] + Kp;
  }
  std::vector<double> fwd(std::max<int64_t>(qoff[M], 1)), bwd(std::max<int64_t>(qoff[M], 1));
  std::vector<double> lam(std::max<int64_t>(loff[M], 1)), u(std::max(nrc - 1, 1), 0.0);
  std::atomic<int> next{0};
  std::atomic<bool> failed{false};
  auto work = [&]() {
    for (int m = next++; m < Mm; m = next++) {
      const int n0 = m == 0 ? 1 : 0;
      const int K = nrc - m - n0;
      if (K <= 0) continue;
      auto eps = [&](int n) -> ld {
        return (n <= m || n <= 0) ? 0 : sqrtl((ld)(n * n - m * m) / (ld)(4 * n * n - 1));
      };
      auto gram = [&](int n, int nj) -> ld {  // G_{n, nj} (pentadiagonal, symmetric)
        const int lo = std::min(n, nj), hi = std::max(n, nj);
        if (hi == lo) return 1 + eps(lo) * eps(lo) + eps(lo + 1) * eps(lo + 1);
        if (hi == lo + 1) return -2 * eps(hi);
        if (hi == lo + 2) return eps(lo + 1) * eps(lo + 2);
        return 0;
      };
      std::vector<ld> sq(K);
      for (int i = 0; i < K; ++i) {
        const ld n = m + n0 + i;
        sq[i] = sqrtl(n * (n + 1));
      }
      std::vector<double> S((size_t)K * K, 0.0), w, Q;
      for (int i = 0; i < K; ++i)
        for (int j = std::max(0, i - 2); j <= std::min(K - 1, i + 2); ++j)
          S[(size_t)i * K + j] = (double)(sq[i] * gram(m + n0 + i, m + n0 + j) * sq[j] / ell2);
      if (!sym_eig(K, S, w, Q)) {
        failed = true;
        continue;
      }
      double* F = fwd.data() + qoff[m];
      double* B = bwd.data() + qoff[m];
      for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) {
          F[(size_t)i * K + j] = (double)(Q[(size_t)i * K + j] * sq[i]);
          B[(size_t)j * K + i] = (double)(Q[(size_t)i * K + j] / sq[i]);
        }
      std::copy(w.begin(), w.end(), lam.begin() + loff[m]);
      if (m == 0) {
        // b_n = X_{0 n} = G_{0 n} n (n + 1) / ell^2 (n = 1, 2); u_j = sum_n b_n V[n][j]
        for (int j = 0; j < K; ++j) {
          ld acc = 0;
          for (int i = 0; i < std::min(K, 2); ++i) {
            const int n = 1 + i;
            const ld b = gram(0, n) * (ld)n * (n + 1) / ell2;
            acc += b * (ld)Q[(size_t)i * K + j] / sq[i];
          }
          u[j] = (double)acc;
        }
      }
    }
  };
  const unsigned hw = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  const int nthreads = (int)std::min<unsigned>(hw, (unsigned)std::max(Mm, 1));
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  if (failed) return fail(MLG_E_DEVICE, "step setup: eigen-decomposition did not converge");

  double** bufs[] = {&p->d_step_fwd, &p->d_step_bwd, &p->d_step_lam, &p->d_step_u, &p->d_step_w};
  for (double** q : bufs)
    if (*q) (void)hipFree(*q);
  if (p->d_step_qoff) (void)hipFree(p->d_step_qoff);
  if (p->d_step_loff) (void)hipFree(p->d_step_loff);
  if (p->d_logf) (void)hipFree(p->d_logf);
  p->d_logf = nullptr;
  p->d_step_fwd = p->d_step_bwd = p->d_step_lam = p->d_step_u = p->d_step_w = nullptr;
  p->d_step_qoff = p->d_step_loff = nullptr;
  p->step_ready = false;
  auto upl = [&](auto** dst, const auto& v) -> mlg_status {
    using T = typename std::decay_t<decltype(v)>::value_type;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(v.size(), 1) * sizeof(T));
    if (e != hipSuccess) { *dst = nullptr; return fail(MLG_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e)); }
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
      return fail(MLG_E_DEVICE, "hipMemcpy failed");
    return MLG_OK;
  };
  mlg_status st;
  if ((st = upl(&p->d_step_fwd, fwd)) || (st = upl(&p->d_step_bwd, bwd)) || (st = upl(&p->d_step_lam, lam)) ||
      (st = upl(&p->d_step_u, u)) || (st = upl(&p->d_step_qoff, qoff)) || (st = upl(&p->d_step_loff, loff)))
    return st;
  const size_t wel = ((size_t)p->tau + std::max(nrc - 1, 1)) * nz * 2;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->d_step_w), wel * sizeof(double));
  if (e != hipSuccess) {
    p->d_step_w = nullptr;
    return fail(MLG_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  int maxk = 0;
  for (int m = 0; m < Mm; ++m) maxk = std::max(maxk, nrc - m - (m == 0 ? 1 : 0));
  p->step_maxk = maxk;
  p->step_dt = d->dt;
  p->step_nu = d->nu;
  p->step_nuh = d->nu_h;
  p->step_q = d->nu_h > 0 ? d->p / 2 : 1;
  // the dissipation of the logarithmic proxies, a constant forcing of the regular parts (Eq. logproxy)
  std::vector<double> lf;
  proxy_forcing(p, d->nu, d->nu_h, p->step_q, lf);
  if ((st = upl(&p->d_logf, lf))) return st;
  p->step_ready = true;
  return MLG_OK;
}

mlg_status launch_step(const mlg_plan_s* p, int mode, int which, const double* s, const double* a1, const double* a0,
                       double* out, hipStream_t st) {
  StepArgs a{};
  a.s = reinterpret_cast<const double2*>(s);
  a.a1 = reinterpret_cast<const double2*>(a1);
  a.a0 = mode == 1 ? reinterpret_cast<const double2*>(a0) : nullptr;
  a.out = reinterpret_cast<double2*>(out);
  a.W = reinterpret_cast<double2*>(p->d_step_w);
  a.W0 = a.W + (size_t)p->tau * p->nz;
  a.fwd = p->d_step_fwd;
  a.bwd = p->d_step_bwd;
  a.lam = p->d_step_lam;
  a.u = p->d_step_u;
  a.qoff = p->d_step_qoff;
  a.loff = p->d_step_loff;
  a.off = p->d_goff;
  a.M = p->M;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.nzc = p->nzc;
  a.mode = mode;
  a.q = p->step_q;
  a.h = (mode == 1 || which == 0) ? p->step_dt / 2 : p->step_dt;
  a.nu = p->step_nu;
  a.nuh = p->step_nuh;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  const int mz = std::min(p->M, p->nrc);
  p->timing.begin("step", st);
  if (p->step_maxk > 0) {
    a.gx = (p->nz + TC - 1) / TC;
    a.gy = (p->step_maxk + TM - 1) / TM;
    a.gz = mz;
    const dim3 grid(xcd_blocks(a.gx, a.gy, a.gz));
    step_fwd_kernel<<<grid, 256, 0, st>>>(a);
    step_bwd_kernel<<<grid, 256, 0, st>>>(a);
  }
  step_row0_kernel<<<(unsigned)((p->nz + R0C - 1) / R0C), R0C * R0S, 0, st>>>(a);
  p->timing.end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string("step kernels: ") + hipGetErrorString(e));
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

mlg_status launch_filter(const mlg_plan_s* p, int slot, double* spec, hipStream_t st) {
  FilterArgs a{};
  a.spec = reinterpret_cast<double2*>(spec);
  a.row_m = p->d_row_m;
  a.off = p->d_goff;
  a.rows = p->tau;
  a.nz = p->nz;
  a.nzc = p->nzc;
  a.nrc = p->nrc;
  a.M = p->M;
  a.zc = p->filter_zc;
  a.tau = p->filter_tau;
  a.eps_max = p->filter_epsmax;
  a.relax = p->filter_relax;
  a.state = p->d_filter;
  a.part = p->d_filter + 4;
  a.slot = slot;
  const int64_t n = a.rows * a.nz;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  p->timing.begin("filter", st);
  filter_sums_kernel<<<FILTER_BLOCKS, 256, 0, st>>>(a);
  filter_update_kernel<<<1, FILTER_BLOCKS, 0, st>>>(a);
  filter_apply_kernel<<<blocks, 256, 0, st>>>(a);
  p->timing.end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string("filter kernels: ") + hipGetErrorString(e));
  return MLG_OK;
}

}  // namespace mlg
