// Plan creation: grid, basis tables and operator factors, built on the host in FP64
// (long double where it buys accuracy), then copied to the device.
//
// * Gauss-Legendre nodes (Sec. 3.1, Eq. map): Newton iteration on P_N(cos theta) in the
//   angle theta, which keeps 1 - x = 2 sin^2(theta/2) and r = ell cot(theta/2) free of
//   cancellation near x = 1 (r -> infinity).
// * Pbar_n^m (Eq. norm): normalised three-term recurrence in n from
//   Pbar_m^m = sqrt(1/2) prod_j sqrt((2j+1)/(2j)) sin^m theta; its ratios are those of the
//   ln N_n^m accumulation of Sec. 3.1, so no factorial is ever formed.
// * r d/dr Pbar: the three-term derivative identity
//   (1 - x^2) Pbar_n' = (n+1) e_n Pbar_{n-1} - n e_{n+1} Pbar_{n+1}, e_n = sqrt((n^2-m^2)/(4n^2-1)),
//   which needs one extra recurrence row n = N_r^c.
// * Horizontal Laplacian (Eq. laplacian, Eq. del2h-entries): in the normalised basis
//   Dbar_m = -G_m diag(n(n+1)) / ell^2 with G_m = <Pbar_n, (1-x)^2 Pbar_j> the exact
//   (pentadiagonal, symmetric positive definite) Gram matrix, assembled as
//   (I - X)^2 from the Jacobi matrix X of multiplication by x.  G_m is factored L D L^T.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "mlg_internal.h"

namespace mlg {

thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

mlg_status fail(mlg_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

hipEvent_t Timing::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Timing::begin(const char* name, hipStream_t s) {
  if (!enabled) return;
  Rec r{name, get(), get()};
  if (!r.a || !r.b) return;
  (void)hipEventRecord(r.a, s);
  recs.push_back(r);
}

void Timing::end(hipStream_t s) {
  if (!enabled || recs.empty()) return;
  (void)hipEventRecord(recs.back().b, s);
}

Timing::~Timing() {
  for (auto& r : recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

int factor_radices(int n, int* rad) {
  int k = 0;
  while (n % 4 == 0) { rad[k++] = 4; n /= 4; }
  while (n % 2 == 0) { rad[k++] = 2; n /= 2; }
  while (n % 3 == 0) { rad[k++] = 3; n /= 3; }
  while (n % 5 == 0) { rad[k++] = 5; n /= 5; }
  if (n != 1) return -1;
  return k;
}

namespace {

using ld = long double;

// P_N(cos t) and P_{N-1}(cos t) by the Bonnet recurrence.
void legendre_pair(int N, ld c, ld* pn, ld* pnm1) {
  ld p0 = 1, p1 = c;
  if (N == 0) { *pn = 1; *pnm1 = 0; return; }
  for (int k = 2; k <= N; ++k) {
    ld p2 = ((2 * k - 1) * c * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *pnm1 = p0;
}

// Nodes in ascending x, returned as theta (descending) and weights.
void gauss_legendre_theta(int N, std::vector<ld>& theta, std::vector<ld>& w) {
  theta.assign(N, 0);
  w.assign(N, 0);
  const ld pi = acosl(-1.0L);
  for (int k = 1; k <= N; ++k) {
    ld t = pi * (4 * k - 1) / (4 * N + 2);  // k-th root from x = 1
    for (int it = 0; it < 100; ++it) {
      ld pn, pm;
      legendre_pair(N, cosl(t), &pn, &pm);
      // d/dt P_N(cos t) = -N (P_{N-1} - x P_N) / sin t
      ld dp = -N * (pm - cosl(t) * pn) / sinl(t);
      ld dt = pn / dp;
      t -= dt;
      if (fabsl(dt) < 1e-19L * (1 + fabsl(t))) break;
    }
    ld pn, pm;
    legendre_pair(N, cosl(t), &pn, &pm);
    ld s = sinl(t);
    int i = N - k;  // ascending x
    theta[i] = t;
    w[i] = 2 * s * s / ((ld)N * N * pm * pm);
  }
}

// Pbar_n^m(cos t) for n = m .. nmax (inclusive) at one angle; out[n - m].
void pbar_column(int m, int nmax, ld t, ld* out) {
  ld s = sinl(t), c = cosl(t);
  ld pmm = sqrtl(0.5L);
  for (int j = 1; j <= m; ++j) pmm *= sqrtl((ld)(2 * j + 1) / (ld)(2 * j)) * s;
  out[0] = pmm;
  if (nmax >= m + 1) out[1] = sqrtl((ld)(2 * m + 3)) * c * pmm;
  for (int n = m + 2; n <= nmax; ++n) {
    ld a = sqrtl((ld)(4 * n * n - 1) / (ld)(n * n - m * m));
    ld b = sqrtl((ld)((2 * n + 1) * (n - 1 - m) * (n - 1 + m)) / (ld)((2 * n - 3) * (n * n - m * m)));
    out[n - m] = a * c * out[n - 1 - m] - b * out[n - 2 - m];
  }
}

ld eps_nm(int n, int m) {
  if (n <= m || n <= 0) return 0;
  return sqrtl((ld)(n * n - m * m) / (ld)(4 * n * n - 1));
}

template <typename T>
mlg_status upload(T** dst, const std::vector<T>& src) {
  if (src.empty()) { *dst = nullptr; return MLG_OK; }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(T));
  if (e != hipSuccess) { *dst = nullptr; return fail(MLG_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e)); }
  e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  return MLG_OK;
}

void free_plan_device(mlg_plan_s* p) {
  void* ptrs[] = {p->d_Pb, p->d_Pf, p->d_Tb, p->d_Qf, p->d_node, p->d_tw_phi, p->d_tw_z,
                  p->d_row_m, p->d_desc_fwd, p->d_desc_bwd, p->d_gram, p->d_goff,
                  p->d_split_syn[0], p->d_split_syn[1], p->d_split_syn[2], p->d_split_syn[3],
                  p->d_split_syn_off, p->d_split_syn_kpad, p->d_split_prj[0], p->d_split_prj[1],
                  p->d_split_prj_off, p->d_split_zdft, p->d_step_fwd,
                  p->d_step_bwd, p->d_step_lam, p->d_step_u, p->d_step_qoff, p->d_step_loff, p->d_step_w,
                  p->d_filter, p->d_logf, p->d_qfl, p->d_qfr, p->d_poisson, p->d_Pb32, p->d_Tb32, p->d_Pf32};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
}

// float -> bfloat16 bits, round to nearest even (finite inputs)
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_float(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
void split_into(double x, uint16_t* hi, uint16_t* lo) {
  const float f = (float)x;
  *hi = bf16_bits(f);
  *lo = bf16_bits(f - bf16_float(*hi));
}

}  // namespace

void proxy_forcing(const mlg_plan_s* p, double nu, double nuh, int q, std::vector<double>& out) {
  const int nrc = p->nrc;
  const ld ell2 = (ld)p->g.ell * (ld)p->g.ell;
  // g: (1/ell^2)(4/3 P_0 - 2 P_1 + 2/3 P_2) on the normalised Pbar_n^0 = sqrt((2n+1)/2) P_n
  std::vector<ld> g(nrc, 0), v(nrc, 0), w(nrc, 0);
  const ld un[3] = {4.0L / 3.0L, -2.0L, 2.0L / 3.0L};
  for (int n = 0; n < 3 && n < nrc; ++n) g[n] = un[n] / sqrtl((ld)(2 * n + 1) / 2.0L) / ell2;
  // -Dbar_0 v = G diag(n(n+1)) v / ell^2 with the exact Gram matrix G of the m = 0 block
  auto minus_dbar = [&](const std::vector<ld>& a, std::vector<ld>& b) {
    for (int n = 0; n < nrc; ++n) {
      ld acc = 0;
      for (int j = std::max(0, n - 2); j <= std::min(nrc - 1, n + 2); ++j) {
        ld G = 0;
        const int lo = std::min(n, j), d = std::abs(n - j);
        const ld e1 = eps_nm(lo + 1, 0), e2 = eps_nm(lo + 2, 0);
        if (d == 0) G = 1 + eps_nm(lo, 0) * eps_nm(lo, 0) + e1 * e1;
        else if (d == 1) G = -2 * e1;
        else G = e1 * e2;
        acc += G * (ld)j * (ld)(j + 1) * a[j];
      }
      b[n] = acc / ell2;
    }
  };
  v = g;
  for (int i = 1; i < q; ++i) {
    minus_dbar(v, w);
    v.swap(w);
  }
  out.assign(nrc, 0.0);
  for (int n = 0; n < nrc; ++n) out[n] = (double)((ld)nu * g[n] + (q >= 1 && nuh != 0.0 ? (ld)nuh * v[n] : 0.0L));
}

void gl_theta(int N, std::vector<long double>& theta, std::vector<long double>& w) { gauss_legendre_theta(N, theta, w); }
void pbar_col(int m, int nmax, long double t, long double* out) { pbar_column(m, nmax, t, out); }

mlg_status build_plan(mlg_plan_s* p) {
  const mlg_grid& g = p->g;
  const int nr = p->nr, nrc = p->nrc, M = p->M, nz = p->nz;
  // ---------------- nodes
  std::vector<ld> th, wl;
  gauss_legendre_theta(nr, th, wl);
  p->x.resize(nr); p->w.resize(nr); p->r.resize(nr); p->theta.resize(nr);
  p->one_minus_x.resize(nr); p->one_plus_x.resize(nr); p->q.resize(nr); p->rinv.resize(nr);
  for (int i = 0; i < nr; ++i) {
    ld t = th[i];
    ld sh = sinl(t / 2), ch = cosl(t / 2);
    ld omx = 2 * sh * sh, opx = 2 * ch * ch;
    p->theta[i] = (double)t;
    p->x[i] = (double)cosl(t);
    p->w[i] = (double)wl[i];
    p->one_minus_x[i] = (double)omx;
    p->one_plus_x[i] = (double)opx;
    p->r[i] = (double)((ld)g.ell * ch / sh);
    p->rinv[i] = (double)(sh / (ch * (ld)g.ell));
    p->q[i] = (double)(omx * omx / ((ld)g.ell * (ld)g.ell));
  }
  // ---------------- triangular offsets
  p->off.assign(M + 1, 0);
  for (int m = 0; m < M; ++m) p->off[m + 1] = p->off[m] + std::max(nrc - m, 0);
  p->tau = p->off[M];
  // ---------------- tables
  const size_t tsz = (size_t)p->tau * nr;
  std::vector<double> Pb(tsz), Pf(tsz), Tb(tsz), Qf(tsz);
  std::vector<ld> col(nrc + 2);
  for (int m = 0; m < M; ++m) {
    const int K = nrc - m;
    if (K <= 0) continue;
    const size_t base = (size_t)p->off[m] * nr;
    for (int i = 0; i < nr; ++i) {
      pbar_column(m, nrc, th[i], col.data());  // rows n = m .. nrc (one extra)
      ld opx = 2 * cosl(th[i] / 2) * cosl(th[i] / 2);
      for (int n = m; n < nrc; ++n) {
        ld P = col[n - m];
        ld Pm1 = (n - 1 >= m) ? col[n - 1 - m] : 0;
        ld Pp1 = col[n + 1 - m];
        ld T = (n + 1) * eps_nm(n, m) * Pm1 - n * eps_nm(n + 1, m) * Pp1;
        ld Q = T - 2 * opx * P;
        Pb[base + (size_t)(n - m) * nr + i] = (double)P;
        Tb[base + (size_t)(n - m) * nr + i] = (double)T;
        Pf[base + (size_t)i * K + (n - m)] = (double)(wl[i] * P);
        Qf[base + (size_t)i * K + (n - m)] = (double)(wl[i] * Q);
      }
    }
  }
  // ---------------- FP32 tables (MLG_FP32 plans: products on FP32 MFMA)
  if (p->prec == MLG_FP32) {
    std::vector<float> pb(Pb.begin(), Pb.end()), tb(Tb.begin(), Tb.end()), pf(Pf.begin(), Pf.end());
    mlg_status st2;
    if ((st2 = upload(&p->d_Pb32, pb)) || (st2 = upload(&p->d_Tb32, tb)) || (st2 = upload(&p->d_Pf32, pf))) return st2;
  }
  // ---------------- split-bfloat16 tables (MLG_SPLIT_BF16 plans only)
  if (p->prec == MLG_SPLIT_BF16) {
    std::vector<int64_t> soff(M + 1, 0), poff(M + 1, 0);
    std::vector<int32_t> kpad(M, 0);
    const int ipad = (nr + 31) / 32 * 32;
    p->split_ipad = ipad;
    for (int m = 0; m < M; ++m) {
      const int K = std::max(nrc - m, 0);
      kpad[m] = (K + 31) / 32 * 32;
      soff[m + 1] = soff[m] + (int64_t)nr * kpad[m];
      poff[m + 1] = poff[m] + (int64_t)K * ipad;
    }
    std::vector<uint16_t> sy[4], pj[2];
    for (int t = 0; t < 4; ++t) sy[t].assign(std::max<int64_t>(soff[M], 1), 0);
    for (int t = 0; t < 2; ++t) pj[t].assign(std::max<int64_t>(poff[M], 1), 0);
    for (int m = 0; m < M; ++m) {
      const int K = std::max(nrc - m, 0);
      const size_t base = (size_t)p->off[m] * nr;
      for (int kk = 0; kk < K; ++kk)
        for (int i = 0; i < nr; ++i) {
          const double P = Pb[base + (size_t)kk * nr + i];
          const double T = Tb[base + (size_t)kk * nr + i];
          const double WP = Pf[base + (size_t)i * K + kk];
          const int64_t s1 = soff[m] + (int64_t)i * kpad[m] + kk;  // [i][n - m]
          const int64_t s2 = poff[m] + (int64_t)kk * ipad + i;     // [n - m][i]
          split_into(P, &sy[0][s1], &sy[1][s1]);
          split_into(T, &sy[2][s1], &sy[3][s1]);
          split_into(WP, &pj[0][s2], &pj[1][s2]);
        }
    }
    mlg_status st2;
    for (int t = 0; t < 4; ++t)
      if ((st2 = upload(&p->d_split_syn[t], sy[t]))) return st2;
    for (int t = 0; t < 2; ++t)
      if ((st2 = upload(&p->d_split_prj[t], pj[t]))) return st2;
    if ((st2 = upload(&p->d_split_syn_off, soff)) || (st2 = upload(&p->d_split_syn_kpad, kpad)) ||
        (st2 = upload(&p->d_split_prj_off, poff)))
      return st2;
    if (nz == 256) {
      // z transforms as two radix-16 DFT products (n = 16 n1 + n2, k = k1 + 16 k2).  Per direction
      // (0: inverse, exp(+i ...); 1: forward, exp(-i ...)) and lane l = 16 g + c, 40 words: the
      // stage-1 B operands (column k1 = c, contraction rows n1 = g + 4 j, re / im interleaved) of
      // the real and imaginary outputs, the stage-2 A operands (row k2 = c, contraction n2 = 4 g + j),
      // each as bfloat16 hi and lo, then the FP32 twiddles W_256^(n2 k1), n2 = 4 g + j, k1 = c.
      std::vector<uint32_t> zt((size_t)2 * 64 * 40, 0);
      const ld pi2 = 2 * acosl(-1.0L);
      for (int d = 0; d < 2; ++d) {
        const ld sg = d == 0 ? 1.0L : -1.0L;
        for (int l = 0; l < 64; ++l) {
          const int gg = l >> 4, c = l & 15;
          uint16_t h[8][8], lo[8][8];  // [operand][element]: B1re, B1im, A2re, A2im (hi / lo)
          float tw[8];
          for (int j = 0; j < 4; ++j) {
            const ld a1 = pi2 * (ld)(((gg + 4 * j) * c) & 15) / 16.0L;
            const ld a2 = pi2 * (ld)((c * (4 * gg + j)) & 15) / 16.0L;
            const ld a3 = pi2 * (ld)(((4 * gg + j) * c) & 255) / 256.0L;
            const double c1 = (double)cosl(a1), s1 = (double)(sg * sinl(a1));
            const double c2 = (double)cosl(a2), s2 = (double)(sg * sinl(a2));
            const double vals[4][2] = {{c1, -s1}, {s1, c1}, {c2, -s2}, {s2, c2}};
            for (int o = 0; o < 4; ++o)
              for (int q = 0; q < 2; ++q) split_into(vals[o][q], &h[o][2 * j + q], &lo[o][2 * j + q]);
            tw[2 * j] = (float)cosl(a3);
            tw[2 * j + 1] = (float)(sg * sinl(a3));
          }
          uint32_t* w = &zt[((size_t)d * 64 + l) * 40];
          for (int o = 0; o < 4; ++o)
            for (int e = 0; e < 4; ++e) {
              w[8 * o + e] = (uint32_t)h[o][2 * e] | ((uint32_t)h[o][2 * e + 1] << 16);
              w[8 * o + 4 + e] = (uint32_t)lo[o][2 * e] | ((uint32_t)lo[o][2 * e + 1] << 16);
            }
          std::memcpy(&w[32], tw, sizeof(tw));
        }
      }
      if ((st2 = upload(&p->d_split_zdft, zt))) return st2;
    }
  }
  // ---------------- Gram factors for the elliptic solves
  GramFactors gf;
  gf.goff.assign(M + 1, 0);
  for (int m = 0; m < M; ++m) gf.goff[m + 1] = gf.goff[m] + std::max(nrc - m, 0);
  p->ngram = gf.goff[M];
  gf.g0.assign(p->ngram, 0); gf.g1.assign(p->ngram, 0); gf.g2.assign(p->ngram, 0);
  gf.d.assign(p->ngram, 0); gf.l1.assign(p->ngram, 0); gf.l2.assign(p->ngram, 0);
  for (int m = 0; m < M; ++m) {
    for (int n = m; n < nrc; ++n) {
      const int64_t k = gf.goff[m] + (n - m);
      ld en = eps_nm(n, m), en1 = eps_nm(n + 1, m), en2 = eps_nm(n + 2, m);
      gf.g0[k] = (double)(1 + en * en + en1 * en1);  // exact Galerkin incl. degree nrc
      gf.g1[k] = (double)(-2 * en1);
      gf.g2[k] = (double)(en1 * en2);
    }
    const int n0 = std::max(m, 1);
    for (int n = n0; n < nrc; ++n) {
      const int64_t k = gf.goff[m] + (n - m);
      ld l2 = 0, l1 = 0;
      if (n - 2 >= n0) l2 = (ld)gf.g2[k - 2] / (ld)gf.d[k - 2];
      if (n - 1 >= n0) {
        ld a = gf.g1[k - 1];
        if (n - 2 >= n0) a -= l2 * (ld)gf.d[k - 2] * (ld)gf.l1[k - 1];
        l1 = a / (ld)gf.d[k - 1];
      }
      ld d = gf.g0[k];
      if (n - 1 >= n0) d -= l1 * l1 * (ld)gf.d[k - 1];
      if (n - 2 >= n0) d -= l2 * l2 * (ld)gf.d[k - 2];
      gf.l1[k] = (double)l1;
      gf.l2[k] = (double)l2;
      gf.d[k] = (double)d;
    }
  }
  // U D U^T factors of the same matrices (unit upper U with superdiagonals u1, u2), so that a
  // solve can start from the highest degree
  std::vector<double> du(p->ngram, 0), u1(p->ngram, 0), u2(p->ngram, 0);
  for (int m = 0; m < M; ++m) {
    const int n0 = std::max(m, 1);
    for (int n = nrc - 1; n >= n0; --n) {
      const int64_t k = gf.goff[m] + (n - m);
      ld a2 = 0, a1 = 0;
      if (n + 2 < nrc) a2 = (ld)gf.g2[k] / (ld)du[k + 2];
      if (n + 1 < nrc) {
        ld t = gf.g1[k];
        if (n + 2 < nrc) t -= a2 * (ld)du[k + 2] * (ld)u1[k + 1];
        a1 = t / (ld)du[k + 1];
      }
      ld d = gf.g0[k];
      if (n + 1 < nrc) d -= a1 * a1 * (ld)du[k + 1];
      if (n + 2 < nrc) d -= a2 * a2 * (ld)du[k + 2];
      u1[k] = (double)a1;
      u2[k] = (double)a2;
      du[k] = (double)d;
    }
  }
  std::vector<double> gram(9 * (size_t)std::max<int64_t>(p->ngram, 1));
  for (int64_t k = 0; k < p->ngram; ++k) {
    gram[0 * p->ngram + k] = gf.g0[k];
    gram[1 * p->ngram + k] = gf.g1[k];
    gram[2 * p->ngram + k] = gf.g2[k];
    gram[3 * p->ngram + k] = gf.d[k] != 0 ? 1.0 / gf.d[k] : 0.0;   // reciprocal pivots
    gram[4 * p->ngram + k] = gf.l1[k];
    gram[5 * p->ngram + k] = gf.l2[k];
    gram[6 * p->ngram + k] = du[k] != 0 ? 1.0 / du[k] : 0.0;
    gram[7 * p->ngram + k] = u1[k];
    gram[8 * p->ngram + k] = u2[k];
  }
  // ---------------- factors of the q operator of the projection, G + kap^2 ell^2 L^-1 (L =
  // diag(n (n + 1))), per active (m, k) column: L D L^T over the solved degrees (m = 0: n >= 1)
  {
    int mmax = 0, kmax = 0;
    active_columns(p, &mmax, &kmax);
    // columns in the aligned blocks of the projection (padded index; inactive entries stay zero)
    const ColBlocks cb = col_blocks(kmax, nz);
    const int ncolp = 8 * cb.nblk;
    const int rows = nrc + 2;
    const size_t cells = (size_t)std::max(mmax, 0) * rows * ncolp;
    std::vector<double2> qfl(std::max<size_t>(cells, 1), make_double2(0.0, 0.0));
    std::vector<double> qfr(std::max<size_t>(cells, 1), 0.0);
    const ld kap0 = 2 * acosl(-1.0L) / (ld)p->g.lz, ell2 = (ld)p->g.ell * (ld)p->g.ell;
    std::vector<ld> d(rows), l1(rows);
    for (int m = 0; m < mmax; ++m) {
      const int cnt = nrc - m, i0 = std::max(m, 1) - m;
      const int64_t gb = gf.goff[m];
      for (int a = 0; a < ncolp; ++a) {
        bool act = false;
        const int kk = colblk_kk(cb, a, kmax, nz, act);
        if (!act) continue;
        const int k = (2 * kk < nz) ? kk : kk - nz;
        const ld sk = kap0 * kap0 * (ld)k * (ld)k * ell2;
        for (int t = i0; t < cnt; ++t) {
          const size_t o = ((size_t)m * rows + t) * ncolp + a;
          if (k == 0) {  // q = -Zhat: no solve
            qfr[o] = 1.0;
            continue;
          }
          const ld n = (ld)(m + t);
          ld l2 = 0, l1t = 0;
          if (t - 2 >= i0) l2 = (ld)gf.g2[gb + t - 2] / d[t - 2];
          if (t - 1 >= i0) {
            ld c = gf.g1[gb + t - 1];
            if (t - 2 >= i0) c -= l2 * d[t - 2] * l1[t - 1];
            l1t = c / d[t - 1];
          }
          ld dt = (ld)gf.g0[gb + t] + sk / (n * (n + 1));
          if (t - 1 >= i0) dt -= l1t * l1t * d[t - 1];
          if (t - 2 >= i0) dt -= l2 * l2 * d[t - 2];
          d[t] = dt;
          l1[t] = l1t;
          qfl[o] = make_double2((double)l1t, (double)l2);
          qfr[o] = (double)(1.0L / dt);
        }
      }
    }
    mlg_status st2;
    if ((st2 = upload(&p->d_qfl, qfl)) || (st2 = upload(&p->d_qfr, qfr))) return st2;
  }
  // ---------------- nodal vectors, twiddles, row orders, GEMM descriptors
  std::vector<double> node(4 * nr);
  for (int i = 0; i < nr; ++i) {
    node[i] = p->rinv[i];
    node[nr + i] = p->q[i];
    node[2 * nr + i] = p->one_plus_x[i];
    // area weight: r dr = ell^2 / (1 - x)^2 dx, times the Gauss-Legendre weight
    const ld omx = 2 * sinl(th[i] / 2) * sinl(th[i] / 2);
    node[3 * nr + i] = (double)(wl[i] * (ld)p->g.ell * (ld)p->g.ell / (omx * omx));
  }
  auto twiddles = [](int n) {
    std::vector<double> tw(2 * n);
    const ld pi = acosl(-1.0L);
    for (int t = 0; t < n; ++t) {
      ld a = -2 * pi * t / n;
      tw[2 * t] = (double)cosl(a);
      tw[2 * t + 1] = (double)sinl(a);
    }
    return tw;
  };
  std::vector<double> twp = twiddles(p->nphi), twz = twiddles(nz);
  std::vector<int32_t> rowm(std::max<int64_t>(p->tau, 1));
  for (int m = 0; m < M; ++m)
    for (int64_t k = p->off[m]; k < p->off[m + 1]; ++k) rowm[k] = m;
  std::vector<GemmDesc> dfwd(M), dbwd(M);
  const int ncol = 2 * nz;
  p->max_rows_fwd = 0;
  p->max_rows_bwd = 0;
  for (int m = 0; m < M; ++m) {
    const int K = std::max(nrc - m, 0);
    GemmDesc b{};
    b.a_off = (int64_t)p->off[m] * nr; b.lda = nr; b.K = K; b.rows = nr;  // K = 0: zero harmonics
    b.b_off = (int64_t)p->off[m] * ncol; b.c_off = (int64_t)m * nr * ncol; b.m = m;
    dbwd[m] = b;
    GemmDesc f{};
    f.a_off = (int64_t)p->off[m] * nr; f.lda = std::max(K, 1); f.K = K > 0 ? nr : 0; f.rows = K;
    f.b_off = (int64_t)m * nr * ncol; f.c_off = (int64_t)p->off[m] * ncol; f.m = m;
    dfwd[m] = f;
    p->max_rows_fwd = std::max(p->max_rows_fwd, f.rows);
    p->max_rows_bwd = std::max(p->max_rows_bwd, b.rows);
  }
  // ---------------- inverse Laplacian, m = k = 0 block (Eq. logproxy): the response shat^g of the
  // solved degrees n >= 1 to the image g of grad_h^2 Lambda, Dbar_0[1:, 1:] shat^g = g[1:] (as
  // G[1:, 1:] y = -ell^2 g[1:], y = L shat^g), and den = g_0 - Dbar_{0,1:} shat^g, in long double
  std::vector<double> poisson(std::max(nrc, 1), 0.0);
  {
    const ld ell2 = (ld)g.ell * (ld)g.ell;
    const ld un[3] = {4.0L / 3.0L, -2.0L, 2.0L / 3.0L};
    std::vector<ld> gv(nrc + 1, 0), G0(nrc + 2, 0), G1(nrc + 2, 0), G2(nrc + 2, 0);
    for (int n = 0; n < 3 && n < nrc; ++n) gv[n] = un[n] / sqrtl((ld)(2 * n + 1) / 2.0L) / ell2;
    for (int n = 0; n < nrc; ++n) {
      const ld e0 = eps_nm(n, 0), e1 = eps_nm(n + 1, 0), e2 = eps_nm(n + 2, 0);
      G0[n] = 1 + e0 * e0 + e1 * e1;
      G1[n] = -2 * e1;
      G2[n] = e1 * e2;
    }
    std::vector<ld> d(nrc + 1, 0), l1(nrc + 1, 0), l2(nrc + 1, 0), z(nrc + 1, 0), y(nrc + 3, 0);
    for (int n = 1; n < nrc; ++n) {
      if (n - 2 >= 1) l2[n] = G2[n - 2] / d[n - 2];
      if (n - 1 >= 1) l1[n] = (G1[n - 1] - (n - 2 >= 1 ? l2[n] * d[n - 2] * l1[n - 1] : 0)) / d[n - 1];
      d[n] = G0[n] - (n - 1 >= 1 ? l1[n] * l1[n] * d[n - 1] : 0) - (n - 2 >= 1 ? l2[n] * l2[n] * d[n - 2] : 0);
      z[n] = -ell2 * gv[n] - (n - 1 >= 1 ? l1[n] * z[n - 1] : 0) - (n - 2 >= 1 ? l2[n] * z[n - 2] : 0);
    }
    for (int n = nrc - 1; n >= 1; --n)
      y[n] = z[n] / d[n] - (n + 1 < nrc ? l1[n + 1] * y[n + 1] : 0) - (n + 2 < nrc ? l2[n + 2] * y[n + 2] : 0);
    ld den = gv[0];
    if (nrc > 1) den += G1[0] * y[1] / ell2;
    if (nrc > 2) den += G2[0] * y[2] / ell2;
    poisson[0] = (double)den;
    for (int n = 1; n < nrc; ++n) poisson[n] = (double)(y[n] / ((ld)n * (n + 1)));
  }
  mlg_status st;
  if ((st = upload(&p->d_poisson, poisson))) return st;
  if ((st = upload(&p->d_Pb, Pb)) || (st = upload(&p->d_Pf, Pf)) || (st = upload(&p->d_Tb, Tb)) ||
      (st = upload(&p->d_Qf, Qf)) || (st = upload(&p->d_node, node)) || (st = upload(&p->d_tw_phi, twp)) ||
      (st = upload(&p->d_tw_z, twz)) || (st = upload(&p->d_row_m, rowm)) ||
      (st = upload(&p->d_desc_fwd, dfwd)) || (st = upload(&p->d_desc_bwd, dbwd)) ||
      (st = upload(&p->d_gram, gram)) || (st = upload(&p->d_goff, gf.goff)))
    return st;
  // ---------------- workspace: 7 mixed + 5 triangular arrays
  p->mixed_elems = (size_t)M * nr * nz;
  p->tri_elems = (size_t)p->tau * nz;
  p->ws_bytes = (7 * p->mixed_elems * 2 + 5 * p->tri_elems * 2) * sizeof(double) + 1024;
  return MLG_OK;
}

void destroy_plan(mlg_plan_s* p) {
  if (!p) return;
  free_plan_device(p);
  delete p;
}

}  // namespace mlg
