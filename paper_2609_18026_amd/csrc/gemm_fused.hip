// Fused radial products for the toroidal-poloidal RHS on FP64 MFMA (v_mfma_f64_16x16x4f64).
//
// Both kernels work per azimuthal order m on a block tile of 64 rows x 16 complex columns (one
// complex column = one axial wavenumber slot).  B tiles are stored in LDS as [k][re 0..15 |
// im 16..31], so a lane's accumulators hold the real and imaginary part of the same complex
// output and the complex epilogue needs no lane exchange.  Four waves stack along the rows; each
// wave owns 16 rows x 16 complex columns per product.
//
// synth: from psi, chi (packed triangular, k spectral) and the tables Pbar, Tbar (per m [n-m][i])
//   computes A1 = Pbar psi, A2 = Tbar psi, A3 = Pbar (L psi), B1 = Pbar chi, B2 = Tbar chi,
//   B3 = Pbar (L chi), B4 = Tbar (L chi) (L = n(n+1)) and writes the harmonics of
//   u_r = (i m A1 + i kap B2)/r, u_phi = (-A2 - m kap B1)/r, u_z = q B3,
//   w_r = i (kap A2 + m q B3 + m kap^2 B1)/r, w_phi = (-m kap A1 - q (B4 - 2(1+x) B3) - kap^2 B2)/r,
//   w_z = q A3   (q = (1-x)^2/ell^2), i.e. Eq. tp and its curl per (m, k) harmonic.
// proj: from the harmonics of a = N_r/r, b = N_phi/r, c = N_z (mixed layout, k spectral) and the
//   weighted tables W Pbar, W Q (per m [i][n-m]) computes Pa, Qa, Pb, Qb, Pc and writes
//   C = -Qb - i m Pa, K' = -i kap Qa - m kap Pb and Zhat = Pc (triangular), the Galerkin
//   sources of the curl / curl-curl projection; only active (m, k) columns are computed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

using namespace ::mlg::dev;

constexpr int TM = 64;   // rows per block
constexpr int TC = 16;   // complex columns per block
constexpr int TK = 16;   // k depth per LDS stage

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }

#define MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

struct SynthArgs {
  const double* Pb;        // backward Pbar tables
  const double* Tb;        // backward Tbar tables
  const double2* psi;      // packed triangular
  const double2* chi;
  double2* out[6];         // mixed layout [m][i][kk]
  const int64_t* off;      // triangular row offsets (M + 1)
  const double* node;      // rinv[nr], q[nr], opx[nr]
  int nr, nrc, nz, M;
  double kap0;
  int mkeep, kmax;         // the two-thirds mask on the potentials (orders above mkeep, |k| > kmax read as zero)
};

__global__ __launch_bounds__(256) void synth_gemm_kernel(SynthArgs a) {
  const int m = blockIdx.z;
  const int row0 = blockIdx.y * TM;
  const int kk0 = blockIdx.x * TC;
  if (row0 >= a.nr || kk0 >= a.nz) return;
  const int K = (a.nrc > m && m <= a.mkeep) ? a.nrc - m : 0;  // a masked order synthesizes zeros
  const int nr = a.nr, nz = a.nz;
  const double* __restrict__ P = a.Pb + a.off[m] * nr;
  const double* __restrict__ T = a.Tb + a.off[m] * nr;
  const double2* __restrict__ ps = a.psi + a.off[m] * nz;
  const double2* __restrict__ ch = a.chi + a.off[m] * nz;

  __shared__ double As[2][2][TK][TM];      // [buf][P, T][k][row]
  __shared__ double Bs[2][2][TK][2 * TC];  // [buf][psi, chi][k][re | im]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double4_t acc[7][2];  // [product][re, im]
#pragma unroll
  for (int p = 0; p < 7; ++p) acc[p][0] = acc[p][1] = double4_t{0.0, 0.0, 0.0, 0.0};

  double ra[2][4];
  double2 rb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kr = e >> 6, rr = e & 63;
      const int k = k0 + kr, row = row0 + rr;
      const bool ok = k < K && row < nr;
      ra[0][t] = ok ? P[(int64_t)k * nr + row] : 0.0;
      ra[1][t] = ok ? T[(int64_t)k * nr + row] : 0.0;
    }
    const int kr = tid >> 4, cc = tid & 15;
    const int k = k0 + kr, kk = kk0 + cc;
    const int kv = kval(kk < nz ? kk : 0, nz);
    const bool ok = k < K && kk < nz && (kv < 0 ? -kv : kv) <= a.kmax;
    rb[0] = ok ? ps[(int64_t)k * nz + kk] : make_double2(0.0, 0.0);
    rb[1] = ok ? ch[(int64_t)k * nz + kk] : make_double2(0.0, 0.0);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kr = e >> 6, rr = e & 63;
      As[buf][0][kr][rr] = ra[0][t];
      As[buf][1][kr][rr] = ra[1][t];
    }
    const int kr = tid >> 4, cc = tid & 15;
    Bs[buf][0][kr][cc] = rb[0].x;
    Bs[buf][0][kr][TC + cc] = rb[0].y;
    Bs[buf][1][kr][cc] = rb[1].x;
    Bs[buf][1][kr][TC + cc] = rb[1].y;
  };

  const int nk = (K + TK - 1) / TK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      const double n = (double)(kt * TK + kr + m);
      const double Ln = n * (n + 1.0);
      const double aP = As[buf][0][kr][wave * 16 + (lane & 15)];
      const double aT = As[buf][1][kr][wave * 16 + (lane & 15)];
      const double bpr = Bs[buf][0][kr][lane & 15], bpi = Bs[buf][0][kr][TC + (lane & 15)];
      const double bcr = Bs[buf][1][kr][lane & 15], bci = Bs[buf][1][kr][TC + (lane & 15)];
      const double lpr = Ln * bpr, lpi = Ln * bpi, lcr = Ln * bcr, lci = Ln * bci;
      acc[0][0] = MFMA(aP, bpr, acc[0][0]);  acc[0][1] = MFMA(aP, bpi, acc[0][1]);   // A1
      acc[1][0] = MFMA(aT, bpr, acc[1][0]);  acc[1][1] = MFMA(aT, bpi, acc[1][1]);   // A2
      acc[2][0] = MFMA(aP, lpr, acc[2][0]);  acc[2][1] = MFMA(aP, lpi, acc[2][1]);   // A3
      acc[3][0] = MFMA(aP, bcr, acc[3][0]);  acc[3][1] = MFMA(aP, bci, acc[3][1]);   // B1
      acc[4][0] = MFMA(aT, bcr, acc[4][0]);  acc[4][1] = MFMA(aT, bci, acc[4][1]);   // B2
      acc[5][0] = MFMA(aP, lcr, acc[5][0]);  acc[5][1] = MFMA(aP, lci, acc[5][1]);   // B3
      acc[6][0] = MFMA(aT, lcr, acc[6][0]);  acc[6][1] = MFMA(aT, lci, acc[6][1]);   // B4
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }
  // epilogue: lane holds rows wave*16 + lane/16 + 4v, column kk0 + lane%16
  const int kk = kk0 + (lane & 15);
  if (kk >= nz) return;
  const double kap = a.kap0 * kval(kk, nz);
  const double fm = (double)m;
  const double* rinvp = a.node;
  const double* qp = a.node + nr;
  const double* opxp = a.node + 2 * nr;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = row0 + wave * 16 + (lane >> 4) + 4 * v;
    if (i >= nr) continue;
    const double rinv = rinvp[i], q = qp[i], opx = opxp[i];
    const double2 A1 = make_double2(acc[0][0][v], acc[0][1][v]);
    const double2 A2 = make_double2(acc[1][0][v], acc[1][1][v]);
    const double2 A3 = make_double2(acc[2][0][v], acc[2][1][v]);
    const double2 B1 = make_double2(acc[3][0][v], acc[3][1][v]);
    const double2 B2 = make_double2(acc[4][0][v], acc[4][1][v]);
    const double2 B3 = make_double2(acc[5][0][v], acc[5][1][v]);
    const double2 B4 = make_double2(acc[6][0][v], acc[6][1][v]);
    const double2 ur = make_double2(-(fm * A1.y + kap * B2.y) * rinv, (fm * A1.x + kap * B2.x) * rinv);
    const double2 up = make_double2((-A2.x - fm * kap * B1.x) * rinv, (-A2.y - fm * kap * B1.y) * rinv);
    const double2 uz = make_double2(q * B3.x, q * B3.y);
    const double tr = kap * A2.x + fm * q * B3.x + fm * kap * kap * B1.x;
    const double ti = kap * A2.y + fm * q * B3.y + fm * kap * kap * B1.y;
    const double2 wr = make_double2(-ti * rinv, tr * rinv);
    const double2 wp = make_double2((-fm * kap * A1.x - q * (B4.x - 2.0 * opx * B3.x) - kap * kap * B2.x) * rinv,
                                    (-fm * kap * A1.y - q * (B4.y - 2.0 * opx * B3.y) - kap * kap * B2.y) * rinv);
    const double2 wz = make_double2(q * A3.x, q * A3.y);
    const int64_t o = ((int64_t)m * nr + i) * nz + kk;
    a.out[0][o] = ur;
    a.out[1][o] = up;
    a.out[2][o] = uz;
    a.out[3][o] = wr;
    a.out[4][o] = wp;
    a.out[5][o] = wz;
  }
}

struct ProjGemmArgs {
  const double* Pf;        // forward W Pbar tables, per m [i][n-m]
  const double* Qf;        // forward W Q tables
  const double2* in[3];    // harmonics of N_r/r, N_phi/r, N_z (mixed [m][i][kk])
  double2* out[3];         // C, K', Zhat (packed triangular)
  const int64_t* off;
  int nr, nrc, nz, kmax, nkact;
  double kap0;
};

__device__ __forceinline__ int active_kk(int a, int kmax, int nz) {
  return (a <= kmax) ? a : nz - (2 * kmax + 1 - a);
}

__global__ __launch_bounds__(256) void proj_gemm_kernel(ProjGemmArgs a) {
  const int m = blockIdx.z;
  const int row0 = blockIdx.y * TM;
  const int c0 = blockIdx.x * TC;  // active column index
  const int rows = a.nrc > m ? a.nrc - m : 0;
  if (row0 >= rows || c0 >= a.nkact) return;
  const int nr = a.nr, nz = a.nz;
  const double* __restrict__ P = a.Pf + a.off[m] * nr;
  const double* __restrict__ Q = a.Qf + a.off[m] * nr;
  const double2* __restrict__ X0 = a.in[0] + (int64_t)m * nr * nz;
  const double2* __restrict__ X1 = a.in[1] + (int64_t)m * nr * nz;
  const double2* __restrict__ X2 = a.in[2] + (int64_t)m * nr * nz;

  __shared__ double As[2][2][TK][TM];      // [buf][P, Q][k = i][row = n - m]
  __shared__ double Bs[2][3][TK][2 * TC];  // [buf][a, b, c][k][re | im]

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double4_t acc[5][2];  // Pa, Qa, Pb, Qb, Pc
#pragma unroll
  for (int p = 0; p < 5; ++p) acc[p][0] = acc[p][1] = double4_t{0.0, 0.0, 0.0, 0.0};

  const int cl = tid & 15;
  const int ca = c0 + cl;
  const int kkl = (ca < a.nkact) ? active_kk(ca, a.kmax, nz) : 0;
  double ra[2][4];
  double2 rb[3];
  auto load = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kr = e >> 6, rr = e & 63;
      const int k = k0 + kr, row = row0 + rr;
      const bool ok = k < nr && row < rows;
      ra[0][t] = ok ? P[(int64_t)k * rows + row] : 0.0;
      ra[1][t] = ok ? Q[(int64_t)k * rows + row] : 0.0;
    }
    const int kr = tid >> 4;
    const int k = k0 + kr;
    const bool ok = k < nr && ca < a.nkact;
    const int64_t idx = (int64_t)k * nz + kkl;
    rb[0] = ok ? X0[idx] : make_double2(0.0, 0.0);
    rb[1] = ok ? X1[idx] : make_double2(0.0, 0.0);
    rb[2] = ok ? X2[idx] : make_double2(0.0, 0.0);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kr = e >> 6, rr = e & 63;
      As[buf][0][kr][rr] = ra[0][t];
      As[buf][1][kr][rr] = ra[1][t];
    }
    const int kr = tid >> 4;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      Bs[buf][f][kr][cl] = rb[f].x;
      Bs[buf][f][kr][TC + cl] = rb[f].y;
    }
  };

  const int nk = (nr + TK - 1) / TK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      const int kr = ks + (lane >> 4);
      const double aP = As[buf][0][kr][wave * 16 + (lane & 15)];
      const double aQ = As[buf][1][kr][wave * 16 + (lane & 15)];
      const double ar_ = Bs[buf][0][kr][lane & 15], ai_ = Bs[buf][0][kr][TC + (lane & 15)];
      const double br_ = Bs[buf][1][kr][lane & 15], bi_ = Bs[buf][1][kr][TC + (lane & 15)];
      const double cr_ = Bs[buf][2][kr][lane & 15], ci_ = Bs[buf][2][kr][TC + (lane & 15)];
      acc[0][0] = MFMA(aP, ar_, acc[0][0]);  acc[0][1] = MFMA(aP, ai_, acc[0][1]);   // Pa
      acc[1][0] = MFMA(aQ, ar_, acc[1][0]);  acc[1][1] = MFMA(aQ, ai_, acc[1][1]);   // Qa
      acc[2][0] = MFMA(aP, br_, acc[2][0]);  acc[2][1] = MFMA(aP, bi_, acc[2][1]);   // Pb
      acc[3][0] = MFMA(aQ, br_, acc[3][0]);  acc[3][1] = MFMA(aQ, bi_, acc[3][1]);   // Qb
      acc[4][0] = MFMA(aP, cr_, acc[4][0]);  acc[4][1] = MFMA(aP, ci_, acc[4][1]);   // Pc
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }
  const int cidx = c0 + (lane & 15);
  if (cidx >= a.nkact) return;
  const int kk = active_kk(cidx, a.kmax, nz);
  const double kap = a.kap0 * kval(kk, nz);
  const double fm = (double)m;
  const int64_t tb = a.off[m];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = row0 + wave * 16 + (lane >> 4) + 4 * v;  // degree n = m + r
    if (r >= rows) continue;
    const double2 Pa = make_double2(acc[0][0][v], acc[0][1][v]);
    const double2 Qa = make_double2(acc[1][0][v], acc[1][1][v]);
    const double2 Pb = make_double2(acc[2][0][v], acc[2][1][v]);
    const double2 Qb = make_double2(acc[3][0][v], acc[3][1][v]);
    const double2 Pc = make_double2(acc[4][0][v], acc[4][1][v]);
    const int64_t o = (tb + r) * nz + kk;
    a.out[0][o] = make_double2(-Qb.x + fm * Pa.y, -Qb.y - fm * Pa.x);
    a.out[1][o] = make_double2(kap * Qa.y - fm * kap * Pb.x, -kap * Qa.x - fm * kap * Pb.y);
    a.out[2][o] = Pc;
  }
}

mlg_status check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MLG_OK;
}

}  // namespace

mlg_status launch_synth_gemm(const mlg_plan_s* p, const double* psi, const double* chi, double* const* out6,
                             hipStream_t s, const SynthMask& mask) {
  if (p->use_fold && p->nr % 2 == 0) return launch_synth_fold(p, psi, chi, out6, s, mask);
  if (mask.skip) return fail(MLG_E_UNSUPPORTED, "synthesis: skipping masked blocks needs the folded products");
  SynthArgs a{};
  a.Pb = p->d_Pb;
  a.Tb = p->d_Tb;
  a.psi = reinterpret_cast<const double2*>(psi);
  a.chi = reinterpret_cast<const double2*>(chi);
  for (int i = 0; i < 6; ++i) a.out[i] = reinterpret_cast<double2*>(out6[i]);
  a.off = p->d_goff;
  a.node = p->d_node;
  a.nr = p->nr;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.M = p->M;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  a.mkeep = mask.mkeep;
  a.kmax = mask.kmax;
  dim3 grid((unsigned)((p->nz + TC - 1) / TC), (unsigned)((p->nr + TM - 1) / TM), (unsigned)p->M);
  p->timing.begin("synth_gemm", s);
  synth_gemm_kernel<<<grid, 256, 0, s>>>(a);
  p->timing.end(s);
  return check("synth_gemm_kernel");
}

mlg_status launch_proj_gemm(const mlg_plan_s* p, double* const* in3, double* const* out3, int mmax, int kmax,
                            hipStream_t s) {
  if (p->use_fold && p->nr % 2 == 0) return launch_proj_fold(p, in3, out3, mmax, kmax, s);
  ProjGemmArgs a{};
  a.Pf = p->d_Pf;
  a.Qf = p->d_Qf;
  for (int i = 0; i < 3; ++i) {
    a.in[i] = reinterpret_cast<const double2*>(in3[i]);
    a.out[i] = reinterpret_cast<double2*>(out3[i]);
  }
  a.off = p->d_goff;
  a.nr = p->nr;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.kmax = kmax;
  a.nkact = (p->nz == 1) ? 1 : 2 * kmax + 1;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  if (mmax <= 0 || a.nkact <= 0) return MLG_OK;
  dim3 grid((unsigned)((a.nkact + TC - 1) / TC), (unsigned)((p->nrc + TM - 1) / TM), (unsigned)mmax);
  p->timing.begin("proj_gemm", s);
  proj_gemm_kernel<<<grid, 256, 0, s>>>(a);
  p->timing.end(s);
  return check("proj_gemm_kernel");
}

}  // namespace mlg
