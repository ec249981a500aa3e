// Parity-folded radial products (even N_r): the Gauss-Legendre nodes are symmetric,
// x_{N-1-i} = -x_i, and Pbar_n^m(-x) = (-1)^(n-m) Pbar_n^m(x), Tbar_n^m(-x) = -(-1)^(n-m) Tbar_n^m(x)
// (Tbar = (1 - x^2) dPbar/dx).  Each product is split over even and odd j = n - m and contracted
// over half the nodes, which halves the flops of the synthesis and of the projection.
//
// synthesis (backward): with E = sum_{j even}, O = sum_{j odd} over the half nodes i < N/2,
//   Pbar-type product at node i: E + O, at its mirror i' = N-1-i: E - O;
//   Tbar-type product at node i: E + O, at i': O - E.
// projection (forward): with X_s = X_i + X_i', X_d = X_i - X_i' (i < N/2) and w symmetric,
//   sum_i w Pbar_n X_i = sum_{i<N/2} w Pbar_n (j even ? X_s : X_d);
//   Q = Tbar - 2(1 + x) Pbar = Q_A - 2 Pbar with Q_A = Tbar - 2 x Pbar of parity -(-1)^j, so
//   sum_i w Q_n X_i = sum_{i<N/2} w Q_A,n (j even ? X_d : X_s) - 2 sum_i w Pbar_n X_i.
// Tiles, MFMA layout and epilogues follow gemm_fused.hip (v_mfma_f64_16x16x4f64, accumulator
// value v of lane l = C[l/16 + 4v][l%16]).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

using namespace ::mlg::dev;

constexpr int TM = 64;  // rows per block (half nodes, or pairs of degrees)
constexpr int TC8 = 8;  // complex columns per block (re and im share the 16 MFMA columns)

typedef float float4_t __attribute__((ext_vector_type(4)));

// The 16 x 16 x 4 MFMA in the real type R of a plan's radial products: FP64 plans use
// v_mfma_f64_16x16x4f64, MLG_FP32 plans v_mfma_f32_16x16x4f32.  Both take A[l % 16][l / 16] and
// B[l / 16][l % 16] from lane l; accumulator value v of lane l holds C[row(l, v)][l % 16] with
// row = l / 16 + 4 v (f64) or 4 (l / 16) + v (f32).
template <typename R>
struct Mma;
template <>
struct Mma<double> {
  typedef double4_t acc;
  typedef double pair __attribute__((ext_vector_type(2)));
  typedef double pair_u __attribute__((ext_vector_type(2), aligned(8)));
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
};
template <>
struct Mma<float> {
  typedef float4_t acc;
  typedef float pair __attribute__((ext_vector_type(2)));
  typedef float pair_u __attribute__((ext_vector_type(2), aligned(4)));
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
};
#define MFMA(a, b, c) Mma<R>::op((a), (b), (c))

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }

// the value of lane l ^ 8 within each row of 16 lanes: a DPP rotation of the row by 8 (a VALU move,
// no LDS round trip as with __shfl_xor)
__device__ __forceinline__ double xor8(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)x, 0x128, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), 0x128, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename R, typename C2>
struct FoldSynthArgs {
  const R* Pb;             // backward Pbar tables, per m [n-m][i]
  const R* Tb;             // backward Tbar tables
  const C2* psi;
  const C2* chi;
  C2* out[6];              // mixed layout [m][i][kk]
  const int64_t* off;
  const double* node;      // rinv[nr], q[nr], opx[nr]
  int nr, nrc, nz;
  int gx, gy, gz;          // tiles: column blocks, row blocks, orders
  double kap0;
  int mkeep, kmax;         // the two-thirds mask on the potentials (orders above mkeep, |k| > kmax read as zero)
  int cbmap;               // 1: column tile x is aligned block x of cb (only the kept slots), 0: slots 8 x ..
  ColBlocks cb;
};

// the Eq. tp harmonics of u and omega at node i from the seven products
template <typename R, typename C2>
__device__ __forceinline__ void synth_write(const FoldSynthArgs<R, C2>& a, int m, int i, int kk, double kap,
                                            const double2 (&p)[7]) {
  const int nr = a.nr, nz = a.nz;
  const double rinv = a.node[i], q = a.node[nr + i], opx = a.node[2 * nr + i];
  const double fm = (double)m;
  const double2 A1 = p[0], A2 = p[1], A3 = p[2], B1 = p[3], B2 = p[4], B3 = p[5], B4 = p[6];
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
  st2(a.out[0] + o, ur);
  st2(a.out[1] + o, up);
  st2(a.out[2] + o, uz);
  st2(a.out[3] + o, wr);
  st2(a.out[4] + o, wp);
  st2(a.out[5] + o, wz);
}

// Block tile: 64 half nodes x 8 complex columns; wavefront w takes 16 half nodes.  The 16 MFMA
// columns hold [re 0..7 | im 0..7], so lane l accumulates the real (l%16 < 8) or imaginary part of
// complex column (l%16) % 8; partner lanes l and l ^ 8 exchange their parts in the epilogue, then
// one writes node i and the other its mirror.  Each wavefront loads its own operands straight into
// the MFMA layouts, D k-steps (of 4 pairs) ahead in a register ring: the table rows of its 16
// nodes (private to it) and the spectra of the block's 8 columns (which the four wavefronts read
// alike, from the L1 cache).  No LDS and no block barrier, so the kernel holds 3 waves per SIMD
// (with LDS staging and a barrier per stage it held 2 and ran 8% longer).  Loads are clamped into
// the tables; degrees past the column are zeroed on the spectrum side.
template <typename R, typename C2, int D>
__global__ __launch_bounds__(256, 2) void synth_fold_kernel(FoldSynthArgs<R, C2> a) {
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  const int half = a.nr / 2;
  const int row0 = tl.y * TM;
  bool act0;
  const int kk0 = a.cbmap ? colblk_kk(a.cb, tl.x * TC8, a.kmax, a.nz, act0) : tl.x * TC8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (row0 + wave * 16 >= half || kk0 >= a.nz) return;
  const int K = (a.nrc > m && m <= a.mkeep) ? a.nrc - m : 0;  // a masked order synthesizes zeros
  const int KP = (K + 1) / 2;
  const int nr = a.nr, nz = a.nz;
  const R* __restrict__ P = a.Pb + a.off[m] * nr;
  const R* __restrict__ T = a.Tb + a.off[m] * nr;
  const R* __restrict__ ps = reinterpret_cast<const R*>(a.psi + a.off[m] * nz);
  const R* __restrict__ ch = reinterpret_cast<const R*>(a.chi + a.off[m] * nz);
  const int cl = lane & 15, kq = lane >> 4;
  const int inode = min(row0 + wave * 16 + cl, half - 1);
  const int kk = kk0 + (cl & 7), part = cl >> 3;
  const bool colok = kk < nz;
  const int kv = kval(colok ? kk : 0, nz);
  const bool kin = colok && (kv < 0 ? -kv : kv) <= a.kmax;  // slots past the mask enter as zero
  const int boff = 2 * (colok ? kk : 0) + part;  // real component of column kk (re or im)
  typename Mma<R>::acc acc[2][7];
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
    for (int p = 0; p < 7; ++p) acc[s2][p] = Mma<R>::zero();
  struct Step {
    R p[2], t[2], bp[2], bc[2];
  };
  Step st[D];
  const int Kc = K > 0 ? K - 1 : 0;
  auto load = [&](int ks, Step& d) {
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int j = min(2 * (4 * ks + kq) + par, Kc);
      d.p[par] = P[(int64_t)j * nr + inode];
      d.t[par] = T[(int64_t)j * nr + inode];
      d.bp[par] = ps[(int64_t)j * 2 * nz + boff];
      d.bc[par] = ch[(int64_t)j * 2 * nz + boff];
    }
  };
  auto compute = [&](int ks, const Step& d) {
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const int j = 2 * (4 * ks + kq) + par;
      const bool ok = j < K && kin;
      const R n = (R)(m + j);
      const R Ln = n * (n + R(1));
      const R bp = ok ? d.bp[par] : R(0), bc = ok ? d.bc[par] : R(0);
      const R lp = Ln * bp, lc = Ln * bc;
      typename Mma<R>::acc(&c)[7] = acc[par];
      c[0] = MFMA(d.p[par], bp, c[0]);
      c[1] = MFMA(d.t[par], bp, c[1]);
      c[2] = MFMA(d.p[par], lp, c[2]);
      c[3] = MFMA(d.p[par], bc, c[3]);
      c[4] = MFMA(d.t[par], bc, c[4]);
      c[5] = MFMA(d.p[par], lc, c[5]);
      c[6] = MFMA(d.t[par], lc, c[6]);
    }
  };
  const int nks = (KP + 3) / 4;
  if (nks > 0) {
#pragma unroll
    for (int d = 0; d < D; ++d) load(d, st[d]);
    for (int k0 = 0; k0 < nks; k0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (k0 + d < nks) compute(k0 + d, st[d]);
        load(k0 + d + D, st[d]);
      }
    }
  }
  const bool hi = cl >= 8;
  const double kap = a.kap0 * kval(colok ? kk : 0, nz);
  constexpr bool tsign[7] = {false, true, false, false, true, false, true};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = row0 + wave * 16 + Mma<R>::row(lane, v);
    double2 val[7];
#pragma unroll
    for (int p = 0; p < 7; ++p) {
      const double e = (double)acc[0][p][v], o = (double)acc[1][p][v];
      const double e2 = xor8(e), o2 = xor8(o);
      const double er = hi ? e2 : e, ei = hi ? e : e2, orr = hi ? o2 : o, oi = hi ? o : o2;
      val[p] = !hi ? make_double2(er + orr, ei + oi)
                   : (tsign[p] ? make_double2(orr - er, oi - ei) : make_double2(er - orr, ei - oi));
    }
    if (i < half && colok) synth_write(a, m, hi ? nr - 1 - i : i, kk, kap, val);
  }
}

template <typename C2>
struct FoldProjArgs {
  const double* Pf;        // forward W Pbar tables, per m [i][n-m]
  const double* Qf;        // forward W Q tables
  const C2* in[3];         // harmonics of N_r/r, N_phi/r, N_z (mixed [m][i][kk]; float2 for reduced plans)
  double2* out[3];         // C, K', Zhat (packed triangular)
  const int64_t* off;
  int nr, nrc, nz, kmax;
  ColBlocks cb;            // the aligned blocks of 8 active axial slots
  int gx, gy, gz;          // tiles: column blocks, pair blocks, orders
  double kap0;
};

// Block tile: 64 RG pairs of degrees (even and odd n - m) x 8 complex columns, [re | im] packed in
// the 16 MFMA columns as in synth_fold_kernel; wavefront w takes RG groups of 16 pairs, the low
// lane of a partner pair writes the even degree, the high lane the odd one.  Register-fed like the
// synthesis: each wavefront loads its table rows (its pairs, both parities) and the block's field
// values at a half node and its mirror straight into the MFMA layouts, D k-steps (of 4 half nodes)
// ahead, and forms the sums, differences and W Q_A = W Q + 2 W Pbar in registers.  No LDS and no
// barrier.  With RG = 2 the six field loads of a k-step feed 20 MFMAs instead of 10, at 2 waves per
// SIMD: 0.236 -> 0.222 ms at 256^3 against RG = 1 at 4 waves per SIMD (and with LDS staging the
// kernel held 2 waves and ran 12% longer than RG = 1); each pair's two table entries then come in
// one 16-byte load (10 loads per 20 MFMAs), 0.220 -> 0.211 ms.  Loads
// are clamped; half nodes past the last are zeroed on the field side, and the entries of pairs
// past the column and of inactive columns are computed but not stored.  Fields are float2 on
// reduced-precision plans (converted after the load has landed).
typedef double PairLd __attribute__((ext_vector_type(2), aligned(8)));  // two adjacent table entries
constexpr int PROJ_RG = 2;  // row groups of 16 pairs per wavefront

template <typename C2, int D, int RG>
__global__ __launch_bounds__(256, RG == 1 ? 4 : 2) void proj_fold_kernel(FoldProjArgs<C2> a) {
  typedef double R;
  typedef decltype(C2().x) S;  // storage real type of the fields
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  const int rows = a.nrc > m ? a.nrc - m : 0;
  const int KP = (rows + 1) / 2;
  const int row0 = tl.y * TM * RG;
  const int c0 = tl.x * TC8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pr0 = row0 + wave * 16 * RG;
  if (pr0 >= KP) return;
  const int ng = min(RG, (KP - pr0 + 15) / 16);  // row groups of this wavefront holding pairs
  const int nr = a.nr, nz = a.nz, half = a.nr / 2;
  const double* __restrict__ P = a.Pf + a.off[m] * nr;
  const double* __restrict__ Q = a.Qf + a.off[m] * nr;
  const int cl = lane & 15, kq = lane >> 4;
  int j0[RG];  // even degree of the lane's pair in each group (clamped into the column)
#pragma unroll
  for (int g = 0; g < RG; ++g) j0[g] = min(2 * (pr0 + 16 * g + cl), rows - 1);
  bool cact;
  const int kc = colblk_kk(a.cb, c0 + (cl & 7), a.kmax, nz, cact);
  const int kk = cact ? kc : 0;
  const int part = cl >> 3;
  const S* __restrict__ X[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) X[f] = reinterpret_cast<const S*>(a.in[f] + (int64_t)m * nr * nz) + 2 * kk + part;
  double4_t acc[RG][2][5];
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
      for (int p = 0; p < 5; ++p) acc[g][s2][p] = double4_t{0.0, 0.0, 0.0, 0.0};
  struct Step {
    R p[RG][2], q[RG][2];
    S x[3], y[3];
  };
  Step st[D];
  auto load = [&](int ks, Step& d) {
    const int i = min(4 * ks + kq, half - 1);
    // the even and odd degree of a pair are adjacent in the [i][n - m] tables: one 16-byte load
    // (8-byte aligned) takes both.  Where j0 is the column's last degree the second value is the
    // first entry of node i + 1 (i < N_r / 2, inside the table), read for a row that is not stored
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const PairLd pv = *reinterpret_cast<const PairLd*>(P + (int64_t)i * rows + j0[g]);
      const PairLd qv = *reinterpret_cast<const PairLd*>(Q + (int64_t)i * rows + j0[g]);
      d.p[g][0] = pv.x;
      d.p[g][1] = pv.y;
      d.q[g][0] = qv.x;
      d.q[g][1] = qv.y;
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      d.x[f] = X[f][(int64_t)i * 2 * nz];
      d.y[f] = X[f][(int64_t)(nr - 1 - i) * 2 * nz];
    }
  };
  auto compute = [&](int ks, const Step& d) {
    const bool iv = 4 * ks + kq < half;
    double sm[3], df[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const double x = iv ? (double)d.x[f] : 0.0, y = iv ? (double)d.y[f] : 0.0;
      sm[f] = x + y;
      df[f] = x - y;
    }
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      if (g >= ng) break;
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const double aP = d.p[g][par], aQ = d.q[g][par] + 2.0 * d.p[g][par];  // w Q_A = w Q + 2 w Pbar
        const double* bp = par ? df : sm;  // Pbar: even rows use sums
        const double* bq = par ? sm : df;  // Q_A: even rows use differences
        double4_t(&c)[5] = acc[g][par];
        c[0] = MFMA(aP, bp[0], c[0]);
        c[1] = MFMA(aQ, bq[0], c[1]);
        c[2] = MFMA(aP, bp[1], c[2]);
        c[3] = MFMA(aQ, bq[1], c[3]);
        c[4] = MFMA(aP, bp[2], c[4]);
      }
    }
  };
  const int nks = (half + 3) / 4;
#pragma unroll
  for (int d = 0; d < D; ++d) load(d, st[d]);
  for (int k0 = 0; k0 < nks; k0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (k0 + d < nks) compute(k0 + d, st[d]);
      load(k0 + d + D, st[d]);
    }
  }
  const bool hi = cl >= 8;
  const double kap = a.kap0 * kval(kk, nz);
  const double fm = (double)m;
  const int64_t tb = a.off[m];
  const int par = hi ? 1 : 0;
#pragma unroll
  for (int g = 0; g < RG; ++g) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int jj = pr0 + 16 * g + (lane >> 4) + 4 * v;
      double2 val[5];
#pragma unroll
      for (int p = 0; p < 5; ++p) {
        const double e = acc[g][0][p][v], o = acc[g][1][p][v];
        const double send = hi ? e : o;
        const double recv = xor8(send);
        const double mine = hi ? o : e;
        val[p] = hi ? make_double2(recv, mine) : make_double2(mine, recv);
      }
      const int r = 2 * jj + par;
      if (r >= rows || !cact) continue;
      const double2 Pa = val[0], Pb = val[2], Pc = val[4];
      const double2 Qa = make_double2(val[1].x - 2.0 * Pa.x, val[1].y - 2.0 * Pa.y);
      const double2 Qb = make_double2(val[3].x - 2.0 * Pb.x, val[3].y - 2.0 * Pb.y);
      const int64_t o = (tb + r) * nz + kk;
      a.out[0][o] = make_double2(-Qb.x + fm * Pa.y, -Qb.y - fm * Pa.x);
      a.out[1][o] = make_double2(kap * Qa.y - fm * kap * Pb.x, -kap * Qa.x - fm * kap * Pb.y);
      a.out[2][o] = Pc;
    }
  }
}

// ---------------------------------------------------------------- scalar transforms, folded
// The radial products of one scalar field (real columns: re and im of each axial slot).  Tiles of 64
// rows x 64 real columns; wavefront w takes 16 rows and all four 16-column MFMA blocks, with an even
// and an odd accumulator per block.  Loads are issued with clamped indices and zeros applied at the
// LDS store (see synth_fold_kernel); every lane loads two adjacent entries at once (16 bytes in
// FP64): half the load instructions of one entry per lane, 0.36 -> 0.34 ms for the transform pair.
constexpr int SC_N = 64;  // real columns per block
constexpr int SC_P = 8;   // pairs (backward) or half nodes (forward) per LDS stage

template <typename R>
struct ScalarFoldArgs {
  const R* A;        // backward: Pbar [m][n-m][i]; forward: w Pbar [m][i][n-m]
  const R* B;        // backward: spectral rows [tau][ncol]; forward: harmonics [m][i][ncol]
  R* C;              // backward: harmonics [m][i][ncol]; forward: spectral rows [tau][ncol]
  const int64_t* off;
  int nr, nrc, ncol;
  int gx, gy, gz;
};

// backward: f(i) = E(i) + O(i), f(N-1-i) = E(i) - O(i), E / O over even / odd n - m, i < N/2
template <typename R>
__global__ __launch_bounds__(256, 3) void scal_bwd_fold_kernel(ScalarFoldArgs<R> a) {
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  const int half = a.nr / 2, nr = a.nr, ncol = a.ncol;
  const int row0 = tl.y * TM, col0 = tl.x * SC_N;
  if (row0 >= half || col0 >= ncol) return;
  const int K = a.nrc > m ? a.nrc - m : 0;
  const int KP = (K + 1) / 2;
  const R* __restrict__ A = a.A + a.off[m] * nr;
  const R* __restrict__ B = a.B + a.off[m] * ncol;
  R* __restrict__ C = a.C + (int64_t)m * nr * ncol;
  __shared__ R As[2][2][SC_P][TM];    // [buf][parity][pair][half node]
  __shared__ R Bs[2][2][SC_P][SC_N];  // [buf][parity][pair][column]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, cl = lane & 15;
  typename Mma<R>::acc acc[2][4];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[q][c] = Mma<R>::zero();
  // two register sets taken in turn, as in synth_fold_kernel: clamped unconditional loads two
  // stages ahead, zeros applied at the LDS store
  constexpr int NL = SC_P / 4;  // 16-byte loads (two adjacent nodes or columns) per thread and stage of each operand
  typedef typename Mma<R>::pair P2;
  struct Stage {
    P2 a[NL], b[NL];
  };
  Stage sx, sy;
  const int Kc = K > 0 ? K - 1 : 0;
  auto load = [&](int p0, Stage& d) {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + 256 * t;  // [parity][pair][32 pairs of nodes or columns]
      const int par = e / (32 * SC_P), kr = (e / 32) % SC_P, c2 = 2 * (e % 32);
      const int jc = min(2 * (p0 + kr) + par, Kc);
      const int ic = min(row0 + c2, nr - 2);  // exact for every kept node (< N_r / 2)
      const int cc2 = min(col0 + c2, ncol - 2);
      d.a[t] = *reinterpret_cast<const P2*>(A + (int64_t)jc * nr + ic);
      d.b[t] = *reinterpret_cast<const P2*>(B + (int64_t)jc * ncol + cc2);
    }
  };
  auto store = [&](int buf, int p0, const Stage& d) {
#pragma unroll
    for (int t = 0; t < NL; ++t) {
      const int e = tid + 256 * t;
      const int par = e / (32 * SC_P), kr = (e / 32) % SC_P, c2 = 2 * (e % 32);
      const bool jin = 2 * (p0 + kr) + par < K;
      As[buf][par][kr][c2] = (jin && row0 + c2 < half) ? d.a[t].x : R(0);
      As[buf][par][kr][c2 + 1] = (jin && row0 + c2 + 1 < half) ? d.a[t].y : R(0);
      Bs[buf][par][kr][c2] = (jin && col0 + c2 < ncol) ? d.b[t].x : R(0);
      Bs[buf][par][kr][c2 + 1] = (jin && col0 + c2 + 1 < ncol) ? d.b[t].y : R(0);
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < SC_P; ks += 4) {
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const R av = As[buf][par][kr][wave * 16 + cl];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[par][c] = MFMA(av, Bs[buf][par][kr][c * 16 + cl], acc[par][c]);
      }
    }
  };
  const int nk = (KP + SC_P - 1) / SC_P;
  if (nk > 0) {
    load(0, sx);
    store(0, 0, sx);
    load(SC_P, sy);
    __syncthreads();
    int kt = 0;
    for (; kt + 1 < nk; kt += 2) {
      load((kt + 2) * SC_P, sx);
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      __builtin_amdgcn_sched_barrier(0);
      store(1, (kt + 1) * SC_P, sy);
      __syncthreads();
      load((kt + 3) * SC_P, sy);
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      __builtin_amdgcn_sched_barrier(0);
      store(0, (kt + 2) * SC_P, sx);
      __syncthreads();
    }
    if (kt < nk) compute(0);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = col0 + c * 16 + cl;
    if (col >= ncol) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = row0 + wave * 16 + Mma<R>::row(lane, v);
      if (i >= half) continue;
      const R e = acc[0][c][v], o = acc[1][c][v];
      C[(int64_t)i * ncol + col] = e + o;
      C[(int64_t)(nr - 1 - i) * ncol + col] = e - o;
    }
  }
}

// forward: even n - m rows contract with X_i + X_{N-1-i}, odd rows with the difference, i < N/2.
// One block of 8 wavefronts covers 2 TM pairs of an order for 64 columns: wavefronts 0..3 the first
// TM of them, 4..7 the next TM, both halves on the same staged sums and differences of the
// fields (with two blocks of TM pairs, each staged them; the second was partly empty on every order
// at N_r = 256): 0.335 -> 0.328 ms for the transform pair at 256^3.
template <typename R>
__global__ __launch_bounds__(512) void scal_fwd_fold_kernel(ScalarFoldArgs<R> a) {
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  const int K = a.nrc > m ? a.nrc - m : 0;
  const int KP = (K + 1) / 2;
  const int half = a.nr / 2, nr = a.nr, ncol = a.ncol;
  const int rowb = tl.y * 2 * TM, col0 = tl.x * SC_N;  // the block covers pairs rowb .. rowb + 2 TM - 1
  if (rowb >= KP || col0 >= ncol) return;
  const R* __restrict__ A = a.A + a.off[m] * nr;      // [i][n-m], row length K
  const R* __restrict__ B = a.B + (int64_t)m * nr * ncol;
  R* __restrict__ C = a.C + a.off[m] * ncol;
  __shared__ R As[2][2][SC_P][2 * TM];  // [buf][parity][half node][pair]
  __shared__ R Bs[2][2][SC_P][SC_N];  // [buf][sum, difference][half node][column]
  const int tid = threadIdx.x, lane = tid & 63, wave = (tid >> 6) & 3, cl = lane & 15;
  const int rloc = (tid >> 8) * TM, row0 = rowb + rloc;  // waves 4..7 take the block's pairs TM .. 2 TM - 1
  typename Mma<R>::acc acc[2][4];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[q][c] = Mma<R>::zero();
  // wavefront w takes the block's columns 16 w .. 16 w + 15 for all its pairs, in 4 groups of 16;
  // groups wholly past the column (the second row tile of a short order) are skipped by every
  // wavefront alike, so the SIMDs stay evenly loaded (with 16 pairs per wavefront, the one that
  // held the first pairs worked on every tile and the others idled on short orders)
  const int ng = max(0, min(4, (KP - row0 + 15) / 16));
  // 16-byte loads: the even and odd degree of a pair (adjacent in the [i][n - m] table; the odd one
  // of a last unpaired degree is the first entry of node i + 1, inside the table, and is not stored),
  // and two adjacent columns of the harmonics
  constexpr int NA = SC_P / 4, NX = SC_P / 8;  // table and field loads per thread and stage
  typedef typename Mma<R>::pair P2;
  typedef typename Mma<R>::pair_u P2u;  // 8-byte aligned (rows of odd length)
  struct Stage {
    P2u a[NA];
    P2 x[NX], y[NX];
  };
  Stage sx, sy;
  const int Kc = K - 1;  // K > 0 here (rowb < KP)
  auto load = [&](int i0, Stage& d) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int e = tid + 512 * t;  // [half node][pair]
      const int kr = e / 128, rr = e % 128;
      const int ic = min(i0 + kr, half - 1);
      const int jc = min(2 * (rowb + rr), Kc);
      d.a[t] = *reinterpret_cast<const P2u*>(A + (int64_t)ic * K + jc);
    }
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      // [half node][32 pairs of columns]; threads 256..511 repeat the loads of 0..255 (unconditional
      // loads keep the wait counts uniform) and do not store them
      const int e = (tid & 255) + 256 * t;
      const int kr = e / 32, c2 = 2 * (e % 32);
      const int ic = min(i0 + kr, half - 1);
      const int cc2 = min(col0 + c2, ncol - 2);
      d.x[t] = *reinterpret_cast<const P2*>(B + (int64_t)ic * ncol + cc2);
      d.y[t] = *reinterpret_cast<const P2*>(B + (int64_t)(nr - 1 - ic) * ncol + cc2);
    }
  };
  auto store = [&](int buf, int i0, const Stage& d) {
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int e = tid + 512 * t;
      const int kr = e / 128, rr = e % 128;
      const bool iok = i0 + kr < half;
      As[buf][0][kr][rr] = (iok && 2 * (rowb + rr) < K) ? d.a[t].x : R(0);
      As[buf][1][kr][rr] = (iok && 2 * (rowb + rr) + 1 < K) ? d.a[t].y : R(0);
    }
    if (tid >= 256) return;
#pragma unroll
    for (int t = 0; t < NX; ++t) {
      const int e = tid + 256 * t;
      const int kr = e / 32, c2 = 2 * (e % 32);
      const bool iok = i0 + kr < half;
      const bool ok0 = iok && col0 + c2 < ncol, ok1 = iok && col0 + c2 + 1 < ncol;
      Bs[buf][0][kr][c2] = ok0 ? d.x[t].x + d.y[t].x : R(0);
      Bs[buf][1][kr][c2] = ok0 ? d.x[t].x - d.y[t].x : R(0);
      Bs[buf][0][kr][c2 + 1] = ok1 ? d.x[t].y + d.y[t].y : R(0);
      Bs[buf][1][kr][c2 + 1] = ok1 ? d.x[t].y - d.y[t].y : R(0);
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < SC_P; ks += 4) {
      const int kr = ks + (lane >> 4);
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        // even degrees contract with sums, odd with differences
        const R bv = Bs[buf][par][kr][wave * 16 + cl];
#pragma unroll
        for (int g = 0; g < 4; ++g)
          if (g < ng) acc[par][g] = MFMA(As[buf][par][kr][rloc + g * 16 + cl], bv, acc[par][g]);
      }
    }
  };
  const int nk = (half + SC_P - 1) / SC_P;
  load(0, sx);
  store(0, 0, sx);
  load(SC_P, sy);
  __syncthreads();
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    load((kt + 2) * SC_P, sx);
    __builtin_amdgcn_sched_barrier(0);
    compute(0);
    __builtin_amdgcn_sched_barrier(0);
    store(1, (kt + 1) * SC_P, sy);
    __syncthreads();
    load((kt + 3) * SC_P, sy);
    __builtin_amdgcn_sched_barrier(0);
    compute(1);
    __builtin_amdgcn_sched_barrier(0);
    store(0, (kt + 2) * SC_P, sx);
    __syncthreads();
  }
  if (kt < nk) compute(0);
  const int col = col0 + wave * 16 + cl;
  if (col >= ncol) return;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int pr = row0 + g * 16 + Mma<R>::row(lane, v);
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const int j = 2 * pr + par;
        if (j < K) C[(int64_t)j * ncol + col] = acc[par][g][v];
      }
    }
  }
}

mlg_status check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MLG_OK;
}

}  // namespace

template <typename R, typename C2>
static void synth_fold_go(const mlg_plan_s* p, const R* Pb, const R* Tb, const double* psi, const double* chi,
                          double* const* out6, hipStream_t s, const SynthMask& mask) {
  FoldSynthArgs<R, C2> a{};
  a.Pb = Pb;
  a.Tb = Tb;
  a.psi = reinterpret_cast<const C2*>(psi);
  a.chi = reinterpret_cast<const C2*>(chi);
  for (int i = 0; i < 6; ++i) a.out[i] = reinterpret_cast<C2*>(out6[i]);
  a.off = p->d_goff;
  a.node = p->d_node;
  a.nr = p->nr;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  a.mkeep = mask.mkeep;
  a.kmax = mask.kmax;
  a.gx = (p->nz + TC8 - 1) / TC8;
  a.gy = (p->nr / 2 + TM - 1) / TM;
  a.gz = p->M;
  a.cbmap = 0;
  if (mask.skip) {  // only the kept orders and the aligned blocks of the kept slots
    a.gz = std::min(p->M, mask.mkeep + 1);
    a.cb = col_blocks(mask.kmax, p->nz);
    a.cbmap = 1;
    a.gx = a.cb.nblk;
  }
  synth_fold_kernel<R, C2, 2><<<dim3(xcd_blocks(a.gx, a.gy, a.gz)), 256, 0, s>>>(a);
}

// psi, chi: spectral arrays of the plan's data type; out6: mixed harmonics (float2 on MLG_FP32
// plans, whose products run on FP32 MFMA with the FP32 tables)
mlg_status launch_synth_fold(const mlg_plan_s* p, const double* psi, const double* chi, double* const* out6,
                             hipStream_t s, const SynthMask& mask) {
  p->timing.begin("synth_gemm", s);
  if (p->prec == MLG_FP32)
    synth_fold_go<float, float2>(p, p->d_Pb32, p->d_Tb32, psi, chi, out6, s, mask);
  else
    synth_fold_go<double, double2>(p, p->d_Pb, p->d_Tb, psi, chi, out6, s, mask);
  p->timing.end(s);
  return check("synth_fold_kernel");
}

template <typename C2>
static void proj_fold_go(const mlg_plan_s* p, double* const* in3, double* const* out3, int kmax, int mmax,
                         hipStream_t s) {
  FoldProjArgs<C2> a{};
  a.Pf = p->d_Pf;
  a.Qf = p->d_Qf;
  for (int i = 0; i < 3; ++i) {
    a.in[i] = reinterpret_cast<const C2*>(in3[i]);
    a.out[i] = reinterpret_cast<double2*>(out3[i]);
  }
  a.off = p->d_goff;
  a.nr = p->nr;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.kmax = kmax;
  a.cb = col_blocks(kmax, p->nz);
  a.kap0 = 2.0 * M_PI / p->g.lz;
  const int kp = (p->nrc + 1) / 2;
  a.gx = a.cb.nblk;
  a.gy = (kp + TM * PROJ_RG - 1) / (TM * PROJ_RG);
  a.gz = mmax;
  proj_fold_kernel<C2, 1, PROJ_RG><<<dim3(xcd_blocks(a.gx, a.gy, a.gz)), 256, 0, s>>>(a);
}

// in3: harmonics of N (float2 on reduced-precision plans); out3: FP64 sources in every case
mlg_status launch_proj_fold(const mlg_plan_s* p, double* const* in3, double* const* out3, int mmax, int kmax,
                            hipStream_t s) {
  const int nkact = (p->nz == 1) ? 1 : 2 * kmax + 1;
  if (mmax <= 0 || nkact <= 0) return MLG_OK;
  p->timing.begin("proj_gemm", s);
  if (p->prec != MLG_FP64)
    proj_fold_go<float2>(p, in3, out3, kmax, mmax, s);
  else
    proj_fold_go<double2>(p, in3, out3, kmax, mmax, s);
  p->timing.end(s);
  return check("proj_fold_kernel");
}

template <typename R>
static void scalar_fold_go(const mlg_plan_s* p, int dir, const R* A, const double* B, double* C, hipStream_t s) {
  ScalarFoldArgs<R> a{};
  a.A = A;
  a.B = reinterpret_cast<const R*>(B);
  a.C = reinterpret_cast<R*>(C);
  a.off = p->d_goff;
  a.nr = p->nr;
  a.nrc = p->nrc;
  a.ncol = 2 * p->nz;
  a.gx = (a.ncol + SC_N - 1) / SC_N;
  a.gy = dir > 0 ? (p->nr / 2 + TM - 1) / TM : ((p->nrc + 1) / 2 + 2 * TM - 1) / (2 * TM);
  a.gz = p->M;
  if (dir > 0)
    scal_bwd_fold_kernel<R><<<dim3(xcd_blocks(a.gx, a.gy, a.gz)), 256, 0, s>>>(a);
  else
    scal_fwd_fold_kernel<R><<<dim3(xcd_blocks(a.gx, a.gy, a.gz)), 512, 0, s>>>(a);
}

mlg_status launch_scalar_fold(const mlg_plan_s* p, int dir, const double* B, double* C, hipStream_t s) {
  p->timing.begin("radial_gemm", s);
  if (p->prec == MLG_FP32)
    scalar_fold_go<float>(p, dir, dir > 0 ? p->d_Pb32 : p->d_Pf32, B, C, s);
  else
    scalar_fold_go<double>(p, dir, dir > 0 ? p->d_Pb : p->d_Pf, B, C, s);
  p->timing.end(s);
  return check(dir > 0 ? "scal_bwd_fold_kernel" : "scal_fwd_fold_kernel");
}

}  // namespace mlg
