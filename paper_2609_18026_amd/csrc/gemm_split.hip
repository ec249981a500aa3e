// Split-bfloat16 radial products for the toroidal-poloidal RHS (plans of precision
// MLG_SPLIT_BF16).  Every operand x is represented as hi + lo with hi = bf16(x) and
// lo = bf16(x - hi); a product is accumulated in FP32 as hi_a hi_b + hi_a lo_b + lo_a hi_b
// (the lo_a lo_b term, ~2^-18 relative, is dropped) with v_mfma_f32_16x16x32_bf16.
// Tables are split once on the host; the data (float / float2: split plans keep their fields in FP32)
// are split while they are staged in LDS.
// The epilogues, layouts and outputs are those of the FP64 kernels in gemm_fused.hip.
//
// MFMA operand layout (16x16x32 bf16): lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and
// B[8(l/16) .. +7][l%16]; FP32 accumulator value v of lane l is C[4(l/16) + v][l%16].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

using namespace ::mlg::dev;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64;  // rows per block (4 waves x 16)
constexpr int TC = 16;  // complex columns per block
constexpr int TK = 32;  // one MFMA k step

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
__device__ __forceinline__ void split2(double x, unsigned short& hi, unsigned short& lo) {
  const float f = (float)x;
  hi = bf16_bits(f);
  lo = bf16_bits(f - bf16_to_float(hi));
}

__device__ __forceinline__ floatx4 mfma3(bf16x8 ah, bf16x8 al, bf16x8 bh, bf16x8 bl, floatx4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  return c;
}

__device__ __forceinline__ bf16x8 ldfrag(const unsigned short* p) {
  const u16x8 v = *reinterpret_cast<const u16x8*>(p);
  return __builtin_bit_cast(bf16x8, v);
}

template <typename C2>
struct SplitSynthArgs {
  const unsigned short* tab[4];  // Pbar hi, Pbar lo, Tbar hi, Tbar lo: per m [i][kpad], k = n - m
  const int64_t* toff;           // per m element offset of the split tables
  const int32_t* kpad;           // per m padded K (multiple of 32)
  const C2* psi;                 // spectra of the plan's data type (float2 on split plans)
  const C2* chi;
  C2* out[6];
  const int64_t* off;
  const double* node;
  int nr, nrc, nz;
  int gx, gy, gz;                // tiles: column blocks, row blocks, orders
  double kap0;
  int mkeep, kmax;               // the two-thirds mask on the potentials (read as zero beyond it)
  int nbpos, nstart;             // nbpos > 0: column tile x < nbpos starts at slot TC x, the others at
                                 // nstart + TC (x - nbpos) (the aligned tiles of the kept slots)
};

// B staging: [buf][var][col][k] with var = input(psi, chi) x scaled(1, L) x part(re, im) x (hi, lo).
// The raw operands of the next two K stages and the table fragments of the next one are held in
// registers as raw loads; the scaling by L and the bf16 split happen when they are written to LDS,
// after the MFMAs of the current stage, so the loads stay in flight across them.  At 3 waves per
// SIMD (156 VGPRs, the accumulators leave the AGPRs) the latency of the next stage is better hidden.
template <typename C2>
__global__ __launch_bounds__(256, 3) void split_synth_kernel(SplitSynthArgs<C2> a) {
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  const int row0 = tl.y * TM;
  const int kk0 = (a.nbpos > 0 && tl.x >= a.nbpos) ? a.nstart + (tl.x - a.nbpos) * TC : tl.x * TC;
  if (row0 >= a.nr || kk0 >= a.nz) return;
  const int K = (a.nrc > m && m <= a.mkeep) ? a.nrc - m : 0;  // a masked order synthesizes zeros
  const int nr = a.nr, nz = a.nz;
  const int kp = a.kpad[m];
  const C2* __restrict__ ps = a.psi + a.off[m] * nz;
  const C2* __restrict__ ch = a.chi + a.off[m] * nz;
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][16][TC][TK];  // 32 KB
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rowl = row0 + wave * 16 + (lane & 15);
  const int kg = 8 * (lane >> 4);
  const bool rowok = rowl < nr;
  const unsigned short* tp[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) tp[t] = a.tab[t] + a.toff[m] + (int64_t)(rowok ? rowl : 0) * kp + kg;

  floatx4 acc[7][2];
#pragma unroll
  for (int p = 0; p < 7; ++p) acc[p][0] = acc[p][1] = floatx4{0.f, 0.f, 0.f, 0.f};

  // each thread stages 2 (k, col) entries of psi and chi per chunk
  struct Stage {
    C2 p[2], c[2];
  };
  auto load = [&](int k0, Stage& d) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + 256 * h;
      const int k = k0 + (e >> 4), kk = kk0 + (e & 15);
      const int kv = kval(kk < nz ? kk : 0, nz);
      const bool ok = k < K && kk < nz && (kv < 0 ? -kv : kv) <= a.kmax;
      d.p[h] = ok ? ps[(int64_t)k * nz + kk] : czero<C2>();
      d.c[h] = ok ? ch[(int64_t)k * nz + kk] : czero<C2>();
    }
  };
  auto store = [&](int buf, int k0, const Stage& d) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + 256 * h;
      const int kr = e >> 4, c = e & 15;
      const double Ln = (double)(k0 + kr + m) * (k0 + kr + m + 1.0);
      const double vals[8] = {d.p[h].x,      d.p[h].y, Ln * d.p[h].x, Ln * d.p[h].y,
                              d.c[h].x,      d.c[h].y, Ln * d.c[h].x, Ln * d.c[h].y};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        unsigned short hi, lo;
        split2(vals[q], hi, lo);
        Bs[buf][2 * q][c][kr] = hi;
        Bs[buf][2 * q + 1][c][kr] = lo;
      }
    }
  };
  auto frags = [&](int kt, bf16x8 (&f)[4]) {
    const int64_t ko = (int64_t)kt * TK;
#pragma unroll
    for (int t = 0; t < 4; ++t) f[t] = ldfrag(tp[t] + ko);
  };

  const int nk = (K + TK - 1) / TK;
  Stage ra, rn;
  bf16x8 fa[4], fn[4];
  if (nk > 0) {
    frags(0, fa);  // issued first, so that the wait for the staged operands covers it
    load(0, ra);
    store(0, 0, ra);
  }
  if (nk > 1) load(TK, ra);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 2 < nk) load((kt + 2) * TK, rn);
    if (kt + 1 < nk) frags(kt + 1, fn);
    const int c = lane & 15;
    // var index: q = 0 psi re, 1 psi im, 2 Lpsi re, 3 Lpsi im, 4 chi re, 5 chi im, 6 Lchi re, 7 Lchi im
    bf16x8 bh[8], bl[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      bh[q] = ldfrag(&Bs[buf][2 * q][c][kg]);
      bl[q] = ldfrag(&Bs[buf][2 * q + 1][c][kg]);
    }
#pragma unroll
    for (int ri = 0; ri < 2; ++ri) {
      acc[0][ri] = mfma3(fa[0], fa[1], bh[0 + ri], bl[0 + ri], acc[0][ri]);  // A1 = P psi
      acc[1][ri] = mfma3(fa[2], fa[3], bh[0 + ri], bl[0 + ri], acc[1][ri]);  // A2 = T psi
      acc[2][ri] = mfma3(fa[0], fa[1], bh[2 + ri], bl[2 + ri], acc[2][ri]);  // A3 = P L psi
      acc[3][ri] = mfma3(fa[0], fa[1], bh[4 + ri], bl[4 + ri], acc[3][ri]);  // B1 = P chi
      acc[4][ri] = mfma3(fa[2], fa[3], bh[4 + ri], bl[4 + ri], acc[4][ri]);  // B2 = T chi
      acc[5][ri] = mfma3(fa[0], fa[1], bh[6 + ri], bl[6 + ri], acc[5][ri]);  // B3 = P L chi
      acc[6][ri] = mfma3(fa[2], fa[3], bh[6 + ri], bl[6 + ri], acc[6][ri]);  // B4 = T L chi
    }
    if (kt + 1 < nk) store(buf ^ 1, (kt + 1) * TK, ra);
    ra = rn;
#pragma unroll
    for (int t = 0; t < 4; ++t) fa[t] = fn[t];
    __syncthreads();
  }
  const int kk = kk0 + (lane & 15);
  if (kk >= nz) return;
  const double kap = a.kap0 * kval(kk, nz);
  const double fm = (double)m;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = row0 + wave * 16 + 4 * (lane >> 4) + v;
    if (i >= nr) continue;
    const double rinv = a.node[i], q = a.node[nr + i], opx = a.node[2 * nr + i];
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
    st2(a.out[0] + o, ur);
    st2(a.out[1] + o, up);
    st2(a.out[2] + o, uz);
    st2(a.out[3] + o, wr);
    st2(a.out[4] + o, wp);
    st2(a.out[5] + o, wz);
  }
}

struct SplitScalarArgs {
  const unsigned short* tab[2];  // hi, lo: backward Pbar [i][kpad] (split synthesis tables),
                                 // forward W Pbar [n-m][ipad] (split projection tables)
  const int64_t* toff;           // per m element offset of the tables
  const int32_t* kpad;           // backward: per m row stride
  int ipad;                      // forward: row stride
  const float2* in;              // backward: spectrum [tau][nz]; forward: harmonics [m][i][nz]
  float2* out;                   // backward: harmonics [m][i][nz]; forward: spectrum [tau][nz]
  const int64_t* off;            // packed offset of each order
  int nr, nrc, nz;
  int gx, gy, gz;                // tiles: column blocks, row blocks, orders
};

// Radial products of the scalar transform pair (Sec. 4.1) with split-bfloat16 operands:
// backward f_m[i][kk] = sum_n Pbar_n^m(x_i) s[n][kk], forward s[n][kk] = sum_i w_i Pbar_n^m(x_i)
// f_m[i][kk].  The real table is the MFMA A operand; the re and im parts of the complex data are
// two B operands.  The raw operands of the next two K stages and the table fragments of the next one
// are held in registers as raw loads and split into bf16 at the LDS store (as in split_synth_kernel).
template <bool FWD>
__global__ __launch_bounds__(256) void split_scalar_kernel(SplitScalarArgs a) {
  Tile3 tl;
  if (!xcd_tile(a.gx, a.gy, a.gz, tl)) return;
  const int m = tl.z;
  const int K = a.nrc > m ? a.nrc - m : 0;
  const int rows = FWD ? K : a.nr;  // output rows of this order
  const int kdim = FWD ? a.nr : K;  // contraction length
  const int row0 = tl.y * TM;
  const int kk0 = tl.x * TC;
  if (row0 >= rows || kk0 >= a.nz) return;
  const int nz = a.nz;
  const int ld = FWD ? a.ipad : a.kpad[m];
  const float2* __restrict__ X = a.in + (FWD ? (int64_t)m * a.nr : a.off[m]) * nz;
  float2* __restrict__ Y = a.out + (FWD ? a.off[m] : (int64_t)m * a.nr) * nz;
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][4][TC][TK];  // [buf][re hi, re lo, im hi, im lo]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rowl = row0 + wave * 16 + (lane & 15);
  const int kg = 8 * (lane >> 4);
  const bool rowok = rowl < rows;
  const unsigned short* tp[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) tp[t] = a.tab[t] + a.toff[m] + (int64_t)(rowok ? rowl : 0) * ld + kg;
  floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
  struct Stage {
    float2 v[2];
  };
  auto load = [&](int k0, Stage& d) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + 256 * h;
      const int k = k0 + (e >> 4), kk = kk0 + (e & 15);
      d.v[h] = (k < kdim && kk < nz) ? X[(int64_t)k * nz + kk] : make_float2(0.f, 0.f);
    }
  };
  auto store = [&](int buf, const Stage& d) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = tid + 256 * h;
      const int kr = e >> 4, c = e & 15;
      unsigned short hi, lo;
      split2(d.v[h].x, hi, lo);
      Bs[buf][0][c][kr] = hi;
      Bs[buf][1][c][kr] = lo;
      split2(d.v[h].y, hi, lo);
      Bs[buf][2][c][kr] = hi;
      Bs[buf][3][c][kr] = lo;
    }
  };
  auto frags = [&](int kt, bf16x8 (&f)[2]) {
    const int64_t ko = (int64_t)kt * TK;
    f[0] = ldfrag(tp[0] + ko);
    f[1] = ldfrag(tp[1] + ko);
  };
  const int nk = (kdim + TK - 1) / TK;
  Stage ra, rn;
  bf16x8 fa[2], fn[2];
  if (nk > 0) {
    frags(0, fa);  // issued first, so that the wait for the staged operands covers it
    load(0, ra);
    store(0, ra);
  }
  if (nk > 1) load(TK, ra);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 2 < nk) load((kt + 2) * TK, rn);
    if (kt + 1 < nk) frags(kt + 1, fn);
    const int c = lane & 15;
    const bf16x8 rh = ldfrag(&Bs[buf][0][c][kg]), rl = ldfrag(&Bs[buf][1][c][kg]);
    const bf16x8 ih = ldfrag(&Bs[buf][2][c][kg]), il = ldfrag(&Bs[buf][3][c][kg]);
    acc[0] = mfma3(fa[0], fa[1], rh, rl, acc[0]);
    acc[1] = mfma3(fa[0], fa[1], ih, il, acc[1]);
    if (kt + 1 < nk) store(buf ^ 1, ra);
    ra = rn;
    fa[0] = fn[0];
    fa[1] = fn[1];
    __syncthreads();
  }
  const int kk = kk0 + (lane & 15);
  if (kk >= nz) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = row0 + wave * 16 + 4 * (lane >> 4) + v;
    if (r < rows) Y[(int64_t)r * nz + kk] = make_float2(acc[0][v], acc[1][v]);
  }
}

// ---------------------------------------------------------------- z transforms as DFT products
// N_z = 256 = 16 x 16 (Cooley-Tukey): with n = 16 n1 + n2 and k = k1 + 16 k2,
//   X[k1 + 16 k2] = sum_n2 W16^(n2 k2) W256^(n2 k1) sum_n1 W16^(n1 k1) x[16 n1 + n2],
// W_N = exp(+-2 pi i / N).  Both radix-16 stages are 16 x 16 complex matrix products on MFMA in the
// real form [[Fr, -Fi], [Fi, Fr]] with split-bfloat16 operands and FP32 accumulation.  Stage 1
// takes the line as its A operand: lane l = 16 g + n2 supplies x[l + 64 j], j = 0..3 (n1 = g + 4 j,
// re and im interleaved along the contraction), so the loads are coalesced.  Its accumulators hold
// Y[k1 = l % 16][n2 = 4 g + v], v = 0..3, which after the twiddle W256^(n2 k1) are exactly the
// lane's B operand of stage 2 (contraction over n2 = 4 g + v); stage 2 leaves X[l % 16 + 16 (4 g + v)]
// in the lane.  No LDS and no lane exchange; the per-lane constants come from a plan table.
struct ZdftArgs {
  const uint4* tab;     // [dir][lane][10] (40 words, see plan construction)
  const float2* in[6];  // split plans keep their fields as float2
  float2* out[6];
  int64_t rows;         // lines per field
  int64_t lines;        // rows x fields
  int nzc;
  const int32_t* row_m;
  int mask_m, mask_k;
};
constexpr int ZD_LPW = 4;  // lines per wave, loaded together

__device__ __forceinline__ bool zkept(int kk, int nzc) {
  const int k = (kk < 128) ? kk : kk - 256;
  return k != -128 && (k < 0 ? -k : k) < nzc;
}
// spectral slot kk of a line of order mrow kept by the chop and the masks (as launch_zfft)
__device__ __forceinline__ bool zspec_keep(const ZdftArgs& a, int mrow, int kk) {
  const int k = (kk < 128) ? kk : kk - 256;
  return zkept(kk, a.nzc) && (a.mask_k < 0 || (k < 0 ? -k : k) <= a.mask_k) && (!a.row_m || mrow <= a.mask_m);
}

template <bool INV>
__global__ __launch_bounds__(256) void split_zdft_kernel(ZdftArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t L0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * ZD_LPW;
  if (L0 >= a.lines) return;
  const int g = lane >> 4, c = lane & 15;
  float2 d[ZD_LPW][4];
#pragma unroll
  for (int t = 0; t < ZD_LPW; ++t) {
    const int64_t L = L0 + t < a.lines ? L0 + t : L0;  // the last wave may hold fewer lines
    const int64_t f = L / a.rows, row = L - f * a.rows;
    const float2* __restrict__ x = a.in[f] + row * 256;
#pragma unroll
    for (int j = 0; j < 4; ++j) d[t][j] = x[lane + 64 * j];
  }
  const uint4* __restrict__ T = a.tab + ((INV ? 0 : 1) * 64 + lane) * 10;
  const bf16x8 b1rh = __builtin_bit_cast(bf16x8, T[0]), b1rl = __builtin_bit_cast(bf16x8, T[1]);
  const bf16x8 b1ih = __builtin_bit_cast(bf16x8, T[2]), b1il = __builtin_bit_cast(bf16x8, T[3]);
  const bf16x8 a2rh = __builtin_bit_cast(bf16x8, T[4]), a2rl = __builtin_bit_cast(bf16x8, T[5]);
  const bf16x8 a2ih = __builtin_bit_cast(bf16x8, T[6]), a2il = __builtin_bit_cast(bf16x8, T[7]);
  const float4 t01 = __builtin_bit_cast(float4, T[8]), t23 = __builtin_bit_cast(float4, T[9]);
  const float twr[4] = {t01.x, t01.z, t23.x, t23.z}, twi[4] = {t01.y, t01.w, t23.y, t23.w};
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < ZD_LPW; ++t) {
    const int64_t L = L0 + t;
    if (L >= a.lines) break;
    const int64_t f = L / a.rows, row = L - f * a.rows;
    const int mrow = a.row_m ? a.row_m[row] : 0;
    // stage 1: A operand (re, im of x[l + 64 j]); the inverse transform drops the unkept slots
    u16x8 ah, al;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float2 v = d[t][j];
      if (INV && !zspec_keep(a, mrow, lane + 64 * j)) v = make_float2(0.f, 0.f);
      unsigned short h, l;
      split2(v.x, h, l);
      ah[2 * j] = h;
      al[2 * j] = l;
      split2(v.y, h, l);
      ah[2 * j + 1] = h;
      al[2 * j + 1] = l;
    }
    const bf16x8 xh = __builtin_bit_cast(bf16x8, ah), xl = __builtin_bit_cast(bf16x8, al);
    const floatx4 yr = mfma3(xh, xl, b1rh, b1rl, zero);
    const floatx4 yi = mfma3(xh, xl, b1ih, b1il, zero);
    // twiddle, then the stage-2 B operand (re, im of Y'[k1][4 g + v])
    u16x8 bh, bl;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float re = yr[v] * twr[v] - yi[v] * twi[v];
      const float im = yr[v] * twi[v] + yi[v] * twr[v];
      unsigned short h, l;
      split2(re, h, l);
      bh[2 * v] = h;
      bl[2 * v] = l;
      split2(im, h, l);
      bh[2 * v + 1] = h;
      bl[2 * v + 1] = l;
    }
    const bf16x8 yh = __builtin_bit_cast(bf16x8, bh), yl = __builtin_bit_cast(bf16x8, bl);
    const floatx4 zr = mfma3(a2rh, a2rl, yh, yl, zero);
    const floatx4 zi = mfma3(a2ih, a2il, yh, yl, zero);
    float2* __restrict__ y = a.out[f] + row * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int kk = c + 16 * (4 * g + v);
      double2 o = make_double2((double)zr[v], (double)zi[v]);
      if (!INV) {
        o = make_double2(o.x * (1.0 / 256.0), o.y * (1.0 / 256.0));
        if (!zspec_keep(a, mrow, kk)) o = make_double2(0.0, 0.0);
      }
      st2(y + kk, o);
    }
  }
}

mlg_status check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MLG_OK;
}

}  // namespace

mlg_status launch_split_synth(const mlg_plan_s* p, const double* psi, const double* chi, double* const* out6,
                              hipStream_t s, const SynthMask& mask) {
  SplitSynthArgs<float2> a{};
  for (int t = 0; t < 4; ++t) a.tab[t] = p->d_split_syn[t];
  a.toff = p->d_split_syn_off;
  a.kpad = p->d_split_syn_kpad;
  a.psi = reinterpret_cast<const float2*>(psi);
  a.chi = reinterpret_cast<const float2*>(chi);
  for (int i = 0; i < 6; ++i) a.out[i] = reinterpret_cast<float2*>(out6[i]);
  a.off = p->d_goff;
  a.node = p->d_node;
  a.nr = p->nr;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  a.mkeep = mask.mkeep;
  a.kmax = mask.kmax;
  a.gx = (p->nz + TC - 1) / TC;
  a.gy = (p->nr + TM - 1) / TM;
  a.gz = p->M;
  a.nbpos = 0;
  if (mask.skip) {  // only the kept orders and the TC-aligned tiles of the kept slots |k| <= kmax
    a.gz = std::min(p->M, mask.mkeep + 1);
    a.nbpos = (mask.kmax + TC) / TC;                    // tiles from slot 0 through slot kmax
    a.nstart = ((p->nz - mask.kmax) / TC) * TC;         // the first tile holding slot nz - kmax
    const int nneg = mask.kmax >= 1 ? (p->nz - a.nstart + TC - 1) / TC : 0;
    if (a.nstart < TC * a.nbpos) {                      // the two ranges meet: every tile
      a.nbpos = 0;
    } else {
      a.gx = a.nbpos + nneg;
    }
  }
  p->timing.begin("synth_gemm", s);
  split_synth_kernel<float2><<<xcd_blocks(a.gx, a.gy, a.gz), 256, 0, s>>>(a);
  p->timing.end(s);
  return check("split_synth_kernel");
}

mlg_status launch_split_scalar(const mlg_plan_s* p, int dir, const double* in, double* out, hipStream_t s) {
  const bool fwd = dir < 0;
  SplitScalarArgs a{};
  for (int t = 0; t < 2; ++t) a.tab[t] = fwd ? p->d_split_prj[t] : p->d_split_syn[t];
  a.toff = fwd ? p->d_split_prj_off : p->d_split_syn_off;
  a.kpad = p->d_split_syn_kpad;
  a.ipad = p->split_ipad;
  a.in = reinterpret_cast<const float2*>(in);
  a.out = reinterpret_cast<float2*>(out);
  a.off = p->d_goff;
  a.nr = p->nr;
  a.nrc = p->nrc;
  a.nz = p->nz;
  a.gx = (p->nz + TC - 1) / TC;
  a.gy = ((fwd ? p->nrc : p->nr) + TM - 1) / TM;
  a.gz = p->M;
  p->timing.begin("radial_gemm", s);
  if (fwd)
    split_scalar_kernel<true><<<xcd_blocks(a.gx, a.gy, a.gz), 256, 0, s>>>(a);
  else
    split_scalar_kernel<false><<<xcd_blocks(a.gx, a.gy, a.gz), 256, 0, s>>>(a);
  p->timing.end(s);
  return check("split_scalar_kernel");
}

mlg_status launch_split_zdft(const mlg_plan_s* p, const double* const* in, double* const* out, int nf, int64_t rows,
                             int dir, const int32_t* row_m, int mask_m, int mask_k, hipStream_t s) {
  if (rows <= 0 || nf <= 0) return MLG_OK;
  if (nf > 6) return fail(MLG_E_ARG, "z transform: 1 to 6 fields per launch");
  if (p->nz != 256 || !p->d_split_zdft) return fail(MLG_E_UNSUPPORTED, "split z transform: N_z = 256 split plans only");
  ZdftArgs a{};
  a.tab = reinterpret_cast<const uint4*>(p->d_split_zdft);
  for (int i = 0; i < nf; ++i) {
    a.in[i] = reinterpret_cast<const float2*>(in[i]);
    a.out[i] = reinterpret_cast<float2*>(out[i]);
  }
  a.rows = rows;
  a.lines = rows * nf;
  a.nzc = p->nzc;
  a.row_m = row_m;
  a.mask_m = mask_m;
  a.mask_k = mask_k;
  const int64_t waves = (a.lines + ZD_LPW - 1) / ZD_LPW;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  p->timing.begin("z_fft", s);
  if (dir > 0)
    split_zdft_kernel<true><<<blocks, 256, 0, s>>>(a);
  else
    split_zdft_kernel<false><<<blocks, 256, 0, s>>>(a);
  p->timing.end(s);
  return check("split_zdft_kernel");
}

}  // namespace mlg
