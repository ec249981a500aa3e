// 256-point FFTs for gfx950 held in registers: a line is spread over the 32 lanes of half a
// wavefront, lane s owning the 8 samples x[s + 32 j].  The DFT factors as 8 x 8 x 4 (fft256w):
// a radix-8 pass in registers, a twiddle, an LDS exchange inside the wavefront, a second radix-8
// pass, a twiddle, an exchange and two radix-4 DFTs per lane, which leaves X[s + 32 k] in the same
// registers: input and output share one distribution, so inverse -> pointwise -> forward chains
// need no reshuffle.
//
// Kernels: the z transforms over contiguous lines (loads and stores straight from registers, 512
// contiguous bytes per 32 lanes, up to six fields per launch), and the azimuthal stages (the
// harmonics of 8 lines are gathered through LDS so that every global access covers 8 consecutive
// lines = 128 bytes): the scalar forward / backward transforms, the scalar nonlinear terms and the
// fused vector stage of the toroidal-poloidal RHS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

using namespace ::mlg::dev;

constexpr double kR2 = 0.70710678118654752;   // sqrt(2)/2

// multiply by w8^J, w8 = exp(-+ 2 pi i / 8) (forward: minus), J = 1, 2, 3
template <bool INV, int J>
__device__ __forceinline__ double2 tw8(double2 a) {
  constexpr double sg = INV ? 1.0 : -1.0;
  if constexpr (J == 1) return cmul(a, make_double2(kR2, sg * kR2));
  else if constexpr (J == 2) return cmul_mi(a, INV);
  else return cmul(a, make_double2(-kR2, sg * kR2));  // J == 3
}

template <bool INV>
__device__ __forceinline__ void dft4(double2& a, double2& b, double2& c, double2& d) {
  const double2 t0 = cadd(a, c), t1 = csub(a, c);
  const double2 t2 = cadd(b, d), t3 = cmul_mi(csub(b, d), INV);
  a = cadd(t0, t2);
  b = cadd(t1, t3);
  c = csub(t0, t2);
  d = csub(t1, t3);
}

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }
__device__ __forceinline__ bool kkept(int kk, int nz, int nzc) {
  const int k = kval(kk, nz);
  if (nz % 2 == 0 && nz > 1 && k == -(nz / 2)) return false;
  return (k < 0 ? -k : k) < nzc;
}

// ---------------------------------------------------------------- azimuthal stages
// Line q = i N_z + l; physical samples at (l N_r + i) 256 + j; harmonic m at m * nlines + q.
constexpr int PL = 8;  // lines per block

struct Phi256 {
  int nr, nz, M, mkeep;
  int64_t nlines;
};

__device__ __forceinline__ int64_t phys_off(const Phi256& g, int64_t q) {
  const int64_t i = q / g.nz;
  const int64_t l = q - i * g.nz;
  return (l * g.nr + i) * 256;
}

// ---------------------------------------------------------------- 32-lane lines
// The vector stage keeps four nodal fields of a line in registers while the last pair is
// transformed; at 16 lanes per line that state allows one wavefront per SIMD.  Here a line is
// spread over 32 lanes with 8 samples each (lane s holds x[s + 32 j]) and the 256-point DFT
// factors as 8 x 8 x 4: a radix-8 pass over j, a twiddle, an LDS exchange, a radix-8 pass over
// the lane's high bits, a twiddle, an exchange and two radix-4 DFTs per lane.  Taking the radix-4
// groups (s, s + 32) returns X[s + 32 j] in v[j]: input and output share one distribution.  The
// 32 lanes of a line lie in one wavefront, so the exchanges need only wavefront-level ordering.
constexpr int WL = 32;       // lanes per line
constexpr int VB = PL * WL;  // threads per block: 8 lines, 4 wavefronts
// LDS entries per line (harmonics at zpos(p), both exchanges).  286 = 14 (mod 16): the 8 lines of a
// block sit at distinct even entry offsets modulo 16 (the 64 banks), so the gathers and scatters
// that touch one order of all 8 lines (and the next order in the next 8 lanes) are conflict-free;
// with the twiddles a block stays within 40 KB of LDS (four blocks per CU)
constexpr int WROW = 286;

__device__ __forceinline__ int zpos(int p) { return 33 * (p >> 5) + (p & 31); }

// Orders the LDS accesses of one wavefront: earlier writes are seen by later reads of other lanes
// and earlier reads complete before later writes (LDS instructions of a wavefront execute in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-register 8-point DFT: v[n] -> V[k] = sum_n v[n] w8^(n k) (radix 2 over two 4-point DFTs).
template <bool INV>
__device__ __forceinline__ void dft8(double2 (&v)[8]) {
  dft4<INV>(v[0], v[2], v[4], v[6]);  // E[k] at v[2 k]
  dft4<INV>(v[1], v[3], v[5], v[7]);  // O[k] at v[2 k + 1]
  const double2 o1 = tw8<INV, 1>(v[3]), o2 = tw8<INV, 2>(v[5]), o3 = tw8<INV, 3>(v[7]);
  double2 x[8];
  x[0] = cadd(v[0], v[1]);
  x[4] = csub(v[0], v[1]);
  x[1] = cadd(v[2], o1);
  x[5] = csub(v[2], o1);
  x[2] = cadd(v[4], o2);
  x[6] = csub(v[4], o2);
  x[3] = cadd(v[6], o3);
  x[7] = csub(v[6], o3);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = x[k];
}

// v[c] *= w^(e c), c = 1..7, from the three table entries w^e, w^(2e), w^(4e) (w = exp(-2 pi i/256),
// conjugated for the inverse); every factor is at most two roundings from the exact twiddle.
template <bool INV>
__device__ __forceinline__ void twiddle8(double2 (&v)[8], const double2* __restrict__ tw, int e) {
  double2 w1 = tw[e], w2 = tw[2 * e], w4 = tw[4 * e];
  if (INV) {
    w1 = cconj(w1);
    w2 = cconj(w2);
    w4 = cconj(w4);
  }
  const double2 w3 = cmul(w1, w2), w6 = cmul(w4, w2);
  v[1] = cmul(v[1], w1);
  v[2] = cmul(v[2], w2);
  v[3] = cmul(v[3], w3);
  v[4] = cmul(v[4], w4);
  v[5] = cmul(v[5], cmul(w4, w1));
  v[6] = cmul(v[6], w6);
  v[7] = cmul(v[7], cmul(w6, w1));
}

// 256-point DFT of one line over its 32 lanes: on entry v[j] = x[s + 32 j], on exit
// v[j] = X[s + 32 j] (unscaled).  W is the line's LDS area (WROW entries); the caller orders any
// later writes to W after these reads.  With n = s + 32 j, s = a + 4 b and k = k2 + 8 c + 64 d:
// X[k] = sum_a w4^(a d) w32^(a c) sum_b w8^(b c) w256^(s k2) sum_j w8^(j k2) x[n].
template <bool INV>
__device__ __forceinline__ void fft256w(double2 (&v)[8], double2* W, int s, const double2* __restrict__ tw) {
  dft8<INV>(v);            // v[k2] = sum_j w8^(j k2) x[s + 32 j]
  twiddle8<INV>(v, tw, s);  // * w256^(s k2)
  wave_sync();
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) W[36 * k2 + s] = v[k2];
  wave_sync();
  const int a = s & 3, kb = s >> 2;  // this lane's (a, k2) for the second pass
#pragma unroll
  for (int b = 0; b < 8; ++b) v[b] = W[36 * kb + a + 4 * b];
  dft8<INV>(v);                // v[c] = sum_b w8^(b c) (...)
  twiddle8<INV>(v, tw, 8 * a);  // * w32^(a c)
  wave_sync();
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int gi = 8 * c + kb;
    W[4 * gi + a + (gi >> 2)] = v[c];
  }
  wave_sync();
  // radix-4 over a for the (c, k2) groups gi = s and s + 32: outputs k = s + 64 d and s + 32 + 64 d
  double2 p[4], r[4];
  const int g0 = s, g1 = s + 32;
#pragma unroll
  for (int aa = 0; aa < 4; ++aa) {
    p[aa] = W[4 * g0 + aa + (g0 >> 2)];
    r[aa] = W[4 * g1 + aa + (g1 >> 2)];
  }
  dft4<INV>(p[0], p[1], p[2], p[3]);
  dft4<INV>(r[0], r[1], r[2], r[3]);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    v[2 * d] = p[d];
    v[2 * d + 1] = r[d];
  }
}

// Harmonics of a field pair for the block's lines, held in registers so that their loads are in
// flight while another pair is transformed.  Entry it covers e = t + VB it: line e % PL, order
// e / PL.  The per-lane byte offset is 32-bit (the launcher bounds the line count) and the rest of
// the address is uniform.  Orders >= min(M, 128, mkeep + 1) read as zero; GUARD (the last block,
// or fewer than 128 stored orders) also reads lines past the end as zero.
template <typename S2>
struct PairRegs {
  S2 a[PL * 128 / VB], b[PL * 128 / VB];
};

template <bool GUARD, typename S2>
__device__ __forceinline__ void load_pair(PairRegs<S2>& r, const Phi256& g, int64_t q0, const S2* __restrict__ fa,
                                          const S2* __restrict__ fb) {
  const int t = threadIdx.x;
  const uint32_t off = (uint32_t)((t >> 3) * g.nlines + (t & 7)) * (uint32_t)sizeof(S2);
  // orders read: those stored (up to 128) and, under the two-thirds mask, those it keeps (the
  // synthesis and the z transforms before this stage leave the others unwritten)
  const int mmax = min(g.M < 128 ? g.M : 128, g.mkeep + 1);
  const bool line_ok = q0 + (t & 7) < g.nlines;
#pragma unroll
  for (int it = 0; it < PL * 128 / VB; ++it) {
    const int64_t base = q0 + (int64_t)(VB / PL) * it * g.nlines;
    const char* pa = reinterpret_cast<const char*>(fa + base) + off;
    const char* pb = reinterpret_cast<const char*>(fb + base) + off;
    if (!GUARD && mmax >= 128) {
      r.a[it] = *reinterpret_cast<const S2*>(pa);
      r.b[it] = *reinterpret_cast<const S2*>(pb);
    } else {
      const bool ok = (!GUARD || line_ok) && (t >> 3) + (VB / PL) * it < mmax;
      r.a[it] = ok ? *reinterpret_cast<const S2*>(pa) : czero<S2>();
      r.b[it] = ok ? *reinterpret_cast<const S2*>(pb) : czero<S2>();
    }
  }
}

// Writes the pair into Z as the Hermitian spectrum of a + i b.  Orders 1..127 fill positions
// m and 256 - m, order 0 position 0; only the Nyquist position 128 is cleared.  Starts with a
// barrier (earlier readers of Z are done) and ends with one.
template <typename S2>
__device__ __forceinline__ void store_pair(const PairRegs<S2>& r, double2 (*Z)[WROW]) {
  const int t = threadIdx.x;
  __syncthreads();
  if (t < PL) Z[t][zpos(128)] = make_double2(0.0, 0.0);
#pragma unroll
  for (int it = 0; it < PL * 128 / VB; ++it) {
    const int e = t + VB * it;
    const int ll = e & (PL - 1), m = e >> 3;
    const double2 a = to_d2(r.a[it]), b = to_d2(r.b[it]);
    if (m == 0) {
      Z[ll][0] = make_double2(a.x, b.x);
    } else {
      Z[ll][zpos(m)] = make_double2(a.x - b.y, a.y + b.x);
      Z[ll][zpos(256 - m)] = make_double2(a.x + b.y, -a.y + b.x);
    }
  }
  __syncthreads();
}

// Scatters the spectrum X (v[j] = X[s + 32 j]) of z = a + i b of each line to the harmonics of a
// and b (orders m <= mkeep and m < M, scaled by 1/256).  The orders above mkeep (the two-thirds
// mask of the RHS) are not written: the forward z transforms and the projection read only the
// orders the mask keeps.  Barriers at both ends.
template <typename S2>
__device__ __forceinline__ void scatter_pair_w(const double2 (&v)[8], double2 (*Z)[WROW], const Phi256& g,
                                               int64_t q0, int ll, int s, S2* fa, S2* fb) {
  __syncthreads();  // every line's exchange reads are complete
#pragma unroll
  for (int j = 0; j < 8; ++j) Z[ll][33 * j + s] = v[j];
  __syncthreads();
  const int t = threadIdx.x;
  const int mmax = g.M < 128 ? g.M : 128;
  const int mout = g.M < g.mkeep + 1 ? g.M : g.mkeep + 1;
  for (int e = t; e < PL * mout; e += VB) {
    const int l2 = e & (PL - 1), m = e >> 3;
    const int64_t q = q0 + l2;
    if (q >= g.nlines) continue;
    double2 A = make_double2(0.0, 0.0), B = A;
    if (m < mmax) {
      const double2 zm = Z[l2][zpos(m)];
      const double2 zc = cconj(Z[l2][zpos((256 - m) & 255)]);
      A = cscale(cadd(zm, zc), 0.5 / 256.0);
      const double2 d = csub(zm, zc);
      B = make_double2(0.5 / 256.0 * d.y, -0.5 / 256.0 * d.x);
    }
    st2(fa + (int64_t)m * g.nlines + q, A);
    if (fb) st2(fb + (int64_t)m * g.nlines + q, B);
  }
  __syncthreads();
}

template <typename S2>
struct Six256 {
  S2* f[6];
};

// TAPS: also store the nodal u, omega and N (the parity taps); without them the kernel fits 3
// waves per SIMD (156 VGPRs against 212 with the tap stores)
template <bool GUARD, bool TAPS, typename S2>
__global__ __launch_bounds__(VB) void phi_vec256_kernel(Phi256 g, const double2* __restrict__ twg, Six256<S2> fs,
                                                        const double* __restrict__ rinv, double Ux, double Uy,
                                                        double Uz, double* __restrict__ taps, int64_t blk0) {
  __shared__ double2 Z[PL][WROW];
  __shared__ double2 tw[256];  // exp(-2 pi i j / 256): twiddles and the node angles
  const int t = threadIdx.x, ll = t / WL, s = t % WL;
  const int64_t q0 = (blk0 + blockIdx.x) * PL;
  const int64_t q = q0 + ll;
  tw[t] = twg[t];  // VB == 256; visible after the first barrier of store_pair
  double2 v[8];
  double ur[8], up[8], uz[8], wr[8];
  PairRegs<S2> pr;
  // pair 0: (u_r, u_phi); the loads of each next pair are issued before the current transform
  load_pair<GUARD>(pr, g, q0, fs.f[0], fs.f[1]);
  store_pair(pr, Z);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = Z[ll][33 * j + s];
  load_pair<GUARD>(pr, g, q0, fs.f[2], fs.f[3]);
  fft256w<true>(v, Z[ll], s, tw);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    ur[k] = v[k].x;
    up[k] = v[k].y;
  }
  // pair 1: (u_z, w_r)
  store_pair(pr, Z);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = Z[ll][33 * j + s];
  load_pair<GUARD>(pr, g, q0, fs.f[4], fs.f[5]);
  fft256w<true>(v, Z[ll], s, tw);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    uz[k] = v[k].x;
    wr[k] = v[k].y;
  }
  // pair 2: (w_phi, w_z)
  store_pair(pr, Z);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = Z[ll][33 * j + s];
  fft256w<true>(v, Z[ll], s, tw);
  // nodal cross product at phi_j, j = s + 32 k: cos(phi_j) = tw[j].x, sin(phi_j) = -tw[j].y
  const bool valid = q < g.nlines;
  const double ri = valid ? rinv[q / g.nz] : 0.0;
  const int64_t pe = g.nlines * 256;
  double nzr[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int j = s + 32 * k;
    const double2 c = tw[j];
    const double cphi = c.x, sphi = -c.y;
    const double wp = v[k].x, wz = v[k].y;
    const double Ur = ur[k] + Ux * cphi + Uy * sphi;
    const double Up = up[k] - Ux * sphi + Uy * cphi;
    const double Uzz = uz[k] + Uz;
    const double Nr = Up * wz - Uzz * wp;
    const double Np = Uzz * wr[k] - Ur * wz;
    const double Nz = Ur * wp - Up * wr[k];
    if (TAPS && valid) {
      const int64_t o = phys_off(g, q) + j;
      taps[0 * pe + o] = ur[k];
      taps[1 * pe + o] = up[k];
      taps[2 * pe + o] = uz[k];
      taps[3 * pe + o] = wr[k];
      taps[4 * pe + o] = wp;
      taps[5 * pe + o] = wz;
      taps[6 * pe + o] = Nr;
      taps[7 * pe + o] = Np;
      taps[8 * pe + o] = Nz;
    }
    v[k] = make_double2(Nr * ri, Np * ri);
    nzr[k] = Nz;
  }
  fft256w<false>(v, Z[ll], s, tw);
  scatter_pair_w(v, Z, g, q0, ll, s, fs.f[0], fs.f[1]);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = make_double2(nzr[k], 0.0);
  fft256w<false>(v, Z[ll], s, tw);
  scatter_pair_w(v, Z, g, q0, ll, s, fs.f[2], (S2*)nullptr);
}

// ---------------------------------------------------------------- scalar phi stages (32-lane lines)
// Two real lines (2p, 2p+1) travel as one complex line z = a + i b, so a block of 8 line groups
// covers 16 real lines and every 256-point transform is used for two of them.  The backward stage
// packs the pair's harmonics as the Hermitian pair spectrum; the forward stage transforms the pair
// and separates the harmonics of both lines from its spectrum.  Gathers and scatters touch one
// order of 16 consecutive lines (256 contiguous bytes).  The twiddles are staged in LDS as in the
// vector stage; the block barrier of the gather publishes them.
constexpr int PL2 = 2 * PL;  // real lines per block of the scalar stages

// Z[pr] = the pair spectrum of lines q0 + 2 pr and q0 + 2 pr + 1 (orders m < min(M, 128); the
// Nyquist position cleared).  Ends with a block barrier.
template <typename S2>
__device__ __forceinline__ void gather_pairs16(double2 (*Z)[WROW], const Phi256& g, const S2* __restrict__ mixed,
                                               int64_t q0) {
  const int t = threadIdx.x;
  if (t < PL) Z[t][zpos(128)] = make_double2(0.0, 0.0);
  const int mmax = g.M < 128 ? g.M : 128;
#pragma unroll
  for (int it = 0; it < PL * 128 / VB; ++it) {
    const int e = t + VB * it;
    const int pr = e & (PL - 1), m = e >> 3;
    const int64_t qa = q0 + 2 * pr, qb = qa + 1;
    const double2 a = (m < mmax && qa < g.nlines) ? ld2(mixed + (int64_t)m * g.nlines + qa) : make_double2(0.0, 0.0);
    const double2 b = (m < mmax && qb < g.nlines) ? ld2(mixed + (int64_t)m * g.nlines + qb) : make_double2(0.0, 0.0);
    double2* Zp = Z[pr];
    if (m == 0) {
      Zp[0] = make_double2(a.x, b.x);
    } else {
      Zp[zpos(m)] = make_double2(a.x - b.y, a.y + b.x);
      Zp[zpos(256 - m)] = make_double2(a.x + b.y, -a.y + b.x);
    }
  }
  __syncthreads();
}

// Scatters the spectrum X (v[j] = X[s + 32 j]) of each group's pair to the harmonics of its two
// lines (orders m < M, scaled by 1/256; orders above mkeep written as zero).  Barriers at both ends.
template <typename S2>
__device__ __forceinline__ void scatter_pairs16(const double2 (&v)[8], double2 (*Z)[WROW], const Phi256& g,
                                                int64_t q0, int ll, int s, S2* __restrict__ out) {
  __syncthreads();  // every group's exchange reads are complete
#pragma unroll
  for (int j = 0; j < 8; ++j) Z[ll][33 * j + s] = v[j];
  __syncthreads();
  const int t = threadIdx.x;
  const int mmax = g.M < 128 ? g.M : 128;
  for (int e = t; e < PL2 * g.M; e += VB) {
    const int l2 = e & (PL2 - 1), m = e >> 4;
    const int64_t q = q0 + l2;
    if (q >= g.nlines) continue;
    double2 r = make_double2(0.0, 0.0);
    if (m < mmax && m <= g.mkeep) {
      const double2* Zp = Z[l2 >> 1];
      const double2 zm = Zp[zpos(m)];
      const double2 zc = cconj(Zp[zpos((256 - m) & 255)]);
      if ((l2 & 1) == 0) {
        r = cscale(cadd(zm, zc), 0.5 / 256.0);
      } else {
        const double2 d = csub(zm, zc);
        r = make_double2(0.5 / 256.0 * d.y, -0.5 / 256.0 * d.x);
      }
    }
    st2(out + (int64_t)m * g.nlines + q, r);
  }
  __syncthreads();
}

template <typename S2, typename S>
__global__ __launch_bounds__(VB) void phi_bwd256_kernel(Phi256 g, const double2* __restrict__ twg,
                                                        const S2* __restrict__ mixed, S* __restrict__ phys) {
  __shared__ double2 Z[PL][WROW];
  __shared__ double2 tw[256];
  const int t = threadIdx.x, ll = t / WL, s = t % WL;
  const int64_t q0 = (int64_t)blockIdx.x * PL2;
  tw[t] = twg[t];
  gather_pairs16(Z, g, mixed, q0);
  double2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = Z[ll][33 * j + s];
  fft256w<true>(v, Z[ll], s, tw);
  const int64_t qa = q0 + 2 * ll, qb = qa + 1;
  if (qa < g.nlines) {
    const int64_t o = phys_off(g, qa) + s;
#pragma unroll
    for (int k = 0; k < 8; ++k) st1(phys + o + 32 * k, v[k].x);
  }
  if (qb < g.nlines) {
    const int64_t o = phys_off(g, qb) + s;
#pragma unroll
    for (int k = 0; k < 8; ++k) st1(phys + o + 32 * k, v[k].y);
  }
}

template <typename S, typename S2>
__global__ __launch_bounds__(VB) void phi_fwd256_kernel(Phi256 g, const double2* __restrict__ twg,
                                                        const S* __restrict__ phys, S2* __restrict__ mixed) {
  __shared__ double2 Z[PL][WROW];
  __shared__ double2 tw[256];
  const int t = threadIdx.x, ll = t / WL, s = t % WL;
  const int64_t q0 = (int64_t)blockIdx.x * PL2;
  tw[t] = twg[t];
  const int64_t qa = q0 + 2 * ll, qb = qa + 1;
  const int64_t oa = qa < g.nlines ? phys_off(g, qa) + s : 0, ob = qb < g.nlines ? phys_off(g, qb) + s : 0;
  double2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double a = (qa < g.nlines) ? ld1(phys + oa + 32 * j) : 0.0;
    const double b = (qb < g.nlines) ? ld1(phys + ob + 32 * j) : 0.0;
    v[j] = make_double2(a, b);
  }
  __syncthreads();  // the twiddle table is staged
  fft256w<false>(v, Z[ll], s, tw);
  scatter_pairs16(v, Z, g, q0, ll, s, mixed);
}

// Scalar nonlinear term of Sec. 3.3 / Sec. 5.2 on two lines per group: inverse transform of the
// pair, u^2 or gamma u (1 - u) on each real line, forward transform of the pair of products.
template <int MODE, typename S2>
__global__ __launch_bounds__(VB) void phi_scalar256_kernel(Phi256 g, const double2* __restrict__ twg, S2* mixed,
                                                           double gamma) {
  __shared__ double2 Z[PL][WROW];
  __shared__ double2 tw[256];
  const int t = threadIdx.x, ll = t / WL, s = t % WL;
  const int64_t q0 = (int64_t)blockIdx.x * PL2;
  tw[t] = twg[t];
  gather_pairs16(Z, g, mixed, q0);
  double2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = Z[ll][33 * j + s];
  fft256w<true>(v, Z[ll], s, tw);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double ua = v[k].x, ub = v[k].y;
    v[k] = (MODE == MLG_RHS_U2) ? make_double2(ua * ua, ub * ub)
                                : make_double2(gamma * ua * (1.0 - ua), gamma * ub * (1.0 - ub));
  }
  fft256w<false>(v, Z[ll], s, tw);
  scatter_pairs16(v, Z, g, q0, ll, s, mixed);
}

// Contiguous lines of 256 samples, up to six fields per launch (blocks field-major).  Lane s of a
// line loads x[s + 32 j] straight into registers (32 lanes cover 512 contiguous bytes), fft256w
// transforms the line within its wavefront and the lane stores X[s + 32 j]: the only block
// barrier is the one after the twiddle table is staged.  In place when in == out.
template <typename S2>
struct ZFields {
  const S2* in[6];
  S2* out[6];
};

// kept_only (forward): slots outside the chop and the masks are not stored at all (for callers that
// read only the kept slots) instead of being written as zero
template <bool INV, typename S2>
__global__ __launch_bounds__(VB) void zfft256w_kernel(const double2* __restrict__ twg, ZFields<S2> fs, int64_t rows,
                                                      int64_t per_field, int nzc, const int32_t* __restrict__ row_m,
                                                      int mask_m, int mask_k, int kept_only) {
  __shared__ double2 Z[PL][WROW];
  __shared__ double2 tw[256];
  const int t = threadIdx.x, ll = t / WL, s = t % WL;
  tw[t] = twg[t];
  __syncthreads();
  // consecutive blocks take the same rows of every field, last rows first: the stage before wrote
  // them last, so they are the ones still held by the last-level cache
  const int64_t nf = gridDim.x / per_field;
  const int64_t f = blockIdx.x % nf;
  const int64_t row = (per_field - 1 - blockIdx.x / nf) * PL + ll;
  if (row >= rows) return;  // no block barrier follows
  const S2* __restrict__ x = fs.in[f] + row * 256;
  const int mrow = row_m ? row_m[row] : 0;
  // spectral slots kept by the chop and the masks: the backward transform does not read the others
  // (they may not have been written), the forward one writes them as zero
  auto keep = [&](int kk) {
    const int k = kval(kk, 256);
    return kkept(kk, 256, nzc) && (mask_k < 0 || (k < 0 ? -k : k) <= mask_k) && (!row_m || mrow <= mask_m);
  };
  double2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kk = s + 32 * j;
    v[j] = make_double2(0.0, 0.0);
    if (!INV || keep(kk)) v[j] = ld2(x + kk);
  }
  fft256w<INV>(v, Z[ll], s, tw);
  S2* __restrict__ y = fs.out[f] + row * 256;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kk = s + 32 * j;
    double2 a = v[j];
    if (!INV) {
      a = cscale(a, 1.0 / 256.0);
      if (!keep(kk)) {
        if (kept_only) continue;
        a = make_double2(0.0, 0.0);
      }
    }
    st2(y + kk, a);
  }
}

Phi256 phi256_geom(const mlg_plan_s* p, bool masked) {
  Phi256 g{};
  g.nr = p->nr;
  g.nz = p->nz;
  g.M = p->M;
  g.mkeep = masked ? p->dealias_m : (1 << 30);
  g.nlines = (int64_t)p->nr * p->nz;
  return g;
}

mlg_status check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MLG_OK;
}

}  // namespace

// Reduced-precision plans (MLG_FP32, MLG_SPLIT_BF16) keep their fields as float / float2.
static bool reduced(const mlg_plan_s* p) { return p->prec != MLG_FP64; }

template <typename S2>
static void zfft256_go(const mlg_plan_s* p, const double* const* in, double* const* out, int nf, int64_t rows, int dir,
                       const int32_t* row_m, int mask_m, int mask_k, bool kept_only, hipStream_t s) {
  ZFields<S2> fs{};
  for (int i = 0; i < nf; ++i) {
    fs.in[i] = reinterpret_cast<const S2*>(in[i]);
    fs.out[i] = reinterpret_cast<S2*>(out[i]);
  }
  const double2* tw = reinterpret_cast<const double2*>(p->d_tw_z);
  const int64_t per = (rows + PL - 1) / PL;
  dim3 grid((unsigned)(per * nf));
  if (dir > 0)
    zfft256w_kernel<true, S2><<<grid, VB, 0, s>>>(tw, fs, rows, per, p->nzc, row_m, mask_m, mask_k, 0);
  else
    zfft256w_kernel<false, S2><<<grid, VB, 0, s>>>(tw, fs, rows, per, p->nzc, row_m, mask_m, mask_k, kept_only ? 1 : 0);
}

mlg_status launch_zfft256(const mlg_plan_s* p, const double* const* in, double* const* out, int nf, int64_t rows,
                          int dir, const int32_t* row_m, int mask_m, int mask_k, hipStream_t s, bool kept_only) {
  if (nf < 1 || nf > 6) return fail(MLG_E_ARG, "z transform: 1 to 6 fields per launch");
  p->timing.begin("z_fft", s);
  if (reduced(p))
    zfft256_go<float2>(p, in, out, nf, rows, dir, row_m, mask_m, mask_k, kept_only, s);
  else
    zfft256_go<double2>(p, in, out, nf, rows, dir, row_m, mask_m, mask_k, kept_only, s);
  p->timing.end(s);
  return check("zfft256w_kernel");
}

mlg_status launch_phi256_forward(const mlg_plan_s* p, const double* phys, double* mixed, hipStream_t s) {
  Phi256 g = phi256_geom(p, false);
  dim3 grid((unsigned)((g.nlines + PL2 - 1) / PL2));
  const double2* tw = reinterpret_cast<const double2*>(p->d_tw_phi);
  p->timing.begin("phi_fft", s);
  if (reduced(p))
    phi_fwd256_kernel<float, float2><<<grid, VB, 0, s>>>(g, tw, reinterpret_cast<const float*>(phys),
                                                         reinterpret_cast<float2*>(mixed));
  else
    phi_fwd256_kernel<double, double2><<<grid, VB, 0, s>>>(g, tw, phys, reinterpret_cast<double2*>(mixed));
  p->timing.end(s);
  return check("phi_fwd256_kernel");
}

mlg_status launch_phi256_backward(const mlg_plan_s* p, const double* mixed, double* phys, hipStream_t s) {
  Phi256 g = phi256_geom(p, false);
  dim3 grid((unsigned)((g.nlines + PL2 - 1) / PL2));
  const double2* tw = reinterpret_cast<const double2*>(p->d_tw_phi);
  p->timing.begin("phi_fft", s);
  if (reduced(p))
    phi_bwd256_kernel<float2, float><<<grid, VB, 0, s>>>(g, tw, reinterpret_cast<const float2*>(mixed),
                                                         reinterpret_cast<float*>(phys));
  else
    phi_bwd256_kernel<double2, double><<<grid, VB, 0, s>>>(g, tw, reinterpret_cast<const double2*>(mixed), phys);
  p->timing.end(s);
  return check("phi_bwd256_kernel");
}

template <typename S2>
static void phi_scalar_go(const mlg_plan_s* p, const Phi256& g, int kind, double gamma, double* mixed, hipStream_t s) {
  dim3 grid((unsigned)((g.nlines + PL2 - 1) / PL2));
  const double2* tw = reinterpret_cast<const double2*>(p->d_tw_phi);
  if (kind == MLG_RHS_U2)
    phi_scalar256_kernel<MLG_RHS_U2, S2><<<grid, VB, 0, s>>>(g, tw, reinterpret_cast<S2*>(mixed), gamma);
  else
    phi_scalar256_kernel<MLG_RHS_KPP, S2><<<grid, VB, 0, s>>>(g, tw, reinterpret_cast<S2*>(mixed), gamma);
}

mlg_status launch_phi256_scalar(const mlg_plan_s* p, int kind, double gamma, double* mixed, hipStream_t s) {
  Phi256 g = phi256_geom(p, p->g.dealias != 0);
  p->timing.begin("phi_fft", s);
  if (reduced(p))
    phi_scalar_go<float2>(p, g, kind, gamma, mixed, s);
  else
    phi_scalar_go<double2>(p, g, kind, gamma, mixed, s);
  p->timing.end(s);
  return check("phi_scalar256_kernel");
}

template <typename S2>
static void phi_vec_go(const mlg_plan_s* p, const Phi256& g, const double* U, double* const* f6, double* taps,
                       hipStream_t s) {
  Six256<S2> six;
  for (int i = 0; i < 6; ++i) six.f[i] = reinterpret_cast<S2*>(f6[i]);
  const double2* tw = reinterpret_cast<const double2*>(p->d_tw_phi);
  // interior blocks (all 8 lines present, 128 stored orders) load without guards; one more
  // launch covers the last partial block, if any
  const int64_t full = g.M >= 128 ? g.nlines / PL : 0;
  const int64_t nblk = (g.nlines + PL - 1) / PL;
  const double* node = p->d_node;
  if (full > 0) {
    if (taps)
      phi_vec256_kernel<false, true, S2><<<dim3((unsigned)full), VB, 0, s>>>(g, tw, six, node, U[0], U[1], U[2], taps, 0);
    else
      phi_vec256_kernel<false, false, S2><<<dim3((unsigned)full), VB, 0, s>>>(g, tw, six, node, U[0], U[1], U[2], taps, 0);
  }
  if (nblk > full) {
    const dim3 grid((unsigned)(nblk - full));
    if (taps)
      phi_vec256_kernel<true, true, S2><<<grid, VB, 0, s>>>(g, tw, six, node, U[0], U[1], U[2], taps, full);
    else
      phi_vec256_kernel<true, false, S2><<<grid, VB, 0, s>>>(g, tw, six, node, U[0], U[1], U[2], taps, full);
  }
}

mlg_status launch_phi256_vec(const mlg_plan_s* p, const double* U, double* const* f6, double* taps, hipStream_t s) {
  Phi256 g = phi256_geom(p, p->g.dealias != 0);
  p->timing.begin("phi_fft", s);
  if (reduced(p))
    phi_vec_go<float2>(p, g, U, f6, taps, s);
  else
    phi_vec_go<double2>(p, g, U, f6, taps, s);
  p->timing.end(s);
  return check("phi_vec256_kernel");
}

}  // namespace mlg
