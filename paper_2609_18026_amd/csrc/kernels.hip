// HIP kernels for gfx950 (CDNA4): radial transforms on FP64 MFMA, LDS Stockham FFTs in phi
// and z, the fused pseudospectral phi stages, the toroidal-poloidal epilogue and the
// projection solves.  All launches are validated on the host against the plan's sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

using namespace ::mlg::dev;

// =====================================================================================
// Radial transform: batched C = A^T B on MFMA f64 16x16x4.
//   Workgroup tile 64 x 64 (rows x columns), K staged through LDS 16 at a time.
//   Four waves in a 2 x 2 arrangement, each owning a 32 x 32 sub-tile (2 x 2 MFMA blocks).
// MFMA operand layout (v_mfma_f64_16x16x4f64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator value v of lane l is C[l/16 + 4 v][l%16] (checked on gfx950).
// =====================================================================================
constexpr int GT_M = 64, GT_N = 64, GT_K = 16;

__global__ __launch_bounds__(256) void radial_gemm_f64(GemmProds prods, const GemmDesc* __restrict__ desc,
                                                        int nbatch, int ncol) {
  const int z = blockIdx.z;
  const int prod = z / nbatch;
  const int bi = z - prod * nbatch;
  const GemmDesc d = desc[bi];
  const int row0 = blockIdx.y * GT_M;
  const int col0 = blockIdx.x * GT_N;
  if (row0 >= d.rows || col0 >= ncol) return;  // K == 0 (orders m >= N_r^c) writes zeros
  const double* __restrict__ A = prods.A[prod] + d.a_off;
  const double* __restrict__ B = prods.B[prod] + d.b_off;
  double* __restrict__ C = prods.C[prod] + d.c_off;
  const int lscale = prods.lscale[prod];

  __shared__ double As[2][GT_K][GT_M];
  __shared__ double Bs[2][GT_K][GT_N];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  // raw loads with indices clamped into the operands (no branch around a load); the zeros outside
  // the operands and the n(n+1) scaling are applied at the LDS store, so the loads of the next
  // stage stay in flight across this stage's MFMAs.  Loads run only when d.K >= 1 (nk > 0); with
  // K == 0 (orders m >= N_r^c) the tile writes zeros.
  double ra[4], rb[4];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kk = e >> 6, cc = e & 63;
      const int k = k0 + kk, kc = k < d.K ? k : d.K - 1;
      const int row = row0 + cc, rc = row < d.rows ? row : d.rows - 1;
      const int col = col0 + cc, ccl = col < ncol ? col : ncol - 1;
      ra[t] = A[(int64_t)kc * d.lda + rc];
      rb[t] = B[(int64_t)kc * ncol + ccl];
    }
  };
  auto store_tiles = [&](int buf, int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kk = e >> 6, cc = e & 63;
      const int k = k0 + kk;
      const bool kin = k < d.K;
      As[buf][kk][cc] = (kin && row0 + cc < d.rows) ? ra[t] : 0.0;
      double v = rb[t];
      if (lscale) {
        const double n = (double)(k + d.m);
        v *= n * (n + 1.0);
      }
      Bs[buf][kk][cc] = (kin && col0 + cc < ncol) ? v : 0.0;
    }
  };
  const int nk = (d.K + GT_K - 1) / GT_K;
  if (nk > 0) {
    load_tiles(0);
    store_tiles(0, 0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tiles((kt + 1) * GT_K);
#pragma unroll
    for (int ks = 0; ks < GT_K; ks += 4) {
      const int kr = ks + (lane >> 4);
      double a0 = As[buf][kr][wr * 32 + (lane & 15)];
      double a1 = As[buf][kr][wr * 32 + 16 + (lane & 15)];
      double b0 = Bs[buf][kr][wc * 32 + (lane & 15)];
      double b1 = Bs[buf][kr][wc * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tiles(buf ^ 1, (kt + 1) * GT_K);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = col0 + wc * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * v;
        if (row < d.rows && col < ncol) C[(int64_t)row * ncol + col] = acc[i][j][v];
      }
    }
}

// =====================================================================================
// Stockham FFT in LDS on 'nlines' lines of length n (line stride 'ls'), radices 2,3,4,5.
// Pass with radix R and current span Ns (Ns = product of previous radices):
//   v_r = in[j + r n/R] * w^(r (j mod Ns) n/(Ns R)),  V = DFT_R(v),  out[(j/Ns) Ns R + j mod Ns + r Ns] = V_r.
// Forward uses w = exp(-2 pi i / n); inverse the conjugate (no scaling).
// =====================================================================================
struct FftRadices {
  int n, nrad;
  int rad[12];
};

template <int R>
__device__ __forceinline__ void dft_small(double2* v, const double2* __restrict__ tw, int n, bool inv) {
  if constexpr (R == 2) {
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    double2 t2 = cadd(v[1], v[3]), t3 = cmul_mi(csub(v[1], v[3]), inv);
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
  } else {
    double2 out[R];
    const int step = n / R;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double2 s = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 w = tw[((r * q) % R) * step];
        if (inv) w = cconj(w);
        s = cadd(s, cmul(v[r], w));
      }
      out[q] = s;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = out[q];
  }
}

template <int R>
__device__ __forceinline__ void fft_pass_r(const double2* in, double2* out, int n, int Ns, const double2* __restrict__ tw,
                                           bool inv, int nlines, int lsi, int lso, int tid, int nth) {
  const int nb = n / R;
  const int total = nlines * nb;
  const int tfac = n / (Ns * R);
  for (int idx = tid; idx < total; idx += nth) {
    const int line = idx / nb;
    const int j = idx - line * nb;
    const double2* src = in + line * lsi;
    double2* dst = out + line * lso;
    const int jm = j % Ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 w = tw[(jm * r * tfac) % n];
        if (inv) w = cconj(w);
        v[r] = cmul(v[r], w);
      }
    }
    dft_small<R>(v, tw, n, inv);
    const int o = (j / Ns) * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[o + r * Ns] = v[r];
  }
}

// Runs all passes; returns the buffer holding the result (x or y).  Line strides lsx / lsy
// belong to x / y.  Contains barriers: every thread of the block must call it.
__device__ double2* fft_lds(double2* x, double2* y, const FftRadices& fr, const double2* __restrict__ tw, bool inv,
                            int nlines, int lsx, int lsy) {
  const int tid = threadIdx.x, nth = blockDim.x;
  int Ns = 1;
  double2* a = x;
  double2* b = y;
  int la = lsx, lb = lsy;
  for (int p = 0; p < fr.nrad; ++p) {
    const int R = fr.rad[p];
    if (R == 4) fft_pass_r<4>(a, b, fr.n, Ns, tw, inv, nlines, la, lb, tid, nth);
    else if (R == 2) fft_pass_r<2>(a, b, fr.n, Ns, tw, inv, nlines, la, lb, tid, nth);
    else if (R == 3) fft_pass_r<3>(a, b, fr.n, Ns, tw, inv, nlines, la, lb, tid, nth);
    else fft_pass_r<5>(a, b, fr.n, Ns, tw, inv, nlines, la, lb, tid, nth);
    __syncthreads();
    Ns *= R;
    double2* t = a;
    a = b;
    b = t;
    int ts = la;
    la = lb;
    lb = ts;
  }
  return a;
}

// ---------------------------------------------------------------- phi lines
// A "line" q = i * N_z + l is the azimuthal line at (r_i, z_l).  Physical data of line q
// starts at (l * N_r + i) * N_phi; its harmonic m lives in a mixed array at m * N_r N_z + q.
struct PhiGeom {
  int nr, nz, nphi, M, mkeep;  // modes m < M stored, m <= mkeep written non-zero
  int64_t nlines;              // N_r * N_z
};

__device__ __forceinline__ int64_t phys_line_off(const PhiGeom& g, int64_t q) {
  const int64_t i = q / g.nz, l = q - (q / g.nz) * g.nz;
  return (l * g.nr + i) * g.nphi;
}

// Unpack the spectrum Z of z = a + i b (a, b real) into the harmonics of a and b.
__device__ __forceinline__ void hermitian_unpack(const double2* Z, int n, int m, double scale, double2* A, double2* B) {
  const double2 zm = Z[m];
  const double2 zc = cconj(Z[(n - m) % n]);
  *A = cscale(cadd(zm, zc), 0.5 * scale);
  const double2 d = csub(zm, zc);  // = 2 i B
  *B = make_double2(0.5 * scale * d.y, -0.5 * scale * d.x);
}

template <int MODE>
__device__ __forceinline__ double pointwise_scalar(double u, double gamma) {
  if constexpr (MODE == MLG_RHS_U2) return u * u;
  else return gamma * u * (1.0 - u);
}

// Forward phi transform: phys -> mixed (1/N_phi scaling), pairs of lines share one complex FFT.
__global__ __launch_bounds__(256) void phi_forward_kernel(PhiGeom g, FftRadices fr, const double2* __restrict__ tw,
                                                          const double* __restrict__ phys, double2* __restrict__ mixed,
                                                          int lb) {
  extern __shared__ double2 smem[];
  const int n = g.nphi;
  const int npair = (lb + 1) / 2;
  double2* X = smem;
  double2* Y = smem + npair * n;
  const int64_t q0 = (int64_t)blockIdx.x * lb;
  for (int e = threadIdx.x; e < npair * n; e += blockDim.x) {
    const int p = e / n, j = e - (e / n) * n;
    const int64_t qa = q0 + 2 * p, qb = qa + 1;
    double a = (qa < g.nlines) ? phys[phys_line_off(g, qa) + j] : 0.0;
    double b = (qb < g.nlines && 2 * p + 1 < lb) ? phys[phys_line_off(g, qb) + j] : 0.0;
    X[p * n + j] = make_double2(a, b);
  }
  __syncthreads();
  double2* Z = fft_lds(X, Y, fr, tw, false, npair, n, n);
  const double scale = 1.0 / n;
  for (int e = threadIdx.x; e < g.M * lb; e += blockDim.x) {
    const int m = e / lb, ll = e - (e / lb) * lb;
    const int64_t q = q0 + ll;
    if (q >= g.nlines) continue;
    double2 A, B;
    hermitian_unpack(Z + (ll >> 1) * n, n, m % n, scale, &A, &B);
    double2 v = (ll & 1) ? B : A;
    if (2 * m >= n || m > g.mkeep) v = make_double2(0.0, 0.0);
    mixed[(int64_t)m * g.nlines + q] = v;
  }
}

// Backward phi transform: mixed -> phys.
__global__ __launch_bounds__(256) void phi_backward_kernel(PhiGeom g, FftRadices fr, const double2* __restrict__ tw,
                                                           const double2* __restrict__ mixed, double* __restrict__ phys,
                                                           int lb) {
  extern __shared__ double2 smem[];
  const int n = g.nphi;
  const int npair = (lb + 1) / 2;
  double2* X = smem;
  double2* Y = smem + npair * n;
  const int64_t q0 = (int64_t)blockIdx.x * lb;
  const int half = (n + 1) / 2;  // orders with 2m < n
  for (int e = threadIdx.x; e < npair * n; e += blockDim.x) X[e] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int e = threadIdx.x; e < npair * half; e += blockDim.x) {
    const int p = e / half, m = e - (e / half) * half;
    if (m >= g.M) continue;
    const int64_t qa = q0 + 2 * p, qb = qa + 1;
    double2 a = (qa < g.nlines) ? mixed[(int64_t)m * g.nlines + qa] : make_double2(0.0, 0.0);
    double2 b = (qb < g.nlines && 2 * p + 1 < lb) ? mixed[(int64_t)m * g.nlines + qb] : make_double2(0.0, 0.0);
    if (m == 0) {
      X[p * n] = make_double2(a.x, b.x);
    } else {
      // Z_m = A_m + i B_m ; Z_{n-m} = conj(A_m) + i conj(B_m)
      X[p * n + m] = make_double2(a.x - b.y, a.y + b.x);
      X[p * n + n - m] = make_double2(a.x + b.y, -a.y + b.x);
    }
  }
  __syncthreads();
  double2* Z = fft_lds(X, Y, fr, tw, true, npair, n, n);
  for (int e = threadIdx.x; e < lb * n; e += blockDim.x) {
    const int ll = e / n, j = e - (e / n) * n;
    const int64_t q = q0 + ll;
    if (q >= g.nlines) continue;
    const double2 v = Z[(ll >> 1) * n + j];
    phys[phys_line_off(g, q) + j] = (ll & 1) ? v.y : v.x;
  }
}

// Fused scalar pseudospectral stage, in place on 'mixed': c2r, g(u), r2c.
template <int MODE>
__global__ __launch_bounds__(256) void phi_scalar_kernel(PhiGeom g, FftRadices fr, const double2* __restrict__ tw,
                                                         double2* __restrict__ mixed, double gamma, int lb) {
  extern __shared__ double2 smem[];
  const int n = g.nphi;
  const int npair = (lb + 1) / 2;
  double2* X = smem;
  double2* Y = smem + npair * n;
  const int64_t q0 = (int64_t)blockIdx.x * lb;
  const int half = (n + 1) / 2;
  for (int e = threadIdx.x; e < npair * n; e += blockDim.x) X[e] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int e = threadIdx.x; e < npair * half; e += blockDim.x) {
    const int p = e / half, m = e - (e / half) * half;
    if (m >= g.M) continue;
    const int64_t qa = q0 + 2 * p, qb = qa + 1;
    double2 a = (qa < g.nlines) ? mixed[(int64_t)m * g.nlines + qa] : make_double2(0.0, 0.0);
    double2 b = (qb < g.nlines && 2 * p + 1 < lb) ? mixed[(int64_t)m * g.nlines + qb] : make_double2(0.0, 0.0);
    if (m == 0) {
      X[p * n] = make_double2(a.x, b.x);
    } else {
      X[p * n + m] = make_double2(a.x - b.y, a.y + b.x);
      X[p * n + n - m] = make_double2(a.x + b.y, -a.y + b.x);
    }
  }
  __syncthreads();
  double2* Z = fft_lds(X, Y, fr, tw, true, npair, n, n);
  for (int e = threadIdx.x; e < npair * n; e += blockDim.x) {
    const double2 v = Z[e];
    Z[e] = make_double2(pointwise_scalar<MODE>(v.x, gamma), pointwise_scalar<MODE>(v.y, gamma));
  }
  __syncthreads();
  double2* other = (Z == X) ? Y : X;
  double2* W = fft_lds(Z, other, fr, tw, false, npair, n, n);
  const double scale = 1.0 / n;
  for (int e = threadIdx.x; e < g.M * lb; e += blockDim.x) {
    const int m = e / lb, ll = e - (e / lb) * lb;
    const int64_t q = q0 + ll;
    if (q >= g.nlines) continue;
    double2 A, B;
    hermitian_unpack(W + (ll >> 1) * n, n, m % n, scale, &A, &B);
    double2 v = (ll & 1) ? B : A;
    if (2 * m >= n || m > g.mkeep) v = make_double2(0.0, 0.0);
    mixed[(int64_t)m * g.nlines + q] = v;
  }
}

// Fused vector stage: six harmonic fields (u_r, u_phi, u_z, w_r, w_phi, w_z) -> nodal values ->
// N = (U + u) x w -> harmonics of N_r / r, N_phi / r, N_z written over fields 0, 1, 2.
// Per line: three complex inverse FFTs (pairs of fields) and two forward FFTs.
struct Six {
  double2* f[6];
};

__global__ __launch_bounds__(256) void phi_vec_kernel(PhiGeom g, FftRadices fr, const double2* __restrict__ tw,
                                                      Six fs, const double* __restrict__ rinv, double Ux, double Uy,
                                                      double Uz, double* __restrict__ taps, int lb) {
  extern __shared__ double2 smem[];
  const int n = g.nphi;
  // per line: three pair buffers P0, P1, P2 and one scratch S, each n complex
  double2* Pb = smem;                       // [lb][3][n]
  double2* Sb = smem + (size_t)lb * 3 * n;  // [lb][n]
  const int64_t q0 = (int64_t)blockIdx.x * lb;
  const int half = (n + 1) / 2;
  for (int e = threadIdx.x; e < lb * 3 * n; e += blockDim.x) Pb[e] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int e = threadIdx.x; e < lb * 3 * half; e += blockDim.x) {
    const int m = e % half;
    const int rest = e / half;
    const int pr = rest % 3, ll = rest / 3;
    if (m >= g.M) continue;
    const int64_t q = q0 + ll;
    double2 a = make_double2(0.0, 0.0), b = a;
    if (q < g.nlines) {
      a = fs.f[2 * pr][(int64_t)m * g.nlines + q];
      b = fs.f[2 * pr + 1][(int64_t)m * g.nlines + q];
    }
    double2* buf = Pb + ((size_t)ll * 3 + pr) * n;
    if (m == 0) {
      buf[0] = make_double2(a.x, b.x);
    } else {
      buf[m] = make_double2(a.x - b.y, a.y + b.x);
      buf[n - m] = make_double2(a.x + b.y, -a.y + b.x);
    }
  }
  __syncthreads();
  // three inverse transforms, each over lb lines (buffers strided by 3n)
  for (int pr = 0; pr < 3; ++pr) {
    double2* Z = fft_lds(Pb + (size_t)pr * n, Sb, fr, tw, true, lb, 3 * n, n);
    if (Z != Pb + (size_t)pr * n) {
      // result landed in the scratch (line stride n): copy home
      for (int e = threadIdx.x; e < lb * n; e += blockDim.x) {
        const int ll = e / n, j = e - (e / n) * n;
        Pb[((size_t)ll * 3 + pr) * n + j] = Sb[(size_t)ll * n + j];
      }
      __syncthreads();
    }
  }
  // cross product at every node; nodal (u, w) and N optionally copied to taps
  const int64_t pe = (int64_t)g.nlines * n;  // physical elements per field
  for (int e = threadIdx.x; e < lb * n; e += blockDim.x) {
    const int ll = e / n, j = e - (e / n) * n;
    const int64_t q = q0 + ll;
    double2* b0 = Pb + ((size_t)ll * 3 + 0) * n;
    double2* b1 = Pb + ((size_t)ll * 3 + 1) * n;
    double2* b2 = Pb + ((size_t)ll * 3 + 2) * n;
    const double ur = b0[j].x, up = b0[j].y, uz = b1[j].x, wr = b1[j].y, wp = b2[j].x, wz = b2[j].y;
    double sphi, cphi;
    sincospi(2.0 * j / n, &sphi, &cphi);
    const double Ur = ur + Ux * cphi + Uy * sphi;
    const double Up = up - Ux * sphi + Uy * cphi;
    const double Uzz = uz + Uz;
    const double Nr = Up * wz - Uzz * wp;
    const double Np = Uzz * wr - Ur * wz;
    const double Nz = Ur * wp - Up * wr;
    if (taps != nullptr && q < g.nlines) {
      const int64_t o = phys_line_off(g, q) + j;
      taps[0 * pe + o] = ur; taps[1 * pe + o] = up; taps[2 * pe + o] = uz;
      taps[3 * pe + o] = wr; taps[4 * pe + o] = wp; taps[5 * pe + o] = wz;
      taps[6 * pe + o] = Nr; taps[7 * pe + o] = Np; taps[8 * pe + o] = Nz;
    }
    const double ri = (q < g.nlines) ? rinv[q / g.nz] : 0.0;
    b0[j] = make_double2(Nr * ri, Np * ri);
    b1[j] = make_double2(Nz, 0.0);
  }
  __syncthreads();
  for (int pr = 0; pr < 2; ++pr) {
    double2* Z = fft_lds(Pb + (size_t)pr * n, Sb, fr, tw, false, lb, 3 * n, n);
    if (Z != Pb + (size_t)pr * n) {
      for (int e = threadIdx.x; e < lb * n; e += blockDim.x) {
        const int ll = e / n, j = e - (e / n) * n;
        Pb[((size_t)ll * 3 + pr) * n + j] = Sb[(size_t)ll * n + j];
      }
      __syncthreads();
    }
  }
  const double scale = 1.0 / n;
  for (int e = threadIdx.x; e < g.M * lb; e += blockDim.x) {
    const int m = e / lb, ll = e - (e / lb) * lb;
    const int64_t q = q0 + ll;
    if (q >= g.nlines) continue;
    double2 A, B, Cz, Dz;
    hermitian_unpack(Pb + ((size_t)ll * 3 + 0) * n, n, m % n, scale, &A, &B);
    hermitian_unpack(Pb + ((size_t)ll * 3 + 1) * n, n, m % n, scale, &Cz, &Dz);
    const bool zero = (2 * m >= n || m > g.mkeep);
    const double2 z0 = make_double2(0.0, 0.0);
    fs.f[0][(int64_t)m * g.nlines + q] = zero ? z0 : A;
    fs.f[1][(int64_t)m * g.nlines + q] = zero ? z0 : B;
    fs.f[2][(int64_t)m * g.nlines + q] = zero ? z0 : Cz;
  }
}

// ---------------------------------------------------------------- z transform
struct ZGeom {
  int nz, nzc, mask_m, mask_k;
  int64_t rows;
};

__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }
__device__ __forceinline__ bool kkept(int kk, int nz, int nzc) {
  const int k = kval(kk, nz);
  if (nz % 2 == 0 && nz > 1 && k == -(nz / 2)) return false;
  return (k < 0 ? -k : k) < nzc;
}
// spectral slot kk of line 'row' kept by the chop and the masks (the backward transform reads only
// these, the forward one writes the others as zero): |k| <= mask_k when mask_k >= 0, and the row's
// order at most mask_m when row_m is given
__device__ __forceinline__ bool zspec_keep(const ZGeom& g, const int32_t* row_m, int64_t row, int kk) {
  const int k = kval(kk, g.nz);
  return kkept(kk, g.nz, g.nzc) && (g.mask_k < 0 || (k < 0 ? -k : k) <= g.mask_k) &&
         (row_m == nullptr || row_m[row] <= g.mask_m);
}

__global__ __launch_bounds__(256) void zfft_kernel(ZGeom g, FftRadices fr, const double2* __restrict__ tw,
                                                   const double2* __restrict__ in, double2* __restrict__ out, int dir,
                                                   const int32_t* __restrict__ row_m, int lb) {
  extern __shared__ double2 smem[];
  const int n = g.nz;
  double2* X = smem;
  double2* Y = smem + (size_t)lb * n;
  const int64_t r0 = (int64_t)blockIdx.x * lb;
  for (int e = threadIdx.x; e < lb * n; e += blockDim.x) {
    const int ll = e / n, kk = e - (e / n) * n;
    const int64_t row = r0 + ll;
    double2 v = make_double2(0.0, 0.0);
    if (row < g.rows && (dir < 0 || zspec_keep(g, row_m, row, kk))) v = in[row * n + kk];
    X[e] = v;
  }
  __syncthreads();
  double2* Z = fft_lds(X, Y, fr, tw, dir > 0, lb, n, n);
  const double scale = (dir > 0) ? 1.0 : 1.0 / n;
  for (int e = threadIdx.x; e < lb * n; e += blockDim.x) {
    const int ll = e / n, kk = e - (e / n) * n;
    const int64_t row = r0 + ll;
    if (row >= g.rows) continue;
    double2 v = cscale(Z[e], scale);
    if (dir < 0 && !zspec_keep(g, row_m, row, kk)) v = make_double2(0.0, 0.0);
    out[row * n + kk] = v;
  }
}

// ---------------------------------------------------------------- projection solves
// Per active (m, k slot) column (kept by the axial chop and, with dealiasing, by the two-thirds
// mask).  Inputs (triangular, k spectral) from the projection products: the curl source
// C = [z . curl N]^, K' = -i kap [(1/r) d_r(r N_r)]^ - m kap [N_phi/r]^ and Zhat = [N_z]^.
//   K = K' - Dbar Zhat,  Dbar = -G L / ell^2.
//   psi: G (L psi) = ell^2 C              (L D L^T of G, per order)
//   q:   q = -Zhat at k = 0, else (G + kap^2 ell^2 L^-1)(L q) = -ell^2 K   (L D L^T per column,
//        a plan constant)
//   chi: G (L chi) = -ell^2 q             (U D U^T of G, started from the top degree)
// For m = 0 the unknowns n >= 1 use G restricted to n >= 1 and n = 0 follows from the decay
// gauge sum_n sqrt((2n+1)/2) s_n = 0.
//
// Every substitution is a linear recurrence of order two, y_t = a_t - al_t y_(t-+1) - be_t y_(t-+2),
// so its value on a run of degrees is affine in the two values entering the run.  A column is
// solved by the PS_SEG lanes of one half wave, each owning a run of at most SMAX consecutive
// degrees: a lane sweeps its run from a zero entering state while carrying the two homogeneous
// solutions (the 2 x 2 map of the entering state), the entering states follow from an exclusive
// scan of the run maps across the half wave (lane shuffles; composition of affine maps is
// associative), and the lane adds the homogeneous part.  Four such rounds: the forward
// substitutions of psi and q, their back substitutions (then psi and q are final), the chi sweep
// U w = -ell^2 q, and its back substitution.  Every intermediate stays in registers, and no round
// waits for another wave.
struct ProjArgs {
  const double2* __restrict__ Cs;
  const double2* __restrict__ Kp;
  const double2* __restrict__ Pc;
  void* __restrict__ psi;        // outputs: double2, or float2 on reduced-precision plans
  void* __restrict__ chi;
  double2* __restrict__ taps;    // C, K, Zhat (triangular) or null
  const double* __restrict__ gram;
  const int64_t* __restrict__ off;
  const double2* __restrict__ qfl;  // q-operator factors (l1, l2), [m][t][padded column], nrc + 2 rows per m
  const double* __restrict__ qfr;   // and reciprocal pivots
  const int32_t* __restrict__ row_m;  // order of each triangular row
  int64_t ngram, tri_elems, rows;
  int nz, nrc, kmax, mmax;
  ColBlocks cb;                  // the aligned column blocks (one per block of the grid's x)
  double ell2, kap0;
};

constexpr int PS_SEG = 32;  // lanes (runs of degrees) per column: half a wave
constexpr int PS_COL = 8;   // columns per block (two per wave)
constexpr int PJ_PAD = 2;   // zero entries before and after each per-m coefficient table

// LDS: 11 per-m tables of nrc + 2 PJ_PAD entries (doubles), each with one spare double after
// every 8 entries: the lanes of a half wave read entries 8 apart (one run each), which would
// otherwise fall on 4 banks
__host__ __device__ constexpr int proj_table_stride(int nrc) {
  return (nrc + 2 * PJ_PAD) + (nrc + 2 * PJ_PAD) / 8 + 2;
}
__host__ __device__ constexpr size_t proj_tables_len(int nrc) { return 11 * (size_t)proj_table_stride(nrc); }

// entry t (t >= -PJ_PAD) of a per-m table that starts PJ_PAD doubles into its slot
struct PTab {
  double* p;
  __device__ __forceinline__ double& operator[](int t) const { return p[t + ((t + 8) >> 3)]; }
};

// The affine map of a run: (y_last, y_before) = (c, p) + [h0 h1; h2 h3] (entering y_1, y_2)
struct RunMap {
  double2 c, p;
  double h0, h1, h2, h3;
};

__device__ __forceinline__ double2 fms2(double2 a, double al, double2 y1, double be, double2 y2) {
  return make_double2(a.x - al * y1.x - be * y2.x, a.y - al * y1.y - be * y2.y);
}

// Sweep of one run, in storage order j = 0..len-1 (UP) or len-1..0 (down), from a zero entering
// state; coef(j, al, be) gives the recurrence coefficients of entry j.
template <int SMAX, bool UP, class Coef>
__device__ __forceinline__ RunMap sweep_run(double2 (&y)[SMAX], const double2 (&a)[SMAX], int len, Coef coef) {
  double2 yc = make_double2(0.0, 0.0), yp = yc;
  double e1c = 1.0, e1p = 0.0, e2c = 0.0, e2p = 1.0;
#pragma unroll
  for (int jj = 0; jj < SMAX; ++jj) {
    const int j = UP ? jj : SMAX - 1 - jj;
    if (j < len) {
      double al, be;
      coef(j, al, be);
      const double2 v = fms2(a[j], al, yc, be, yp);
      yp = yc;
      yc = v;
      y[j] = v;
      const double n1 = -al * e1c - be * e1p, n2 = -al * e2c - be * e2p;
      e1p = e1c;
      e1c = n1;
      e2p = e2c;
      e2c = n2;
    }
  }
  return RunMap{yc, yp, e1c, e2c, e1p, e2p};
}

// A o B: the map of run B followed by run A
__device__ __forceinline__ RunMap compose(const RunMap& A, const RunMap& B) {
  RunMap o;
  o.c = make_double2(A.c.x + A.h0 * B.c.x + A.h1 * B.p.x, A.c.y + A.h0 * B.c.y + A.h1 * B.p.y);
  o.p = make_double2(A.p.x + A.h2 * B.c.x + A.h3 * B.p.x, A.p.y + A.h2 * B.c.y + A.h3 * B.p.y);
  o.h0 = A.h0 * B.h0 + A.h1 * B.h2;
  o.h1 = A.h0 * B.h1 + A.h1 * B.h3;
  o.h2 = A.h2 * B.h0 + A.h3 * B.h2;
  o.h3 = A.h2 * B.h1 + A.h3 * B.h3;
  return o;
}

// DPP lane moves of a double (two 32-bit moves): lanes whose source lies outside the pattern, and
// rows outside ROWMASK, keep 'old'.  The moves are VALU operations and need no LDS round trip.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_d(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)x, CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int DPP_ROW_SHL = 0x100, DPP_ROW_SHR = 0x110, DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138,
              DPP_ROW_BCAST15 = 0x142;

// the map of the lane the pattern names; lanes without a source receive the identity map
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ RunMap dpp_map(const RunMap& q) {
  RunMap o;
  o.c = make_double2(dpp_d<CTRL, ROWMASK>(0.0, q.c.x), dpp_d<CTRL, ROWMASK>(0.0, q.c.y));
  o.p = make_double2(dpp_d<CTRL, ROWMASK>(0.0, q.p.x), dpp_d<CTRL, ROWMASK>(0.0, q.p.y));
  o.h0 = dpp_d<CTRL, ROWMASK>(1.0, q.h0);
  o.h1 = dpp_d<CTRL, ROWMASK>(0.0, q.h1);
  o.h2 = dpp_d<CTRL, ROWMASK>(0.0, q.h2);
  o.h3 = dpp_d<CTRL, ROWMASK>(1.0, q.h3);
  return o;
}

// every lane of a group of 32 reads lane 16 of its group (ds_swizzle, bit mode with or-mask 16)
__device__ __forceinline__ double swz_lane16(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)x, 16 << 5);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(x >> 32), 16 << 5);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Entering state (y_1, y_2) of run r, the composition of the runs before it applied to a zero
// state (UP: runs 0..r-1 in order, else PS_SEG-1 down to r+1).  The column's 32 lanes are two
// rows of 16: an inclusive scan of the maps within each row by DPP row shifts of 1, 2, 4, 8 (lanes
// past the row's edge compose with the identity), then the rows join: ascending, the second row
// composes with the last lane of the first (DPP row broadcast); descending, the first row composes
// with the first lane of the second (swizzle).  The state left by the previous run is then a
// one-lane DPP wave shift.  Against a Kogge-Stone scan over 32 lanes with LDS permutes, 0.173 ->
// 0.158 ms for the solves at 256^3.
template <bool UP>
__device__ __forceinline__ void enter_state(RunMap q, int r, double2& in1, double2& in2) {
  static_assert(PS_SEG == 32, "two DPP rows of 16 lanes per column");
  if (UP) {
    q = compose(q, dpp_map<DPP_ROW_SHR + 1>(q));
    q = compose(q, dpp_map<DPP_ROW_SHR + 2>(q));
    q = compose(q, dpp_map<DPP_ROW_SHR + 4>(q));
    q = compose(q, dpp_map<DPP_ROW_SHR + 8>(q));
    q = compose(q, dpp_map<DPP_ROW_BCAST15, 0xa>(q));  // lane 15 (47) into the lanes of row 1 (3)
    in1 = make_double2(dpp_d<DPP_WAVE_SHR1>(0.0, q.c.x), dpp_d<DPP_WAVE_SHR1>(0.0, q.c.y));
    in2 = make_double2(dpp_d<DPP_WAVE_SHR1>(0.0, q.p.x), dpp_d<DPP_WAVE_SHR1>(0.0, q.p.y));
  } else {
    q = compose(q, dpp_map<DPP_ROW_SHL + 1>(q));
    q = compose(q, dpp_map<DPP_ROW_SHL + 2>(q));
    q = compose(q, dpp_map<DPP_ROW_SHL + 4>(q));
    q = compose(q, dpp_map<DPP_ROW_SHL + 8>(q));
    RunMap o;
    o.c = make_double2(swz_lane16(q.c.x), swz_lane16(q.c.y));
    o.p = make_double2(swz_lane16(q.p.x), swz_lane16(q.p.y));
    o.h0 = swz_lane16(q.h0);
    o.h1 = swz_lane16(q.h1);
    o.h2 = swz_lane16(q.h2);
    o.h3 = swz_lane16(q.h3);
    if (r >= 16) o = RunMap{make_double2(0.0, 0.0), make_double2(0.0, 0.0), 1.0, 0.0, 0.0, 1.0};
    q = compose(q, o);
    in1 = make_double2(dpp_d<DPP_WAVE_SHL1>(0.0, q.c.x), dpp_d<DPP_WAVE_SHL1>(0.0, q.c.y));
    in2 = make_double2(dpp_d<DPP_WAVE_SHL1>(0.0, q.p.x), dpp_d<DPP_WAVE_SHL1>(0.0, q.p.y));
  }
  if (UP ? r == 0 : r == PS_SEG - 1) {  // the first run in sweep order enters from zero
    in1 = make_double2(0.0, 0.0);
    in2 = in1;
  }
}

// Adds the homogeneous solution started from the entering state (in1, in2)
template <int SMAX, bool UP, class Coef>
__device__ __forceinline__ void add_entering(double2 (&y)[SMAX], int len, double2 in1, double2 in2, Coef coef) {
#pragma unroll
  for (int jj = 0; jj < SMAX; ++jj) {
    const int j = UP ? jj : SMAX - 1 - jj;
    if (j < len) {
      double al, be;
      coef(j, al, be);
      const double2 d = make_double2(-al * in1.x - be * in2.x, -al * in1.y - be * in2.y);
      in2 = in1;
      in1 = d;
      y[j] = cadd(y[j], d);
    }
  }
}

template <bool TAPS, int SMAX, typename O2>
__global__ __launch_bounds__(PS_SEG * PS_COL, SMAX <= 8 ? 2 : 1) void projection_kernel(ProjArgs a) {
  extern __shared__ double sm[];
  const int m = blockIdx.y;
  const int nrc = a.nrc;
  const int cnt = nrc - m;  // degrees n = m .. nrc-1 at index t = n - m
  const int i0 = (m > 0 ? m : 1) - m;  // first solved index (m = 0: n = 0 is the gauge row)
  const int len_t = cnt + 2 * PJ_PAD;
  const int tstr = proj_table_stride(nrc);
  const PTab sg0{sm + PJ_PAD}, sg1{sg0.p + tstr}, sg2{sg1.p + tstr}, srd{sg2.p + tstr}, sl1{srd.p + tstr},
      sl2{sl1.p + tstr}, sru{sl2.p + tstr}, su1{sru.p + tstr}, su2{su1.p + tstr}, srL{su2.p + tstr}, sgw{srL.p + tstr};
  const int64_t gbase = a.off[m];
  const int lane = threadIdx.x & 63;
  const int c = (threadIdx.x >> 6) * 2 + (lane >> 5), r = lane & (PS_SEG - 1);  // column, run
  const int nz = a.nz;
  const int slot = blockIdx.x * PS_COL + c;  // padded column index
  bool active;
  const int kc = colblk_kk(a.cb, slot, a.kmax, nz, active);
  const int kk = active ? kc : 0;  // inactive lanes load column 0 and store nothing
  const int k = kval(kk, nz);
  const bool k0 = k == 0;
  const int nsol = cnt - i0;
  const int S = (nsol + PS_SEG - 1) / PS_SEG;
  const int s0 = i0 + r * S;
  const int len = max(0, min(s0 + S, cnt) - s0);
  const double2 z0 = make_double2(0.0, 0.0);
  const double ell2 = a.ell2, inv_ell2 = 1.0 / a.ell2;
  const double2* __restrict__ Cs = a.Cs + gbase * nz + kk;
  const double2* __restrict__ Kp = a.Kp + gbase * nz + kk;
  const double2* __restrict__ Zc = a.Pc + gbase * nz + kk;
  O2* __restrict__ ps = reinterpret_cast<O2*>(a.psi) + gbase * nz + kk;
  O2* __restrict__ chv = reinterpret_cast<O2*>(a.chi) + gbase * nz + kk;
  const int qrows = nrc + 2;
  const int ncolp = 8 * a.cb.nblk;
  const double2* __restrict__ qfl = a.qfl + (int64_t)m * qrows * ncolp + slot;
  const double* __restrict__ qfr = a.qfr + (int64_t)m * qrows * ncolp + slot;
  auto tcl = [&](int t) { return t < 0 ? 0 : (t < cnt ? t : cnt - 1); };  // clamped into the column
  auto lzv = [&](int t, double2 z) {
    const double n = (double)(m + t);
    return cscale(z, n * (n + 1.0));
  };
  // (G L Zhat)_t from L Zhat at t-2..t+2 (entries outside the column meet zero-padded couplings)
  auto glz = [&](int t, double2 zm2, double2 zm1, double2 zc, double2 zp1, double2 zp2) {
    double2 g = cscale(zc, sg0[t]);
    g = cadd(g, cscale(zm1, sg1[t - 1]));
    g = cadd(g, cscale(zm2, sg2[t - 2]));
    g = cadd(g, cscale(zp1, sg1[t]));
    return cadd(g, cscale(zp2, sg2[t]));
  };

  // ---- the source loads of round 1 go out first: they need nothing from LDS, and they stay in
  // flight while the block clears the inactive entries and stages its tables
  double2 yp[SMAX], yq[SMAX];
  double2 qf[SMAX], qx[2];
  double qr[SMAX];
  double2 zw[SMAX + 4];  // Zhat at t = s0 - 2 + i
  // the sweeps of round 1 overwrite their sources in place (entry j is read before it is written)
  double2 (&ap)[SMAX] = yp;
  double2 (&aq)[SMAX] = yq;
#pragma unroll
  for (int i = 0; i < SMAX + 4; ++i) zw[i] = Zc[(int64_t)tcl(s0 - 2 + i) * nz];
#pragma unroll
  for (int j = 0; j < SMAX; ++j) {
    const int t = tcl(s0 + j);
    ap[j] = Cs[(int64_t)t * nz];
    aq[j] = Kp[(int64_t)t * nz];
  }
  {
    // every block first clears its share of the entries whose (m, k) column is not solved (the
    // stores drain while the solves wait on their loads): (1) a contiguous share of the rows of
    // the orders m >= mmax, (2) its share of the rows of its own order m, slots kmax+1 .. nz-kmax-1
    // (the |k| outside the kept band; empty when nz = 1)
    const double2 z = make_double2(0.0, 0.0);
    auto clear = [&](int64_t e) {
      st2(reinterpret_cast<O2*>(a.psi) + e, z);
      st2(reinterpret_cast<O2*>(a.chi) + e, z);
      if (TAPS) {
        a.taps[e] = z;
        a.taps[a.tri_elems + e] = z;
        a.taps[2 * a.tri_elems + e] = z;
      }
    };
    const int64_t zb = a.off[a.mmax] * a.nz, total = a.rows * a.nz - zb;
    const int64_t nb = (int64_t)gridDim.x * gridDim.y, b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int64_t per = (total + nb - 1) / nb;
    const int64_t e1 = min(total, (b + 1) * per);
    for (int64_t e = b * per + threadIdx.x; e < e1; e += blockDim.x) clear(zb + e);
    const int band = a.nz - 2 * a.kmax - 1;
    if (band > 0) {
      const int rows_m = a.nrc - m;
      const int nrow = rows_m > (int)blockIdx.x ? (rows_m - (int)blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
      const int64_t base = a.off[m] * a.nz + a.kmax + 1;
      for (int e = threadIdx.x; e < nrow * band; e += blockDim.x) {
        const int i = e / band;
        clear(base + (int64_t)(blockIdx.x + i * gridDim.x) * a.nz + (e - i * band));
      }
    }
  }
  for (int e = threadIdx.x; e < len_t; e += blockDim.x) {
    const int t = e - PJ_PAD;
    const bool in = t >= 0 && t < cnt;
    const int64_t g = gbase + (in ? t : 0);
    const bool sol = in && t >= i0;
    sg0[t] = in ? a.gram[g] : 0.0;
    sg1[t] = in && t + 1 < cnt ? a.gram[a.ngram + g] : 0.0;
    sg2[t] = in && t + 2 < cnt ? a.gram[2 * a.ngram + g] : 0.0;
    srd[t] = sol ? a.gram[3 * a.ngram + g] : 0.0;
    sl1[t] = sol && t - 1 >= i0 ? a.gram[4 * a.ngram + g] : 0.0;
    sl2[t] = sol && t - 2 >= i0 ? a.gram[5 * a.ngram + g] : 0.0;
    sru[t] = sol ? a.gram[6 * a.ngram + g] : 0.0;
    su1[t] = sol && t + 1 < cnt ? a.gram[7 * a.ngram + g] : 0.0;
    su2[t] = sol && t + 2 < cnt ? a.gram[8 * a.ngram + g] : 0.0;
    const double n = (double)(m + t);
    srL[t] = in && m + t > 0 ? 1.0 / (n * (n + 1.0)) : 0.0;
    sgw[t] = in ? sqrt((2.0 * n + 1.0) * 0.5) : 0.0;
  }
  __syncthreads();


  // ---- round 1 (ascending): sources, forward substitutions of psi and q
  {
#pragma unroll
    for (int j = 0; j < SMAX; ++j) {
      if (j < len) {
        const int t = s0 + j;
        const double2 g = glz(t, lzv(t - 2, zw[j]), lzv(t - 1, zw[j + 1]), lzv(t, zw[j + 2]), lzv(t + 1, zw[j + 3]),
                              lzv(t + 2, zw[j + 4]));
        const double2 K = make_double2(aq[j].x + g.x * inv_ell2, aq[j].y + g.y * inv_ell2);
        if (TAPS && active) {
          const int64_t idx = (gbase + t) * nz + kk;
          a.taps[idx] = ap[j];
          a.taps[a.tri_elems + idx] = K;
          a.taps[2 * a.tri_elems + idx] = zw[j + 2];
        }
        ap[j] = cscale(ap[j], ell2);
        aq[j] = k0 ? zw[j + 2] : cscale(K, -ell2);  // k = 0: the identity solve keeps Zhat
      }
    }
    if (TAPS && active && r == 0 && i0 > 0) {  // m = 0: the gauge row's sources
      const double2 za = Zc[0], zb = Zc[(int64_t)tcl(1) * nz], zc2 = Zc[(int64_t)tcl(2) * nz];
      const double2 g = glz(0, z0, z0, lzv(0, za), lzv(1, zb), lzv(2, zc2));
      const double2 Kq = Kp[0];
      a.taps[gbase * nz + kk] = Cs[0];
      a.taps[a.tri_elems + gbase * nz + kk] = make_double2(Kq.x + g.x * inv_ell2, Kq.y + g.y * inv_ell2);
      a.taps[2 * a.tri_elems + gbase * nz + kk] = za;
    }
    // the q-operator factors load only now, when Zhat is no longer held, and arrive while the psi
    // sweep and its scan run; the factors of round 2 follow the q scan.  Against loading them with
    // the sources (216 registers, the psi and q sweeps side by side): 178 registers and 0.158 ->
    // 0.137 ms at 256^3
#pragma unroll
    for (int j = 0; j < SMAX; ++j) qf[j] = qfl[(int64_t)(s0 + j < qrows ? s0 + j : 0) * ncolp];
    auto cp = [&](int j, double& al, double& be) {
      al = sl1[s0 + j];
      be = sl2[s0 + j];
    };
    auto cq = [&](int j, double& al, double& be) {
      al = qf[j].x;
      be = qf[j].y;
    };
    const RunMap mp = sweep_run<SMAX, true>(yp, ap, len, cp);
    double2 p1, p2, q1, q2;
    enter_state<true>(mp, r, p1, p2);
    add_entering<SMAX, true>(yp, len, p1, p2, cp);
    const RunMap mq = sweep_run<SMAX, true>(yq, aq, len, cq);
    enter_state<true>(mq, r, q1, q2);
    // the factors of round 2 alone
#pragma unroll
    for (int j = 0; j < SMAX; ++j) qr[j] = qfr[(int64_t)(s0 + j < qrows ? s0 + j : 0) * ncolp];
#pragma unroll
    for (int j = 0; j < 2; ++j) qx[j] = qfl[(int64_t)(s0 + SMAX + j < qrows ? s0 + SMAX + j : 0) * ncolp];
    add_entering<SMAX, true>(yq, len, q1, q2, cq);
  }

  // ---- round 2 (descending): back substitutions of psi and q; psi is final
  double gpr = 0.0, gpi = 0.0;
  {
    // couplings to t + 1 and t + 2, from the factors loaded in round 1 (ascending j reads
    // entries j + 1 and j + 2 before they are replaced)
#pragma unroll
    for (int j = 0; j < SMAX; ++j) {
      const double2 f1 = j + 1 < SMAX ? qf[j + 1] : qx[j + 1 - SMAX];
      const double2 f2 = j + 2 < SMAX ? qf[j + 2] : qx[j + 2 - SMAX];
      qf[j] = make_double2(f1.x, f2.y);
    }
#pragma unroll
    for (int j = 0; j < SMAX; ++j) {
      if (j < len) {
        yp[j] = cscale(yp[j], srd[s0 + j]);
        yq[j] = cscale(yq[j], qr[j]);
      }
    }
    auto cp = [&](int j, double& al, double& be) {
      al = sl1[s0 + j + 1];
      be = sl2[s0 + j + 2];
    };
    auto cq = [&](int j, double& al, double& be) {
      al = qf[j].x;
      be = qf[j].y;
    };
    double2 (&bp)[SMAX] = yp;  // in place, as in round 1
    double2 (&bq)[SMAX] = yq;
    double2 p1, p2, q1, q2;
    const RunMap mp = sweep_run<SMAX, false>(bp, yp, len, cp);
    enter_state<false>(mp, r, p1, p2);
    add_entering<SMAX, false>(bp, len, p1, p2, cp);
    const RunMap mq = sweep_run<SMAX, false>(bq, yq, len, cq);
    enter_state<false>(mq, r, q1, q2);
    add_entering<SMAX, false>(bq, len, q1, q2, cq);
#pragma unroll
    for (int j = 0; j < SMAX; ++j) {
      if (j < len) {
        const int t = s0 + j;
        const double2 v = cscale(bp[j], srL[t]);
        if (active) st2(ps + (int64_t)t * nz, v);
        gpr += sgw[t] * v.x;
        gpi += sgw[t] * v.y;
        yq[j] = cscale(cscale(bq[j], k0 ? -1.0 : srL[t]), -ell2);  // the chi source -ell^2 q
      }
    }
  }

  // ---- round 3 (descending): U w = -ell^2 q
  {
    auto cw = [&](int j, double& al, double& be) {
      al = su1[s0 + j];
      be = su2[s0 + j];
    };
    double2 w1, w2;
    enter_state<false>(sweep_run<SMAX, false>(yp, yq, len, cw), r, w1, w2);
    add_entering<SMAX, false>(yp, len, w1, w2, cw);
#pragma unroll
    for (int j = 0; j < SMAX; ++j)
      if (j < len) yp[j] = cscale(yp[j], sru[s0 + j]);
  }

  // ---- round 4 (ascending): D U^T y = w; chi is final
  double gcr = 0.0, gci = 0.0;
  {
    auto cu = [&](int j, double& al, double& be) {
      al = su1[s0 + j - 1];
      be = su2[s0 + j - 2];
    };
    double2 c1, c2;
    enter_state<true>(sweep_run<SMAX, true>(yq, yp, len, cu), r, c1, c2);
    add_entering<SMAX, true>(yq, len, c1, c2, cu);
#pragma unroll
    for (int j = 0; j < SMAX; ++j) {
      if (j < len) {
        const int t = s0 + j;
        const double2 v = cscale(yq[j], srL[t]);
        if (active) st2(chv + (int64_t)t * nz, v);
        gcr += sgw[t] * v.x;
        gci += sgw[t] * v.y;
      }
    }
  }

  // ---- m = 0: the gauge row n = 0 from the sums over the column
  if (m == 0) {
    // sums over the column's runs (a butterfly over its half wave, the same order on every lane)
#pragma unroll
    for (int d = PS_SEG / 2; d >= 1; d /= 2) {
      gpr += __shfl_xor(gpr, d, PS_SEG);
      gpi += __shfl_xor(gpi, d, PS_SEG);
      gcr += __shfl_xor(gcr, d, PS_SEG);
      gci += __shfl_xor(gci, d, PS_SEG);
    }
    if (r == 0 && active) {
      st2(ps, make_double2(-gpr / sgw[0], -gpi / sgw[0]));
      st2(chv, make_double2(-gcr / sgw[0], -gci / sgw[0]));
    }
  }
}

// ---------------------------------------------------------------- axial modal energy
// With the velocity harmonics f_m(i, kk) in the mixed layout [m][i][kk], a real field is
// Re f_0 + 2 Re sum_{m>=1} f_m exp(i m phi) (the azimuthal Nyquist order is not synthesised), so
// its axial coefficient at slot kk is f_0,kk + sum_{m>=1} (f_m,kk e^{i m phi} + conj(f_m,-kk) e^{-i m phi})
// and, by Parseval in phi,
//   energy[kk] = (L_z/2) 2 pi sum_i W_i (|f_0,kk|^2 + sum_{m>=1} (|f_m,kk|^2 + |f_m,-kk|^2)),
// summed over u_r, u_phi, u_z, with W_i = w_i ell^2/(1-x_i)^2.  Stage 1: block b sums the rows
// [b EN_ROWS, (b+1) EN_ROWS) of every axial slot into part[b][kk] (lanes over kk, coalesced);
// stage 2 adds the parts in block order.
constexpr int EN_ROWS = 64;

__global__ __launch_bounds__(256) void energy_part_kernel(const double2* __restrict__ ur,
                                                          const double2* __restrict__ up,
                                                          const double2* __restrict__ uz,
                                                          const double* __restrict__ area, int nr, int nz,
                                                          int nphi, int64_t rows, double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.x * EN_ROWS;
  const int64_t r1 = r0 + EN_ROWS < rows ? r0 + EN_ROWS : rows;
  for (int kk = threadIdx.x; kk < nz; kk += blockDim.x) {
    const int kn = kk == 0 ? 0 : nz - kk;  // slot of -k
    double acc = 0.0;
    for (int64_t row = r0; row < r1; ++row) {
      const int m = (int)(row / nr), i = (int)(row - (int64_t)m * nr);
      if (2 * m == nphi) continue;  // the Nyquist order carries no physical field
      const int64_t o = row * nz;
      const double2 a = ur[o + kk], b = up[o + kk], d = uz[o + kk];
      double e = a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y + d.x * d.x + d.y * d.y;
      if (m > 0) {
        const double2 a2 = ur[o + kn], b2 = up[o + kn], d2 = uz[o + kn];
        e += a2.x * a2.x + a2.y * a2.y + b2.x * b2.x + b2.y * b2.y + d2.x * d2.x + d2.y * d2.y;
      }
      acc += area[i] * e;
    }
    part[(int64_t)blockIdx.x * nz + kk] = acc;
  }
}

__global__ __launch_bounds__(256) void energy_sum_kernel(const double* __restrict__ part, int nparts, int nz,
                                                         double scale, double* __restrict__ energy) {
  const int kk = blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= nz) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += part[(int64_t)b * nz + kk];
  energy[kk] = scale * acc;
}

// ---------------------------------------------------------------- pointwise evaluation of one harmonic
// f(r_j) = sum_{n=m}^{N_r^c-1} s[n][kk] Pbar_n^m(x(r_j)) (Eq. expansion for one (m, k) column), with
// x = (r^2 - ell^2) / (r^2 + ell^2) and sqrt(1 - x^2) = 2 ell r / (r^2 + ell^2) (Eq. map), Pbar by
// the normalised recurrence of the plan tables in FP64: one thread per radius, coefficients read
// in order by every thread.
__global__ __launch_bounds__(256) void eval_harmonic_kernel(const double2* __restrict__ col, int64_t stride, int m,
                                                            int nrc, double ell, const double* __restrict__ r,
                                                            int64_t npts, double2* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= npts) return;
  const double rr = r[j], d = rr * rr + ell * ell;
  const double x = (rr * rr - ell * ell) / d, sn = 2.0 * ell * rr / d;
  double p0 = sqrt(0.5);
  for (int i = 1; i <= m; ++i) p0 *= sqrt((double)(2 * i + 1) / (double)(2 * i)) * sn;
  double2 acc = make_double2(0.0, 0.0);
  if (m < nrc) {
    double2 c = col[0];
    acc = make_double2(c.x * p0, c.y * p0);
  }
  double p1 = sqrt((double)(2 * m + 3)) * x * p0;
  if (m + 1 < nrc) {
    double2 c = col[stride];
    acc.x += c.x * p1;
    acc.y += c.y * p1;
  }
  for (int n = m + 2; n < nrc; ++n) {
    const double a = sqrt((double)(4 * n * n - 1) / (double)(n * n - m * m));
    const double b = sqrt((double)((2 * n + 1) * (n - 1 - m) * (n - 1 + m)) / (double)((2 * n - 3) * (n * n - m * m)));
    const double p2 = a * x * p1 - b * p0;
    const double2 c = col[(int64_t)(n - m) * stride];
    acc.x += c.x * p2;
    acc.y += c.y * p2;
    p0 = p1;
    p1 = p2;
  }
  out[j] = acc;
}

// ---------------------------------------------------------------- logarithmic proxy (Eq. logproxy)
// Potentials psi~ + c_psi Lambda, chi~ + c_chi Lambda with Lambda = ln(r^2 + ell^2): at node i, with
// q = (1 - x)^2 / ell^2 = grad_h^2 Lambda and r (1 - x) / ell^2 = 2 r / (r^2 + ell^2), the proxy parts
// add u_phi = -c_psi r sqrt(q) / ell, u_z = -c_chi q, w_phi = -2 c_chi r q^{3/2} / ell, w_z = -c_psi q
// to the m = 0, k = 0 harmonics (mixed layout, before the inverse z transforms).
__global__ void proxy_fields_kernel(double2* __restrict__ up, double2* __restrict__ uz, double2* __restrict__ wp,
                                    double2* __restrict__ wz, const double* __restrict__ node, int nr, int nz,
                                    double cpsi, double cchi, double ell) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const double r = 1.0 / node[i], q = node[nr + i], sq = sqrt(q);
  const int64_t o = (int64_t)i * nz;  // order 0, node i, axial slot 0
  up[o].x += -cpsi * r * sq / ell;
  uz[o].x += -cchi * q;
  wp[o].x += -2.0 * cchi * r * q * sq / ell;
  wz[o].x += -cpsi * q;
}

// The regular parts evolve with the constant forcing c L Lambda on the m = 0, k = 0 column.
__global__ void proxy_force_kernel(double2* __restrict__ psi_n, double2* __restrict__ chi_n,
                                   const double* __restrict__ f, int nrc, int nz, double cpsi, double cchi) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nrc) return;
  psi_n[(int64_t)n * nz].x += cpsi * f[n];
  chi_n[(int64_t)n * nz].x += cchi * f[n];
}

// Zero every entry of the packed arrays whose (m, k) column is not active.
template <typename O2>
__global__ void zero_inactive_kernel(O2* __restrict__ x0, O2* __restrict__ x1, double2* __restrict__ x2,
                                     double2* __restrict__ x3, double2* __restrict__ x4,
                                     const int32_t* __restrict__ row_m, int64_t rows, int nz, int nzc, int mmax,
                                     int kmax) {
  const int64_t total = rows * nz;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / nz;
    const int kk = (int)(e - row * nz);
    const int k = kval(kk, nz);
    const bool active = row_m[row] < mmax && (k < 0 ? -k : k) <= kmax && kkept(kk, nz, nzc);
    if (active) continue;
    const double2 z = make_double2(0.0, 0.0);
    st2(x0 + e, z);
    st2(x1 + e, z);
    if (x2) { x2[e] = z; x3[e] = z; x4[e] = z; }
  }
}

__global__ void mask_tri_kernel(double2* spec, const int32_t* __restrict__ row_m, int64_t rows, int nz, int mask_m,
                                int mask_k) {
  const int64_t total = rows * nz;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / nz;
    const int kk = (int)(e - row * nz);
    const int k = kval(kk, nz);
    if (row_m[row] > mask_m || (k < 0 ? -k : k) > mask_k) spec[e] = make_double2(0.0, 0.0);
  }
}

FftRadices make_radices(int n, const int* rad, int nrad) {
  FftRadices f{};
  f.n = n;
  f.nrad = nrad;
  for (int i = 0; i < nrad; ++i) f.rad[i] = rad[i];
  return f;
}

PhiGeom phi_geom(const mlg_plan_s* p, bool masked) {
  PhiGeom g{};
  g.nr = p->nr;
  g.nz = p->nz;
  g.nphi = p->nphi;
  g.M = p->M;
  g.mkeep = masked ? p->dealias_m : (1 << 30);
  g.nlines = (int64_t)p->nr * p->nz;
  return g;
}

int phi_lines_per_block(int n) {
  int lb = 2048 / n;  // two buffers of lb/2 complex lines each: 16 * lb * n bytes <= 32 KB
  if (lb < 2) lb = 2;
  if (lb > 16) lb = 16;
  return lb & ~1;
}

mlg_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MLG_OK;
}

}  // namespace

mlg_status launch_gemm(const mlg_plan_s* p, const GemmProds& prods, const GemmDesc* d_desc, int max_rows, int ncol,
                       hipStream_t stream) {
  if (max_rows <= 0 || prods.nprod <= 0) return MLG_OK;
  dim3 grid((ncol + GT_N - 1) / GT_N, (max_rows + GT_M - 1) / GT_M, p->M * prods.nprod);
  p->timing.begin("radial_gemm", stream);
  radial_gemm_f64<<<grid, 256, 0, stream>>>(prods, d_desc, p->M, ncol);
  p->timing.end(stream);
  return check_launch("radial_gemm_f64");
}

mlg_status launch_phi_forward(const mlg_plan_s* p, const double* phys, double* mixed, hipStream_t s) {
  if (p->nphi == 256 && p->use_fast_fft) return launch_phi256_forward(p, phys, mixed, s);
  if (p->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "reduced-precision plans need N_phi = 256");
  PhiGeom g = phi_geom(p, false);
  const int lb = phi_lines_per_block(p->nphi);
  const int npair = lb / 2;
  const size_t shm = (size_t)2 * npair * p->nphi * sizeof(double2);
  dim3 grid((unsigned)((g.nlines + lb - 1) / lb));
  p->timing.begin("phi_fft", s);
  phi_forward_kernel<<<grid, 256, shm, s>>>(g, make_radices(p->nphi, p->phi_rad, p->phi_nrad),
                                            reinterpret_cast<const double2*>(p->d_tw_phi), phys,
                                            reinterpret_cast<double2*>(mixed), lb);
  p->timing.end(s);
  return check_launch("phi_forward_kernel");
}

mlg_status launch_phi_backward(const mlg_plan_s* p, const double* mixed, double* phys, hipStream_t s) {
  if (p->nphi == 256 && p->use_fast_fft) return launch_phi256_backward(p, mixed, phys, s);
  if (p->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "reduced-precision plans need N_phi = 256");
  PhiGeom g = phi_geom(p, false);
  const int lb = phi_lines_per_block(p->nphi);
  const size_t shm = (size_t)2 * (lb / 2) * p->nphi * sizeof(double2);
  dim3 grid((unsigned)((g.nlines + lb - 1) / lb));
  p->timing.begin("phi_fft", s);
  phi_backward_kernel<<<grid, 256, shm, s>>>(g, make_radices(p->nphi, p->phi_rad, p->phi_nrad),
                                             reinterpret_cast<const double2*>(p->d_tw_phi),
                                             reinterpret_cast<const double2*>(mixed), phys, lb);
  p->timing.end(s);
  return check_launch("phi_backward_kernel");
}

mlg_status launch_phi_scalar_rhs(const mlg_plan_s* p, int kind, double gamma, double* mixed, hipStream_t s) {
  if (p->nphi == 256 && p->use_fast_fft) return launch_phi256_scalar(p, kind, gamma, mixed, s);
  if (p->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "reduced-precision plans need N_phi = 256");
  PhiGeom g = phi_geom(p, p->g.dealias != 0);
  const int lb = phi_lines_per_block(p->nphi);
  const size_t shm = (size_t)2 * (lb / 2) * p->nphi * sizeof(double2);
  dim3 grid((unsigned)((g.nlines + lb - 1) / lb));
  FftRadices fr = make_radices(p->nphi, p->phi_rad, p->phi_nrad);
  const double2* tw = reinterpret_cast<const double2*>(p->d_tw_phi);
  p->timing.begin("phi_fft", s);
  if (kind == MLG_RHS_U2)
    phi_scalar_kernel<MLG_RHS_U2><<<grid, 256, shm, s>>>(g, fr, tw, reinterpret_cast<double2*>(mixed), gamma, lb);
  else
    phi_scalar_kernel<MLG_RHS_KPP><<<grid, 256, shm, s>>>(g, fr, tw, reinterpret_cast<double2*>(mixed), gamma, lb);
  p->timing.end(s);
  return check_launch("phi_scalar_kernel");
}

mlg_status launch_phi_vec_rhs(const mlg_plan_s* p, const double* U, double* const* f6, double* taps, hipStream_t s) {
  // the 256-point kernel forms per-lane byte offsets of up to 31 lines of orders in 32 bits
  if (p->nphi == 256 && p->use_fast_fft && (int64_t)p->nr * p->nz <= (int64_t(1) << 23))
    return launch_phi256_vec(p, U, f6, taps, s);
  if (p->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "reduced-precision plans need N_phi = 256");
  PhiGeom g = phi_geom(p, p->g.dealias != 0);
  int lb = 1024 / p->nphi;  // 4 buffers of n complex per line: 64 * lb * n bytes <= 64 KB
  if (lb < 1) lb = 1;
  if (lb > 8) lb = 8;
  const size_t shm = (size_t)4 * lb * p->nphi * sizeof(double2);
  dim3 grid((unsigned)((g.nlines + lb - 1) / lb));
  Six six;
  for (int i = 0; i < 6; ++i) six.f[i] = reinterpret_cast<double2*>(f6[i]);
  p->timing.begin("phi_fft", s);
  phi_vec_kernel<<<grid, 256, shm, s>>>(g, make_radices(p->nphi, p->phi_rad, p->phi_nrad),
                                        reinterpret_cast<const double2*>(p->d_tw_phi), six, p->d_node, U[0], U[1], U[2],
                                        taps, lb);
  p->timing.end(s);
  return check_launch("phi_vec_kernel");
}

mlg_status launch_zfft_fields(const mlg_plan_s* p, const double* const* in, double* const* out, int nf, int64_t rows,
                              int dir, const int32_t* row_m, int mask_m, int mask_k, hipStream_t s, bool fp64_only,
                              bool kept_only) {
  if (rows <= 0 || nf <= 0) return MLG_OK;
  if (p->nz == 256 && p->prec == MLG_SPLIT_BF16 && !fp64_only)
    return launch_split_zdft(p, in, out, nf, rows, dir, row_m, mask_m, mask_k, s);
  if (p->nz == 256 && p->use_fast_fft)
    return launch_zfft256(p, in, out, nf, rows, dir, row_m, mask_m, mask_k, s, kept_only);
  if (p->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "reduced-precision plans need N_z = 256");
  for (int i = 0; i < nf; ++i)
    if (mlg_status st = launch_zfft(p, in[i], out[i], rows, dir, row_m, mask_m, mask_k, s)) return st;
  return MLG_OK;
}

mlg_status launch_zfft(const mlg_plan_s* p, const double* in, double* out, int64_t rows, int dir, const int32_t* row_m,
                       int mask_m, int mask_k, hipStream_t s) {
  if (rows <= 0) return MLG_OK;
  if (p->nz == 256 && p->prec == MLG_SPLIT_BF16) return launch_split_zdft(p, &in, &out, 1, rows, dir, row_m, mask_m, mask_k, s);
  if (p->nz == 256 && p->use_fast_fft) return launch_zfft256(p, &in, &out, 1, rows, dir, row_m, mask_m, mask_k, s);
  if (p->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "reduced-precision plans need N_z = 256");
  ZGeom g{};
  g.nz = p->nz;
  g.nzc = p->nzc;
  g.mask_m = mask_m;
  g.mask_k = mask_k;
  g.rows = rows;
  int lb = 1024 / p->nz;  // two buffers: 32 * lb * n bytes <= 32 KB
  if (lb < 1) lb = 1;
  if (lb > 64) lb = 64;
  const size_t shm = (size_t)2 * lb * p->nz * sizeof(double2);
  dim3 grid((unsigned)((rows + lb - 1) / lb));
  p->timing.begin("z_fft", s);
  zfft_kernel<<<grid, 256, shm, s>>>(g, make_radices(p->nz, p->z_rad, p->z_nrad),
                                     reinterpret_cast<const double2*>(p->d_tw_z), reinterpret_cast<const double2*>(in),
                                     reinterpret_cast<double2*>(out), dir, row_m, lb);
  p->timing.end(s);
  return check_launch("zfft_kernel");
}

void active_columns(const mlg_plan_s* p, int* mmax_out, int* kmax_out) {
  // chop-kept k (never the Nyquist slot) and, when dealiasing, the two-thirds mask
  int kmax = p->nzc - 1;
  if (p->nz % 2 == 0 && p->nz > 1) kmax = std::min(kmax, p->nz / 2 - 1);
  int mmax = std::min(p->M, p->nrc);
  if (2 * (p->M - 1) >= p->nphi) mmax = std::min(mmax, p->nphi / 2);  // no Nyquist order
  if (p->g.dealias) {
    kmax = std::min(kmax, p->dealias_k);
    mmax = std::min(mmax, p->dealias_m + 1);
  }
  *mmax_out = mmax;
  *kmax_out = kmax;
}

mlg_status launch_projection(const mlg_plan_s* p, const double* const* src3, double* psi_n, double* chi_n,
                             double* taps_src, hipStream_t s) {
  ProjArgs a{};
  a.Cs = reinterpret_cast<const double2*>(src3[0]);
  a.Kp = reinterpret_cast<const double2*>(src3[1]);
  a.Pc = reinterpret_cast<const double2*>(src3[2]);
  a.psi = psi_n;
  a.chi = chi_n;
  const bool red = p->prec != MLG_FP64;  // outputs in the plan's data type
  a.taps = reinterpret_cast<double2*>(taps_src);
  a.gram = p->d_gram;
  a.off = p->d_goff;  // the Gram offsets coincide with the triangular row offsets
  a.qfl = p->d_qfl;
  a.qfr = p->d_qfr;
  a.row_m = p->d_row_m;
  a.rows = p->tau;
  a.ngram = p->ngram;
  a.tri_elems = (int64_t)p->tri_elems;
  a.nz = p->nz;
  a.nrc = p->nrc;
  int mmax, kmax;
  active_columns(p, &mmax, &kmax);
  a.kmax = kmax;
  a.cb = col_blocks(kmax, p->nz);
  const int nkact = p->nz == 1 ? 1 : 2 * kmax + 1;
  a.mmax = mmax;
  a.ell2 = p->g.ell * p->g.ell;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  // runs of at most SMAX degrees: ceil((nrc - 1) / PS_SEG) for the longest column (m = 0)
  if (p->nrc - 1 > 16 * PS_SEG) return fail(MLG_E_UNSUPPORTED, "projection solves: nrc above 513");
  const int64_t total = p->tau * p->nz;
  const bool solve = mmax > 0 && nkact > 0;
  if (total > 0 && !solve) {  // otherwise the solve blocks clear the inactive entries
    int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
    double2* t0 = a.taps;
    p->timing.begin("projection", s);
    if (red)
      zero_inactive_kernel<float2><<<blocks, 256, 0, s>>>(
          reinterpret_cast<float2*>(psi_n), reinterpret_cast<float2*>(chi_n), t0, t0 ? t0 + p->tri_elems : nullptr,
          t0 ? t0 + 2 * p->tri_elems : nullptr, p->d_row_m, p->tau, p->nz, p->nzc, mmax, kmax);
    else
      zero_inactive_kernel<double2><<<blocks, 256, 0, s>>>(
          reinterpret_cast<double2*>(psi_n), reinterpret_cast<double2*>(chi_n), t0, t0 ? t0 + p->tri_elems : nullptr,
          t0 ? t0 + 2 * p->tri_elems : nullptr, p->d_row_m, p->tau, p->nz, p->nzc, mmax, kmax);
    p->timing.end(s);
    if (mlg_status st = check_launch("zero_inactive_kernel")) return st;
  }
  if (solve) {
    dim3 grid((unsigned)a.cb.nblk, (unsigned)mmax);
    const size_t shm = proj_tables_len(p->nrc) * sizeof(double);
    const bool wide = p->nrc - 1 > 8 * PS_SEG;
    p->timing.begin("projection", s);
    if (red) {
      if (a.taps) {
        if (wide) projection_kernel<true, 16, float2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
        else projection_kernel<true, 8, float2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
      } else {
        if (wide) projection_kernel<false, 16, float2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
        else projection_kernel<false, 8, float2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
      }
    } else if (a.taps) {
      if (wide) projection_kernel<true, 16, double2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
      else projection_kernel<true, 8, double2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
    } else {
      if (wide) projection_kernel<false, 16, double2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
      else projection_kernel<false, 8, double2><<<grid, PS_SEG * PS_COL, shm, s>>>(a);
    }
    p->timing.end(s);
  }
  return check_launch("projection_kernel");
}

mlg_status launch_energy(const mlg_plan_s* p, double* const* u3, double* energy, double* scratch, hipStream_t s) {
  const int64_t rows = (int64_t)p->M * p->nr;
  const int nparts = (int)((rows + EN_ROWS - 1) / EN_ROWS);
  if (rows <= 0) return fail(MLG_E_ARG, "energy: empty plan");
  // the scratch (a triangular workspace array, 2 tri_elems doubles) holds nparts * nz partial sums
  if ((int64_t)nparts * p->nz > 2 * (int64_t)p->tri_elems) return fail(MLG_E_UNSUPPORTED, "energy: scratch too small");
  const double scale = 0.5 * p->g.lz * 2.0 * M_PI;
  energy_part_kernel<<<nparts, 256, 0, s>>>(reinterpret_cast<const double2*>(u3[0]),
                                            reinterpret_cast<const double2*>(u3[1]),
                                            reinterpret_cast<const double2*>(u3[2]), p->d_node + 3 * p->nr, p->nr,
                                            p->nz, p->nphi, rows, scratch);
  if (mlg_status st = check_launch("energy_part_kernel")) return st;
  energy_sum_kernel<<<(p->nz + 255) / 256, 256, 0, s>>>(scratch, nparts, p->nz, scale, energy);
  return check_launch("energy_sum_kernel");
}

mlg_status launch_mask_tri(const mlg_plan_s* p, double* spec, hipStream_t s) {
  const int64_t total = (int64_t)p->tau * p->nz;
  if (total == 0) return MLG_OK;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
  p->timing.begin("mask", s);
  mask_tri_kernel<<<blocks, 256, 0, s>>>(reinterpret_cast<double2*>(spec), p->d_row_m, p->tau, p->nz, p->dealias_m,
                                         p->dealias_k);
  p->timing.end(s);
  return check_launch("mask_tri_kernel");
}

mlg_status launch_eval_harmonic(const mlg_plan_s* p, const double* spec, int m, int kk, const double* r, int64_t npts,
                                double* out, hipStream_t s) {
  if (npts <= 0) return MLG_OK;
  // the packed row offset of order m comes from the plan's host copy of the offsets
  const double2* col = reinterpret_cast<const double2*>(spec) + p->off[m] * p->nz + kk;
  eval_harmonic_kernel<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(col, p->nz, m, p->nrc, p->g.ell, r, npts,
                                                                     reinterpret_cast<double2*>(out));
  return check_launch("eval_harmonic_kernel");
}

mlg_status launch_proxy_fields(const mlg_plan_s* p, double* const* f6, hipStream_t s) {
  if (p->log_cpsi == 0.0 && p->log_cchi == 0.0) return MLG_OK;
  proxy_fields_kernel<<<(p->nr + 255) / 256, 256, 0, s>>>(
      reinterpret_cast<double2*>(f6[1]), reinterpret_cast<double2*>(f6[2]), reinterpret_cast<double2*>(f6[4]),
      reinterpret_cast<double2*>(f6[5]), p->d_node, p->nr, p->nz, p->log_cpsi, p->log_cchi, p->g.ell);
  return check_launch("proxy_fields_kernel");
}

mlg_status launch_proxy_force(const mlg_plan_s* p, double* psi_n, double* chi_n, hipStream_t s) {
  if ((p->log_cpsi == 0.0 && p->log_cchi == 0.0) || !p->d_logf) return MLG_OK;
  proxy_force_kernel<<<(p->nrc + 255) / 256, 256, 0, s>>>(reinterpret_cast<double2*>(psi_n),
                                                           reinterpret_cast<double2*>(chi_n), p->d_logf, p->nrc,
                                                           p->nz, p->log_cpsi, p->log_cchi);
  return check_launch("proxy_force_kernel");
}
}  // namespace mlg

