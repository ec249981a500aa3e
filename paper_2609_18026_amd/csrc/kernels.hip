// HIP kernels for gfx950 (CDNA4): radial transforms on FP64 MFMA, LDS Stockham FFTs in phi
// and z, the fused pseudospectral phi stages, the toroidal-poloidal epilogue and the
// projection solves.  All launches are validated on the host against the plan's sizes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "mlg_internal.h"

namespace mlg {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ double2 cmul_mi(double2 a, bool inv) {
  return inv ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

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
  if (row0 >= d.rows || col0 >= ncol || d.K <= 0) return;
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

  double ra[4], rb[4];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kk = e >> 6, cc = e & 63;
      const int k = k0 + kk;
      const int row = row0 + cc;
      ra[t] = (k < d.K && row < d.rows) ? A[(int64_t)k * d.lda + row] : 0.0;
      const int col = col0 + cc;
      double v = (k < d.K && col < ncol) ? B[(int64_t)k * ncol + col] : 0.0;
      if (lscale) {
        const double n = (double)(k + d.m);
        v *= n * (n + 1.0);
      }
      rb[t] = v;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 256 * t;
      const int kk = e >> 6, cc = e & 63;
      As[buf][kk][cc] = ra[t];
      Bs[buf][kk][cc] = rb[t];
    }
  };

  const int nk = (d.K + GT_K - 1) / GT_K;
  load_tiles(0);
  store_tiles(0);
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
    if (kt + 1 < nk) {
      store_tiles(buf ^ 1);
    }
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
    if (row < g.rows) {
      v = in[row * n + kk];
      if (dir > 0 && !kkept(kk, n, g.nzc)) v = make_double2(0.0, 0.0);
    }
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
    if (dir < 0) {
      bool keep = kkept(kk, n, g.nzc);
      if (row_m != nullptr) {
        const int k = kval(kk, n);
        keep = keep && row_m[row] <= g.mask_m && (k < 0 ? -k : k) <= g.mask_k;
      }
      if (!keep) v = make_double2(0.0, 0.0);
    }
    out[row * n + kk] = v;
  }
}

// ---------------------------------------------------------------- toroidal-poloidal epilogue
// In place over the seven radial products A1 = Pbar psi, A2 = T psi, A3 = Pbar(L psi), B1 = Pbar chi,
// B2 = T chi, B3 = Pbar(L chi), B4 = T(L chi) (mixed layout, k spectral), writing the harmonics
//   u_r = (i m A1 + i kap B2)/r, u_phi = (-A2 - m kap B1)/r, u_z = q B3,
//   w_r = (i kap A2 + i m q B3 + i m kap^2 B1)/r, w_phi = (-m kap A1 - q (B4 - 2(1+x) B3) - kap^2 B2)/r,
//   w_z = q A3   into buffers 0..5.
struct Seven {
  double2* f[7];
};

__global__ __launch_bounds__(256) void vec_epilogue_kernel(Seven s, const double* __restrict__ node, int nr, int nz,
                                                           int M, double kap0) {
  const int64_t total = (int64_t)M * nr * nz;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int kk = (int)(e % nz);
    const int64_t mi = e / nz;
    const int i = (int)(mi % nr);
    const int m = (int)(mi / nr);
    const double kap = kap0 * kval(kk, nz);
    const double rinv = node[i], q = node[nr + i], opx = node[2 * nr + i];
    const double2 A1 = s.f[0][e], A2 = s.f[1][e], A3 = s.f[2][e];
    const double2 B1 = s.f[3][e], B2 = s.f[4][e], B3 = s.f[5][e], B4 = s.f[6][e];
    const double fm = (double)m;
    // i*m*A1 + i*kap*B2
    double2 ur = make_double2(-(fm * A1.y + kap * B2.y), fm * A1.x + kap * B2.x);
    double2 up = make_double2(-A2.x - fm * kap * B1.x, -A2.y - fm * kap * B1.y);
    double2 uz = cscale(B3, q);
    // i*(kap*A2 + m*q*B3 + m*kap^2*B1)
    double2 t = make_double2(kap * A2.x + fm * q * B3.x + fm * kap * kap * B1.x,
                             kap * A2.y + fm * q * B3.y + fm * kap * kap * B1.y);
    double2 wr = make_double2(-t.y, t.x);
    double2 wp = make_double2(-fm * kap * A1.x - q * (B4.x - 2.0 * opx * B3.x) - kap * kap * B2.x,
                              -fm * kap * A1.y - q * (B4.y - 2.0 * opx * B3.y) - kap * kap * B2.y);
    double2 wz = cscale(A3, q);
    s.f[0][e] = cscale(ur, rinv);
    s.f[1][e] = cscale(up, rinv);
    s.f[2][e] = uz;
    s.f[3][e] = cscale(wr, rinv);
    s.f[4][e] = cscale(wp, rinv);
    s.f[5][e] = wz;
  }
}

// ---------------------------------------------------------------- projection solves
// One thread per (m, k slot) column.  Inputs (triangular, k spectral): Pa = Pbar^T W (N_r/r),
// Qa = Q^T W (N_r/r), Pb = Pbar^T W (N_phi/r), Qb = Q^T W (N_phi/r), Pc = Pbar^T W N_z.
//   C = -Qb - i m Pa,  K = -i kap Qa - m kap Pb - Dbar Pc,  Dbar = -G L / ell^2.
//   psi: G (L psi) = ell^2 C ;  q = -Pc at k = 0, else (G + kap^2 ell^2 L^-1)(L q) = -ell^2 K ;
//   chi: G (L chi) = -ell^2 q.  For m = 0 the unknowns n >= 1 are solved with G restricted to
//   n >= 1 and n = 0 follows from the gauge sum_n sqrt((2n+1)/2) s_n = 0.
struct ProjArgs {
  const double2* Pa;
  const double2* Qa;
  const double2* Pb;
  const double2* Qb;
  const double2* Pc;
  double2* psi;
  double2* chi;
  double* scratch;       // 5 reals per (column, degree)
  double2* taps;         // C, K, Zhat (triangular) or null
  const double* gram;    // g0 g1 g2 d l1 l2, each ngram long
  const int64_t* goff;
  const int64_t* off;    // triangular offsets (device)
  int64_t ngram, tri_elems;
  int M, nz, nrc, nzc, mask_m, mask_k, dealias;
  double ell2, kap0;
};

__global__ __launch_bounds__(64) void projection_kernel(ProjArgs a) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncols = (int64_t)a.M * a.nz;
  if (col >= ncols) return;
  const int m = (int)(col / a.nz);
  const int kk = (int)(col - (int64_t)m * a.nz);
  if (m >= a.nrc) return;
  const int nz = a.nz;
  const int64_t base = a.off[m];  // row of n = m
  auto at = [&](int n) -> int64_t { return (base + (n - m)) * nz + kk; };
  const int k = kval(kk, nz);
  bool keep = kkept(kk, nz, a.nzc);
  if (a.dealias) keep = keep && m <= a.mask_m && (k < 0 ? -k : k) <= a.mask_k;
  const double2 z0 = make_double2(0.0, 0.0);
  if (!keep) {
    for (int n = m; n < a.nrc; ++n) {
      a.psi[at(n)] = z0;
      a.chi[at(n)] = z0;
      if (a.taps) {
        a.taps[at(n)] = z0;
        a.taps[a.tri_elems + at(n)] = z0;
        a.taps[2 * a.tri_elems + at(n)] = z0;
      }
    }
    return;
  }
  const double kap = a.kap0 * k;
  const double fm = (double)m;
  const double* g0 = a.gram;
  const double* g1 = a.gram + a.ngram;
  const double* g2 = a.gram + 2 * a.ngram;
  const double* dd = a.gram + 3 * a.ngram;
  const double* l1 = a.gram + 4 * a.ngram;
  const double* l2 = a.gram + 5 * a.ngram;
  const int64_t gb = a.goff[m] - m;  // index of degree n is gb + n
  const int n0 = m > 0 ? m : 1;
  const int64_t sstride = ncols;     // scratch: [slot][n][col]
  auto sidx = [&](int slot, int n) -> int64_t { return ((int64_t)slot * a.nrc + n) * sstride + col; };
  auto Lf = [](int n) { return (double)n * (n + 1.0); };

  // ---- pass 1 (ascending): sources, forward substitution for psi and for q
  double2 zpsi1 = z0, zpsi2 = z0;  // z_{n-1}, z_{n-2}
  double2 zq1 = z0, zq2 = z0;
  double dq1 = 0, dq2 = 0, lq1p = 0;  // d'_{n-1}, d'_{n-2}, l1'_{n-1}
  const double s = kap * kap * a.ell2;
  // Zhat window for Dbar Pc: (L Z)_j for j = n-2 .. n+2
  auto LZ = [&](int j) -> double2 {
    if (j < m || j >= a.nrc) return z0;
    return cscale(a.Pc[at(j)], Lf(j));
  };
  double2 lz_m2 = LZ(m - 2), lz_m1 = LZ(m - 1), lz_0 = LZ(m), lz_p1 = LZ(m + 1), lz_p2 = LZ(m + 2);
  for (int n = m; n < a.nrc; ++n) {
    const int64_t idx = at(n);
    const double2 pa = a.Pa[idx], qa = a.Qa[idx], pb = a.Pb[idx], qb = a.Qb[idx];
    // (G L Z)_n = g2_{n-2} LZ_{n-2} + g1_{n-1} LZ_{n-1} + g0_n LZ_n + g1_n LZ_{n+1} + g2_n LZ_{n+2}
    double2 glz = cscale(lz_0, g0[gb + n]);
    if (n - 1 >= m) glz = cadd(glz, cscale(lz_m1, g1[gb + n - 1]));
    if (n - 2 >= m) glz = cadd(glz, cscale(lz_m2, g2[gb + n - 2]));
    if (n + 1 < a.nrc) glz = cadd(glz, cscale(lz_p1, g1[gb + n]));
    if (n + 2 < a.nrc) glz = cadd(glz, cscale(lz_p2, g2[gb + n]));
    // C = -Qb - i m Pa
    const double2 C = make_double2(-qb.x + fm * pa.y, -qb.y - fm * pa.x);
    // K = -i kap Qa - m kap Pb + (G L Z)/ell^2
    const double2 K = make_double2(kap * qa.y - fm * kap * pb.x + glz.x / a.ell2,
                                   -kap * qa.x - fm * kap * pb.y + glz.y / a.ell2);
    if (a.taps) {
      a.taps[idx] = C;
      a.taps[a.tri_elems + idx] = K;
      a.taps[2 * a.tri_elems + idx] = a.Pc[idx];
    }
    // slide the L Z window
    lz_m2 = lz_m1; lz_m1 = lz_0; lz_0 = lz_p1; lz_p1 = lz_p2; lz_p2 = LZ(n + 3);
    if (n < n0) continue;  // m = 0, n = 0: gauge row
    // psi forward substitution with the precomputed unit-lower factor
    {
      double2 b = cscale(C, a.ell2);
      if (n - 1 >= n0) b = csub(b, cscale(zpsi1, l1[gb + n]));
      if (n - 2 >= n0) b = csub(b, cscale(zpsi2, l2[gb + n]));
      zpsi2 = zpsi1;
      zpsi1 = b;
      a.psi[idx] = b;
    }
    if (k != 0) {
      // on-the-fly L D L^T of A' = G + s L^-1 (same off-diagonals as G)
      const double diag = g0[gb + n] + s / Lf(n);
      double l2n = 0, l1n = 0;
      if (n - 2 >= n0) l2n = g2[gb + n - 2] / dq2;
      if (n - 1 >= n0) {
        double t = g1[gb + n - 1];
        if (n - 2 >= n0) t -= l2n * dq2 * lq1p;
        l1n = t / dq1;
      }
      double dn = diag;
      if (n - 1 >= n0) dn -= l1n * l1n * dq1;
      if (n - 2 >= n0) dn -= l2n * l2n * dq2;
      double2 b = cscale(K, -a.ell2);
      if (n - 1 >= n0) b = csub(b, cscale(zq1, l1n));
      if (n - 2 >= n0) b = csub(b, cscale(zq2, l2n));
      zq2 = zq1;
      zq1 = b;
      dq2 = dq1;
      dq1 = dn;
      lq1p = l1n;
      a.scratch[sidx(0, n)] = b.x;
      a.scratch[sidx(1, n)] = b.y;
      a.scratch[sidx(2, n)] = l1n;
      a.scratch[sidx(3, n)] = l2n;
      a.scratch[sidx(4, n)] = dn;
    }
  }
  // ---- pass 2 (descending): back substitution for psi and q
  double2 ypsi1 = z0, ypsi2 = z0, yq1 = z0, yq2 = z0;
  double l1q_n1 = 0, l2q_n2 = 0, l2q_n1 = 0;  // l1'_{n+1}, l2'_{n+2}, l2'_{n+1}
  double gauge_psi_re = 0, gauge_psi_im = 0;
  for (int n = a.nrc - 1; n >= n0; --n) {
    const int64_t idx = at(n);
    {
      double2 y = cscale(a.psi[idx], 1.0 / dd[gb + n]);
      if (n + 1 < a.nrc) y = csub(y, cscale(ypsi1, l1[gb + n + 1]));
      if (n + 2 < a.nrc) y = csub(y, cscale(ypsi2, l2[gb + n + 2]));
      ypsi2 = ypsi1;
      ypsi1 = y;
      const double2 v = cscale(y, 1.0 / Lf(n));
      a.psi[idx] = v;
      const double gw = sqrt((2.0 * n + 1.0) * 0.5);
      gauge_psi_re += gw * v.x;
      gauge_psi_im += gw * v.y;
    }
    double2 qn;
    if (k != 0) {
      const double2 zb = make_double2(a.scratch[sidx(0, n)], a.scratch[sidx(1, n)]);
      const double dn = a.scratch[sidx(4, n)];
      double2 y = cscale(zb, 1.0 / dn);
      if (n + 1 < a.nrc) y = csub(y, cscale(yq1, l1q_n1));
      if (n + 2 < a.nrc) y = csub(y, cscale(yq2, l2q_n2));
      yq2 = yq1;
      yq1 = y;
      l2q_n2 = l2q_n1;
      l1q_n1 = a.scratch[sidx(2, n)];
      l2q_n1 = a.scratch[sidx(3, n)];
      qn = cscale(y, 1.0 / Lf(n));
    } else {
      qn = cscale(a.Pc[idx], -1.0);
    }
    a.scratch[sidx(0, n)] = qn.x;
    a.scratch[sidx(1, n)] = qn.y;
  }
  if (m == 0) a.psi[at(0)] = make_double2(-gauge_psi_re / sqrt(0.5), -gauge_psi_im / sqrt(0.5));
  // ---- pass 3 (ascending): chi forward substitution, G (L chi) = -ell^2 q
  double2 zc1 = z0, zc2 = z0;
  for (int n = n0; n < a.nrc; ++n) {
    const double2 qn = make_double2(a.scratch[sidx(0, n)], a.scratch[sidx(1, n)]);
    double2 b = cscale(qn, -a.ell2);
    if (n - 1 >= n0) b = csub(b, cscale(zc1, l1[gb + n]));
    if (n - 2 >= n0) b = csub(b, cscale(zc2, l2[gb + n]));
    zc2 = zc1;
    zc1 = b;
    a.chi[at(n)] = b;
  }
  // ---- pass 4 (descending): chi back substitution
  double2 yc1 = z0, yc2 = z0;
  double gauge_chi_re = 0, gauge_chi_im = 0;
  for (int n = a.nrc - 1; n >= n0; --n) {
    const int64_t idx = at(n);
    double2 y = cscale(a.chi[idx], 1.0 / dd[gb + n]);
    if (n + 1 < a.nrc) y = csub(y, cscale(yc1, l1[gb + n + 1]));
    if (n + 2 < a.nrc) y = csub(y, cscale(yc2, l2[gb + n + 2]));
    yc2 = yc1;
    yc1 = y;
    const double2 v = cscale(y, 1.0 / Lf(n));
    a.chi[idx] = v;
    const double gw = sqrt((2.0 * n + 1.0) * 0.5);
    gauge_chi_re += gw * v.x;
    gauge_chi_im += gw * v.y;
  }
  if (m == 0) a.chi[at(0)] = make_double2(-gauge_chi_re / sqrt(0.5), -gauge_chi_im / sqrt(0.5));
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

mlg_status launch_zfft(const mlg_plan_s* p, const double* in, double* out, int64_t rows, int dir, const int32_t* row_m,
                       int mask_m, int mask_k, hipStream_t s) {
  if (rows <= 0) return MLG_OK;
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

mlg_status launch_vec_epilogue(const mlg_plan_s* p, double* const* prod7, hipStream_t s) {
  Seven sv;
  for (int i = 0; i < 7; ++i) sv.f[i] = reinterpret_cast<double2*>(prod7[i]);
  const int64_t total = (int64_t)p->M * p->nr * p->nz;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
  const double kap0 = 2.0 * M_PI / p->g.lz;
  p->timing.begin("vec_epilogue", s);
  vec_epilogue_kernel<<<blocks, 256, 0, s>>>(sv, p->d_node, p->nr, p->nz, p->M, kap0);
  p->timing.end(s);
  return check_launch("vec_epilogue_kernel");
}

mlg_status launch_projection(const mlg_plan_s* p, const double* const* src5, double* psi_n, double* chi_n,
                             double* scratch, double* taps_src, hipStream_t s) {
  ProjArgs a{};
  a.Pa = reinterpret_cast<const double2*>(src5[0]);
  a.Qa = reinterpret_cast<const double2*>(src5[1]);
  a.Pb = reinterpret_cast<const double2*>(src5[2]);
  a.Qb = reinterpret_cast<const double2*>(src5[3]);
  a.Pc = reinterpret_cast<const double2*>(src5[4]);
  a.psi = reinterpret_cast<double2*>(psi_n);
  a.chi = reinterpret_cast<double2*>(chi_n);
  a.scratch = scratch;
  a.taps = reinterpret_cast<double2*>(taps_src);
  a.gram = p->d_gram;
  a.goff = p->d_goff;
  a.ngram = p->ngram;
  a.tri_elems = (int64_t)p->tri_elems;
  a.M = p->M;
  a.nz = p->nz;
  a.nrc = p->nrc;
  a.nzc = p->nzc;
  a.mask_m = p->dealias_m;
  a.mask_k = p->dealias_k;
  a.dealias = p->g.dealias;
  a.ell2 = p->g.ell * p->g.ell;
  a.kap0 = 2.0 * M_PI / p->g.lz;
  a.off = p->d_goff;  // the Gram offsets coincide with the triangular row offsets
  const int64_t ncols = (int64_t)p->M * p->nz;
  dim3 grid((unsigned)((ncols + 63) / 64));
  p->timing.begin("projection", s);
  projection_kernel<<<grid, 64, 0, s>>>(a);
  p->timing.end(s);
  return check_launch("projection_kernel");
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

}  // namespace mlg
