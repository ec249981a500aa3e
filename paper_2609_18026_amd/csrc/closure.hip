// Learned coarse-grid closure for the toroidal-poloidal nonlinear term.
//
// A small network maps the coefficients of one (m, k) column of a coarse state to a correction
// of that column of the coarse nonlinear term, so that RHS_c + C approaches the truncation of the
// fine-grid term.  Truncation of spectral coefficients between grids is exact: the mapped
// Legendre functions Pbar_n^m (Sec. 3.1, Eq. expansion) do not depend on N_r.
//
// Network (per column, batch rows = columns):
//   x (258 features, padded to 288) -> tanh(W1 x + b1) (256) -> tanh(W2 h1 + b2) (256)
//     -> W3 h2 + b3 (256 outputs)
// Features of column (m, k): Re/Im of psi_n and chi_n for n < 64 at positions
// [0, 64) Re psi, [64, 128) Im psi, [128, 192) Re chi, [192, 256) Im chi (zero where n < m),
// then m / M and k / k_max; each multiplied by a per-feature scale.  Outputs use the same 256
// positions, multiplied by per-output scales, and correct (psi_n, chi_n).
//
// Products run on v_mfma_f32_16x16x32_bf16: operands in bfloat16 (round to nearest even),
// FP32 accumulation.  bfloat16 is stored for the inputs, the weight copies used by the products,
// the activations h1, h2 and the gradients dy, dz2, dz1; tanh values are also kept in FP32 for
// the derivative; biases, master weights and Adam moments are FP32.
//
// MFMA operand layout (16x16x32 bf16): lane l supplies A[l%16][8(l/16) .. +7] and
// B[8(l/16) .. +7][l%16]; FP32 accumulator value v of lane l is C[4(l/16) + v][l%16].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dev_common.h"
#include "mlg_internal.h"

namespace mlg {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int NIN = MLG_CLOSURE_NIN;     // 258 features
constexpr int KIN = 288;                 // padded input width (multiple of 32)
constexpr int HID = MLG_CLOSURE_HIDDEN;  // 256
constexpr int NOUT = MLG_CLOSURE_NOUT;   // 256
constexpr int NCOEF = 64;                // degrees per field in the features
// internal FP32 parameter vector (W1 padded to KIN columns)
constexpr int P_W1 = 0;
constexpr int P_B1 = P_W1 + HID * KIN;
constexpr int P_W2 = P_B1 + HID;
constexpr int P_B2 = P_W2 + HID * HID;
constexpr int P_W3 = P_B2 + HID;
constexpr int P_B3 = P_W3 + NOUT * HID;
constexpr int P_TOTAL = P_B3 + NOUT;
constexpr int EXT_TOTAL = HID * NIN + HID + HID * HID + HID + NOUT * HID + NOUT;
constexpr int NSPLIT_MAX = 16;  // K splits of the weight-gradient products
constexpr int NORM_BLOCKS = 256;

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
__device__ __forceinline__ int kval(int kk, int nz) { return (2 * kk < nz) ? kk : kk - nz; }

enum Epi { EPI_F32 = 0, EPI_TANH = 1, EPI_LOSS = 2, EPI_OUT = 3, EPI_DTANH = 4 };

struct MMArgs {
  const unsigned short* A;
  const unsigned short* B;
  int lda, ldb;
  int M, N, K;        // C is M x N; K and kchunk are multiples of 32; M, N multiples of 8
  int kchunk;         // contraction rows per blockIdx.z
  float* Cf;          // EPI_F32: Cf + z * cf_split + row * ldc + col; EPI_OUT: Cf + row * ldc + col
  int64_t cf_split;
  int ldc;
  unsigned short* Cb;  // bfloat16 output (TANH, LOSS, DTANH)
  float* Hf;           // TANH: FP32 tanh output; DTANH: the forward tanh values (input)
  const float* bias;
  const float* T;      // LOSS: normalised targets
  float* part;         // LOSS: per-block partial sums of squared residuals
  const float* yscale; // OUT: output scales
  int nvalid;          // rows below nvalid are samples
  float gscale;        // LOSS: 2 / (nvalid * N)
};

// Stage a 64 x 32 tile (rows r0.., contraction k0..) into Xs[row][k].  KC: element (r, k) at
// src[r * ld + k]; otherwise at src[k * ld + r].  Rows >= R read as zero.
template <bool KC>
__device__ __forceinline__ void load_tile(const unsigned short* __restrict__ src, int ld, int r0, int R, int k0,
                                          unsigned short (*Xs)[40], int tid) {
  if (KC) {
    const int r = tid >> 2, k8 = (tid & 3) * 8;
    u16x8 v = (u16x8)(0);
    if (r0 + r < R) v = *reinterpret_cast<const u16x8*>(src + (int64_t)(r0 + r) * ld + k0 + k8);
    *reinterpret_cast<u16x8*>(&Xs[r][k8]) = v;
  } else {
    const int k = tid >> 3, r8 = (tid & 7) * 8;
    u16x8 v = (u16x8)(0);
    if (r0 + r8 < R) v = *reinterpret_cast<const u16x8*>(src + (int64_t)(k0 + k) * ld + r0 + r8);
#pragma unroll
    for (int i = 0; i < 8; ++i) Xs[r8 + i][k] = v[i];
  }
}

__device__ __forceinline__ bf16x8 frag(const unsigned short* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(p));
}

// C = op(A) op(B) on 64 x 64 tiles, 4 waves of 32 x 32, with the layer epilogues.
template <bool AK, bool BK, int EPI>
__global__ __launch_bounds__(256) void mm_kernel(MMArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned short As[64][40];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[64][40];
  __shared__ float red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kbeg = blockIdx.z * a.kchunk;
  const int kend = min(a.K, kbeg + a.kchunk);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    load_tile<AK>(a.A, a.lda, m0, a.M, k0, As, tid);
    load_tile<BK>(a.B, a.ldb, n0, a.N, k0, Bs, tid);
    __syncthreads();
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) af[i] = frag(&As[wm + 16 * i + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < 2; ++j) bfr[j] = frag(&Bs[wn + 16 * j + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  float ls = 0.f;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + v;
        const int col = n0 + wn + 16 * j + (lane & 15);
        if (row >= a.M || col >= a.N) continue;
        const float c = acc[i][j][v];
        const int64_t e = (int64_t)row * a.ldc + col;
        if (EPI == EPI_F32) {
          a.Cf[blockIdx.z * a.cf_split + e] = c;
        } else if (EPI == EPI_TANH) {
          const float h = tanhf(c + a.bias[col]);
          a.Hf[e] = h;
          a.Cb[e] = bf16_bits(h);
        } else if (EPI == EPI_LOSS) {
          if (row < a.nvalid) {
            const float d = c + a.bias[col] - a.T[e];
            a.Cb[e] = bf16_bits(a.gscale * d);
            ls += d * d;
          } else {
            a.Cb[e] = 0;
          }
        } else if (EPI == EPI_OUT) {
          if (row < a.nvalid) a.Cf[e] = (c + a.bias[col]) * a.yscale[col];
        } else {  // EPI_DTANH
          const float h = a.Hf[e];
          a.Cb[e] = bf16_bits(c * (1.f - h * h));
        }
      }
  if (EPI == EPI_LOSS) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ls += __shfl_xor(ls, o);
    if (lane == 0) red[wave] = ls;
    __syncthreads();
    if (tid == 0) a.part[blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Bias gradients: partial column sums of dy, dz2, dz1 over the rows of split z.
__global__ __launch_bounds__(256) void colsum_kernel(const unsigned short* dy, const unsigned short* dz2,
                                                     const unsigned short* dz1, int rows, int kchunk, float* part) {
  const int z = blockIdx.x, layer = blockIdx.y, o = threadIdx.x;
  const unsigned short* src = layer == 0 ? dy : (layer == 1 ? dz2 : dz1);
  const int dst = layer == 0 ? P_B3 : (layer == 1 ? P_B2 : P_B1);
  const int r0 = z * kchunk, r1 = min(rows, r0 + kchunk);
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += bf16_f(src[(int64_t)r * HID + o]);
  part[(int64_t)z * P_TOTAL + dst + o] = s;
}

// Gradient = sum of the split partials (fixed order), then Adam with bias correction.
__global__ __launch_bounds__(256) void adam_kernel(const float* part, int nsplit, float* grad, float* p, float* mom,
                                                   float* vel, unsigned short* wb, float lr, float b1, float b2,
                                                   float bc1, float bc2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P_TOTAL) return;
  float g = 0.f;
  for (int z = 0; z < nsplit; ++z) g += part[(int64_t)z * P_TOTAL + i];
  grad[i] = g;
  const float m = b1 * mom[i] + (1.f - b1) * g;
  const float v = b2 * vel[i] + (1.f - b2) * g * g;
  mom[i] = m;
  vel[i] = v;
  const float np = p[i] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
  p[i] = np;
  wb[i] = bf16_bits(np);
}

__global__ __launch_bounds__(256) void loss_kernel(const float* part, int n, float inv_count, float* loss) {
  __shared__ float s[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = s[0] * inv_count;
}

// Training / evaluation inputs from raw rows: X = bf16(x * xs) padded to KIN, T = y / ys.
// idx (optional) selects rows of the data; an index outside [0, count) marks flags[0] and
// yields a zero row.
__global__ __launch_bounds__(256) void prep_kernel(const float* data_x, const float* data_y, const int32_t* idx,
                                                   int64_t count, int nb, int rows, const float* xs,
                                                   const float* ys, unsigned short* X, float* T, int* flags) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nx = (int64_t)rows * KIN;
  if (e < nx) {
    const int r = (int)(e / KIN), j = (int)(e - (int64_t)r * KIN);
    float v = 0.f;
    if (r < nb && j < NIN) {
      int64_t s = idx ? (int64_t)idx[r] : (int64_t)r;
      if (s < 0 || s >= count) {
        if (j == 0) flags[0] = 1;
      } else {
        v = data_x[s * NIN + j] * xs[j];
      }
    }
    X[e] = bf16_bits(v);
  }
  if (data_y && e < (int64_t)rows * NOUT) {
    const int r = (int)(e / NOUT), o = (int)(e - (int64_t)r * NOUT);
    float v = 0.f;
    if (r < nb) {
      const int64_t s = idx ? (int64_t)idx[r] : (int64_t)r;
      if (s >= 0 && s < count) v = data_y[s * NOUT + o] / ys[o];
    }
    T[e] = v;
  }
}

struct ColMap {
  const int32_t* slot;     // active slot of column index jk
  const int32_t* row_m;    // azimuthal order of every triangular row
  const int64_t* off;      // triangular row offsets (M + 1)
  int M, nrc, nz, nk, kmax;
};

__device__ __forceinline__ float feature(const ColMap& c, const double2* psi, const double2* chi, int col, int j) {
  const int m = col / c.nk, jk = col - m * c.nk;
  const int slot = c.slot[jk];
  if (j < 4 * NCOEF) {
    const int n = j & (NCOEF - 1), part = (j >> 6) & 1;
    if (n < m || n >= c.nrc) return 0.f;
    const double2 z = ((j >> 7) ? chi : psi)[(c.off[m] + n - m) * c.nz + slot];
    return (float)(part ? z.y : z.x);
  }
  if (j == 4 * NCOEF) return (float)m / (float)c.M;
  return c.kmax > 0 ? (float)kval(slot, c.nz) / (float)c.kmax : 0.f;
}

// Raw features [ncols][NIN] (FP32), or the network input [rows][KIN] (bfloat16, scaled).
__global__ __launch_bounds__(256) void features_kernel(ColMap c, const double2* psi, const double2* chi, int ncols,
                                                       int rows, float* raw, const float* xs, unsigned short* X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (raw) {
    if (e >= (int64_t)ncols * NIN) return;
    const int col = (int)(e / NIN), j = (int)(e - (int64_t)col * NIN);
    raw[e] = feature(c, psi, chi, col, j);
  } else {
    if (e >= (int64_t)rows * KIN) return;
    const int col = (int)(e / KIN), j = (int)(e - (int64_t)col * KIN);
    const float v = (col < ncols && j < NIN) ? feature(c, psi, chi, col, j) * xs[j] : 0.f;
    X[e] = bf16_bits(v);
  }
}

// Raw targets [ncols][NOUT]: (ref - coarse) at the output positions.
__global__ __launch_bounds__(256) void targets_kernel(ColMap c, const double2* rp, const double2* rc,
                                                      const double2* cp, const double2* cc, int ncols, float* y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ncols * NOUT) return;
  const int col = (int)(e / NOUT), o = (int)(e - (int64_t)col * NOUT);
  const int m = col / c.nk, jk = col - m * c.nk;
  const int slot = c.slot[jk];
  const int n = o & (NCOEF - 1), part = (o >> 6) & 1;
  float v = 0.f;
  if (n >= m && n < c.nrc) {
    const int64_t i = (c.off[m] + n - m) * c.nz + slot;
    const double2 r = (o >> 7) ? rc[i] : rp[i];
    const double2 q = (o >> 7) ? cc[i] : cp[i];
    v = (float)(part ? r.y - q.y : r.x - q.x);
  }
  y[e] = v;
}

// The correction of one spectral element of field f (0 psi, 1 chi); m = 0 columns are made
// Hermitian in k: C(0, k) <- (C(0, k) + conj(C(0, -k))) / 2.
__device__ __forceinline__ double2 correction(const ColMap& c, const int32_t* col_of_slot, const float* Y, int f,
                                              int64_t row, int slot) {
  const int jk = col_of_slot[slot];
  if (jk < 0) return make_double2(0.0, 0.0);
  const int m = c.row_m[row];
  const int n = m + (int)(row - c.off[m]);
  const int o = f * 2 * NCOEF + n;
  const float* y = Y + (int64_t)(m * c.nk + jk) * NOUT;
  double re = y[o], im = y[o + NCOEF];
  if (m == 0) {
    const int ns = slot == 0 ? 0 : c.nz - slot;
    const float* yn = Y + (int64_t)col_of_slot[ns] * NOUT;
    re = 0.5 * (re + (double)yn[o]);
    im = 0.5 * (im - (double)yn[o + NCOEF]);
  }
  return make_double2(re, im);
}

// Norm partials of the judge, per block: |C|^2, |RHS|^2 and, when the reference term Ar of the
// plain solver on a finer grid is given, |RHS + C - Ar|^2 and |RHS - Ar|^2 (both fields).
__global__ __launch_bounds__(256) void norm_kernel(ColMap c, const int32_t* col_of_slot, const float* Y,
                                                   const double2* rp, const double2* rc, const double2* arp,
                                                   const double2* arc, int64_t nel, double* part) {
  __shared__ double s[4][256];
  double cs = 0.0, rs = 0.0, as = 0.0, bs = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * nel; e += (int64_t)gridDim.x * blockDim.x) {
    const int f = e >= nel;
    const int64_t i = e - f * nel;
    const int64_t row = i / c.nz;
    const int slot = (int)(i - row * c.nz);
    const double2 cv = correction(c, col_of_slot, Y, f, row, slot);
    const double2 r = f ? rc[i] : rp[i];
    cs += cv.x * cv.x + cv.y * cv.y;
    rs += r.x * r.x + r.y * r.y;
    if (arp) {
      const double2 q = f ? arc[i] : arp[i];
      const double dx = r.x - q.x, dy = r.y - q.y;
      as += (dx + cv.x) * (dx + cv.x) + (dy + cv.y) * (dy + cv.y);
      bs += dx * dx + dy * dy;
    }
  }
  s[0][threadIdx.x] = cs;
  s[1][threadIdx.x] = rs;
  s[2][threadIdx.x] = as;
  s[3][threadIdx.x] = bs;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) part[4 * blockIdx.x + q] = s[q][0];
}

// Judge and apply: every block reduces the norm partials in the same order and takes the same
// decision; accepted corrections are added to (rp, rc).  Accepted: finite norms, ||C|| <= beta ||RHS||
// and, with a reference term, ||RHS + C - Ar|| <= ||RHS - Ar||.  flags[1] = fallback of this call,
// flags[2] counts fallbacks, flags[3] counts calls.
__global__ __launch_bounds__(256) void apply_kernel(ColMap c, const int32_t* col_of_slot, const float* Y,
                                                    double2* rp, double2* rc, int64_t nel, const double* part,
                                                    int nparts, double beta, int has_ref, int* flags) {
  __shared__ double s[4][256];
  __shared__ int accept;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nparts; i += 256)
    for (int q = 0; q < 4; ++q) v[q] += part[4 * i + q];
  for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double cn = s[0][0], rn = s[1][0], an = s[2][0], bn = s[3][0];
    int ok = isfinite(cn) && isfinite(rn) && sqrt(cn) <= beta * sqrt(rn);
    if (has_ref) ok = ok && isfinite(an) && isfinite(bn) && an <= bn;
    accept = ok;
    if (blockIdx.x == 0) {
      flags[1] = !ok;
      flags[2] += !ok;
      flags[3] += 1;
    }
  }
  __syncthreads();
  if (!accept) return;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * nel; e += (int64_t)gridDim.x * blockDim.x) {
    const int f = e >= nel;
    const int64_t i = e - f * nel;
    const int64_t row = i / c.nz;
    const int slot = (int)(i - row * c.nz);
    const double2 cv = correction(c, col_of_slot, Y, f, row, slot);
    double2* r = f ? rc : rp;
    r[i] = make_double2(r[i].x + cv.x, r[i].y + cv.y);
  }
}

// Spectral truncation / zero extension between two FP64 plans with equal ell and L_z: every
// destination coefficient (m, n, k) takes the source coefficient of the same (m, n, k) when the
// source stores it and the destination chop keeps k, and zero otherwise.
struct TruncArgs {
  const double2* src;
  double2* dst;
  const int32_t* row_m_d;
  const int64_t* off_d;
  const int64_t* off_s;
  int64_t nel_d;
  int nz_d, nzc_d, nz_s, nzc_s, M_s, nrc_s;
};

__global__ __launch_bounds__(256) void truncate_kernel(TruncArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nel_d) return;
  const int64_t row = e / a.nz_d;
  const int slot = (int)(e - row * a.nz_d);
  const int m = a.row_m_d[row];
  const int n = m + (int)(row - a.off_d[m]);
  const int k = kval(slot, a.nz_d);
  const int ka = k < 0 ? -k : k;
  const bool keep_d = ka < a.nzc_d && !(a.nz_d % 2 == 0 && a.nz_d > 1 && k == -(a.nz_d / 2));
  const bool have_s = m < a.M_s && n < a.nrc_s && ka < a.nzc_s && 2 * ka <= a.nz_s &&
                      !(a.nz_s % 2 == 0 && a.nz_s > 1 && k == -(a.nz_s / 2)) && (a.nz_s > 1 || k == 0);
  double2 v = make_double2(0.0, 0.0);
  if (keep_d && have_s) {
    const int ss = k < 0 ? k + a.nz_s : k;
    v = a.src[(a.off_s[m] + n - m) * a.nz_s + ss];
  }
  a.dst[e] = v;
}

int blocks_for(int64_t n, int t = 256) { return (int)std::max<int64_t>(1, (n + t - 1) / t); }

template <typename T>
mlg_status dalloc(T** p, size_t n) {
  *p = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(MLG_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return MLG_OK;
}

template <bool AK, bool BK, int EPI>
mlg_status mm(const MMArgs& a, int splits, hipStream_t s) {
  dim3 grid((a.N + 63) / 64, (a.M + 63) / 64, splits);
  hipLaunchKernelGGL((mm_kernel<AK, BK, EPI>), grid, dim3(256), 0, s, a);
  MLG_HIP_TRY(hipGetLastError());
  return MLG_OK;
}

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int round_up(int v, int q) { return (v + q - 1) / q * q; }

}  // namespace
}  // namespace mlg

struct mlg_closure_s {
  const mlg_plan_s* plan = nullptr;
  int device = 0;
  double beta = 0.0;
  int max_batch = 0, ncols = 0, nk = 0, kmax = 0, rows = 0;  // rows: allocated batch rows (multiple of 64)
  int64_t step = 0;
  int last_nb = 0;
  int32_t* d_slot = nullptr;
  int32_t* d_col_of_slot = nullptr;
  float* d_p = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_g = nullptr;
  float* d_part = nullptr;       // NSPLIT_MAX x P_TOTAL
  float* d_loss_part = nullptr;  // (rows / 64) x (NOUT / 64)
  float* d_loss = nullptr;
  unsigned short* d_wb = nullptr;
  float* d_xs = nullptr;
  float* d_ys = nullptr;
  unsigned short* d_x = nullptr;
  unsigned short* d_h1b = nullptr;
  unsigned short* d_h2b = nullptr;
  unsigned short* d_dy = nullptr;
  unsigned short* d_dz2 = nullptr;
  unsigned short* d_dz1 = nullptr;
  float* d_h1f = nullptr;
  float* d_h2f = nullptr;
  float* d_t = nullptr;
  float* d_y = nullptr;
  double* d_norm = nullptr;
  int* d_flags = nullptr;  // [0] bad index, [1] last fallback, [2] fallbacks, [3] calls
  // reference judge (mlg_closure_set_reference): the plain term on a finer plan
  const mlg_plan_s* ref = nullptr;
  double Uref[3] = {0.0, 0.0, 0.0};
  void* d_ref_ws = nullptr;
  double* d_ref_buf = nullptr;  // psi, chi, A_psi, A_chi on the reference plan; A_psi, A_chi truncated

  mlg::ColMap colmap() const {
    mlg::ColMap c{};
    c.slot = d_slot;
    c.row_m = plan->d_row_m;
    c.off = plan->d_goff;
    c.M = plan->M;
    c.nrc = plan->nrc;
    c.nz = plan->nz;
    c.nk = nk;
    c.kmax = kmax;
    return c;
  }
};

namespace mlg {
namespace {

void free_closure(mlg_closure_s* c) {
  void* ptrs[] = {c->d_slot, c->d_col_of_slot, c->d_p, c->d_m, c->d_v, c->d_g, c->d_part, c->d_loss_part,
                  c->d_loss, c->d_wb, c->d_xs, c->d_ys, c->d_x, c->d_h1b, c->d_h2b, c->d_dy, c->d_dz2,
                  c->d_dz1, c->d_h1f, c->d_h2f, c->d_t, c->d_y, c->d_norm, c->d_flags, c->d_ref_ws,
                  c->d_ref_buf};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
}

// Forward pass over 'rows' rows of c->d_x; training (targets in d_t) or inference (out != null).
mlg_status run_forward(mlg_closure_s* c, int rows, int nvalid, float* out, hipStream_t s) {
  MMArgs a{};
  a.M = rows;
  a.N = HID;
  a.kchunk = KIN;
  a.A = c->d_x;
  a.lda = KIN;
  a.B = c->d_wb + P_W1;
  a.ldb = KIN;
  a.K = KIN;
  a.ldc = HID;
  a.bias = c->d_p + P_B1;
  a.Hf = c->d_h1f;
  a.Cb = c->d_h1b;
  if (mlg_status st = mm<true, true, EPI_TANH>(a, 1, s)) return st;
  a.A = c->d_h1b;
  a.lda = HID;
  a.B = c->d_wb + P_W2;
  a.ldb = HID;
  a.K = HID;
  a.kchunk = HID;
  a.bias = c->d_p + P_B2;
  a.Hf = c->d_h2f;
  a.Cb = c->d_h2b;
  if (mlg_status st = mm<true, true, EPI_TANH>(a, 1, s)) return st;
  a.A = c->d_h2b;
  a.B = c->d_wb + P_W3;
  a.N = NOUT;
  a.ldc = NOUT;
  a.bias = c->d_p + P_B3;
  a.nvalid = nvalid;
  if (out) {
    a.Cf = out;
    a.yscale = c->d_ys;
    return mm<true, true, EPI_OUT>(a, 1, s);
  }
  a.T = c->d_t;
  a.Cb = c->d_dy;
  a.part = c->d_loss_part;
  a.gscale = 2.0f / ((float)nvalid * (float)NOUT);
  return mm<true, true, EPI_LOSS>(a, 1, s);
}

mlg_status run_backward(mlg_closure_s* c, int rows, float lr, hipStream_t s) {
  const int nsplit = std::max(1, std::min(NSPLIT_MAX, rows / 256));
  const int kchunk = round_up((rows + nsplit - 1) / nsplit, 32);
  // weight gradients: gW[o][j] = sum_b dZ[b][o] H[b][j]
  MMArgs g{};
  g.M = HID;
  g.K = rows;
  g.kchunk = kchunk;
  g.cf_split = P_TOTAL;
  g.lda = NOUT;
  g.A = c->d_dy;
  g.B = c->d_h2b;
  g.ldb = HID;
  g.N = HID;
  g.ldc = HID;
  g.Cf = c->d_part + P_W3;
  if (mlg_status st = mm<false, false, EPI_F32>(g, nsplit, s)) return st;
  // dz2 = bf16((dy W3) * (1 - h2^2))
  MMArgs d{};
  d.M = rows;
  d.N = HID;
  d.K = NOUT;
  d.kchunk = NOUT;
  d.A = c->d_dy;
  d.lda = NOUT;
  d.B = c->d_wb + P_W3;
  d.ldb = HID;
  d.ldc = HID;
  d.Hf = c->d_h2f;
  d.Cb = c->d_dz2;
  if (mlg_status st = mm<true, false, EPI_DTANH>(d, 1, s)) return st;
  g.A = c->d_dz2;
  g.lda = HID;
  g.B = c->d_h1b;
  g.Cf = c->d_part + P_W2;
  if (mlg_status st = mm<false, false, EPI_F32>(g, nsplit, s)) return st;
  d.A = c->d_dz2;
  d.lda = HID;
  d.K = HID;
  d.kchunk = HID;
  d.B = c->d_wb + P_W2;
  d.Hf = c->d_h1f;
  d.Cb = c->d_dz1;
  if (mlg_status st = mm<true, false, EPI_DTANH>(d, 1, s)) return st;
  g.A = c->d_dz1;
  g.B = c->d_x;
  g.ldb = KIN;
  g.N = KIN;
  g.ldc = KIN;
  g.Cf = c->d_part + P_W1;
  if (mlg_status st = mm<false, false, EPI_F32>(g, nsplit, s)) return st;
  hipLaunchKernelGGL(colsum_kernel, dim3(nsplit, 3), dim3(256), 0, s, c->d_dy, c->d_dz2, c->d_dz1, rows, kchunk,
                     c->d_part);
  MLG_HIP_TRY(hipGetLastError());
  c->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 - std::pow(b1, (double)c->step));
  const float bc2 = (float)(1.0 - std::pow(b2, (double)c->step));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(P_TOTAL)), dim3(256), 0, s, c->d_part, nsplit, c->d_g, c->d_p,
                     c->d_m, c->d_v, c->d_wb, lr, (float)b1, (float)b2, bc1, bc2, 1e-8f);
  MLG_HIP_TRY(hipGetLastError());
  return MLG_OK;
}

mlg_status check_closure(mlg_closure c) {
  if (!c) return fail(MLG_E_ARG, "closure is NULL");
  return MLG_OK;
}

// external (W1 [256][258]) <-> internal (W1 [256][288]) parameter order
void to_internal(const float* ext, std::vector<float>& in) {
  in.assign(P_TOTAL, 0.f);
  size_t o = 0;
  for (int r = 0; r < HID; ++r)
    for (int j = 0; j < NIN; ++j) in[P_W1 + (size_t)r * KIN + j] = ext[o++];
  for (int i = 0; i < P_TOTAL - P_B1; ++i) in[P_B1 + i] = ext[o++];
}
void to_external(const std::vector<float>& in, float* ext) {
  size_t o = 0;
  for (int r = 0; r < HID; ++r)
    for (int j = 0; j < NIN; ++j) ext[o++] = in[P_W1 + (size_t)r * KIN + j];
  for (int i = 0; i < P_TOTAL - P_B1; ++i) ext[o++] = in[P_B1 + i];
}

}  // namespace

// Internal entry used by the time integrator: features -> network -> judge -> add.
mlg_status closure_correct(mlg_closure_s* c, const double* psi, const double* chi, double* rpsi, double* rchi,
                           hipStream_t s) {
  const mlg_plan_s* p = c->plan;
  const ColMap cm = c->colmap();
  const int rows = round_up(c->ncols, 64);
  hipLaunchKernelGGL(features_kernel, dim3(blocks_for((int64_t)rows * KIN)), dim3(256), 0, s, cm,
                     reinterpret_cast<const double2*>(psi), reinterpret_cast<const double2*>(chi), c->ncols, rows,
                     (float*)nullptr, c->d_xs, c->d_x);
  MLG_HIP_TRY(hipGetLastError());
  if (mlg_status st = run_forward(c, rows, c->ncols, c->d_y, s)) return st;
  const int64_t nel = p->tau * p->nz;
  const double2* arp = nullptr;
  const double2* arc = nullptr;
  if (c->ref) {
    // the plain term of the same coarse state on the finer reference plan, truncated back
    const mlg_plan_s* q = c->ref;
    const size_t qe = (size_t)q->tau * q->nz * 2;
    double* b = c->d_ref_buf;
    double *qp = b, *qc = b + qe, *qap = b + 2 * qe, *qac = b + 3 * qe;
    double *tap = b + 4 * qe, *tac = tap + (size_t)nel * 2;
    mlg_status st;
    if ((st = mlg_truncate(const_cast<mlg_plan_s*>(p), const_cast<mlg_plan_s*>(q), psi, qp, s)) ||
        (st = mlg_truncate(const_cast<mlg_plan_s*>(p), const_cast<mlg_plan_s*>(q), chi, qc, s)) ||
        (st = mlg_rhs_tp(const_cast<mlg_plan_s*>(q), c->Uref, qp, qc, qap, qac, nullptr, c->d_ref_ws, s)) ||
        (st = mlg_truncate(const_cast<mlg_plan_s*>(q), const_cast<mlg_plan_s*>(p), qap, tap, s)) ||
        (st = mlg_truncate(const_cast<mlg_plan_s*>(q), const_cast<mlg_plan_s*>(p), qac, tac, s)))
      return st;
    arp = reinterpret_cast<const double2*>(tap);
    arc = reinterpret_cast<const double2*>(tac);
  }
  hipLaunchKernelGGL(norm_kernel, dim3(NORM_BLOCKS), dim3(256), 0, s, cm, c->d_col_of_slot, c->d_y,
                     reinterpret_cast<const double2*>(rpsi), reinterpret_cast<const double2*>(rchi), arp, arc, nel,
                     c->d_norm);
  MLG_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(apply_kernel, dim3(NORM_BLOCKS), dim3(256), 0, s, cm, c->d_col_of_slot, c->d_y,
                     reinterpret_cast<double2*>(rpsi), reinterpret_cast<double2*>(rchi), nel, c->d_norm, NORM_BLOCKS,
                     c->beta, c->ref ? 1 : 0, c->d_flags);
  MLG_HIP_TRY(hipGetLastError());
  return MLG_OK;
}

const mlg_plan_s* closure_plan(const mlg_closure_s* c) { return c->plan; }

}  // namespace mlg

using namespace mlg;

extern "C" {

int32_t mlg_closure_param_count(void) { return EXT_TOTAL; }

mlg_status mlg_closure_create(const mlg_closure_cfg* cfg, mlg_plan coarse, mlg_closure* out) {
  if (!out) return fail(MLG_E_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg || !coarse) return fail(MLG_E_ARG, "cfg or plan is NULL");
  if (coarse->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "the closure needs an FP64 coarse plan");
  if (coarse->nrc > NCOEF) return fail(MLG_E_UNSUPPORTED, "the closure needs N_r^c <= 64 on the coarse plan");
  if (cfg->max_batch < 1 || cfg->max_batch > (1 << 20)) return fail(MLG_E_ARG, "max_batch must be in [1, 2^20]");
  if (!std::isfinite(cfg->beta) || cfg->beta < 0) return fail(MLG_E_ARG, "beta must be finite and >= 0");
  DevGuard guard(coarse->device);
  mlg_closure_s* c = new (std::nothrow) mlg_closure_s();
  if (!c) return fail(MLG_E_ALLOC, "host allocation failed");
  c->plan = coarse;
  c->device = coarse->device;
  c->beta = cfg->beta;
  c->max_batch = cfg->max_batch;
  // active axial slots in FFT order
  std::vector<int32_t> slots, col_of_slot(coarse->nz, -1);
  for (int sl = 0; sl < coarse->nz; ++sl) {
    const int k = (2 * sl < coarse->nz) ? sl : sl - coarse->nz;
    const int ka = std::abs(k);
    const bool nyq = coarse->nz % 2 == 0 && coarse->nz > 1 && k == -(coarse->nz / 2);
    if (ka < coarse->nzc && !nyq) {
      col_of_slot[sl] = (int32_t)slots.size();
      slots.push_back(sl);
      c->kmax = std::max(c->kmax, ka);
    }
  }
  c->nk = (int)slots.size();
  c->ncols = coarse->M * c->nk;
  c->rows = round_up(std::max(c->max_batch, c->ncols), 64);
  const size_t R = (size_t)c->rows;
  mlg_status st = MLG_OK;
  if ((st = dalloc(&c->d_slot, slots.size())) || (st = dalloc(&c->d_col_of_slot, col_of_slot.size())) ||
      (st = dalloc(&c->d_p, P_TOTAL)) || (st = dalloc(&c->d_m, P_TOTAL)) || (st = dalloc(&c->d_v, P_TOTAL)) ||
      (st = dalloc(&c->d_g, P_TOTAL)) || (st = dalloc(&c->d_part, (size_t)NSPLIT_MAX * P_TOTAL)) ||
      (st = dalloc(&c->d_loss_part, (R / 64) * (NOUT / 64))) || (st = dalloc(&c->d_loss, 1)) ||
      (st = dalloc(&c->d_wb, P_TOTAL)) || (st = dalloc(&c->d_xs, KIN)) || (st = dalloc(&c->d_ys, NOUT)) ||
      (st = dalloc(&c->d_x, R * KIN)) || (st = dalloc(&c->d_h1b, R * HID)) || (st = dalloc(&c->d_h2b, R * HID)) ||
      (st = dalloc(&c->d_dy, R * NOUT)) || (st = dalloc(&c->d_dz2, R * HID)) || (st = dalloc(&c->d_dz1, R * HID)) ||
      (st = dalloc(&c->d_h1f, R * HID)) || (st = dalloc(&c->d_h2f, R * HID)) || (st = dalloc(&c->d_t, R * NOUT)) ||
      (st = dalloc(&c->d_y, R * NOUT)) || (st = dalloc(&c->d_norm, 4 * NORM_BLOCKS)) ||
      (st = dalloc(&c->d_flags, 4))) {
    free_closure(c);
    return st;
  }
  std::vector<float> zero(P_TOTAL, 0.f), ones(KIN, 1.f);
  std::vector<unsigned short> zb(P_TOTAL, 0);
  std::vector<int> fl(4, 0);
  hipError_t e = hipSuccess;
  if ((e = hipMemcpy(c->d_slot, slots.data(), slots.size() * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_col_of_slot, col_of_slot.data(), col_of_slot.size() * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_p, zero.data(), P_TOTAL * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_m, zero.data(), P_TOTAL * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_v, zero.data(), P_TOTAL * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_g, zero.data(), P_TOTAL * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_wb, zb.data(), P_TOTAL * 2, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_xs, ones.data(), KIN * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_ys, ones.data(), NOUT * 4, hipMemcpyHostToDevice)) ||
      (e = hipMemcpy(c->d_flags, fl.data(), 16, hipMemcpyHostToDevice))) {
    free_closure(c);
    return fail(MLG_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  *out = c;
  return MLG_OK;
}

mlg_status mlg_closure_destroy(mlg_closure c) {
  if (!c) return MLG_OK;
  DevGuard guard(c->device);
  (void)hipDeviceSynchronize();
  free_closure(c);
  return MLG_OK;
}

mlg_status mlg_closure_columns(mlg_closure c, int32_t* ncols) {
  if (mlg_status st = check_closure(c)) return st;
  if (!ncols) return fail(MLG_E_ARG, "ncols is NULL");
  *ncols = c->ncols;
  return MLG_OK;
}

mlg_status mlg_closure_set_params(mlg_closure c, const float* params) {
  if (mlg_status st = check_closure(c)) return st;
  if (!params) return fail(MLG_E_ARG, "params is NULL");
  DevGuard guard(c->device);
  std::vector<float> in;
  to_internal(params, in);
  std::vector<unsigned short> wb(P_TOTAL);
  for (int i = 0; i < P_TOTAL; ++i) {
    unsigned int u;
    std::memcpy(&u, &in[i], 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    wb[i] = (unsigned short)(u >> 16);
  }
  std::vector<float> zero(P_TOTAL, 0.f);
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(c->d_p, in.data(), P_TOTAL * 4, hipMemcpyHostToDevice));
  MLG_HIP_TRY(hipMemcpy(c->d_wb, wb.data(), P_TOTAL * 2, hipMemcpyHostToDevice));
  MLG_HIP_TRY(hipMemcpy(c->d_m, zero.data(), P_TOTAL * 4, hipMemcpyHostToDevice));
  MLG_HIP_TRY(hipMemcpy(c->d_v, zero.data(), P_TOTAL * 4, hipMemcpyHostToDevice));
  MLG_HIP_TRY(hipMemcpy(c->d_g, zero.data(), P_TOTAL * 4, hipMemcpyHostToDevice));
  c->step = 0;
  return MLG_OK;
}

mlg_status mlg_closure_get_params(mlg_closure c, float* params) {
  if (mlg_status st = check_closure(c)) return st;
  if (!params) return fail(MLG_E_ARG, "params is NULL");
  DevGuard guard(c->device);
  std::vector<float> in(P_TOTAL);
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(in.data(), c->d_p, P_TOTAL * 4, hipMemcpyDeviceToHost));
  to_external(in, params);
  return MLG_OK;
}

mlg_status mlg_closure_get_grads(mlg_closure c, float* grads) {
  if (mlg_status st = check_closure(c)) return st;
  if (!grads) return fail(MLG_E_ARG, "grads is NULL");
  DevGuard guard(c->device);
  std::vector<float> in(P_TOTAL);
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(in.data(), c->d_g, P_TOTAL * 4, hipMemcpyDeviceToHost));
  to_external(in, grads);
  return MLG_OK;
}

mlg_status mlg_closure_set_scales(mlg_closure c, const float* x_scale, const float* y_scale) {
  if (mlg_status st = check_closure(c)) return st;
  if (!x_scale || !y_scale) return fail(MLG_E_ARG, "null scales");
  for (int j = 0; j < NIN; ++j)
    if (!std::isfinite(x_scale[j])) return fail(MLG_E_NONFINITE, "non-finite feature scale");
  for (int o = 0; o < NOUT; ++o)
    if (!std::isfinite(y_scale[o]) || y_scale[o] == 0.f) return fail(MLG_E_ARG, "output scales must be finite, non-zero");
  DevGuard guard(c->device);
  std::vector<float> xs(KIN, 0.f);
  std::copy(x_scale, x_scale + NIN, xs.begin());
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(c->d_xs, xs.data(), KIN * 4, hipMemcpyHostToDevice));
  MLG_HIP_TRY(hipMemcpy(c->d_ys, y_scale, NOUT * 4, hipMemcpyHostToDevice));
  return MLG_OK;
}

mlg_status mlg_closure_get_scales(mlg_closure c, float* x_scale, float* y_scale) {
  if (mlg_status st = check_closure(c)) return st;
  if (!x_scale || !y_scale) return fail(MLG_E_ARG, "null scales");
  DevGuard guard(c->device);
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(x_scale, c->d_xs, NIN * 4, hipMemcpyDeviceToHost));
  MLG_HIP_TRY(hipMemcpy(y_scale, c->d_ys, NOUT * 4, hipMemcpyDeviceToHost));
  return MLG_OK;
}

mlg_status mlg_closure_features(mlg_closure c, const void* psi, const void* chi, float* x_out, void* stream) {
  if (mlg_status st = check_closure(c)) return st;
  if (!psi || !chi || !x_out) return fail(MLG_E_ARG, "null buffer");
  DevGuard guard(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(features_kernel, dim3(blocks_for((int64_t)c->ncols * NIN)), dim3(256), 0, s, c->colmap(),
                     static_cast<const double2*>(psi), static_cast<const double2*>(chi), c->ncols, 0, x_out,
                     (const float*)nullptr, (unsigned short*)nullptr);
  MLG_HIP_TRY(hipGetLastError());
  return MLG_OK;
}

mlg_status mlg_closure_targets(mlg_closure c, const void* ref_psi, const void* ref_chi, const void* psi_n,
                               const void* chi_n, float* y_out, void* stream) {
  if (mlg_status st = check_closure(c)) return st;
  if (!ref_psi || !ref_chi || !psi_n || !chi_n || !y_out) return fail(MLG_E_ARG, "null buffer");
  DevGuard guard(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(targets_kernel, dim3(blocks_for((int64_t)c->ncols * NOUT)), dim3(256), 0, s, c->colmap(),
                     static_cast<const double2*>(ref_psi), static_cast<const double2*>(ref_chi),
                     static_cast<const double2*>(psi_n), static_cast<const double2*>(chi_n), c->ncols, y_out);
  MLG_HIP_TRY(hipGetLastError());
  return MLG_OK;
}

mlg_status mlg_closure_forward(mlg_closure c, const float* x, int32_t nb, float* y, void* stream) {
  if (mlg_status st = check_closure(c)) return st;
  if (!x || !y) return fail(MLG_E_ARG, "null buffer");
  if (nb < 1 || nb > c->rows) return fail(MLG_E_ARG, "nb must be in [1, max(max_batch, columns)]");
  DevGuard guard(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rows = round_up(nb, 64);
  hipLaunchKernelGGL(prep_kernel, dim3(blocks_for((int64_t)rows * KIN)), dim3(256), 0, s, x, (const float*)nullptr,
                     (const int32_t*)nullptr, (int64_t)nb, nb, rows, c->d_xs, c->d_ys, c->d_x, c->d_t, c->d_flags);
  MLG_HIP_TRY(hipGetLastError());
  return run_forward(c, rows, nb, y, s);
}

mlg_status mlg_closure_train_step(mlg_closure c, const float* data_x, const float* data_y, const int32_t* idx,
                                  int64_t count, int32_t nb, float lr, float* loss_out, void* stream) {
  if (mlg_status st = check_closure(c)) return st;
  if (!data_x || !data_y) return fail(MLG_E_ARG, "null buffer");
  if (nb < 1 || nb > c->max_batch) return fail(MLG_E_ARG, "nb must be in [1, max_batch]");
  if (count < 1 || (!idx && count < nb)) return fail(MLG_E_ARG, "count too small for the batch");
  if (!std::isfinite(lr) || lr < 0) return fail(MLG_E_ARG, "lr must be finite and >= 0");
  DevGuard guard(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rows = round_up(nb, 64);
  hipLaunchKernelGGL(prep_kernel, dim3(blocks_for((int64_t)rows * KIN)), dim3(256), 0, s, data_x, data_y, idx, count,
                     nb, rows, c->d_xs, c->d_ys, c->d_x, c->d_t, c->d_flags);
  MLG_HIP_TRY(hipGetLastError());
  if (mlg_status st = run_forward(c, rows, nb, nullptr, s)) return st;
  const int nparts = (rows / 64) * (NOUT / 64);
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, s, c->d_loss_part, nparts,
                     1.0f / ((float)nb * (float)NOUT), c->d_loss);
  MLG_HIP_TRY(hipGetLastError());
  if (mlg_status st = run_backward(c, rows, lr, s)) return st;
  c->last_nb = nb;
  if (loss_out) {
    int fl[4];
    MLG_HIP_TRY(hipMemcpyAsync(loss_out, c->d_loss, 4, hipMemcpyDeviceToHost, s));
    MLG_HIP_TRY(hipMemcpyAsync(fl, c->d_flags, 16, hipMemcpyDeviceToHost, s));
    MLG_HIP_TRY(hipStreamSynchronize(s));
    if (fl[0]) {
      const int zero = 0;
      MLG_HIP_TRY(hipMemcpy(c->d_flags, &zero, 4, hipMemcpyHostToDevice));
      return fail(MLG_E_ARG, "a batch index was outside [0, count)");
    }
  }
  return MLG_OK;
}

mlg_status mlg_closure_infer(mlg_closure c, const void* psi, const void* chi, void* rhs_psi, void* rhs_chi,
                             int32_t* used_fallback, void* stream) {
  if (mlg_status st = check_closure(c)) return st;
  if (!psi || !chi || !rhs_psi || !rhs_chi) return fail(MLG_E_ARG, "null buffer");
  if (rhs_psi == rhs_chi) return fail(MLG_E_ARG, "rhs_psi and rhs_chi must differ");
  DevGuard guard(c->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mlg_status st = closure_correct(c, static_cast<const double*>(psi), static_cast<const double*>(chi),
                                      static_cast<double*>(rhs_psi), static_cast<double*>(rhs_chi), s))
    return st;
  if (used_fallback) {
    int fl[4];
    MLG_HIP_TRY(hipMemcpyAsync(fl, c->d_flags, 16, hipMemcpyDeviceToHost, s));
    MLG_HIP_TRY(hipStreamSynchronize(s));
    *used_fallback = fl[1];
  }
  return MLG_OK;
}

mlg_status mlg_closure_stats(mlg_closure c, int64_t* calls, int64_t* fallbacks) {
  if (mlg_status st = check_closure(c)) return st;
  DevGuard guard(c->device);
  int fl[4];
  MLG_HIP_TRY(hipDeviceSynchronize());
  MLG_HIP_TRY(hipMemcpy(fl, c->d_flags, 16, hipMemcpyDeviceToHost));
  if (calls) *calls = fl[3];
  if (fallbacks) *fallbacks = fl[2];
  return MLG_OK;
}

mlg_status mlg_closure_set_reference(mlg_closure c, mlg_plan ref, const double* U) {
  if (mlg_status st = check_closure(c)) return st;
  DevGuard guard(c->device);
  MLG_HIP_TRY(hipDeviceSynchronize());
  if (c->d_ref_ws) (void)hipFree(c->d_ref_ws);
  if (c->d_ref_buf) (void)hipFree(c->d_ref_buf);
  c->d_ref_ws = nullptr;
  c->d_ref_buf = nullptr;
  c->ref = nullptr;
  if (!ref) return MLG_OK;
  const mlg_plan_s* p = c->plan;
  if (ref->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "the reference plan must be FP64");
  if (ref->device != p->device) return fail(MLG_E_ARG, "reference plan on another device");
  if (ref->g.ell != p->g.ell || ref->g.lz != p->g.lz) return fail(MLG_E_ARG, "reference plan needs equal ell and L_z");
  if (ref->M < p->M || ref->nrc < p->nrc || ref->nzc < p->nzc)
    return fail(MLG_E_ARG, "the reference plan must keep every coefficient of the coarse plan");
  if (ref->nrc > 512) return fail(MLG_E_UNSUPPORTED, "reference plan N_r^c above 512");
  double Uh[3] = {0.0, 0.0, 0.0};
  if (U)
    for (int i = 0; i < 3; ++i) {
      if (!std::isfinite(U[i])) return fail(MLG_E_ARG, "background U must be finite");
      Uh[i] = U[i];
    }
  const size_t qe = (size_t)ref->tau * ref->nz * 2, ce = (size_t)p->tau * p->nz * 2;
  mlg_status st;
  if ((st = dalloc(reinterpret_cast<unsigned char**>(&c->d_ref_ws), ref->ws_bytes)) ||
      (st = dalloc(&c->d_ref_buf, 4 * qe + 2 * ce))) {
    if (c->d_ref_ws) (void)hipFree(c->d_ref_ws);
    c->d_ref_ws = nullptr;
    return st;
  }
  for (int i = 0; i < 3; ++i) c->Uref[i] = Uh[i];
  c->ref = ref;
  return MLG_OK;
}

mlg_status mlg_truncate(mlg_plan from, mlg_plan to, const void* src, void* dst, void* stream) {
  if (!from || !to) return fail(MLG_E_ARG, "plan is NULL");
  if (!src || !dst) return fail(MLG_E_ARG, "null buffer");
  if (src == dst) return fail(MLG_E_ARG, "src and dst must differ");
  if (from->prec != MLG_FP64 || to->prec != MLG_FP64) return fail(MLG_E_UNSUPPORTED, "truncation needs FP64 plans");
  if (from->g.ell != to->g.ell || from->g.lz != to->g.lz)
    return fail(MLG_E_ARG, "truncation needs equal ell and L_z");
  if (from->device != to->device) return fail(MLG_E_ARG, "plans on different devices");
  DevGuard guard(to->device);
  TruncArgs a{};
  a.src = static_cast<const double2*>(src);
  a.dst = static_cast<double2*>(dst);
  a.row_m_d = to->d_row_m;
  a.off_d = to->d_goff;
  a.off_s = from->d_goff;
  a.nel_d = to->tau * to->nz;
  a.nz_d = to->nz;
  a.nzc_d = to->nzc;
  a.nz_s = from->nz;
  a.nzc_s = from->nzc;
  a.M_s = from->M;
  a.nrc_s = from->nrc;
  hipLaunchKernelGGL(truncate_kernel, dim3(blocks_for(a.nel_d)), dim3(256), 0, static_cast<hipStream_t>(stream), a);
  MLG_HIP_TRY(hipGetLastError());
  return MLG_OK;
}

}  // extern "C"
