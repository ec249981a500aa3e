// Batched pseudospectral KPP term for many uneven 2D instances.
//
// For each instance b (N_z = 1): R_b = Mask(F(gamma u (1 - u))), u = B(Mask(u_hat_b)) (Sec. 3.3;
// Sec. 5.2, Eq. kpp; the two-thirds mask holds for the field entering the product too).  Three persistent launches (a fixed number of blocks per CU, each block
// walking its share of the phase's work list) run the phases; the kernel boundaries order them
// (a grid-wide barrier inside one cooperative launch costs about 50 us on this part, against a few
// microseconds for a launch boundary):
//   1. backward radial transform per (instance, m): f_m(r_i) = sum_n Pbar_n^m(x_i) u_hat_n^m;
//      Pbar either streamed from per-instance tables or regenerated in the kernel by the
//      normalised three-term recurrence (FP64) from Pbar_m^m(x_i);
//   2. per (instance, group of azimuthal lines): inverse real FFT in phi, gamma u (1 - u),
//      forward FFT, two-thirds mask;
//   3. forward radial projection per (instance, m): u_hat_n^m = sum_i w_i Pbar_n^m(x_i) g_m(r_i).
// Work lists of each phase are sorted by cost (largest first) and dealt round-robin to the
// blocks.  Data may be FP64 or FP32 (template T); recurrences and tables are built in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "mlg_internal.h"

namespace mlg {

struct BatchInst {
  int nr, nphi, M, nrc, mkeep, nrad;
  int rad[8];
  int64_t spec_off;   // complex elements into the packed spectra
  int64_t mix_off;    // complex elements into the workspace (M x nr harmonics)
  int64_t tb_off;     // backward table Pbar [m][n-m][i]  (reals)
  int64_t tf_off;     // forward table w Pbar [m][i][n-m] (reals)
  int64_t rec_off;    // recurrence data: per m, (nrc - m) pairs (a_n, b_n)
  int64_t start_off;  // Pbar_m^m(x_i): [m][i]
  int64_t node_off;   // x_i
  int64_t tw_off;     // exp(-2 pi i t / N_phi), complex
  int64_t tri_off;    // triangular row offset table start (M + 1 entries) in the int64 array
};

struct BatchConfig {
  int recurrence;   // 1: regenerate Pbar in the kernel in phase 1
  int threads;      // 128 or 256
  int blocks_per_cu;
  int lines;        // azimuthal lines per phase-2 item (even)
};

}  // namespace mlg

struct mlg_batch_s {
  int count = 0;
  int device = 0;
  mlg_precision prec = MLG_FP64;
  double gamma_default = 0.25;
  std::vector<mlg::BatchInst> inst;
  std::vector<int64_t> spec_offsets;  // count + 1
  int64_t spec_total = 0, mix_total = 0;
  mlg::BatchInst* d_inst = nullptr;
  double* d_tab = nullptr;     // FP64 tables (backward, forward, recurrence, start, nodes, twiddles)
  float* d_tab32 = nullptr;    // FP32 copies of the backward / forward tables (FP32 batches)
  int64_t* d_tri = nullptr;
  int32_t* d_items[3] = {nullptr, nullptr, nullptr};  // packed (instance << 16 | index)
  int nitems[3] = {0, 0, 0};
  std::vector<int32_t> items_host[3];
  mlg::BatchConfig cfg{0, 256, 2, 8};
  int tuned = 0;
  int cus = 0;
  size_t ws_bytes = 0;
};

namespace mlg {
namespace {

template <typename T>
struct Cx {
  T x, y;
};
template <typename T>
__device__ __forceinline__ Cx<T> cx(T a, T b) {
  return Cx<T>{a, b};
}
template <typename T>
__device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return cx(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return cx(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return cx(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ Cx<T> conjc(Cx<T> a) { return cx(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ Cx<T> scl(Cx<T> a, T s) { return cx(a.x * s, a.y * s); }

// multiply by -i (forward) or +i (inverse)
template <typename T>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a, bool inv) {
  return inv ? cx(-a.y, a.x) : cx(a.y, -a.x);
}

// In-register DFT of length R (2, 3, 4, 5) with exp(-+ 2 pi i / R) (forward: minus), written out.
template <typename T, int R>
__device__ __forceinline__ void small_dft(Cx<T> (&v)[R], bool inv) {
  if constexpr (R == 2) {
    const Cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 3) {
    constexpr double h = 0.86602540378443864676;  // sqrt(3)/2
    const Cx<T> t1 = v[1] + v[2];
    const Cx<T> t2 = v[0] - scl(t1, (T)0.5);
    const Cx<T> t3 = mul_mi(scl(v[1] - v[2], (T)h), inv);
    v[0] = v[0] + t1;
    v[1] = t2 + t3;
    v[2] = t2 - t3;
  } else if constexpr (R == 4) {
    const Cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
    const Cx<T> t2 = v[1] + v[3], t3 = mul_mi(v[1] - v[3], inv);
    v[0] = t0 + t2;
    v[1] = t1 + t3;
    v[2] = t0 - t2;
    v[3] = t1 - t3;
  } else {
    constexpr double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;  // cos 2pi/5, cos 4pi/5
    constexpr double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;   // sin 2pi/5, sin 4pi/5
    const Cx<T> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
    const Cx<T> r1 = v[0] + scl(t1, (T)c1) + scl(t2, (T)c2);
    const Cx<T> r2 = v[0] + scl(t1, (T)c2) + scl(t2, (T)c1);
    const Cx<T> i1 = mul_mi(scl(t3, (T)s1) + scl(t4, (T)s2), inv);
    const Cx<T> i2 = mul_mi(scl(t3, (T)s2) - scl(t4, (T)s1), inv);
    v[0] = v[0] + t1 + t2;
    v[1] = r1 + i1;
    v[4] = r1 - i1;
    v[2] = r2 + i2;
    v[3] = r2 - i2;
  }
}

// Stockham pass (radix R, span Ns) over 'nl' lines of length n in LDS; tw is the line's table
// exp(-2 pi i t / n) staged in LDS.  The stage twiddle index j_mod_Ns r n / (Ns R) is below n.
template <typename T, int R>
__device__ __forceinline__ void bpass(const Cx<T>* in, Cx<T>* out, int n, int Ns, const Cx<double>* tw, bool inv,
                                      int nl, int tid, int nth) {
  const int nb = n / R;
  const int tfac = n / (Ns * R);
  for (int idx = tid; idx < nl * nb; idx += nth) {
    const int line = idx / nb, j = idx - line * nb;
    const Cx<T>* src = in + line * n;
    Cx<T>* dst = out + line * n;
    const int jm = j % Ns;
    Cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const Cx<double> w = tw[jm * r * tfac];
      v[r] = v[r] * cx((T)w.x, (T)(inv ? -w.y : w.y));
    }
    small_dft<T, R>(v, inv);
    const int od = (j / Ns) * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[od + r * Ns] = v[r];
  }
}

template <typename T>
__device__ __forceinline__ Cx<T>* bfft(Cx<T>* x, Cx<T>* y, const BatchInst& I, const Cx<double>* tw, bool inv, int nl) {
  const int tid = threadIdx.x, nth = blockDim.x;
  int Ns = 1;
  Cx<T>* a = x;
  Cx<T>* b = y;
  for (int p = 0; p < I.nrad; ++p) {
    const int R = I.rad[p];
    if (R == 4) bpass<T, 4>(a, b, I.nphi, Ns, tw, inv, nl, tid, nth);
    else if (R == 2) bpass<T, 2>(a, b, I.nphi, Ns, tw, inv, nl, tid, nth);
    else if (R == 3) bpass<T, 3>(a, b, I.nphi, Ns, tw, inv, nl, tid, nth);
    else bpass<T, 5>(a, b, I.nphi, Ns, tw, inv, nl, tid, nth);
    __syncthreads();
    Ns *= R;
    Cx<T>* t = a;
    a = b;
    b = t;
  }
  return a;
}

template <typename T>
struct BatchArgs {
  const BatchInst* inst;
  const double* tab;
  const T* tabT;         // tables in the data precision (backward / forward)
  const int64_t* tri;
  const Cx<T>* spec_in;
  Cx<T>* spec_out;
  Cx<T>* mix;
  const int32_t* items[3];
  int nitems[3];
  int recurrence;
  int lines;
  T gamma;
};

template <typename T>
__device__ void phase_backward(const BatchArgs<T>& A, int b, int m, char* smem) {
  const BatchInst& I = A.inst[b];
  const int K = (I.nrc > m && m <= I.mkeep) ? I.nrc - m : 0;  // a masked order enters as zero
  Cx<T>* mix = A.mix + I.mix_off + (int64_t)m * I.nr;
  if (K == 0) {
    for (int i = threadIdx.x; i < I.nr; i += blockDim.x) mix[i] = cx<T>(0, 0);
    return;
  }
  const int64_t trow = A.tri[I.tri_off + m];
  Cx<T>* s = reinterpret_cast<Cx<T>*>(smem);
  for (int t = threadIdx.x; t < K; t += blockDim.x) s[t] = A.spec_in[I.spec_off + trow + t];
  double* rec = reinterpret_cast<double*>(smem + 256 * sizeof(Cx<double>));
  if (A.recurrence)
    for (int t = threadIdx.x; t < 2 * K; t += blockDim.x) rec[t] = A.tab[I.rec_off + 2 * trow + t];
  __syncthreads();
  for (int i = threadIdx.x; i < I.nr; i += blockDim.x) {
    Cx<T> acc = cx<T>(0, 0);
    if (A.recurrence) {
      // Pbar_m^m, Pbar_{m+1}^m = sqrt(2m+3) x Pbar_m^m, Pbar_n^m = a_n x Pbar_{n-1} - b_n Pbar_{n-2}
      const double x = A.tab[I.node_off + i];
      double p0 = A.tab[I.start_off + (int64_t)m * I.nr + i];
      double p1 = sqrt(2.0 * m + 3.0) * x * p0;
      double ar = (double)s[0].x * p0, ai = (double)s[0].y * p0;
      if (K > 1) {
        ar += (double)s[1].x * p1;
        ai += (double)s[1].y * p1;
      }
#pragma unroll 8
      for (int t = 2; t < K; ++t) {
        const double p2 = rec[2 * t] * x * p1 - rec[2 * t + 1] * p0;
        ar += (double)s[t].x * p2;
        ai += (double)s[t].y * p2;
        p0 = p1;
        p1 = p2;
      }
      acc = cx<T>((T)ar, (T)ai);
    } else {
      // eight independent partial sums keep eight table loads in flight
      const T* P = A.tabT + I.tb_off + trow * I.nr + i;
      Cx<T> part[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) part[u] = cx<T>(0, 0);
      int t = 0;
      for (; t + 8 <= K; t += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) part[u] = part[u] + scl(s[t + u], P[(int64_t)(t + u) * I.nr]);
      }
      for (; t < K; ++t) part[0] = part[0] + scl(s[t], P[(int64_t)t * I.nr]);
#pragma unroll
      for (int u = 1; u < 8; ++u) part[0] = part[0] + part[u];
      acc = part[0];
    }
    mix[i] = acc;
  }
  __syncthreads();
}

template <typename T>
__device__ void phase_phi(const BatchArgs<T>& A, int b, int q0, char* smem) {
  const BatchInst& I = A.inst[b];
  const int n = I.nphi, L = A.lines, np = L / 2;
  Cx<T>* X = reinterpret_cast<Cx<T>*>(smem);
  Cx<T>* Y = X + np * n;
  // the twiddle table follows the two line buffers (2 np n complex of T: a multiple of 16 bytes)
  Cx<double>* tw = reinterpret_cast<Cx<double>*>(smem + (size_t)2 * np * n * sizeof(Cx<T>));
  const double* twg = A.tab + I.tw_off;
  for (int e = threadIdx.x; e < n; e += blockDim.x) tw[e] = Cx<double>{twg[2 * e], twg[2 * e + 1]};
  Cx<T>* mix = A.mix + I.mix_off;
  for (int e = threadIdx.x; e < np * n; e += blockDim.x) X[e] = cx<T>(0, 0);
  __syncthreads();
  const int half = (n + 1) / 2;
  for (int e = threadIdx.x; e < np * half; e += blockDim.x) {
    const int p = e / half, m = e - p * half;
    if (m >= I.M) continue;
    const int qa = q0 + 2 * p, qb = qa + 1;
    const Cx<T> a = qa < I.nr ? mix[(int64_t)m * I.nr + qa] : cx<T>(0, 0);
    const Cx<T> c = qb < I.nr ? mix[(int64_t)m * I.nr + qb] : cx<T>(0, 0);
    if (m == 0) {
      X[p * n] = cx(a.x, c.x);
    } else {
      X[p * n + m] = cx(a.x - c.y, a.y + c.x);
      X[p * n + n - m] = cx(a.x + c.y, -a.y + c.x);
    }
  }
  __syncthreads();
  Cx<T>* Z = bfft<T>(X, Y, I, tw, true, np);
  for (int e = threadIdx.x; e < np * n; e += blockDim.x) {
    const Cx<T> v = Z[e];
    Z[e] = cx<T>(A.gamma * v.x * ((T)1 - v.x), A.gamma * v.y * ((T)1 - v.y));
  }
  __syncthreads();
  Cx<T>* W = bfft<T>(Z, Z == X ? Y : X, I, tw, false, np);
  const T sc = (T)1 / (T)n;
  for (int e = threadIdx.x; e < I.M * L; e += blockDim.x) {
    const int m = e / L, ll = e - m * L;
    const int q = q0 + ll;
    if (q >= I.nr) continue;
    const Cx<T>* Zp = W + (ll >> 1) * n;
    const Cx<T> zm = Zp[m % n];
    const Cx<T> zc = conjc(Zp[(n - m) % n]);
    Cx<T> v;
    if ((ll & 1) == 0) {
      v = scl(zm + zc, (T)0.5 * sc);
    } else {
      const Cx<T> d = zm - zc;
      v = cx<T>((T)0.5 * sc * d.y, -(T)0.5 * sc * d.x);
    }
    if (2 * m >= n || m > I.mkeep) v = cx<T>(0, 0);
    mix[(int64_t)m * I.nr + q] = v;
  }
  __syncthreads();
}

template <typename T>
__device__ void phase_forward(const BatchArgs<T>& A, int b, int m, char* smem) {
  const BatchInst& I = A.inst[b];
  const int K = I.nrc > m ? I.nrc - m : 0;
  if (K == 0) return;
  const int64_t trow = A.tri[I.tri_off + m];
  Cx<T>* out = A.spec_out + I.spec_off + trow;
  if (m > I.mkeep) {
    for (int t = threadIdx.x; t < K; t += blockDim.x) out[t] = cx<T>(0, 0);
    return;
  }
  Cx<T>* g = reinterpret_cast<Cx<T>*>(smem);
  const Cx<T>* mix = A.mix + I.mix_off + (int64_t)m * I.nr;
  for (int i = threadIdx.x; i < I.nr; i += blockDim.x) g[i] = mix[i];
  __syncthreads();
  const T* P = A.tabT + I.tf_off + trow * I.nr;
  for (int t = threadIdx.x; t < K; t += blockDim.x) {
    // eight independent partial sums keep eight table loads in flight
    Cx<T> part[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) part[u] = cx<T>(0, 0);
    int i = 0;
    for (; i + 8 <= I.nr; i += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) part[u] = part[u] + scl(g[i + u], P[(int64_t)(i + u) * K + t]);
    }
    for (; i < I.nr; ++i) part[0] = part[0] + scl(g[i], P[(int64_t)i * K + t]);
#pragma unroll
    for (int u = 1; u < 8; ++u) part[0] = part[0] + part[u];
    out[t] = part[0];
  }
  __syncthreads();
}

template <typename T, int PHASE>
__global__ void batch_kernel(BatchArgs<T> A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  for (int it = blockIdx.x; it < A.nitems[PHASE]; it += gridDim.x) {
    const int w = A.items[PHASE][it];
    if constexpr (PHASE == 0) phase_backward<T>(A, w >> 16, w & 0xffff, smem);
    else if constexpr (PHASE == 1) phase_phi<T>(A, w >> 16, w & 0xffff, smem);
    else phase_forward<T>(A, w >> 16, w & 0xffff, smem);
  }
}

size_t smem_bytes(const mlg_batch_s* bt, int lines) {
  size_t mx = 256 * sizeof(Cx<double>) + 512 * sizeof(double);
  const size_t cs = bt->prec == MLG_FP32 ? sizeof(Cx<float>) : sizeof(Cx<double>);
  // phase 2: two buffers of lines / 2 complex lines, then the twiddle table (nphi complex FP64)
  for (const auto& I : bt->inst)
    mx = std::max(mx, (size_t)2 * (lines / 2) * I.nphi * cs + (size_t)I.nphi * sizeof(Cx<double>));
  return mx;
}

template <typename T>
mlg_status run_batch(const mlg_batch_s* bt, double gamma, const void* in, void* out, void* ws, hipStream_t s,
                     const BatchConfig& c) {
  BatchArgs<T> A{};
  A.inst = bt->d_inst;
  A.tab = bt->d_tab;
  if constexpr (sizeof(T) == 8)
    A.tabT = reinterpret_cast<const T*>(bt->d_tab);
  else
    A.tabT = reinterpret_cast<const T*>(bt->d_tab32);
  A.tri = bt->d_tri;
  A.spec_in = reinterpret_cast<const Cx<T>*>(in);
  A.spec_out = reinterpret_cast<Cx<T>*>(out);
  A.mix = reinterpret_cast<Cx<T>*>(ws);
  for (int p = 0; p < 3; ++p) {
    A.items[p] = bt->d_items[p];
    A.nitems[p] = bt->nitems[p];
  }
  A.recurrence = c.recurrence;
  A.lines = c.lines;
  A.gamma = (T)gamma;
  const size_t shm = smem_bytes(bt, c.lines);
  // blocks per CU: the configured count, capped by what the phase kernels' registers and LDS allow
  int per_cu = 1 << 30;
  for (const void* k : {reinterpret_cast<const void*>(batch_kernel<T, 0>), reinterpret_cast<const void*>(batch_kernel<T, 1>),
                        reinterpret_cast<const void*>(batch_kernel<T, 2>)}) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, c.threads, shm);
    if (e != hipSuccess || n <= 0) return fail(MLG_E_DEVICE, "batch kernel does not fit on a CU");
    per_cu = std::min(per_cu, n);
  }
  const int blocks = std::max(1, std::min(per_cu, c.blocks_per_cu) * bt->cus);
  batch_kernel<T, 0><<<dim3(blocks), dim3(c.threads), shm, s>>>(A);
  batch_kernel<T, 1><<<dim3(blocks), dim3(c.threads), shm, s>>>(A);
  batch_kernel<T, 2><<<dim3(blocks), dim3(c.threads), shm, s>>>(A);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string("batch kernel launch: ") + hipGetErrorString(e));
  return MLG_OK;
}

using ld = long double;

}  // namespace

mlg_status batch_run(const mlg_batch_s* bt, double gamma, const void* in, void* out, void* ws, hipStream_t s,
                     const BatchConfig& c) {
  if (bt->prec == MLG_FP32) return run_batch<float>(bt, gamma, in, out, ws, s, c);
  return run_batch<double>(bt, gamma, in, out, ws, s, c);
}

size_t batch_smem(const mlg_batch_s* bt, int lines) { return smem_bytes(bt, lines); }

}  // namespace mlg

// ------------------------------------------------------------------------------------ host side
namespace mlg {
namespace {

template <typename V>
mlg_status up(V** dst, const std::vector<typename std::remove_pointer<V*>::type>& src) {
  using E = typename std::remove_pointer<V*>::type;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(src.size(), 1) * sizeof(E));
  if (e != hipSuccess) { *dst = nullptr; return fail(MLG_E_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e)); }
  if (!src.empty()) {
    e = hipMemcpy(*dst, src.data(), src.size() * sizeof(E), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(MLG_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  return MLG_OK;
}

void free_batch(mlg_batch_s* b) {
  if (!b) return;
  void* ptrs[] = {b->d_inst, b->d_tab, b->d_tab32, b->d_tri, b->d_items[0], b->d_items[1], b->d_items[2]};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete b;
}

// Work lists sorted by estimated cost, largest first.
mlg_status build_items(mlg_batch_s* bt, int lines) {
  struct W { double cost; int32_t code; };
  std::vector<W> w[3];
  for (int b = 0; b < bt->count; ++b) {
    const BatchInst& I = bt->inst[b];
    for (int m = 0; m < I.M; ++m) {
      const int K = std::max(I.nrc - m, 0);
      w[0].push_back({(m > I.mkeep ? 1.0 : (double)std::max(K, 1) * I.nr), (b << 16) | m});
      w[2].push_back({(m > I.mkeep ? 1.0 : (double)std::max(K, 1) * I.nr), (b << 16) | m});
    }
    for (int q = 0; q < I.nr; q += lines)
      w[1].push_back({(double)lines * I.nphi * std::log2((double)I.nphi + 1.0), (b << 16) | q});
  }
  for (int p = 0; p < 3; ++p) {
    std::stable_sort(w[p].begin(), w[p].end(), [](const W& a, const W& c) { return a.cost > c.cost; });
    std::vector<int32_t> codes(w[p].size());
    for (size_t i = 0; i < w[p].size(); ++i) codes[i] = w[p][i].code;
    if (bt->d_items[p]) (void)hipFree(bt->d_items[p]);
    bt->d_items[p] = nullptr;
    if (mlg_status st = up(&bt->d_items[p], codes)) return st;
    bt->nitems[p] = (int)codes.size();
    bt->items_host[p] = codes;
  }
  return MLG_OK;
}

}  // namespace
}  // namespace mlg

using namespace mlg;

extern "C" {

mlg_status mlg_batch_create(int count, const mlg_grid* grids, mlg_precision prec, int device, mlg_batch* out) {
  if (!out) return fail(MLG_E_ARG, "out is NULL");
  *out = nullptr;
  if (count <= 0 || count > 16384 || !grids) return fail(MLG_E_ARG, "count must be in [1, 16384] and grids non-NULL");
  if (prec != MLG_FP64 && prec != MLG_FP32) return fail(MLG_E_UNSUPPORTED, "batches support MLG_FP64 and MLG_FP32");
  for (int b = 0; b < count; ++b) {
    const mlg_grid& g = grids[b];
    if (!std::isfinite(g.ell) || !(g.ell > 0)) return fail(MLG_E_ARG, "ell must be positive and finite");
    if (g.nz != 1) return fail(MLG_E_UNSUPPORTED, "batched instances are 2D (N_z = 1)");
    if (g.nr < 2 || g.nr > 256) return fail(MLG_E_UNSUPPORTED, "batched instances need 2 <= N_r <= 256");
    if (g.nphi < 2 || g.nphi > 256) return fail(MLG_E_UNSUPPORTED, "batched instances need 2 <= N_phi <= 256");
    int r[16];
    if (factor_radices(g.nphi, r) < 0) return fail(MLG_E_UNSUPPORTED, "N_phi must have prime factors 2, 3, 5 only");
    if (g.nrc < 0 || g.nrc > g.nr) return fail(MLG_E_ARG, "N_r^c out of range");
    if (g.nphic < 0 || g.nphic > g.nphi / 2 + 1) return fail(MLG_E_ARG, "N_phi^c out of range");
    if (g.dealias != 0 && g.dealias != 1) return fail(MLG_E_ARG, "dealias must be 0 or 1");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(MLG_E_ARG, "device index out of range or no HIP device");
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return fail(MLG_E_DEVICE, "hipSetDevice failed");
  mlg_batch_s* bt = new (std::nothrow) mlg_batch_s();
  if (!bt) return fail(MLG_E_ALLOC, "host allocation failed");
  bt->count = count;
  bt->device = device;
  bt->prec = prec;
  hipDeviceProp_t prop;
  (void)hipGetDeviceProperties(&prop, device);
  bt->cus = prop.multiProcessorCount;
  std::vector<double> tab;
  std::vector<int64_t> tri;
  bt->spec_offsets.assign(count + 1, 0);
  int64_t mix = 0;
  for (int b = 0; b < count; ++b) {
    const mlg_grid& g = grids[b];
    BatchInst I{};
    I.nr = g.nr;
    I.nphi = g.nphi;
    I.nrc = g.nrc ? g.nrc : g.nr;
    I.M = g.nphic ? g.nphic : g.nphi / 2;
    I.mkeep = g.dealias ? (g.nphi - 1) / 3 : (1 << 30);
    I.nrad = factor_radices(g.nphi, I.rad);
    const int nr = I.nr, nrc = I.nrc, M = I.M;
    I.tri_off = (int64_t)tri.size();
    int64_t t = 0;
    for (int m = 0; m < M; ++m) {
      tri.push_back(t);
      t += std::max(nrc - m, 0);
    }
    tri.push_back(t);
    const int64_t tau = t;
    I.spec_off = bt->spec_offsets[b];
    bt->spec_offsets[b + 1] = I.spec_off + tau;
    I.mix_off = mix;
    mix += (int64_t)M * nr;
    std::vector<long double> th, wl;
    gl_theta(nr, th, wl);
    I.tb_off = (int64_t)tab.size();
    tab.resize(tab.size() + tau * nr);
    I.tf_off = (int64_t)tab.size();
    tab.resize(tab.size() + tau * nr);
    I.rec_off = (int64_t)tab.size();
    tab.resize(tab.size() + 2 * tau);
    I.start_off = (int64_t)tab.size();
    tab.resize(tab.size() + (int64_t)M * nr);
    I.node_off = (int64_t)tab.size();
    tab.resize(tab.size() + nr);
    I.tw_off = (int64_t)tab.size();
    tab.resize(tab.size() + 2 * g.nphi);
    std::vector<long double> col(nrc + 2);
    for (int i = 0; i < nr; ++i) tab[I.node_off + i] = (double)cosl(th[i]);
    for (int m = 0; m < M; ++m) {
      const int K = std::max(nrc - m, 0);
      if (K == 0) continue;
      const int64_t tr = tri[I.tri_off + m];
      for (int i = 0; i < nr; ++i) {
        pbar_col(m, nrc, th[i], col.data());
        tab[I.start_off + (int64_t)m * nr + i] = (double)col[0];
        for (int n = m; n < nrc; ++n) {
          tab[I.tb_off + (tr + n - m) * nr + i] = (double)col[n - m];
          tab[I.tf_off + tr * nr + (int64_t)i * K + (n - m)] = (double)(wl[i] * col[n - m]);
        }
      }
      for (int n = m; n < nrc; ++n) {
        ld a = 0, c = 0;
        if (n >= m + 2) {
          a = sqrtl((ld)(4 * n * n - 1) / (ld)(n * n - m * m));
          c = sqrtl((ld)((2 * n + 1) * (n - 1 - m) * (n - 1 + m)) / (ld)((2 * n - 3) * (n * n - m * m)));
        }
        tab[I.rec_off + 2 * (tr + n - m)] = (double)a;
        tab[I.rec_off + 2 * (tr + n - m) + 1] = (double)c;
      }
    }
    const ld pi = acosl(-1.0L);
    for (int q = 0; q < g.nphi; ++q) {
      tab[I.tw_off + 2 * q] = (double)cosl(-2 * pi * q / g.nphi);
      tab[I.tw_off + 2 * q + 1] = (double)sinl(-2 * pi * q / g.nphi);
    }
    bt->inst.push_back(I);
  }
  bt->spec_total = bt->spec_offsets[count];
  bt->mix_total = mix;
  bt->ws_bytes = (size_t)mix * (prec == MLG_FP32 ? 8 : 16) + 256;
  mlg_status st;
  if ((st = up(&bt->d_inst, bt->inst)) || (st = up(&bt->d_tab, tab)) || (st = up(&bt->d_tri, tri))) {
    free_batch(bt);
    if (prev >= 0) (void)hipSetDevice(prev);
    return st;
  }
  if (prec == MLG_FP32) {
    std::vector<float> t32(tab.begin(), tab.end());
    if ((st = up(&bt->d_tab32, t32))) {
      free_batch(bt);
      if (prev >= 0) (void)hipSetDevice(prev);
      return st;
    }
  }
  if ((st = build_items(bt, bt->cfg.lines))) {
    free_batch(bt);
    if (prev >= 0) (void)hipSetDevice(prev);
    return st;
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  *out = bt;
  return MLG_OK;
}

mlg_status mlg_batch_destroy(mlg_batch b) {
  free_batch(b);
  return MLG_OK;
}

mlg_status mlg_batch_query(mlg_batch b, int64_t* spec_offsets, int64_t* workspace_bytes) {
  if (!b) return fail(MLG_E_ARG, "batch is NULL");
  if (spec_offsets)
    for (int i = 0; i <= b->count; ++i) spec_offsets[i] = b->spec_offsets[i];
  if (workspace_bytes) *workspace_bytes = (int64_t)b->ws_bytes;
  return MLG_OK;
}

mlg_status mlg_batch_rhs_scalar(mlg_batch b, double gamma, const void* spec_in, void* spec_out, void* ws,
                                void* stream) {
  if (!b) return fail(MLG_E_ARG, "batch is NULL");
  if (!spec_in || !spec_out || !ws) return fail(MLG_E_ARG, "null buffer");
  if (spec_in == spec_out) return fail(MLG_E_ARG, "spec_in and spec_out must not alias");
  if (!std::isfinite(gamma)) return fail(MLG_E_ARG, "gamma must be finite");
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->device);
  mlg_status st = batch_run(b, gamma, spec_in, spec_out, ws, static_cast<hipStream_t>(stream), b->cfg);
  if (prev >= 0) (void)hipSetDevice(prev);
  return st;
}

mlg_status mlg_batch_set_config(mlg_batch b, const mlg_batch_config* c) {
  if (!b || !c) return fail(MLG_E_ARG, "null argument");
  if ((c->recurrence != 0 && c->recurrence != 1) || (c->threads != 64 && c->threads != 128 && c->threads != 256) ||
      c->blocks_per_cu < 1 || c->blocks_per_cu > 8 || c->lines < 2 || c->lines > 32 || (c->lines & 1))
    return fail(MLG_E_ARG, "invalid batch configuration");
  const size_t shm = batch_smem(b, c->lines);
  if (shm > 65536) return fail(MLG_E_ARG, "configuration needs more than 64 KiB of LDS");
  BatchConfig nc{c->recurrence, c->threads, c->blocks_per_cu, c->lines};
  if (nc.lines != b->cfg.lines) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    mlg_status st = build_items(b, nc.lines);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (st) return st;
  }
  b->cfg = nc;
  return MLG_OK;
}

mlg_status mlg_batch_get_config(mlg_batch b, mlg_batch_config* c) {
  if (!b || !c) return fail(MLG_E_ARG, "null argument");
  c->recurrence = b->cfg.recurrence;
  c->threads = b->cfg.threads;
  c->blocks_per_cu = b->cfg.blocks_per_cu;
  c->lines = b->cfg.lines;
  return MLG_OK;
}

mlg_status mlg_batch_autotune(mlg_batch b, double gamma, const void* spec_in, void* spec_out, void* ws, void* stream,
                              mlg_batch_config* chosen, double* best_ms) {
  if (!b) return fail(MLG_E_ARG, "batch is NULL");
  if (!spec_in || !spec_out || !ws) return fail(MLG_E_ARG, "null buffer");
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(MLG_E_DEVICE, "hipEventCreate failed");
  const int lines_c[] = {4, 8, 16};
  const int thr_c[] = {128, 256};
  const int bpc_c[] = {1, 2, 4, 8};
  BatchConfig best = b->cfg;
  float best_t = 1e30f;
  mlg_status st = MLG_OK;
  for (int lines : lines_c) {
    if (batch_smem(b, lines) > 65536) continue;
    if ((st = build_items(b, lines))) break;
    for (int rec = 0; rec < 2; ++rec)
      for (int thr : thr_c)
        for (int bpc : bpc_c) {
          BatchConfig c{rec, thr, bpc, lines};
          if ((st = batch_run(b, gamma, spec_in, spec_out, ws, s, c))) break;  // warm-up
          (void)hipEventRecord(e0, s);
          for (int r = 0; r < 3; ++r)
            if ((st = batch_run(b, gamma, spec_in, spec_out, ws, s, c))) break;
          (void)hipEventRecord(e1, s);
          if (st) break;
          (void)hipEventSynchronize(e1);
          float ms = 0;
          (void)hipEventElapsedTime(&ms, e0, e1);
          ms /= 3;
          if (ms < best_t) {
            best_t = ms;
            best = c;
          }
        }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == MLG_OK) st = build_items(b, best.lines);
  if (st == MLG_OK) {
    b->cfg = best;
    b->tuned = 1;
    if (chosen) {
      chosen->recurrence = best.recurrence;
      chosen->threads = best.threads;
      chosen->blocks_per_cu = best.blocks_per_cu;
      chosen->lines = best.lines;
    }
    if (best_ms) *best_ms = best_t;
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  return st;
}

}  // extern "C"
