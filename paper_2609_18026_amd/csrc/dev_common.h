// Device-side complex helpers shared by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>

namespace mlg {
namespace dev {

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

// The chip dispatches the blocks of a launch to its 8 XCDs round-robin (block b to XCD b mod 8),
// and each XCD has its own L2.  For per-order products (tiles x, y of order z share the order's
// tables) xcd_tile deals whole orders to the XCDs in turn: XCD c runs the gx * gy tiles of order
// c, then those of c + 8, and so on, so that one L2 serves each order's tables and the triangular
// work (which shrinks with the order) is spread evenly.  The launch has xcd_blocks(gx, gy, gz)
// blocks; xcd_tile returns false for the padding blocks of the last round.
struct Tile3 {
  int x, y, z;
};
__device__ __forceinline__ bool xcd_tile(int gx, int gy, int gz, Tile3& t) {
  const int per = gx * gy;
  const int b = blockIdx.x;
  const int c = b & 7, slot = b >> 3;
  const int tile = slot % per;
  t.z = c + 8 * (slot / per);
  t.x = tile % gx;
  t.y = tile / gx;
  return t.z < gz;
}
__host__ __device__ inline unsigned xcd_blocks(int gx, int gy, int gz) {
  return 8u * (unsigned)gx * (unsigned)gy * (unsigned)((gz + 7) / 8);
}

// Storage conversions: reduced-precision plans keep fields as float / float2 in memory while the
// kernels compute in double.
__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ double2 ld2(const float2* p) {
  const float2 v = *p;
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 to_d2(double2 a) { return a; }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double ld1(const double* p) { return *p; }
__device__ __forceinline__ double ld1(const float* p) { return (double)*p; }
__device__ __forceinline__ void st1(double* p, double v) { *p = v; }
__device__ __forceinline__ void st1(float* p, double v) { *p = (float)v; }
template <typename S2>
__device__ __forceinline__ S2 czero();
template <>
__device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
template <>
__device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }

}  // namespace dev
}  // namespace mlg
