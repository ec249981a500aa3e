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

}  // namespace dev
}  // namespace mlg
