// Shared host/device definitions for the dfx library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <utility>

namespace dfx {

// ---- status / errors -------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
void set_last_error(const std::string& m);

#define DFX_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::dfx::Error(-3, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

// ---- B layout: packed lower triangle of 32x32 function tiles ---------------
// Element (r, c) with r >= c lives in tile (I, J) = (r / 32, c / 32), I >= J, at
// (I (I + 1) / 2 + J) * 1024 + (r % 32) * 32 + c % 32.  Diagonal tiles (I == J)
// hold both triangles.  Functions beyond nbf in the last tile are zero.
constexpr int TILE = 32;
constexpr int TILE2 = TILE * TILE;

__host__ __device__ inline int64_t tile_base(int I, int J) {
  return ((int64_t)I * (I + 1) / 2 + J) * TILE2;
}
__host__ __device__ inline int ntiles_for(int nbf) { return (nbf + TILE - 1) / TILE; }
__host__ __device__ inline int64_t tiled_cols(int nbf) {
  const int nt = ntiles_for(nbf);
  return (int64_t)nt * (nt + 1) / 2 * TILE2;
}

// ---- device view of a shell set --------------------------------------------
struct DevShells {
  const double* ctr;   // [nsh][3]
  const int* l;        // [nsh]
  const int* nprim;    // [nsh]
  const int* poff;     // [nsh] first primitive
  const int* foff;     // [nsh] first spherical function
  const double* exps;  // [nprim total]
  const double* coef;  // [nprim total], multiplies x^i y^j z^k exp(-a r^2)
  int nsh;
};

// ---- compile-time helpers ---------------------------------------------------
__host__ __device__ constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
// power of axis (0 = x, 1 = y, 2 = z) in Cartesian component c of degree l;
// components run x-power descending, then y-power descending.
__host__ __device__ constexpr int cpow(int l, int c, int axis) {
  int n = 0;
  for (int i = l; i >= 0; --i)
    for (int j = l - i; j >= 0; --j) {
      if (n == c) return axis == 0 ? i : (axis == 1 ? j : l - i - j);
      ++n;
    }
  return -1;
}

template <typename F, int... I>
__host__ __device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
// f(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time
template <int N, typename F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

}  // namespace dfx
