// Rys quadrature roots and weights on gfx950 (device side).
//
// The electron-repulsion integrals are evaluated by Rys quadrature (Dupuis,
// Rys & King 1976), the algorithm the paper names in its section "Molecular
// integrals".  For n roots and argument T the quadrature nodes u_i = t_i^2 and
// weights w_i satisfy sum_i w_i u_i^m = F_m(T) (the Boys function) for
// m < 2n.  They come from piecewise polynomial tables (gen_rys_tables.py),
// staged into LDS by each workgroup, and from the large-T Hermite limit.
#pragma once
#include "common.h"
#include "rys_tables.inc"

namespace dfx {

// Device table: for each n, RYS_NINT[n] intervals of [2n functions][RYS_DEG + 1]
// coefficients, each interval padded to an odd number of doubles (rys_blk), then
// n values x_i^2 and n values W_i of the large-T limit.  The lanes of a wave read
// the same coefficient of different intervals; with an even stride (2n (RYS_DEG
// + 1) doubles) those reads fall on a few LDS banks, with an odd one they spread
// over all of them.
__host__ __device__ constexpr int rys_blk(int n) {
  return (2 * n * (RYS_DEG + 1)) | 1;
}
__host__ __device__ constexpr int rys_dev_size(int n) {
  return RYS_NINT[n] * rys_blk(n) + 2 * n;
}
__host__ __device__ constexpr int rys_dev_off(int n) {
  int s = 0;
  for (int m = 1; m < n; ++m) s += rys_dev_size(m);
  return s;
}
constexpr int RYS_DEV_TOTAL = rys_dev_off(RYS_NMAX + 1);

// Per-triplet state: where the root polynomials of this T live.
template <int NR>
struct RysPoint {
  const double* blk;  // coefficient block of the interval (LDS), or the asymptotic constants
  double x;           // local variable of the interval, or 1/T
  double s;           // 1/sqrt(T) in the asymptotic regime
  bool asym;
  __device__ __forceinline__ RysPoint(const double* tab, double T) {
    constexpr double tmax = RYS_TMAX[NR];
    constexpr double h = RYS_HN[NR];
    constexpr double ih = 1.0 / RYS_HN[NR];
    asym = !(T < tmax);
    if (asym) {
      blk = tab + RYS_NINT[NR] * rys_blk(NR);
      x = 1.0 / T;
      s = sqrt(x);
    } else {
      const int k = (int)(T * ih);
      blk = tab + k * rys_blk(NR);
      x = (T - ((double)k * h + 0.5 * h)) * (2.0 * ih);
      s = 0.0;
    }
  }
  __device__ __forceinline__ static double horner(const double* c, double x) {
    double r = c[0];
#pragma unroll
    for (int j = 1; j <= RYS_DEG; ++j) r = fma(r, x, c[j]);
    return r;
  }
  // root u_i and weight w_i
  __device__ __forceinline__ void get(int i, double& u, double& w) const {
    if (asym) {
      u = blk[i] * x;
      w = blk[NR + i] * s;
    } else {
      u = horner(blk + i * (RYS_DEG + 1), x);
      w = horner(blk + (NR + i) * (RYS_DEG + 1), x);
    }
  }
};

// Stage the table for NR roots from global memory into LDS.
template <int NR>
__device__ __forceinline__ void rys_stage(double* lds, const double* __restrict__ g) {
  constexpr int N = rys_dev_size(NR);
  const double* src = g + rys_dev_off(NR);
  for (int i = threadIdx.x; i < N; i += blockDim.x) lds[i] = src[i];
  __syncthreads();
}

// Host: build the device-side table image (coefficients + asymptotic constants).
void rys_host_image(double* out /* RYS_DEV_TOTAL */);

}  // namespace dfx
