// Pieces of the DF-RHF gradient other than the three-index and metric
// derivative integrals: the one-electron derivative terms (overlap, kinetic,
// nuclear attraction) and the element-wise steps that assemble the weights of
// the fitted-integral terms.
//
// One-electron terms, 2 tr(D h^x) - 2 tr(W S^x) with h = T + V: per shell pair
// the Cartesian weight blocks T_a^T (2D) T_b and T_a^T (2W) T_b (the solid-
// harmonic transforms folded in, both orders of an off-diagonal pair counted)
// are formed once; the derivative integrals are then accumulated as scalars.
// Overlap and kinetic factors per axis come from the Obara-Saika overlap
// recurrence with a horizontal transfer, the kinetic one as
// -1/2 [4 b^2 S(i, j+2) - 2 b (2j+1) S(i, j) + j (j-1) S(i, j-2)]; the nuclear
// attraction by Rys quadrature.  Moving a basis centre differentiates its
// Gaussian into 2 alpha x^(i+1) - i x^(i-1); the attraction operator of nucleus
// C moves with C, and since the integral depends on A - C and B - C only, its
// derivative is minus the sum of the two basis-centre derivatives.
#include "grad_kernel.h"

namespace dfx {

// Cartesian weights of one pair: w[i][j] = f s sum_{ma, mb} T_a[ma][i] T_b[mb][j] M[a+ma][b+mb],
// f = 2 for a != b (both orders of the block), for M = D and M = W and the
// energy's factor s = 2 (2 tr D h - 2 tr W S)
template <int LA, int LB>
__global__ void onee_wcart_kernel(OneEGradArgs g, const double* __restrict__ Dw, const double* __restrict__ Ww,
                                  int n, double scale, double* __restrict__ wD, double* __restrict__ wW) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.npairs) return;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  const int sa = g.pf[p], sb = g.ps[p];
  const int fa = g.sh.foff[sa], fb = g.sh.foff[sb];
  const double f = (sa != sb ? 2.0 : 1.0) * scale;
  const int64_t o = g.woff[p];
  sfor<NA>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    sfor<NB>([&](auto ij) {
      constexpr int j = decltype(ij)::value;
      double vd = 0.0, vw = 0.0;
      sfor<2 * LA + 1>([&](auto mai) {
        constexpr int ma = decltype(mai)::value;
        constexpr double ta = sph<LA>(ma, i);
        if constexpr (ta != 0.0)
          sfor<2 * LB + 1>([&](auto mbi) {
            constexpr int mb = decltype(mbi)::value;
            constexpr double tb = sph<LB>(mb, j);
            if constexpr (tb != 0.0) {
              const int64_t e = (int64_t)(fa + ma) * n + fb + mb;
              vd = fma(ta * tb, Dw[e], vd);
              vw = fma(ta * tb, Ww[e], vw);
            }
          });
      });
      wD[o + i * NB + j] = f * vd;
      wW[o + i * NB + j] = f * vw;
    });
  });
}

// 2 alpha F(i + 1) - i F(i - 1) along the moved index (M 0: first, 1: second)
template <int M, int i, int j, class FT>
__device__ __forceinline__ double dmove(const FT& F, double ex2) {
  if constexpr (M == 0) {
    double v = ex2 * F[i + 1][j];
    if constexpr (i > 0) v = fma(-(double)i, F[i - 1][j], v);
    return v;
  } else {
    double v = ex2 * F[i][j + 1];
    if constexpr (j > 0) v = fma(-(double)j, F[i][j - 1], v);
    return v;
  }
}

template <int LA, int LB>
__global__ void __launch_bounds__(64) onee_grad_kernel(OneEGradArgs g) {
  constexpr int NA = ncart(LA), NB = ncart(LB);
  constexpr int NR = (LA + LB + 1) / 2 + 1;
  __shared__ double tab[rys_dev_size(NR)];
  rys_stage<NR>(tab, g.rys);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < g.npairs;
  const int pp = live ? p : g.npairs - 1;
  const int s1 = g.pf[pp], s2 = g.ps[pp];
  const double A[3] = {g.sh.ctr[3 * s1], g.sh.ctr[3 * s1 + 1], g.sh.ctr[3 * s1 + 2]};
  const double B[3] = {g.sh.ctr[3 * s2], g.sh.ctr[3 * s2 + 1], g.sh.ctr[3 * s2 + 2]};
  const double AB[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
  const double rab2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
  const int64_t wo = g.woff[pp];
  double gA[3] = {0.0, 0.0, 0.0}, gB[3] = {0.0, 0.0, 0.0};

  // ---- overlap and kinetic
  for (int i1 = 0; i1 < (live ? g.sh.nprim[s1] : 0); ++i1)
    for (int j1 = 0; j1 < g.sh.nprim[s2]; ++j1) {
      const double al = g.sh.exps[g.sh.poff[s1] + i1], be = g.sh.exps[g.sh.poff[s2] + j1];
      const double pp_ = al + be, h = 0.5 / pp_;
      const double pref = g.sh.coef[g.sh.poff[s1] + i1] * g.sh.coef[g.sh.poff[s2] + j1] *
                          exp(-al * be / pp_ * rab2) * pow(M_PI / pp_, 1.5);
      constexpr int E = LA + LB + 4;
      double S[3][LA + 2][LB + 4], T[3][LA + 2][LB + 2];
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        const double PA = -be / pp_ * AB[x];
        double G[E + 1];
        G[0] = 1.0;
#pragma unroll
        for (int e = 0; e < E; ++e) G[e + 1] = PA * G[e] + (e > 0 ? e * h * G[e - 1] : 0.0);
#pragma unroll
        for (int i = 0; i < LA + 2; ++i) S[x][i][0] = G[i];
#pragma unroll
        for (int b = 1; b < LB + 4; ++b) {
#pragma unroll
          for (int e = 0; e <= E - b; ++e) G[e] = G[e + 1] + AB[x] * G[e];
#pragma unroll
          for (int i = 0; i < LA + 2; ++i) S[x][i][b] = G[i];
        }
#pragma unroll
        for (int i = 0; i < LA + 2; ++i)
#pragma unroll
          for (int j = 0; j < LB + 2; ++j) {
            double t = 4.0 * be * be * S[x][i][j + 2] - 2.0 * be * (2 * j + 1) * S[x][i][j];
            if (j >= 2) t += j * (j - 1) * S[x][i][j >= 2 ? j - 2 : 0];
            T[x][i][j] = -0.5 * t;
          }
      }
      const double a2 = 2.0 * al, b2 = 2.0 * be;
      sfor<NA>([&](auto ia) {
        constexpr int i = decltype(ia)::value;
        constexpr int ax = cpow(LA, i, 0), ay = cpow(LA, i, 1), az = cpow(LA, i, 2);
        sfor<NB>([&](auto ib) {
          constexpr int j = decltype(ib)::value;
          constexpr int bx = cpow(LB, j, 0), by = cpow(LB, j, 1), bz = cpow(LB, j, 2);
          const double wd = pref * g.wD[wo + i * NB + j], ww = pref * g.wW[wo + i * NB + j];
          const double sx = S[0][ax][bx], sy = S[1][ay][by], sz = S[2][az][bz];
          const double tx = T[0][ax][bx], ty = T[1][ay][by], tz = T[2][az][bz];
          // x
          {
            const double dsa = dmove<0, ax, bx>(S[0], a2), dta = dmove<0, ax, bx>(T[0], a2);
            const double dsb = dmove<1, ax, bx>(S[0], b2), dtb = dmove<1, ax, bx>(T[0], b2);
            const double o = ty * sz + sy * tz;
            gA[0] += wd * (dta * sy * sz + dsa * o) - ww * dsa * sy * sz;
            gB[0] += wd * (dtb * sy * sz + dsb * o) - ww * dsb * sy * sz;
          }
          {
            const double dsa = dmove<0, ay, by>(S[1], a2), dta = dmove<0, ay, by>(T[1], a2);
            const double dsb = dmove<1, ay, by>(S[1], b2), dtb = dmove<1, ay, by>(T[1], b2);
            const double o = tx * sz + sx * tz;
            gA[1] += wd * (dta * sx * sz + dsa * o) - ww * dsa * sx * sz;
            gB[1] += wd * (dtb * sx * sz + dsb * o) - ww * dsb * sx * sz;
          }
          {
            const double dsa = dmove<0, az, bz>(S[2], a2), dta = dmove<0, az, bz>(T[2], a2);
            const double dsb = dmove<1, az, bz>(S[2], b2), dtb = dmove<1, az, bz>(T[2], b2);
            const double o = tx * sy + sx * ty;
            gA[2] += wd * (dta * sx * sy + dsa * o) - ww * dsa * sx * sy;
            gB[2] += wd * (dtb * sx * sy + dsb * o) - ww * dsb * sx * sy;
          }
        });
      });
    }

  // ---- nuclear attraction, nucleus by nucleus
  for (int c = 0; c < g.natom; ++c) {
    double gc[3] = {0.0, 0.0, 0.0};
    for (int i1 = 0; i1 < (live ? g.sh.nprim[s1] : 0); ++i1)
      for (int j1 = 0; j1 < g.sh.nprim[s2]; ++j1) {
        const double al = g.sh.exps[g.sh.poff[s1] + i1], be = g.sh.exps[g.sh.poff[s2] + j1];
        const double pp_ = al + be;
        const double cf = g.sh.coef[g.sh.poff[s1] + i1] * g.sh.coef[g.sh.poff[s2] + j1] *
                          exp(-al * be / pp_ * rab2) * 2.0 * M_PI / pp_;
        // P - A = b (B - A) / p, P - C = (P - A) + (A - C): exact for concentric centres
        const double PA[3] = {-be / pp_ * AB[0], -be / pp_ * AB[1], -be / pp_ * AB[2]};
        const double PC[3] = {PA[0] + (A[0] - g.xyz[3 * c]), PA[1] + (A[1] - g.xyz[3 * c + 1]),
                              PA[2] + (A[2] - g.xyz[3 * c + 2])};
        const double Tb = pp_ * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
        const double z = -g.Z[c] * cf;
        const RysPoint<NR> rp(tab, Tb);
        const double a2 = 2.0 * al, b2 = 2.0 * be;
#pragma unroll 1
        for (int r = 0; r < NR; ++r) {
          double u, w;
          rp.get(r, u, w);
          const double B10 = 0.5 / pp_ * (1.0 - u);
          constexpr int E = LA + LB + 1;
          double H[3][LA + 2][LB + 2];
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            const double C00 = PA[x] - u * PC[x];
            double G[E + 1];
            G[0] = (x == 2) ? w * z : 1.0;
#pragma unroll
            for (int e = 0; e < E; ++e) G[e + 1] = C00 * G[e] + (e > 0 ? e * B10 * G[e - 1] : 0.0);
#pragma unroll
            for (int i = 0; i < LA + 2; ++i) H[x][i][0] = i <= E ? G[i <= E ? i : 0] : 0.0;
#pragma unroll
            for (int b = 1; b < LB + 2; ++b) {
#pragma unroll
              for (int e = 0; e <= E - b; ++e) G[e] = G[e + 1] + AB[x] * G[e];
#pragma unroll
              for (int i = 0; i < LA + 2; ++i) H[x][i][b] = i <= E - b ? G[i <= E - b ? i : 0] : 0.0;
            }
          }
          sfor<NA>([&](auto ia) {
            constexpr int i = decltype(ia)::value;
            constexpr int ax = cpow(LA, i, 0), ay = cpow(LA, i, 1), az = cpow(LA, i, 2);
            sfor<NB>([&](auto ib) {
              constexpr int j = decltype(ib)::value;
              constexpr int bx = cpow(LB, j, 0), by = cpow(LB, j, 1), bz = cpow(LB, j, 2);
              const double wd = g.wD[wo + i * NB + j];
              const double hx = H[0][ax][bx], hy = H[1][ay][by], hz = H[2][az][bz];
              const double dax = dmove<0, ax, bx>(H[0], a2) * hy * hz, dbx = dmove<1, ax, bx>(H[0], b2) * hy * hz;
              const double day = hx * dmove<0, ay, by>(H[1], a2) * hz, dby = hx * dmove<1, ay, by>(H[1], b2) * hz;
              const double daz = hx * hy * dmove<0, az, bz>(H[2], a2), dbz = hx * hy * dmove<1, az, bz>(H[2], b2);
              gA[0] = fma(wd, dax, gA[0]); gB[0] = fma(wd, dbx, gB[0]); gc[0] -= wd * (dax + dbx);
              gA[1] = fma(wd, day, gA[1]); gB[1] = fma(wd, dby, gB[1]); gc[1] -= wd * (day + dby);
              gA[2] = fma(wd, daz, gA[2]); gB[2] = fma(wd, dbz, gB[2]); gc[2] -= wd * (daz + dbz);
            });
          });
        }
      }
    // the workgroup is one wave: sum the nucleus's share over its lanes
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double t = gc[k];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
      if (threadIdx.x == 0) g.nbuf[((int64_t)blockIdx.x * g.natom + c) * 3 + k] = t;
    }
  }
  if (live)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      g.pbuf[(int64_t)p * 6 + k] = gA[k];
      g.pbuf[(int64_t)p * 6 + 3 + k] = gB[k];
    }
}

void onee_grad_dispatch(int LA, int LB, OneEGradArgs g, const double* Dw, const double* Ww, int n, double scale,
                        double* wD, double* wW, hipStream_t st) {
  const dim3 blk(64), grd((g.npairs + 63) / 64);
#define OG(X, Y)                                                                                     \
  case X * 8 + Y:                                                                                     \
    hipLaunchKernelGGL((onee_wcart_kernel<X, Y>), grd, blk, 0, st, g, Dw, Ww, n, scale, wD, wW);     \
    hipLaunchKernelGGL((onee_grad_kernel<X, Y>), grd, blk, 0, st, g);                                 \
    break;
  switch (LA * 8 + LB) {
    OG(0, 0) OG(0, 1) OG(0, 2) OG(0, 3) OG(1, 0) OG(1, 1) OG(1, 2) OG(1, 3)
    OG(2, 0) OG(2, 1) OG(2, 2) OG(2, 3) OG(3, 0) OG(3, 1) OG(3, 2) OG(3, 3)
    default: throw Error(DFX_EUNSUPPORTED, "one-electron gradient: unsupported angular momentum class");
  }
#undef OG
}

// ---- assembly of the fitted-integral weights ----------------------------------------

// Gam~ in raw's packed columns for rows q0.. of a chunk: out[q][c] = 4 gam_q D[mu][nu]
// + T[q][mu][nu], (mu, nu) = cols[c] (T = -2 D X_q C^T, dense per row of the chunk)
__global__ void gam_pack_kernel(const double* __restrict__ T, const double* __restrict__ D, int nbf,
                                const double* __restrict__ gam, const int* __restrict__ cmu,
                                const int* __restrict__ cnu, int64_t ncols, double* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int q = blockIdx.y;
  const int64_t e = (int64_t)cmu[c] * nbf + cnu[c];
  out[(int64_t)q * ncols + c] = fma(4.0 * gam[q], D[e], T[(int64_t)q * nbf * nbf + e]);
}

// M -= 2 gam gam^T (n x n)
__global__ void rank1_kernel(double* __restrict__ M, const double* __restrict__ gam, int n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n) return;
  M[i] = fma(-2.0 * gam[i / n], gam[i % n], M[i]);
}

// B = A^T (n x n)
__global__ void transpose_kernel(const double* __restrict__ A, double* __restrict__ B, int n) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = by + k, c = bx + threadIdx.x;
    if (r < n && c < n) t[k][threadIdx.x] = A[(int64_t)r * n + c];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int r = bx + k, c = by + threadIdx.x;
    if (r < n && c < n) B[(int64_t)r * n + c] = t[threadIdx.x][k];
  }
}

// Ce[mu][i] = C[mu][i] eps[i]
__global__ void scale_cols_kernel(const double* __restrict__ C, const double* __restrict__ eps, int n, int no,
                                  double* __restrict__ Ce) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * no) return;
  Ce[i] = C[i] * eps[i % no];
}

void gam_pack(const double* T, const double* D, int nbf, const double* gam, const int* cmu, const int* cnu,
              int64_t ncols, int nq, double* out, hipStream_t st) {
  if (nq <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(gam_pack_kernel, dim3((unsigned)((ncols + 255) / 256), nq), dim3(256), 0, st, T, D, nbf, gam,
                     cmu, cnu, ncols, out);
}
void rank1_sub2(double* M, const double* gam, int n, hipStream_t st) {
  const int64_t t = (int64_t)n * n;
  hipLaunchKernelGGL(rank1_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, M, gam, n);
}
void transpose_sq(const double* A, double* B, int n, hipStream_t st) {
  const dim3 g((n + 31) / 32, (n + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, g, dim3(32, 8), 0, st, A, B, n);
}
void scale_cols(const double* C, const double* eps, int n, int no, double* Ce, hipStream_t st) {
  const int64_t t = (int64_t)n * no;
  hipLaunchKernelGGL(scale_cols_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, C, eps, n, no, Ce);
}

}  // namespace dfx
