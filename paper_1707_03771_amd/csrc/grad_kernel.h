// Nuclear-coordinate derivatives of the three-index integrals (mu nu|P) and of
// the metric (P|Q) by Rys quadrature, contracted on the fly with the weights
// of the DF-RHF gradient (Gam, in raw's packed pair columns, for (mu nu|P);
// Gam2, dense, for (P|Q)).  Section "Molecular integrals" names the integral
// derivatives beside the integrals.
//
// One instantiation per class (LA, LB | LC), ket group, moved centre WHICH (0:
// the lane's first shell, 1: its second) and Cartesian axis AXIS.  Moving a
// centre differentiates its Gaussian into 2 alpha x^(a+1) - a x^(a-1), so the
// 2D integrals are built one order higher on that centre (the ERI kernel's
// recurrences with LA + 1 or LB + 1) and only the AXIS direction is
// differentiated in each product.  The ket centre is not differentiated: the
// integrals depend on the centres' differences only, so its derivative is
// minus the sum of the two bra derivatives, and each launch hands the ket
// minus its own share.
//
// Output, summed in a fixed order on the host: per lane (pair) and ket chunk,
// its weighted derivative; per workgroup and ket shell, minus the sum over the
// workgroup's lanes.
#pragma once
#include "eri3_kernel.h"
#include "kernels.h"

namespace dfx {

struct GradArgs {
  Eri3Args e;              // lists, shells, Rys table; out/ld unused
  const double* gam;       // Gam [P][ldg] (raw's columns, class by class) or Gam2 [P][Q] (UNITB)
  int64_t ldg;
  double* pbuf;            // [gridDim.y][npairs]: per lane and ket chunk
  double* kbuf;            // [nk][gridDim.x]: per ket shell and workgroup
  double scale_off;        // weight of a pair of two different shells (2: both orders)
};

// d/dR along the differentiated direction of one 2D factor: the moved
// centre's power pa (WHICH 0) or pb (WHICH 1) goes up and down by one
template <int WHICH, int pa, int pb, int pc, class HT>
__device__ __forceinline__ double dfac(const HT& H, double ex2) {
  if constexpr (WHICH == 0) {
    double v = ex2 * H[pa + 1][pb][pc];
    if constexpr (pa > 0) v = fma(-(double)pa, H[pa - 1][pb][pc], v);
    return v;
  } else {
    double v = ex2 * H[pa][pb + 1][pc];
    if constexpr (pb > 0) v = fma(-(double)pb, H[pa][pb - 1][pc], v);
    return v;
  }
}

template <int LA, int LB, int LC, int M0, int GN, bool UNITB, int WHICH, int AXIS>
__global__ void __launch_bounds__(ERI_THREADS) eri3_grad_kernel(const GradArgs ga) {
  const Eri3Args& a = ga.e;
  constexpr int XA = LA + (WHICH == 0), XB = LB + (WHICH == 1);
  constexpr int NR = (XA + XB + LC) / 2 + 1;
  constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC);
  constexpr int SA = 2 * LA + 1, SB = UNITB ? 1 : 2 * LB + 1;
  __shared__ double tab[rys_dev_size(NR)];
  __shared__ double red[ERI_THREADS / 64];
  rys_stage<NR>(tab, a.rys);

  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = p < a.npairs;
  const int pp = live ? p : a.npairs - 1;
  const int f = a.pf[pp];
  const int s = UNITB ? f : a.ps[pp];
  const double A0 = a.F.ctr[3 * f], A1 = a.F.ctr[3 * f + 1], A2 = a.F.ctr[3 * f + 2];
  const double B0 = UNITB ? A0 : a.S.ctr[3 * s], B1 = UNITB ? A1 : a.S.ctr[3 * s + 1],
               B2 = UNITB ? A2 : a.S.ctr[3 * s + 2];
  const int nfp = a.F.nprim[f], fpo = a.F.poff[f];
  const int nsp = UNITB ? 1 : a.S.nprim[s], spo = UNITB ? 0 : a.S.poff[s];
  const int foffF = a.F.foff[f];
  const double qab = a.pq ? a.pq[pp] : 1.0;
  // a pair of two different shells stands for both orders of its block
  const double wpair = (!UNITB && f != s) ? ga.scale_off : 1.0;
  const double AB0 = A0 - B0, AB1 = A1 - B1, AB2 = A2 - B2;
  const double rAB2 = AB0 * AB0 + AB1 * AB1 + AB2 * AB2;
  constexpr double TWO_PI_52 = 34.98683665524972;  // 2 pi^(5/2)

  double glane = 0.0;
  const int c0 = blockIdx.y * a.kchunk;
  const int c1 = min(c0 + a.kchunk, a.nk);
  for (int ci = c0; ci < c1; ++ci) {
    const bool eval = live && (UNITB || qab * a.kq[ci] >= a.tau);
    const int kc = a.kl[ci];
    const double C0 = a.K.ctr[3 * kc], C1 = a.K.ctr[3 * kc + 1], C2 = a.K.ctr[3 * kc + 2];
    const int nkp = a.K.nprim[kc], kpo = a.K.poff[kc];

    double acc[NA][NB][GN];
    sfor<NA>([&](auto i) { sfor<NB>([&](auto j) { sfor<GN>([&](auto g) { acc[i][j][g] = 0.0; }); }); });

    for (int ip = 0; ip < (eval ? nfp : 0); ++ip) {
      const double al = a.F.exps[fpo + ip], ca = a.F.coef[fpo + ip];
      for (int jp = 0; jp < nsp; ++jp) {
        const double be = UNITB ? 0.0 : a.S.exps[spo + jp];
        const double cb = UNITB ? 1.0 : a.S.coef[spo + jp];
        const double pp_ = al + be, ip_ = 1.0 / pp_;
        const double bp = be * ip_;  // P - A = b (B - A) / p, as in the ERI kernel
        const double Kab = UNITB ? 1.0 : exp(-al * be * ip_ * rAB2);
        const double PA0 = -bp * AB0, PA1 = -bp * AB1, PA2 = -bp * AB2;
        const double ex2 = 2.0 * (WHICH == 0 ? al : be);  // 2 x the moved primitive's exponent
        for (int kp = 0; kp < nkp; ++kp) {
          const double q = a.K.exps[kpo + kp], cc = a.K.coef[kpo + kp];
          const double pq = pp_ + q, ipq = 1.0 / pq;
          const double PC0 = PA0 + (A0 - C0), PC1 = PA1 + (A1 - C1), PC2 = PA2 + (A2 - C2);
          const double rho = pp_ * q * ipq;
          const double T = rho * (PC0 * PC0 + PC1 * PC1 + PC2 * PC2);
          const double pref = TWO_PI_52 / (pp_ * q * sqrt(pq)) * Kab * ca * cb * cc;
          const RysPoint<NR> rp(tab, T);
          const double qf = q * ipq, pf = pp_ * ipq;
#pragma unroll 1
          for (int r = 0; r < NR; ++r) {
            double u, w;
            rp.get(r, u, w);
            const double B00 = 0.5 * u * ipq;
            const double B10 = 0.5 * ip_ * (1.0 - qf * u);
            const double B01 = 0.5 / q * (1.0 - pf * u);
            double Hx[XA + 1][XB + 1][LC + 1], Hy[XA + 1][XB + 1][LC + 1], Hz[XA + 1][XB + 1][LC + 1];
            rys_2d<XA, XB, LC>(PA0 - qf * u * PC0, pf * u * PC0, B10, B01, B00, AB0, 1.0, Hx);
            rys_2d<XA, XB, LC>(PA1 - qf * u * PC1, pf * u * PC1, B10, B01, B00, AB1, 1.0, Hy);
            rys_2d<XA, XB, LC>(PA2 - qf * u * PC2, pf * u * PC2, B10, B01, B00, AB2, w * pref, Hz);
            sfor<NA>([&](auto ia) {
              constexpr int i = decltype(ia)::value;
              constexpr int ax = cpow(LA, i, 0), ay = cpow(LA, i, 1), az = cpow(LA, i, 2);
              sfor<NB>([&](auto ib) {
                constexpr int j = decltype(ib)::value;
                constexpr int bx = cpow(LB, j, 0), by = cpow(LB, j, 1), bz = cpow(LB, j, 2);
                sfor<NC>([&](auto ic) {
                  constexpr int c = decltype(ic)::value;
                  if constexpr (in_group<LC, M0, GN>(c)) {
                    constexpr int cx = cpow(LC, c, 0), cy = cpow(LC, c, 1), cz = cpow(LC, c, 2);
                    // the derivative along AXIS of the moved centre's factor
                    double v;
                    if constexpr (AXIS == 0)
                      v = dfac<WHICH, ax, bx, cx>(Hx, ex2) * Hy[ay][by][cy] * Hz[az][bz][cz];
                    else if constexpr (AXIS == 1)
                      v = Hx[ax][bx][cx] * dfac<WHICH, ay, by, cy>(Hy, ex2) * Hz[az][bz][cz];
                    else
                      v = Hx[ax][bx][cx] * Hy[ay][by][cy] * dfac<WHICH, az, bz, cz>(Hz, ex2);
                    sfor<GN>([&](auto ig) {
                      constexpr int g = decltype(ig)::value;
                      constexpr double t = sph<LC>(M0 + g, c);
                      if constexpr (t != 0.0) acc[i][j][g] = fma(t, v, acc[i][j][g]);
                    });
                  }
                });
              });
            });
          }
        }
      }
    }

    // bra solid harmonics, contracted with the weights of this block
    const int kfo = a.K.foff[kc];
    double s_ket = 0.0;
    if (eval) {
      sfor<SA>([&](auto mai) {
        constexpr int ma = decltype(mai)::value;
        sfor<SB>([&](auto mbi) {
          constexpr int mb = decltype(mbi)::value;
          sfor<GN>([&](auto ig) {
            constexpr int g = decltype(ig)::value;
            double v = 0.0;
            sfor<NA>([&](auto ia) {
              constexpr int i = decltype(ia)::value;
              constexpr double ta = sph<LA>(ma, i);
              if constexpr (ta != 0.0) {
                sfor<NB>([&](auto ib) {
                  constexpr int j = decltype(ib)::value;
                  constexpr double tb = UNITB ? 1.0 : sph<LB>(mb, j);
                  if constexpr (tb != 0.0) v = fma(ta * tb, acc[i][j][g], v);
                });
              }
            });
            const int P = kfo + M0 + g;
            const double wgt = UNITB ? ga.gam[(int64_t)(foffF + ma) * ga.ldg + P]
                                     : ga.gam[(int64_t)P * ga.ldg + a.cbase + (int64_t)p * (SA * SB) + (ma * SB + mb)];
            s_ket = fma(v, wgt, s_ket);
          });
        });
      });
    }
    s_ket *= wpair;
    glane += s_ket;
    // the ket centre takes minus this block's share: summed over the workgroup
    double t = s_ket;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_down(t, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int wv = 0; wv < ERI_THREADS / 64; ++wv) sum += red[wv];
      ga.kbuf[(int64_t)ci * gridDim.x + blockIdx.x] = -sum;
    }
    __syncthreads();
  }
  if (live) ga.pbuf[(int64_t)blockIdx.y * a.npairs + p] = glane;
}

// ket solid-harmonic components per derivative kernel: the accumulator block
// near 64 doubles per lane (the kernels keep one weighted sum per lane, so the
// block is live only within a ket shell)
__host__ __device__ constexpr int grad_group(int LA, int LB, int LC) {
  const int nab = ncart(LA) * ncart(LB);
  int g = 64 / nab;
  if (g < 1) g = 1;
  if (g > 2 * LC + 1) g = 2 * LC + 1;
  return g;
}

// Every ket group writes its own partial sums for the same lanes and ket
// shells: group k of a class launch writes at pbuf + k pstride, kbuf + k kstride.
template <int LA, int LB, int LC, bool UNITB, int WHICH, int AXIS, int M0 = 0>
void grad_launch_groups(GradArgs ga, dim3 grid, int64_t pstride, int64_t kstride, hipStream_t st) {
  constexpr int G = grad_group(LA, LB, LC);
  constexpr int NS = 2 * LC + 1;
  constexpr int GN = (M0 + G <= NS) ? G : NS - M0;
  hipLaunchKernelGGL((eri3_grad_kernel<LA, LB, LC, M0, GN, UNITB, WHICH, AXIS>), grid, dim3(ERI_THREADS), 0, st, ga);
  if constexpr (M0 + GN < NS) {
    ga.pbuf += pstride;
    ga.kbuf += kstride;
    grad_launch_groups<LA, LB, LC, UNITB, WHICH, AXIS, M0 + GN>(ga, grid, pstride, kstride, st);
  }
}

// number of ket groups of a class (the number of partial-sum slices it writes)
__host__ __device__ constexpr int grad_groups_of(int LA, int LB, int LC) {
  const int G = grad_group(LA, LB, LC);
  return (2 * LC + 1 + G - 1) / G;
}

// One orbital class (LA >= LB), moved centre W and axis AX of the three-index
// derivatives per object file (grad3_class.hip, compiled once per combination),
// the metric derivatives per axis (grad2_class.hip).  Explicit specialisations,
// declared here for every combination.
template <int LA, int LB, int W, int AX>
void grad3_class(int LC, GradArgs ga, dim3 grid, int64_t pstride, int64_t kstride, hipStream_t st);
template <int AX>
void grad2_class(int LA, int LC, GradArgs ga, dim3 grid, int64_t pstride, int64_t kstride, hipStream_t st);

#define DFX_GRAD3_AXES(M, LA, LB, W) M(LA, LB, W, 0) M(LA, LB, W, 1) M(LA, LB, W, 2)
#define DFX_GRAD3_WA(M, LA, LB) DFX_GRAD3_AXES(M, LA, LB, 0) DFX_GRAD3_AXES(M, LA, LB, 1)
#define DFX_GRAD3_ALL(M)                                                                                 \
  DFX_GRAD3_WA(M, 0, 0) DFX_GRAD3_WA(M, 1, 0) DFX_GRAD3_WA(M, 1, 1) DFX_GRAD3_WA(M, 2, 0)                \
  DFX_GRAD3_WA(M, 2, 1) DFX_GRAD3_WA(M, 2, 2) DFX_GRAD3_WA(M, 3, 0) DFX_GRAD3_WA(M, 3, 1)                \
  DFX_GRAD3_WA(M, 3, 2) DFX_GRAD3_WA(M, 3, 3)
#define DFX_GRAD3_DECL(LA, LB, W, AX)                                                                    \
  template <>                                                                                           \
  void grad3_class<LA, LB, W, AX>(int LC, GradArgs ga, dim3 grid, int64_t pstride, int64_t kstride,     \
                                  hipStream_t st);
DFX_GRAD3_ALL(DFX_GRAD3_DECL)
template <> void grad2_class<0>(int, int, GradArgs, dim3, int64_t, int64_t, hipStream_t);
template <> void grad2_class<1>(int, int, GradArgs, dim3, int64_t, int64_t, hipStream_t);
template <> void grad2_class<2>(int, int, GradArgs, dim3, int64_t, int64_t, hipStream_t);

// ---- one-electron derivatives and weight assembly (grad_misc.hip)
struct OneEGradArgs {
  DevShells sh;
  const int* pf;          // [npairs] shell a (angular momentum LA)
  const int* ps;          // [npairs] shell b (LB), a >= b by index
  int npairs;
  const int64_t* woff;    // [npairs] first element of the pair's Cartesian weight block
  const double* wD;       // Cartesian weights of 2D (h terms)
  const double* wW;       // Cartesian weights of 2W (overlap term)
  const double* xyz;      // [natom][3]
  const double* Z;        // [natom]
  int natom;
  const double* rys;
  double* pbuf;           // [npairs][6]: d/dA (x, y, z), d/dB (x, y, z)
  double* nbuf;           // [gridDim.x][natom][3]: the operators' own derivatives
};
void onee_grad_dispatch(int LA, int LB, OneEGradArgs g, const double* Dw, const double* Ww, int n, double scale,
                        double* wD, double* wW, hipStream_t st);
void gam_pack(const double* T, const double* D, int nbf, const double* gam, const int* cmu, const int* cnu,
              int64_t ncols, int nq, double* out, hipStream_t st);
void rank1_sub2(double* M, const double* gam, int n, hipStream_t st);
void transpose_sq(const double* A, double* B, int n, hipStream_t st);
void scale_cols(const double* C, const double* eps, int n, int no, double* Ce, hipStream_t st);

// runtime dispatch (grad.cpp)
void grad3_dispatch(int LA, int LB, int LC, int which, int axis, GradArgs ga, dim3 grid, int64_t pstride,
                    int64_t kstride, hipStream_t st);

}  // namespace dfx
