// Three-index electron-repulsion integrals (mu nu|P) by Rys quadrature, gfx950.
//
// One kernel instantiation per shell-triplet class (LA, LB | LC), LA >= LB,
// and per group of solid-harmonic components of the ket shell.  Each lane owns
// one orbital shell pair; a workgroup walks a chunk of ket (auxiliary) shells
// of angular momentum LC, so the whole wave shares one ket shell.  The raw
// integrals are stored class by class (STORE_CLASS, see eri_args.h): the
// lanes of a wave fill one contiguous block of columns.  Per root of
// the Rys quadrature the lane builds the 2D integrals by the vertical
// recurrence on (a+b, c) and the horizontal transfer to (a, b), then
// accumulates the Cartesian products straight into the real solid harmonics of
// the ket (compile-time sparse transform).  All arithmetic is FP64.
//
// The same kernel evaluates the two-centre Coulomb metric (P|Q) with the
// second bra function replaced by the constant 1 (UNITB).
#pragma once
#include "common.h"
#include "eri_args.h"
#include "rys.h"
#include "sph_tables.inc"

namespace dfx {

constexpr int ERI_THREADS = 128;

template <int L> struct SphTab;
template <> struct SphTab<0> { static constexpr const double (&t)[1][1] = SPH_L0; };
template <> struct SphTab<1> { static constexpr const double (&t)[3][3] = SPH_L1; };
template <> struct SphTab<2> { static constexpr const double (&t)[5][6] = SPH_L2; };
template <> struct SphTab<3> { static constexpr const double (&t)[7][10] = SPH_L3; };
template <> struct SphTab<4> { static constexpr const double (&t)[9][15] = SPH_L4; };
template <int L>
__host__ __device__ constexpr double sph(int m, int c) { return SphTab<L>::t[m][c]; }

// is Cartesian component c of degree L used by any m in [M0, M0 + GN)?
template <int L, int M0, int GN>
__host__ __device__ constexpr bool in_group(int c) {
  for (int g = 0; g < GN; ++g)
    if (sph<L>(M0 + g, c) != 0.0) return true;
  return false;
}


// 2D integrals of one Cartesian direction for one root: VRR to I(e, k),
// e <= LA + LB, k <= LC, then the horizontal transfer to H[a][b][k].
template <int LA, int LB, int LC>
__device__ __forceinline__ void rys_2d(double C00, double D00, double B10, double B01, double B00,
                                       double AB, double I0, double (&H)[LA + 1][LB + 1][LC + 1]) {
  constexpr int E = LA + LB;
  double V[E + 1][LC + 1];
  V[0][0] = I0;
  if constexpr (E > 0) V[1][0] = C00 * I0;
#pragma unroll
  for (int e = 1; e < E; ++e) V[e + 1][0] = fma(C00, V[e][0], (double)e * B10 * V[e - 1][0]);
#pragma unroll
  for (int k = 0; k < LC; ++k) {
    V[0][k + 1] = D00 * V[0][k];
    if (k > 0) V[0][k + 1] = fma((double)k * B01, V[0][k - 1], V[0][k + 1]);
#pragma unroll
    for (int e = 1; e <= E; ++e) {
      double v = fma(D00, V[e][k], (double)e * B00 * V[e - 1][k]);
      if (k > 0) v = fma((double)k * B01, V[e][k - 1], v);
      V[e][k + 1] = v;
    }
  }
#pragma unroll
  for (int k = 0; k <= LC; ++k) {
    double G[E + 1];
#pragma unroll
    for (int e = 0; e <= E; ++e) G[e] = V[e][k];
#pragma unroll
    for (int a = 0; a <= LA; ++a) H[a][0][k] = G[a];
#pragma unroll
    for (int b = 1; b <= LB; ++b) {
#pragma unroll
      for (int e = 0; e <= E - b; ++e) G[e] = fma(AB, G[e], G[e + 1]);
#pragma unroll
      for (int a = 0; a <= LA; ++a) H[a][b][k] = G[a];
    }
  }
}

// LDS written by some lanes of a wave and read by others: LDS operations of one
// wave complete in issue order, so only the compiler has to keep them in place
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LA, int LB, int LC, int M0, int GN, bool UNITB, int MODE>
__global__ void __launch_bounds__(ERI_THREADS) eri3_kernel(const Eri3Args a) {
  constexpr int NR = (LA + LB + LC) / 2 + 1;
  constexpr int NA = ncart(LA), NB = ncart(LB), NC = ncart(LC);
  constexpr int SA = 2 * LA + 1, SB = UNITB ? 1 : 2 * LB + 1;
  // STORE_CLASS: for one ket function a wave's results are one contiguous run
  // of 64 SA SB columns, pair by pair.  Where the workgroup's copy of that run
  // and the Rys table fit in a quarter of the CU's 160 KB of LDS (so that LDS
  // never holds the class below two waves per SIMD) the run goes out through
  // LDS, consecutive lanes storing consecutive columns; otherwise each lane
  // stores its own pair's block.
  constexpr int SASB = SA * SB;
  static_assert(MODE == STORE_CLASS || UNITB, "dense stores are for the two-centre metric");
  constexpr bool STAGE =
      MODE == STORE_CLASS && (ERI_THREADS * SASB + rys_dev_size(NR)) * (int)sizeof(double) <= 40 * 1024;
  constexpr int NSTG = STAGE ? 64 * SASB : 1;
  __shared__ double tab[rys_dev_size(NR)];
  __shared__ double stg[ERI_THREADS / 64][NSTG];
  rys_stage<NR>(tab, a.rys);
  const int lane = threadIdx.x & 63;
  const int p0 = blockIdx.x * blockDim.x + (threadIdx.x - lane);  // first pair of the wave
  if (p0 >= a.npairs) return;  // the whole wave
  // lanes past the end of the class list evaluate nothing; in STORE_CLASS they
  // stay for the stores, which they share with the other lanes
  const bool live = p0 + lane < a.npairs;
  if (MODE != STORE_CLASS && !live) return;
  const int p = live ? p0 + lane : a.npairs - 1;
  const int f = a.pf[p];
  const int s = UNITB ? f : a.ps[p];
  const double A0 = a.F.ctr[3 * f], A1 = a.F.ctr[3 * f + 1], A2 = a.F.ctr[3 * f + 2];
  const double B0 = UNITB ? A0 : a.S.ctr[3 * s], B1 = UNITB ? A1 : a.S.ctr[3 * s + 1],
               B2 = UNITB ? A2 : a.S.ctr[3 * s + 2];
  const int nfp = a.F.nprim[f], fpo = a.F.poff[f];
  const int nsp = UNITB ? 1 : a.S.nprim[s], spo = UNITB ? 0 : a.S.poff[s];
  const int foffF = a.F.foff[f];
  const double qab = a.pq ? a.pq[p] : 1.0;
  const double AB0 = A0 - B0, AB1 = A1 - B1, AB2 = A2 - B2;
  const double rAB2 = AB0 * AB0 + AB1 * AB1 + AB2 * AB2;
  constexpr double TWO_PI_52 = 34.98683665524972;  // 2 pi^(5/2)

  const int c0 = blockIdx.y * a.kchunk;
  const int c1 = min(c0 + a.kchunk, a.nk);
  for (int ci = c0; ci < c1; ++ci) {
    // a screened triplet stores its block of zeros (the raw tensor is not cleared
    // beforehand: every one of its elements is written by exactly one lane)
    const bool keep = MODE != STORE_CLASS || (live && qab * a.kq[ci] >= a.tau);
    const int kc = a.kl[ci];
    const double C0 = a.K.ctr[3 * kc], C1 = a.K.ctr[3 * kc + 1], C2 = a.K.ctr[3 * kc + 2];
    const int nkp = a.K.nprim[kc], kpo = a.K.poff[kc];

    double acc[NA][NB][GN];
    sfor<NA>([&](auto i) { sfor<NB>([&](auto j) { sfor<GN>([&](auto g) { acc[i][j][g] = 0.0; }); }); });

    const int nfp_keep = keep ? nfp : 0;
    for (int ip = 0; ip < nfp_keep; ++ip) {
      const double al = a.F.exps[fpo + ip], ca = a.F.coef[fpo + ip];
      for (int jp = 0; jp < nsp; ++jp) {
        const double be = UNITB ? 0.0 : a.S.exps[spo + jp];
        const double cb = UNITB ? 1.0 : a.S.coef[spo + jp];
        const double pp = al + be, ip_ = 1.0 / pp;
        // P - A = b (B - A) / p from the centre difference: exactly zero for
        // concentric functions and independent of the origin
        const double bp = be * ip_;
        const double Kab = UNITB ? 1.0 : exp(-al * be * ip_ * rAB2);
        const double PA0 = -bp * AB0, PA1 = -bp * AB1, PA2 = -bp * AB2;
        for (int kp = 0; kp < nkp; ++kp) {
          const double q = a.K.exps[kpo + kp], cc = a.K.coef[kpo + kp];
          const double pq = pp + q, ipq = 1.0 / pq;
          const double PC0 = PA0 + (A0 - C0), PC1 = PA1 + (A1 - C1), PC2 = PA2 + (A2 - C2);
          const double rho = pp * q * ipq;
          const double T = rho * (PC0 * PC0 + PC1 * PC1 + PC2 * PC2);
          const double pref = TWO_PI_52 / (pp * q * sqrt(pq)) * Kab * ca * cb * cc;
          const RysPoint<NR> rp(tab, T);
          const double qf = q * ipq, pf = pp * ipq;
#pragma unroll 1
          for (int r = 0; r < NR; ++r) {
            double u, w;
            rp.get(r, u, w);
            const double B00 = 0.5 * u * ipq;
            const double B10 = 0.5 * ip_ * (1.0 - qf * u);
            const double B01 = 0.5 / q * (1.0 - pf * u);
            double Hx[LA + 1][LB + 1][LC + 1], Hy[LA + 1][LB + 1][LC + 1], Hz[LA + 1][LB + 1][LC + 1];
            rys_2d<LA, LB, LC>(PA0 - qf * u * PC0, pf * u * PC0, B10, B01, B00, AB0, 1.0, Hx);
            rys_2d<LA, LB, LC>(PA1 - qf * u * PC1, pf * u * PC1, B10, B01, B00, AB1, 1.0, Hy);
            rys_2d<LA, LB, LC>(PA2 - qf * u * PC2, pf * u * PC2, B10, B01, B00, AB2, w * pref, Hz);
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
                    const double v = Hx[ax][bx][cx] * Hy[ay][by][cy] * Hz[az][bz][cz];
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

    // bra solid harmonics and store
    const int kfo = a.K.foff[kc];
    double* const out = a.out;
    auto bra = [&](auto mai, auto mbi, auto ig) {
      constexpr int ma = decltype(mai)::value, mb = decltype(mbi)::value, g = decltype(ig)::value;
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
      return v;
    };
    if constexpr (STAGE) {
      // the lanes of a wave hold consecutive pairs of the class: per ket
      // function, 64 SA SB consecutive columns from the wave's first pair on
      double* const sw = stg[threadIdx.x >> 6];
      const int nval = min(64, a.npairs - p0) * SASB;
      sfor<GN>([&](auto ig) {
        constexpr int g = decltype(ig)::value;
        sfor<SA>([&](auto mai) {
          constexpr int ma = decltype(mai)::value;
          sfor<SB>([&](auto mbi) {
            constexpr int mb = decltype(mbi)::value;
            sw[lane * SASB + ma * SB + mb] = bra(mai, mbi, ig);
          });
        });
        wave_lds_sync();
        double* const o = out + (int64_t)(kfo + M0 + g) * a.ld + a.cbase + (int64_t)p0 * SASB;
        // a loop rather than an unrolled sequence: unrolled, the compiler
        // keeps every store's lane mask live across the ket loop
#pragma unroll 1
        for (int e = lane; e < nval; e += 64) o[e] = sw[e];
        wave_lds_sync();
      });
    } else if constexpr (MODE == STORE_CLASS) {
      if (live) {
        sfor<SA>([&](auto mai) {
          constexpr int ma = decltype(mai)::value;
          sfor<SB>([&](auto mbi) {
            constexpr int mb = decltype(mbi)::value;
            sfor<GN>([&](auto ig) {
              constexpr int g = decltype(ig)::value;
              out[(int64_t)(kfo + M0 + g) * a.ld + a.cbase + (int64_t)p * SASB + (ma * SB + mb)] =
                  bra(mai, mbi, ig);
            });
          });
        });
      }
    } else {
      sfor<SA>([&](auto mai) {
        constexpr int ma = decltype(mai)::value;
        sfor<GN>([&](auto ig) {
          constexpr int g = decltype(ig)::value;
          out[(int64_t)(foffF + ma) * a.ld + kfo + M0 + g] = bra(mai, std::integral_constant<int, 0>{}, ig);
        });
      });
    }
  }
}

// number of ket solid-harmonic components per kernel instantiation: keep the
// accumulator block near ERI_ACC doubles per lane
#ifndef ERI_ACC
#define ERI_ACC 32
#endif
__host__ __device__ constexpr int eri_group(int LA, int LB, int LC) {
  const int nab = ncart(LA) * ncart(LB);
  int g = ERI_ACC / nab;
  if (g < 1) g = 1;
  if (g > 2 * LC + 1) g = 2 * LC + 1;
  return g;
}

template <int LA, int LB, int LC, bool UNITB, int MODE, int M0 = 0>
void eri3_launch_groups(const Eri3Args& a, dim3 grid, hipStream_t st) {
  constexpr int G = eri_group(LA, LB, LC);
  constexpr int NS = 2 * LC + 1;
  constexpr int GN = (M0 + G <= NS) ? G : NS - M0;
  hipLaunchKernelGGL((eri3_kernel<LA, LB, LC, M0, GN, UNITB, MODE>), grid, dim3(ERI_THREADS), 0, st, a);
  if constexpr (M0 + GN < NS) eri3_launch_groups<LA, LB, LC, UNITB, MODE, M0 + GN>(a, grid, st);
}

// grid for npairs x nk work items
inline dim3 eri3_grid(Eri3Args& a) {
  const int gx = (a.npairs + ERI_THREADS - 1) / ERI_THREADS;
  int chunk = (int)(((int64_t)a.nk * gx + 2047) / 2048);
  if (chunk < 1) chunk = 1;
  if (chunk > a.nk) chunk = a.nk > 0 ? a.nk : 1;
  a.kchunk = chunk;
  const int gy = (a.nk + chunk - 1) / chunk;
  return dim3(gx, gy, 1);
}

void eri3_dispatch(int LA, int LB, int LC, bool unitb, int mode, Eri3Args a, hipStream_t st);
void metric_dispatch(int LA, int LC, Eri3Args a, hipStream_t st);

// class dispatch (eri3_dispatch.hip); one translation unit per (LA, LB)
template <int LA, int LB>
void eri3_dispatch_pair(int LC, Eri3Args a, hipStream_t st);

}  // namespace dfx
