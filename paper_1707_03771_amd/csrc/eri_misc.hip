// Schwarz factors (four-centre diagonal (mu nu|mu nu) by Rys quadrature) and
// one-electron integrals (overlap, kinetic energy, nuclear attraction) on gfx950.
#include "eri3_kernel.h"
#include "kernels.h"

namespace dfx {

// ---------------------------------------------------------------------------
// Sparse rows of the solid-harmonic tables: Cartesian support of each m.
struct SuppRow {
  int n;
  int c[6];
  double t[6];
};
template <int L>
__host__ __device__ constexpr SuppRow make_supp(int m) {
  SuppRow r{0, {0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}};
  for (int c = 0; c < ncart(L); ++c)
    if (sph<L>(m, c) != 0.0) {
      r.c[r.n] = c;
      r.t[r.n] = sph<L>(m, c);
      ++r.n;
    }
  return r;
}
__constant__ SuppRow g_supp[4][7] = {
    {make_supp<0>(0)},
    {make_supp<1>(0), make_supp<1>(1), make_supp<1>(2)},
    {make_supp<2>(0), make_supp<2>(1), make_supp<2>(2), make_supp<2>(3), make_supp<2>(4)},
    {make_supp<3>(0), make_supp<3>(1), make_supp<3>(2), make_supp<3>(3), make_supp<3>(4),
     make_supp<3>(5), make_supp<3>(6)}};

// ---------------------------------------------------------------------------
// Schwarz: Q_ab = sqrt(max_{mu in a, nu in b} (mu nu|mu nu)).  One wave per
// shell pair (LA >= LB after swapping), lanes over the spherical (mu, nu).
// Per root, lanes 0..2 build the four-index 2D integrals of one direction in
// LDS; every lane then sums its sparse spherical combination.
template <int LA, int LB>
__global__ void __launch_bounds__(64) schwarz_kernel(SchwarzArgs a) {
  constexpr int NR = (2 * (LA + LB)) / 2 + 1;
  constexpr int E = LA + LB;
  constexpr int D1 = LA + 1, D2 = LB + 1;
  constexpr int N4 = D1 * D2 * D1 * D2;
  __shared__ double tab[rys_dev_size(NR)];
  __shared__ double H4[3][N4];
  rys_stage<NR>(tab, a.rys);
  const int p = blockIdx.x;
  if (p >= a.npairs) return;
  const int s1 = a.pf[p], s2 = a.ps[p];
  const int lane = threadIdx.x;
  constexpr int SA = 2 * LA + 1, SB = 2 * LB + 1;
  const int ma = lane / SB, mb = lane % SB;
  const bool active = lane < SA * SB;
  const double A[3] = {a.sh.ctr[3 * s1], a.sh.ctr[3 * s1 + 1], a.sh.ctr[3 * s1 + 2]};
  const double B[3] = {a.sh.ctr[3 * s2], a.sh.ctr[3 * s2 + 1], a.sh.ctr[3 * s2 + 2]};
  const double AB[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
  const double rAB2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
  const int n1 = a.sh.nprim[s1], o1 = a.sh.poff[s1];
  const int n2 = a.sh.nprim[s2], o2 = a.sh.poff[s2];
  const SuppRow ra = g_supp[LA][active ? ma : 0], rb = g_supp[LB][active ? mb : 0];
  double acc = 0.0;
  constexpr double TWO_PI_52 = 34.98683665524972;
  for (int i1 = 0; i1 < n1; ++i1)
    for (int j1 = 0; j1 < n2; ++j1) {
      const double al = a.sh.exps[o1 + i1], be = a.sh.exps[o2 + j1];
      const double p1 = al + be;
      // P - A = b (B - A) / p from the centre difference (exact for concentric pairs)
      const double PA[3] = {be / p1 * (B[0] - A[0]), be / p1 * (B[1] - A[1]), be / p1 * (B[2] - A[2])};
      const double K1 = exp(-al * be / p1 * rAB2) * a.sh.coef[o1 + i1] * a.sh.coef[o2 + j1];
      for (int i2 = 0; i2 < n1; ++i2)
        for (int j2 = 0; j2 < n2; ++j2) {
          const double ga = a.sh.exps[o1 + i2], de = a.sh.exps[o2 + j2];
          const double q = ga + de;
          const double QA[3] = {de / q * (B[0] - A[0]), de / q * (B[1] - A[1]), de / q * (B[2] - A[2])};
          const double K2 = exp(-ga * de / q * rAB2) * a.sh.coef[o1 + i2] * a.sh.coef[o2 + j2];
          const double pq = p1 + q;
          const double PQ[3] = {PA[0] - QA[0], PA[1] - QA[1], PA[2] - QA[2]};
          const double T = p1 * q / pq * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
          const double pref = TWO_PI_52 / (p1 * q * sqrt(pq)) * K1 * K2;
          const RysPoint<NR> rp(tab, T);
          for (int r = 0; r < NR; ++r) {
            double u, w;
            rp.get(r, u, w);
            if (lane < 3) {
              const int x = lane;
              const double C00 = PA[x] - q / pq * PQ[x] * u;
              const double D00 = QA[x] + p1 / pq * PQ[x] * u;
              const double B00 = 0.5 * u / pq;
              const double B10 = 0.5 / p1 * (1.0 - q / pq * u);
              const double B01 = 0.5 / q * (1.0 - p1 / pq * u);
              double V[E + 1][E + 1];
              V[0][0] = (x == 2) ? w * pref : 1.0;
#pragma unroll
              for (int e = 0; e < E; ++e)
                V[e + 1][0] = C00 * V[e][0] + (e > 0 ? e * B10 * V[e - 1][0] : 0.0);
#pragma unroll
              for (int f = 0; f < E; ++f)
#pragma unroll
                for (int e = 0; e <= E; ++e)
                  V[e][f + 1] = D00 * V[e][f] + (f > 0 ? f * B01 * V[e][f - 1] : 0.0) +
                                (e > 0 ? e * B00 * V[e - 1][f] : 0.0);
              // bra transfer: W[a1][b1][f]
              double W[D1][D2][E + 1];
#pragma unroll
              for (int f = 0; f <= E; ++f) {
                double G[E + 1];
#pragma unroll
                for (int e = 0; e <= E; ++e) G[e] = V[e][f];
#pragma unroll
                for (int a1 = 0; a1 < D1; ++a1) W[a1][0][f] = G[a1];
#pragma unroll
                for (int b1 = 1; b1 < D2; ++b1) {
#pragma unroll
                  for (int e = 0; e <= E - b1; ++e) G[e] = G[e + 1] + AB[x] * G[e];
#pragma unroll
                  for (int a1 = 0; a1 < D1; ++a1) W[a1][b1][f] = G[a1];
                }
              }
              // ket transfer
#pragma unroll
              for (int a1 = 0; a1 < D1; ++a1)
#pragma unroll
                for (int b1 = 0; b1 < D2; ++b1) {
                  double G[E + 1];
#pragma unroll
                  for (int f = 0; f <= E; ++f) G[f] = W[a1][b1][f];
#pragma unroll
                  for (int a2 = 0; a2 < D1; ++a2) H4[x][((a1 * D2 + b1) * D1 + a2) * D2] = G[a2];
#pragma unroll
                  for (int b2 = 1; b2 < D2; ++b2) {
#pragma unroll
                    for (int f = 0; f <= E - b2; ++f) G[f] = G[f + 1] + AB[x] * G[f];
#pragma unroll
                    for (int a2 = 0; a2 < D1; ++a2)
                      H4[x][((a1 * D2 + b1) * D1 + a2) * D2 + b2] = G[a2];
                  }
                }
            }
            __syncthreads();
            if (active) {
              for (int i = 0; i < ra.n; ++i)
                for (int j = 0; j < rb.n; ++j)
                  for (int k = 0; k < ra.n; ++k)
                    for (int l = 0; l < rb.n; ++l) {
                      const int ci = ra.c[i], cj = rb.c[j], ck = ra.c[k], cl = rb.c[l];
                      double v = ra.t[i] * rb.t[j] * ra.t[k] * rb.t[l];
#pragma unroll
                      for (int x = 0; x < 3; ++x) {
                        const int pa = cpow(LA, ci, x), pb = cpow(LB, cj, x);
                        const int pc = cpow(LA, ck, x), pd = cpow(LB, cl, x);
                        v *= H4[x][((pa * D2 + pb) * D1 + pc) * D2 + pd];
                      }
                      acc += v;
                    }
            }
            __syncthreads();
          }
        }
    }
  // max over the wave
  double m = active ? acc : -1.0;
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (lane == 0) a.q[p] = sqrt(fmax(m, 0.0));
}

void schwarz_dispatch(int LA, int LB, SchwarzArgs a, hipStream_t st) {
  const dim3 g(a.npairs), b(64);
#define SC(X, Y)                                                        \
  case (X)*8 + (Y):                                                     \
    hipLaunchKernelGGL((schwarz_kernel<X, Y>), g, b, 0, st, a);         \
    break;
  switch (LA * 8 + LB) {
    SC(0, 0) SC(1, 0) SC(1, 1) SC(2, 0) SC(2, 1) SC(2, 2) SC(3, 0) SC(3, 1) SC(3, 2) SC(3, 3)
    default:
      throw Error(-6, "schwarz: unsupported angular momentum class");
  }
#undef SC
}

// ---------------------------------------------------------------------------
// One-electron integrals over a shell pair (any order of l), one lane per pair.
// Overlap by the Obara-Saika recursion per direction; kinetic energy from the
// second derivative of the ket, -1/2 <i| d^2/dx^2 |j>; nuclear attraction
// -sum_C Z_C <a| 1/|r - C| |b> by Rys quadrature with T = p |P - C|^2.
template <int LA, int LB>
__global__ void __launch_bounds__(64) onee_st_kernel(OneEArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npairs) return;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  const int s1 = a.pf[p], s2 = a.ps[p];
  double accS[NA][NB], accT[NA][NB];
  sfor<NA>([&](auto i) { sfor<NB>([&](auto j) { accS[i][j] = 0.0; accT[i][j] = 0.0; }); });
  const double A[3] = {a.sh.ctr[3 * s1], a.sh.ctr[3 * s1 + 1], a.sh.ctr[3 * s1 + 2]};
  const double B[3] = {a.sh.ctr[3 * s2], a.sh.ctr[3 * s2 + 1], a.sh.ctr[3 * s2 + 2]};
  for (int i1 = 0; i1 < a.sh.nprim[s1]; ++i1)
    for (int j1 = 0; j1 < a.sh.nprim[s2]; ++j1) {
      const double al = a.sh.exps[a.sh.poff[s1] + i1], be = a.sh.exps[a.sh.poff[s2] + j1];
      const double cf = a.sh.coef[a.sh.poff[s1] + i1] * a.sh.coef[a.sh.poff[s2] + j1];
      const double pp = al + be, h = 0.5 / pp;
      double S[3][LA + 1][LB + 3], K[3][LA + 1][LB + 1];
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        const double XAB = A[x] - B[x];
        // P - A and P - B from the centre difference (exact for concentric pairs)
        const double PA = -be / pp * XAB, PB = al / pp * XAB;
        S[x][0][0] = sqrt(M_PI / pp) * exp(-al * be / pp * XAB * XAB);
#pragma unroll
        for (int j = 0; j < LB + 2; ++j)
          S[x][0][j + 1] = PB * S[x][0][j] + (j > 0 ? h * j * S[x][0][j - 1] : 0.0);
#pragma unroll
        for (int i = 0; i < LA; ++i)
#pragma unroll
          for (int j = 0; j <= LB + 2; ++j)
            S[x][i + 1][j] = PA * S[x][i][j] + h * ((i > 0 ? i * S[x][i - 1][j] : 0.0) +
                                                    (j > 0 ? j * S[x][i][j - 1] : 0.0));
#pragma unroll
        for (int i = 0; i <= LA; ++i)
#pragma unroll
          for (int j = 0; j <= LB; ++j)
            K[x][i][j] = -0.5 * ((j >= 2 ? j * (j - 1) * S[x][i][j - 2] : 0.0) -
                                 2.0 * be * (2 * j + 1) * S[x][i][j] + 4.0 * be * be * S[x][i][j + 2]);
      }
      sfor<NA>([&](auto ia) {
        constexpr int i = decltype(ia)::value;
        constexpr int ax = cpow(LA, i, 0), ay = cpow(LA, i, 1), az = cpow(LA, i, 2);
        sfor<NB>([&](auto ib) {
          constexpr int j = decltype(ib)::value;
          constexpr int bx = cpow(LB, j, 0), by = cpow(LB, j, 1), bz = cpow(LB, j, 2);
          const double sx = S[0][ax][bx], sy = S[1][ay][by], sz = S[2][az][bz];
          accS[i][j] += cf * sx * sy * sz;
          accT[i][j] += cf * (K[0][ax][bx] * sy * sz + sx * K[1][ay][by] * sz + sx * sy * K[2][az][bz]);
        });
      });
    }
  const int fa = a.sh.foff[s1], fb = a.sh.foff[s2];
  sfor<2 * LA + 1>([&](auto mai) {
    constexpr int ma = decltype(mai)::value;
    sfor<2 * LB + 1>([&](auto mbi) {
      constexpr int mb = decltype(mbi)::value;
      double vs = 0.0, vt = 0.0;
      sfor<NA>([&](auto ia) {
        constexpr int i = decltype(ia)::value;
        constexpr double ta = sph<LA>(ma, i);
        if constexpr (ta != 0.0)
          sfor<NB>([&](auto ib) {
            constexpr int j = decltype(ib)::value;
            constexpr double tb = sph<LB>(mb, j);
            if constexpr (tb != 0.0) {
              vs = fma(ta * tb, accS[i][j], vs);
              vt = fma(ta * tb, accT[i][j], vt);
            }
          });
      });
      const int64_t r = fa + ma, c = fb + mb;
      a.S[r * a.n + c] = vs;
      a.S[c * a.n + r] = vs;
      a.T[r * a.n + c] = vt;
      a.T[c * a.n + r] = vt;
    });
  });
}

template <int LA, int LB>
__global__ void __launch_bounds__(64) onee_v_kernel(OneEArgs a) {
  constexpr int NR = (LA + LB) / 2 + 1;
  __shared__ double tab[rys_dev_size(NR)];
  rys_stage<NR>(tab, a.rys);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.npairs) return;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  constexpr int E = LA + LB;
  const int s1 = a.pf[p], s2 = a.ps[p];
  double acc[NA][NB];
  sfor<NA>([&](auto i) { sfor<NB>([&](auto j) { acc[i][j] = 0.0; }); });
  const double A[3] = {a.sh.ctr[3 * s1], a.sh.ctr[3 * s1 + 1], a.sh.ctr[3 * s1 + 2]};
  const double B[3] = {a.sh.ctr[3 * s2], a.sh.ctr[3 * s2 + 1], a.sh.ctr[3 * s2 + 2]};
  const double AB[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
  for (int i1 = 0; i1 < a.sh.nprim[s1]; ++i1)
    for (int j1 = 0; j1 < a.sh.nprim[s2]; ++j1) {
      const double al = a.sh.exps[a.sh.poff[s1] + i1], be = a.sh.exps[a.sh.poff[s2] + j1];
      const double pp = al + be;
      const double cf = a.sh.coef[a.sh.poff[s1] + i1] * a.sh.coef[a.sh.poff[s2] + j1] *
                        exp(-al * be / pp * (AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2])) *
                        2.0 * M_PI / pp;
      // P - A = b (B - A) / p, P - C = (P - A) + (A - C): exact for concentric centres
      const double PA[3] = {-be / pp * AB[0], -be / pp * AB[1], -be / pp * AB[2]};
      for (int c = 0; c < a.natom; ++c) {
        const double PC[3] = {PA[0] + (A[0] - a.xyz[3 * c]), PA[1] + (A[1] - a.xyz[3 * c + 1]),
                              PA[2] + (A[2] - a.xyz[3 * c + 2])};
        const double T = pp * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
        const double z = -a.Z[c] * cf;
        const RysPoint<NR> rp(tab, T);
#pragma unroll 1
        for (int r = 0; r < NR; ++r) {
          double u, w;
          rp.get(r, u, w);
          const double B10 = 0.5 / pp * (1.0 - u);
          double H[3][LA + 1][LB + 1];
#pragma unroll
          for (int x = 0; x < 3; ++x) {
            const double C00 = PA[x] - u * PC[x];
            double G[E + 1];
            G[0] = (x == 2) ? w * z : 1.0;
#pragma unroll
            for (int e = 0; e < E; ++e) G[e + 1] = C00 * G[e] + (e > 0 ? e * B10 * G[e - 1] : 0.0);
#pragma unroll
            for (int i = 0; i <= LA; ++i) H[x][i][0] = G[i];
#pragma unroll
            for (int b = 1; b <= LB; ++b) {
#pragma unroll
              for (int e = 0; e <= E - b; ++e) G[e] = G[e + 1] + AB[x] * G[e];
#pragma unroll
              for (int i = 0; i <= LA; ++i) H[x][i][b] = G[i];
            }
          }
          sfor<NA>([&](auto ia) {
            constexpr int i = decltype(ia)::value;
            constexpr int ax = cpow(LA, i, 0), ay = cpow(LA, i, 1), az = cpow(LA, i, 2);
            sfor<NB>([&](auto ib) {
              constexpr int j = decltype(ib)::value;
              constexpr int bx = cpow(LB, j, 0), by = cpow(LB, j, 1), bz = cpow(LB, j, 2);
              acc[i][j] = fma(H[0][ax][bx] * H[1][ay][by], H[2][az][bz], acc[i][j]);
            });
          });
        }
      }
    }
  const int fa = a.sh.foff[s1], fb = a.sh.foff[s2];
  sfor<2 * LA + 1>([&](auto mai) {
    constexpr int ma = decltype(mai)::value;
    sfor<2 * LB + 1>([&](auto mbi) {
      constexpr int mb = decltype(mbi)::value;
      double v = 0.0;
      sfor<NA>([&](auto ia) {
        constexpr int i = decltype(ia)::value;
        constexpr double ta = sph<LA>(ma, i);
        if constexpr (ta != 0.0)
          sfor<NB>([&](auto ib) {
            constexpr int j = decltype(ib)::value;
            constexpr double tb = sph<LB>(mb, j);
            if constexpr (tb != 0.0) v = fma(ta * tb, acc[i][j], v);
          });
      });
      const int64_t r = fa + ma, c = fb + mb;
      a.V[r * a.n + c] = v;
      a.V[c * a.n + r] = v;
    });
  });
}

void onee_dispatch(int LA, int LB, OneEArgs a, hipStream_t st) {
  const dim3 g((a.npairs + 63) / 64), b(64);
#define OC(X, Y)                                                        \
  case (X)*8 + (Y):                                                     \
    hipLaunchKernelGGL((onee_st_kernel<X, Y>), g, b, 0, st, a);         \
    hipLaunchKernelGGL((onee_v_kernel<X, Y>), g, b, 0, st, a);          \
    break;
  switch (LA * 8 + LB) {
    OC(0, 0) OC(0, 1) OC(0, 2) OC(0, 3) OC(1, 0) OC(1, 1) OC(1, 2) OC(1, 3)
    OC(2, 0) OC(2, 1) OC(2, 2) OC(2, 3) OC(3, 0) OC(3, 1) OC(3, 2) OC(3, 3)
    default:
      throw Error(-6, "one-electron: unsupported angular momentum class");
  }
#undef OC
}

// ---------------------------------------------------------------------------
// Q_C = sqrt(max_{P in C} (P|P)) from the metric diagonal.
__global__ void aux_schwarz_kernel(const double* J, int64_t ld, DevShells aux, double* q) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= aux.nsh) return;
  const int f0 = aux.foff[c], n = 2 * aux.l[c] + 1;
  double m = 0.0;
  for (int i = 0; i < n; ++i) m = fmax(m, J[(int64_t)(f0 + i) * ld + f0 + i]);
  q[c] = sqrt(m);
}

void aux_schwarz(const double* J, int64_t ld, DevShells aux, double* q, hipStream_t st) {
  hipLaunchKernelGGL(aux_schwarz_kernel, dim3((aux.nsh + 127) / 128), dim3(128), 0, st, J, ld, aux, q);
}

}  // namespace dfx
