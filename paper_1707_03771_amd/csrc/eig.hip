// Symmetric eigen-decomposition on the GPU: the two-sided block Jacobi method
// (the cyclic Jacobi method of Golub & Van Loan, "Matrix Computations", 4th
// ed., sec. 8.5, applied to 32 x 32 blocks; parallel orderings as in their
// sec. 8.5.5).  It serves the SCF wherever a full set of eigenpairs is needed
// (section "Standard algorithms": the orthogonaliser of the overlap, the
// orbitals and orbital energies of RHF, UHF and ROHF).
//
// The matrix, zero-padded to N = 64 ceil(n / 64), is split into nb = N / 32
// blocks.  A sweep runs nb - 1 rounds; a round pairs the blocks into nb / 2
// disjoint pairs by the circle method.  Per round:
//   1. ej_pair_kernel: per pair (a, b), one workgroup loads the 64 x 64
//      principal submatrix of blocks a and b into LDS and runs one cyclic
//      Jacobi sweep over it (63 rounds of 32 disjoint rotations, each
//      rotation zeroing its element exactly; a round updates S by 2 x 2
//      blocks, one thread per block, so rows and columns need no barrier in
//      between), accumulating the orthogonal U with U^T S U the reduced
//      submatrix.  S goes back in place, U to a buffer.  One local sweep per
//      visit converges in as many outer sweeps as solving the pair problem
//      to the end (measured in a CPU model of the scheme).
//   2. ej_apply_kernel: the off-diagonal 64 x 64 blocks between pairs,
//      A_IJ <- U_I^T A_IJ U_J (one workgroup per block I > J, writing both
//      A_IJ and A_JI), and the eigenvector columns V_:I <- V_:I U_I.
// A rotation is applied only when |a_pq| > 1e-15 sqrt(|a_pp a_qq|); the
// iteration stops after a sweep without any rotation, so on return every
// off-diagonal element is below that bound.  Padded rows and columns carry
// exact zeros, which no rotation ever touches, so they never mix with the
// matrix's own.  Rotations: t = sign(th) / (|th| + sqrt(1 + th^2)),
// th = (a_qq - a_pp) / (2 a_pq), c = 1 / sqrt(1 + t^2), s = t c; the rotated
// diagonal is a_pp - t a_pq and a_qq + t a_pq (Golub & Van Loan, Alg. 8.5.1).
#include <algorithm>
#include <numeric>
#include <vector>

#include "host.h"
#include "kernels.h"

namespace dfx {

namespace {

constexpr int EJB = 32;       // block
constexpr int EJP = 64;       // pair problem (two blocks)
constexpr int EJT = 256;      // threads per workgroup
constexpr double EJ_TOL = 1e-15;

__device__ __forceinline__ int ej_g(int i, int2 ab) { return i < EJB ? ab.x * EJB + i : ab.y * EJB + (i - EJB); }

// circle method on the 64 local indices: round r in [0, 63), pair k in [0, 32)
__device__ __forceinline__ void ej_local_pair(int r, int k, int& p, int& q) {
  int a, b;
  if (k == 0) {
    a = r;
    b = EJP - 1;
  } else {
    a = (r + k) % (EJP - 1);
    b = (r - k + (EJP - 1)) % (EJP - 1);
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// Aw = (A + A^T) / 2 zero-padded to N x N, V = I
__global__ void ej_init_kernel(const double* __restrict__ A, int n, int N, double* __restrict__ Aw,
                               double* __restrict__ V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  Aw[e] = (i < n && j < n) ? 0.5 * (A[(int64_t)i * n + j] + A[(int64_t)j * n + i]) : 0.0;
  V[e] = i == j ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(EJT) ej_pair_kernel(double* __restrict__ A, int N, const int2* __restrict__ pr,
                                                      double* __restrict__ Ub, int* __restrict__ nrot,
                                                      int* __restrict__ moved) {
  __shared__ double S[EJP][EJP + 1];
  __shared__ double Ut[EJP][EJP + 1];  // Ut[r][k] = U[k][r]: its rows rotate like those of S
  __shared__ double cs_c[EJP / 2], cs_s[EJP / 2], d_p[EJP / 2], d_q[EJP / 2];
  __shared__ unsigned char lp[EJP - 1][EJP / 2], lq[EJP - 1][EJP / 2];  // the local pairs of every round
  __shared__ int any;
  const int2 ab = pr[blockIdx.x];
  const int t = threadIdx.x;
  for (int e = t; e < EJP * EJP; e += EJT) {
    const int i = e / EJP, j = e % EJP;
    S[i][j] = A[(int64_t)ej_g(i, ab) * N + ej_g(j, ab)];
    Ut[i][j] = i == j ? 1.0 : 0.0;
  }
  for (int e = t; e < (EJP - 1) * (EJP / 2); e += EJT) {
    int p, q;
    ej_local_pair(e / (EJP / 2), e % (EJP / 2), p, q);
    lp[e / (EJP / 2)][e % (EJP / 2)] = (unsigned char)p;
    lq[e / (EJP / 2)][e % (EJP / 2)] = (unsigned char)q;
  }
  if (t == 0) any = 0;
  __syncthreads();
  for (int r = 0; r < EJP - 1; ++r) {
    // the rotation of local pair t, and its rotated diagonal
    if (t < EJP / 2) {
      const int p = lp[r][t], q = lq[r][t];
      const double apq = S[p][q], app = S[p][p], aqq = S[q][q];
      double c = 1.0, s = 0.0, dp = app, dq = aqq;
      if (apq != 0.0 && fabs(apq) > EJ_TOL * sqrt(fabs(app * aqq))) {
        const double th = (aqq - app) / (2.0 * apq);
        double tt = 1.0 / (fabs(th) + sqrt(1.0 + th * th));
        if (th < 0.0) tt = -tt;
        c = 1.0 / sqrt(1.0 + tt * tt);
        s = tt * c;
        dp = app - tt * apq;
        dq = aqq + tt * apq;
        any = 1;  // every writer stores the same value
      }
      cs_c[t] = c;
      cs_s[t] = s;
      d_p[t] = dp;
      d_q[t] = dq;
    }
    __syncthreads();
    // S <- J^T S J as 2 x 2 blocks (rows p_k, q_k) x (columns p_k2, q_k2): every
    // element is read and written by one thread, so rows and columns need no
    // barrier between them; the diagonal blocks take the exact rotated values.
    // Thread t takes the column pair k2 = t % 32 and the row pairs t / 32 + 8 m,
    // and issues all its loads before its stores.
    {
      const int k2 = t % (EJP / 2);
      const double c2 = cs_c[k2], s2 = cs_s[k2];
      const int p2 = lp[r][k2], q2 = lq[r][k2];
      int pk[4], qk[4];
      double ck[4], sk[4], x[4][4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = t / (EJP / 2) + 8 * m;
        pk[m] = lp[r][k];
        qk[m] = lq[r][k];
        ck[m] = cs_c[k];
        sk[m] = cs_s[k];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        x[m][0] = S[pk[m]][p2];
        x[m][1] = S[pk[m]][q2];
        x[m][2] = S[qk[m]][p2];
        x[m][3] = S[qk[m]][q2];
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int k = t / (EJP / 2) + 8 * m;
        const int p = pk[m], q = qk[m];
        if (k == k2) {
          if (s2 != 0.0) {
            S[p][p] = d_p[k];
            S[q][q] = d_q[k];
            S[p][q] = 0.0;
            S[q][p] = 0.0;
          }
          continue;
        }
        const double c1 = ck[m], s1 = sk[m];
        if (s1 == 0.0 && s2 == 0.0) continue;
        // rows: J_k^T x, then columns: y J_k2
        const double ypp = c1 * x[m][0] - s1 * x[m][2], ypq = c1 * x[m][1] - s1 * x[m][3];
        const double yqp = s1 * x[m][0] + c1 * x[m][2], yqq = s1 * x[m][1] + c1 * x[m][3];
        S[p][p2] = c2 * ypp - s2 * ypq;
        S[p][q2] = s2 * ypp + c2 * ypq;
        S[q][p2] = c2 * yqp - s2 * yqq;
        S[q][q2] = s2 * yqp + c2 * yqq;
      }
    }
    // rows p, q of U^T: thread t takes column j = t % 64 of the pairs t / 64 + 4 m
    {
      const int j = t % EJP;
      int pk[8], qk[8];
      double u[8], v[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int k = t / EJP + 4 * m;
        pk[m] = lp[r][k];
        qk[m] = lq[r][k];
        u[m] = Ut[pk[m]][j];
        v[m] = Ut[qk[m]][j];
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int k = t / EJP + 4 * m;
        const double s = cs_s[k];
        if (s == 0.0) continue;
        const double c = cs_c[k];
        Ut[pk[m]][j] = c * u[m] - s * v[m];
        Ut[qk[m]][j] = s * u[m] + c * v[m];
      }
    }
    __syncthreads();
  }
  for (int e = t; e < EJP * EJP; e += EJT) {
    const int i = e / EJP, j = e % EJP;
    A[(int64_t)ej_g(i, ab) * N + ej_g(j, ab)] = S[i][j];
    Ub[(int64_t)blockIdx.x * EJP * EJP + e] = Ut[j][i];  // U[i][j]
  }
  if (t == 0) {
    moved[blockIdx.x] = any;  // 0: U is exactly the identity
    if (any) atomicAdd(nrot, 1);
  }
}

// blockIdx.x < ntri: off-diagonal block (I, J), I > J, of the pairs, A_IJ <- U_I^T A_IJ U_J
// (and A_JI its transpose); else the eigenvector columns of pair I over 64 rows of V.
// Pairs whose U is exactly the identity (moved[I] == 0) leave their blocks as they are.
__global__ void __launch_bounds__(EJT) ej_apply_kernel(double* __restrict__ A, double* __restrict__ V, int N,
                                                       const int2* __restrict__ pr, const double* __restrict__ Ub,
                                                       const int* __restrict__ moved, int np, int ntri) {
  __shared__ double X[EJP][EJP + 1];
  __shared__ double U[EJP][EJP + 1];
  const int t = threadIdx.x;
  const int r0 = (t / 16) * 4, c0 = (t % 16) * 4;
  double acc[4][4];
  if ((int)blockIdx.x < ntri) {
    const int b = blockIdx.x;
    int I = (int)((sqrt(8.0 * b + 1.0) + 1.0) * 0.5);
    while (I * (I - 1) / 2 > b) --I;
    while ((I + 1) * I / 2 <= b) ++I;
    const int J = b - I * (I - 1) / 2;
    if (!moved[I] && !moved[J]) return;
    const int2 pI = pr[I], pJ = pr[J];
    for (int e = t; e < EJP * EJP; e += EJT) {
      const int i = e / EJP, j = e % EJP;
      X[i][j] = A[(int64_t)ej_g(i, pI) * N + ej_g(j, pJ)];
      U[i][j] = Ub[(int64_t)I * EJP * EJP + e];
    }
    __syncthreads();
    // T = U_I^T X: T[r][c] = sum_k U_I[k][r] X[k][c]
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k = 0; k < EJP; ++k) {
      double u[4], x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) u[i] = U[k][r0 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = X[k][c0 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(u[i], x[j], acc[i][j]);
    }
    __syncthreads();
    // X <- T^T, U <- U_J
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) X[c0 + j][r0 + i] = acc[i][j];
    for (int e = t; e < EJP * EJP; e += EJT) U[e / EJP][e % EJP] = Ub[(int64_t)J * EJP * EJP + e];
    __syncthreads();
    // R = T U_J: R[r][c] = sum_k T^T[k][r] U_J[k][c]
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
    for (int k = 0; k < EJP; ++k) {
      double u[4], x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = X[k][r0 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) u[j] = U[k][c0 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], u[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gr = ej_g(r0 + i, pI), gc = ej_g(c0 + j, pJ);
        A[(int64_t)gr * N + gc] = acc[i][j];
        A[(int64_t)gc * N + gr] = acc[i][j];
      }
    return;
  }
  // eigenvectors: rows [64 s, 64 s + 64) of V, columns of pair I: V_:I <- V_:I U_I
  const int b = blockIdx.x - ntri;
  const int I = b % np, strip = b / np;
  if (!moved[I]) return;
  const int2 pI = pr[I];
  for (int e = t; e < EJP * EJP; e += EJT) {
    const int i = e / EJP, k = e % EJP;
    X[k][i] = V[(int64_t)(strip * EJP + i) * N + ej_g(k, pI)];  // X[k][i] = V[row i][col k]
    U[i][k] = Ub[(int64_t)I * EJP * EJP + e];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k = 0; k < EJP; ++k) {
    double x[4], u[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = X[k][r0 + i];
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = U[k][c0 + j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], u[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) V[(int64_t)(strip * EJP + r0 + i) * N + ej_g(c0 + j, pI)] = acc[i][j];
}

__global__ void ej_diag_kernel(const double* __restrict__ Aw, int N, int n, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = Aw[(int64_t)i * N + i];
}

// rows of A: eigenvectors in ascending order, w the eigenvalues
__global__ void ej_out_kernel(const double* __restrict__ Aw, const double* __restrict__ V, int N, int n,
                              const int* __restrict__ idx, double* __restrict__ A, double* __restrict__ w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int k = (int)(e / n), mu = (int)(e % n);
  const int c = idx[k];
  A[e] = V[(int64_t)mu * N + c];
  if (mu == 0) w[k] = Aw[(int64_t)c * N + c];
}

struct EjDims {
  int N, nb, np;
};

EjDims ej_dims(int n) {
  EjDims d;
  d.N = (n + EJP - 1) / EJP * EJP;
  d.nb = d.N / EJB;
  d.np = d.nb / 2;
  return d;
}

}  // namespace

size_t sym_eig_work_bytes(int n) {
  const EjDims d = ej_dims(std::max(n, 1));
  auto a = [](size_t x) { return (x + 255) / 256 * 256; };
  return 2 * a(8 * (size_t)d.N * d.N) + a(8 * (size_t)d.np * EJP * EJP) +
         a(sizeof(int) * 2 * (size_t)(d.nb - 1) * d.np) + a(8 * (size_t)d.N) + a(sizeof(int) * (size_t)d.N) +
         a(sizeof(int) * (size_t)d.np) + 512;
}

int sym_eig(double* A, int n, double* w, hipStream_t st) {
  if (n <= 0) return 0;
  const EjDims d = ej_dims(n);
  const int N = d.N, nb = d.nb, np = d.np;
  DevMem Aw(8 * (size_t)N * N), V(8 * (size_t)N * N), Ub(8 * (size_t)np * EJP * EJP);
  // the rounds of a sweep: circle method over the nb blocks
  std::vector<int> prh(2 * (size_t)(nb - 1) * np);
  for (int r = 0; r < nb - 1; ++r)
    for (int k = 0; k < np; ++k) {
      int a, b;
      if (k == 0) {
        a = r;
        b = nb - 1;
      } else {
        a = (r + k) % (nb - 1);
        b = (r - k + (nb - 1)) % (nb - 1);
      }
      prh[2 * ((size_t)r * np + k)] = std::min(a, b);
      prh[2 * ((size_t)r * np + k) + 1] = std::max(a, b);
    }
  DevMem prd = upload(prh, st), cnt(sizeof(int)), dg(8 * (size_t)N), idxd(sizeof(int) * (size_t)N),
      mv(sizeof(int) * (size_t)np);
  const int64_t NN = (int64_t)N * N;
  hipLaunchKernelGGL(ej_init_kernel, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, st, A, n, N,
                     Aw.as<double>(), V.as<double>());
  const int ntri = np * (np - 1) / 2, nstrip = N / EJP;
  int sweeps = 0;
  for (;;) {
    if (sweeps == 40) throw Error(DFX_EHIP, "sym_eig: no convergence in 40 sweeps");
    DFX_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int), st));
    for (int r = 0; r < nb - 1; ++r) {
      const int2* pr = reinterpret_cast<const int2*>(prd.as<int>() + 2 * (size_t)r * np);
      hipLaunchKernelGGL(ej_pair_kernel, dim3(np), dim3(EJT), 0, st, Aw.as<double>(), N, pr, Ub.as<double>(),
                         cnt.as<int>(), mv.as<int>());
      hipLaunchKernelGGL(ej_apply_kernel, dim3(ntri + nstrip * np), dim3(EJT), 0, st, Aw.as<double>(),
                         V.as<double>(), N, pr, Ub.as<double>(), mv.as<int>(), np, ntri);
    }
    ++sweeps;
    int h = 0;
    DFX_HIP(hipMemcpyAsync(&h, cnt.p, sizeof(int), hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
    if (h == 0) break;
  }
  // ascending order (ties by index, so the result is deterministic)
  hipLaunchKernelGGL(ej_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, Aw.as<double>(), N, n,
                     dg.as<double>());
  std::vector<double> dh(n);
  DFX_HIP(hipMemcpyAsync(dh.data(), dg.p, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
  DFX_HIP(hipStreamSynchronize(st));
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return dh[a] < dh[b]; });
  DFX_HIP(hipMemcpyAsync(idxd.p, idx.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, st));
  const int64_t nn = (int64_t)n * n;
  hipLaunchKernelGGL(ej_out_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, Aw.as<double>(),
                     V.as<double>(), N, n, idxd.as<int>(), A, w);
  DFX_HIP(hipGetLastError());
  DFX_HIP(hipStreamSynchronize(st));  // the host index vector goes out of scope
  return sweeps;
}

}  // namespace dfx
