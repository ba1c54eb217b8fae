// Restricted Hartree-Fock with density-fitted J and K (section "Standard
// algorithms": the Fock builder is built on the density-fitting operations).
//
//   D = C_occ C_occ^T,  F = h + 2 J[D] - K[D],  E = tr D (h + F) + E_nn,
//   DIIS (Pulay) on e = X^T (F D S - S D F) X, X the canonical orthogonaliser,
//   aufbau on the lowest nocc eigenvalues of X^T F X.
//
// Everything lives on the GPU; per iteration only E, max|e| and the DIIS
// overlaps (a few doubles) travel to the host, where the (m+1)x(m+1) DIIS
// system is solved.
//
// The occupied space of X^T F X comes from trace-correcting purification
// (Niklasson, Phys. Rev. B 66, 155115 (2002)) -- FP64 matrix products only --
// followed by a Cholesky QR (applied twice) of the projector times the previous
// occupied orbitals; the library's block Jacobi eigensolver (eig.hip) serves
// the first update from the core guess, the final orbitals and energies, and
// any purification that does not converge.  The orthonormal basis is Loewdin's
// S^-1/2 by Newton-Schulz where no function is near the drop threshold.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>

#include "host.h"

namespace dfx {

// ---- element-wise and reduction kernels ----------------------------------------
__global__ void fock_kernel(const double* h, const double* J, const double* K, double* F, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) F[i] = h[i] + 2.0 * J[i] - K[i];
}

// F = h + J - K (one spin of the unrestricted Fock matrices)
__global__ void uhf_fock_kernel(const double* h, const double* J, const double* K, double* F, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) F[i] = h[i] + J[i] - K[i];
}

// Roothaan's effective Fock matrix in the orthonormal basis from F_alpha',
// F_beta' and the projectors P_a, P_b onto the alpha and beta occupied spaces
// (core P_c = P_b, open P_o = P_a - P_b, virtual P_v = I - P_a): core-open
// blocks take F_beta, open-virtual F_alpha, all others A = (F_alpha + F_beta) / 2.
// With Delta = (F_alpha - F_beta) / 2 that is R = A + Z + Z^T, Z = P_o Delta (P_v - P_c).
// Step 1: Delta and P_o.
__global__ void rohf_delta_kernel(const double* Fa, const double* Fb, const double* Pa, const double* Pb,
                                  double* Dl, double* Po, int64_t m2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m2) return;
  Dl[i] = 0.5 * (Fa[i] - Fb[i]);
  Po[i] = Pa[i] - Pb[i];
}
// Step 2: P_v - P_c = I - P_a - P_b.
__global__ void rohf_vc_kernel(const double* Pa, const double* Pb, double* Q, int m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)m * m) return;
  Q[i] = (i / m == i % m ? 1.0 : 0.0) - Pa[i] - Pb[i];
}
// Step 3: R = A + Z + Z^T.
__global__ void rohf_feff_kernel(const double* Fa, const double* Fb, const double* Z, double* R, int m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)m * m) return;
  const int r = (int)(i / m), c = (int)(i % m);
  R[i] = 0.5 * (Fa[i] + Fb[i]) + Z[i] + Z[(int64_t)c * m + r];
}

// F += b (S - T): the level shift of one UHF spin, T = S D_s S
__global__ void shift_ao_kernel(double* F, const double* S, const double* T, double b, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) F[i] += b * (S[i] - T[i]);
}

// F += b (I - D / 2) on an m x m matrix of the orthonormal basis (ROHF level shift)
__global__ void shift_orth_kernel(double* F, const double* D, double b, int m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)m * m) return;
  F[i] += b * ((i / m == i % m ? 1.0 : 0.0) - 0.5 * D[i]);
}

__global__ void add_kernel(const double* a, const double* b, double* c, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) c[i] = a[i] + b[i];
}

// partial sums of a . b (or of a . (b + c) when c != null), fixed order
__global__ void dot_partial_kernel(const double* a, const double* b, const double* c, int64_t n,
                                   double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i] * (c ? b[i] + c[i] : b[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void maxabs_partial_kernel(const double* a, int64_t n, double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s = fmax(s, fabs(a[i]));
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// E = A - A^T
__global__ void antisym_kernel(const double* A, double* E, int n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n) return;
  const int r = (int)(i / n), c = (int)(i % n);
  E[i] = A[i] - A[(int64_t)c * n + r];
}

struct Comb {
  const double* F[16];
  double c[16];
  int m;
};
__global__ void lincomb_kernel(Comb cb, double* out, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  double s = 0.0;
  for (int k = 0; k < cb.m; ++k) s += cb.c[k] * cb.F[k][i];
  out[i] = s;
}

// X[mu][k] = W[ndrop + k][mu] / sqrt(s[ndrop + k]); rows of W are eigenvectors of S
__global__ void build_x_kernel(const double* W, const double* s, int n, int ndrop, int m, double* X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * m) return;
  const int mu = (int)(i / m), k = (int)(i % m);
  X[i] = W[(int64_t)(ndrop + k) * n + mu] / sqrt(s[ndrop + k]);
}

// U[mu][k] = W[ndrop + k][mu]: the kept eigenvectors of S as columns
__global__ void build_u_kernel(const double* W, int n, int ndrop, int m, double* U) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * m) return;
  const int mu = (int)(i / m), k = (int)(i % m);
  U[i] = W[(int64_t)(ndrop + k) * n + mu];
}

// T[k][mu] = sqrt(max(s_k, 0)) W[k][mu]
__global__ void scale_rows_sqrt_kernel(const double* W, const double* s, int n, double* T) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * n) return;
  T[i] = W[i] * sqrt(fmax(s[i / n], 0.0));
}

__global__ void copy_cols_kernel(const double* A, int lda, int rows, int cols, double* B, int ldb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int r = (int)(i / cols), c = (int)(i % cols);
  B[(int64_t)r * ldb + c] = A[(int64_t)r * lda + c];
}

// ---- purification kernels (X^T F X is m x m, row-major) -------------------------
// Gershgorin discs of row r: centre A_rr, radius sum_{j != r} |A_rj|
__global__ void gersh_kernel(const double* __restrict__ A, int m, double* __restrict__ lo, double* __restrict__ hi) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  const double* row = A + (int64_t)r * m;
  double s = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x)
    if (j != r) s += fabs(row[j]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lo[r] = row[r] - red[0];
    hi[r] = row[r] + red[0];
  }
}

// out[0] = min lo, out[1] = max hi (one block)
__global__ void minmax_kernel(const double* __restrict__ lo, const double* __restrict__ hi, int m,
                              double* __restrict__ out) {
  __shared__ double a[256], b[256];
  double x = 1e300, y = -1e300;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    x = fmin(x, lo[i]);
    y = fmax(y, hi[i]);
  }
  a[threadIdx.x] = x;
  b[threadIdx.x] = y;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      a[threadIdx.x] = fmin(a[threadIdx.x], a[threadIdx.x + o]);
      b[threadIdx.x] = fmax(b[threadIdx.x], b[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = a[0];
    out[1] = b[0];
  }
}

// P0 = (emax I - F) / (emax - emin): spectrum mapped into [0, 1], occupied levels high
__global__ void tc2_init_kernel(const double* __restrict__ F, int m, double emax, double inv_w,
                                double* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)m * m) return;
  const int r = (int)(i / m), c = (int)(i % m);
  P[i] = ((r == c ? emax : 0.0) - F[i]) * inv_w;
}

// out[0] = tr P, out[1] = tr P2 (one block, fixed order)
__global__ void trace2_kernel(const double* __restrict__ P, const double* __restrict__ P2, int m,
                              double* __restrict__ out) {
  __shared__ double a[256], b[256];
  double x = 0.0, y = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    x += P[(int64_t)i * m + i];
    y += P2[(int64_t)i * m + i];
  }
  a[threadIdx.x] = x;
  b[threadIdx.x] = y;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      a[threadIdx.x] += a[threadIdx.x + o];
      b[threadIdx.x] += b[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = a[0];
    out[1] = b[0];
  }
}

// P <- 2 P - P2
__global__ void tc2_raise_kernel(double* __restrict__ P, const double* __restrict__ P2, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) P[i] = 2.0 * P[i] - P2[i];
}

// Y[k][j] = V[row0 + j][k]: eigenvectors (rows of V) row0 .. row0 + nocc - 1 as columns
__global__ void rows_to_cols_kernel(const double* __restrict__ V, int m, int row0, int nocc, double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)m * nocc) return;
  const int k = (int)(i / nocc), j = (int)(i % nocc);
  Y[i] = V[(int64_t)(row0 + j) * m + k];
}

// out[0] = min_i |G_ii|, out[1] = max_i |G_ii| (one block)
__global__ void diag_minmax_kernel(const double* __restrict__ G, int k, double* __restrict__ out) {
  __shared__ double a[256], b[256];
  double x = 1e300, y = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double v = fabs(G[(int64_t)i * k + i]);
    x = fmin(x, v);
    y = fmax(y, v);
  }
  a[threadIdx.x] = x;
  b[threadIdx.x] = y;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      a[threadIdx.x] = fmin(a[threadIdx.x], a[threadIdx.x + o]);
      b[threadIdx.x] = fmax(b[threadIdx.x], b[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = a[0];
    out[1] = b[0];
  }
}

// Y[i] uniform in [-1, 1) from a counter hash (SplitMix64 finaliser): a start for
// the Cholesky QR of P Y when there are no previous orbitals
__global__ void rand_fill_kernel(double* __restrict__ Y, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  Y[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// A = -A (element-wise)
__global__ void negate_kernel(double* __restrict__ A, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[i] = -A[i];
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// The calling thread's SCF stream and rocBLAS handle on the current device,
// made on first use and kept until the process ends: a call neither creates
// nor destroys them (the handle also keeps the eigensolver's device scratch
// between calls).
DevCtx& thread_ctx() {
  static thread_local std::map<int, DevCtx> ctx;
  int dev = 0;
  DFX_HIP(hipGetDevice(&dev));
  DevCtx& c = ctx[dev];
  if (!c.st) DFX_HIP(hipStreamCreate(&c.st));
  return c;
}

// Newton-Schulz square roots: Y = S / c, Z = I
__global__ void ns_init_kernel(const double* __restrict__ Sm, int n, double inv_c, double* __restrict__ Y,
                               double* __restrict__ Z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  Y[e] = Sm[e] * inv_c;
  Z[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// T = (3 I - P) / 2 with P = Z Y; P <- P - I, whose largest element is the residual
__global__ void ns_t_kernel(double* __restrict__ P, int n, double* __restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const double d = (e / n == e % n) ? 1.0 : 0.0;
  const double p = P[e];
  T[e] = 1.5 * d - 0.5 * p;
  P[e] = p - d;
}

__global__ void scale_kernel(double* __restrict__ A, int64_t cnt, double a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) A[e] *= a;
}

// y = A x (n x n), one workgroup per row, fixed-order reduction
__global__ void matvec_kernel(const double* __restrict__ A, int n, const double* __restrict__ x,
                              double* __restrict__ y) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) s = fma(A[(int64_t)i * n + j], x[j], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) y[i] = red[0];
}

// ---- driver ---------------------------------------------------------------------------
struct Scf {
  hipStream_t st{};
  int n = 0, m = 0, nocc = 0;
  DevMem part, gw;  // gw: split-K partial products
  DevMem qr_linv, qr_work, qr_z, qr_info;  // Cholesky QR of the purified occupied space
  std::vector<double> hpart;
  EventSpans* eig_spans = nullptr;
  int verbose = 0;

  double reduce_sum(const double* a, const double* b, const double* c, int64_t cnt) {
    const int nb = 512;
    hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(256), 0, st, a, b, c, cnt, part.as<double>());
    hpart.resize(nb);
    DFX_HIP(hipMemcpyAsync(hpart.data(), part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : hpart) s += v;
    return s;
  }
  double reduce_max(const double* a, int64_t cnt) {
    const int nb = 512;
    hipLaunchKernelGGL(maxabs_partial_kernel, dim3(nb), dim3(256), 0, st, a, cnt, part.as<double>());
    hpart.resize(nb);
    DFX_HIP(hipMemcpyAsync(hpart.data(), part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : hpart) s = std::max(s, v);
    return s;
  }
  void gemm(int M, int N, int K, const double* A, int lda, bool ta, const double* B, int ldb, bool tb,
            double* C, int ldc, double alpha = 1.0, double beta = 0.0) {
    GemmF64 g{};
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda; g.ta = ta;
    g.B = B; g.ldb = ldb; g.tb = tb;
    g.C = C; g.ldc = ldc;
    g.alpha = alpha; g.beta = beta; g.batch = 1;
    dgemm_sk(g, gw.p ? gw.as<double>() : nullptr, (int64_t)(gw.n / sizeof(double)), st);
  }
  // S^-1/2 and S^1/2 of the symmetric positive definite n x n matrix Sm by the
  // coupled Newton-Schulz iteration (N. J. Higham, "Functions of Matrices",
  // SIAM 2008, sec. 6.7): with c >= lambda_max(S) (the largest Gershgorin
  // bound), Y0 = S / c, Z0 = I, T = (3 I - Z Y) / 2, Y <- Y T, Z <- T Z; then
  // Y -> (S / c)^1/2 and Z -> (S / c)^-1/2 for any spectrum in (0, c].  Once
  // max |I - Z Y| < 1e-8 one more step reaches the rounding level.  buf: four
  // n x n buffers; on return isq = S^-1/2 and sq = S^1/2 point into them, and
  // lmin estimates lambda_min(S) as 1 / |S^-1/2|_2^2 from 40 power steps
  // (an upper estimate: the power iteration approaches the norm from below).
  // Returns false if S is not numerically positive definite (no convergence
  // in 100 steps, or a non-finite residual).  Synchronous.
  bool inv_sqrt(const double* Sm, int nn, double* const buf[4], double*& isq, double*& sq, double& lmin,
                int& steps) {
    const int64_t n2 = (int64_t)nn * nn;
    DevMem lh(16 * (size_t)nn), vw(16 * (size_t)nn + 16);
    double b[2];
    hipLaunchKernelGGL(gersh_kernel, dim3(nn), dim3(256), 0, st, Sm, nn, lh.as<double>(), lh.as<double>() + nn);
    hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(256), 0, st, lh.as<double>(), lh.as<double>() + nn, nn,
                       part.as<double>());
    DFX_HIP(hipMemcpyAsync(b, part.p, sizeof b, hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
    const double c = b[1];
    if (!(c > 0.0) || !std::isfinite(c)) return false;
    double *Y = buf[0], *Z = buf[1], *T = buf[2], *P = buf[3];
    hipLaunchKernelGGL(ns_init_kernel, dim3(nblk(n2)), dim3(256), 0, st, Sm, nn, 1.0 / c, Y, Z);
    bool last = false, ok = false;
    for (steps = 0; steps < 100; ++steps) {
      gemm(nn, nn, nn, Z, nn, false, Y, nn, false, P, nn);  // Z Y
      hipLaunchKernelGGL(ns_t_kernel, dim3(nblk(n2)), dim3(256), 0, st, P, nn, T);
      const double r = reduce_max(P, n2);
      if (!std::isfinite(r)) return false;
      if (last) {
        ok = r < 1e-10;
        break;
      }
      gemm(nn, nn, nn, Y, nn, false, T, nn, false, P, nn);  // Y T
      std::swap(Y, P);
      gemm(nn, nn, nn, T, nn, false, Z, nn, false, P, nn);  // T Z
      std::swap(Z, P);
      if (r < 1e-8) last = true;
    }
    if (!ok) return false;
    hipLaunchKernelGGL(scale_kernel, dim3(nblk(n2)), dim3(256), 0, st, Z, n2, 1.0 / std::sqrt(c));
    hipLaunchKernelGGL(scale_kernel, dim3(nblk(n2)), dim3(256), 0, st, Y, n2, std::sqrt(c));
    isq = Z;
    sq = Y;
    // |S^-1/2|_2 by power steps from a seeded start
    double* v = vw.as<double>();
    double* w = v + nn;
    hipLaunchKernelGGL(rand_fill_kernel, dim3(nblk(nn)), dim3(256), 0, st, v, (int64_t)nn, (uint64_t)0x2545F4914F6CDD1Dull);
    double nrm = 0.0;
    for (int k = 0; k < 40; ++k) {
      const double vv = reduce_sum(v, v, nullptr, nn);
      if (!(vv > 0.0)) return false;
      hipLaunchKernelGGL(scale_kernel, dim3(nblk(nn)), dim3(256), 0, st, v, (int64_t)nn, 1.0 / std::sqrt(vv));
      hipLaunchKernelGGL(matvec_kernel, dim3(nn), dim3(256), 0, st, Z, nn, v, w);
      nrm = std::sqrt(reduce_sum(w, w, nullptr, nn));
      std::swap(v, w);
    }
    lmin = 1.0 / (nrm * nrm);
    return true;
  }

  // P2 = P P^T, which is P^2 for the symmetric P: the symmetric product (half the
  // FLOPs) where the row stride allows it, else the general product
  void square_sym(const double* P, double* P2) {
    if (m % 2 == 0 && gw.n >= sizeof(double) * syrk_f64_work_elems(m))
      syrk_f64(P, m, m, m, P2, gw.as<double>(), st);
    else
      gemm(m, m, m, P, m, false, P, m, false, P2, m);
  }
  // Occupied space of the symmetric m x m matrix F (the nocc lowest levels) by
  // trace-correcting purification: P0 = (e_max I - F) / (e_max - e_min) with
  // Gershgorin bounds, then P <- P^2 or 2P - P^2, whichever moves tr P toward
  // nocc, until sum lambda (1 - lambda) = tr P - tr P^2 < 1e-9 nocc, plus three
  // more steps.  The projector times the previous occupied orbitals Y, put
  // through a Cholesky QR twice (the library's blocked Cholesky and L^-1, no
  // vendor solver), is the new Y (m x nocc, orthonormal columns).
  // P and P2 are m x m work, Z m x nocc, G nocc x nocc, lohi 2m.  Returns false,
  // Y unchanged, if the iteration does not settle in 100 steps, the trace
  // misses nocc, or Z = P Y is too ill-conditioned (a Cholesky pivot below
  // 1e-4 of the largest).
  bool purify_occ(const double* F, double* P, double* P2, double* Y, double* Z, double* G, double* lohi,
                  int& steps, const char*& why) {
    double b[2];
    hipLaunchKernelGGL(gersh_kernel, dim3(m), dim3(256), 0, st, F, m, lohi, lohi + m);
    hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(256), 0, st, lohi, lohi + m, m, part.as<double>());
    DFX_HIP(hipMemcpyAsync(b, part.p, sizeof b, hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
    const double w = b[1] - b[0];
    why = "spectral bounds";
    if (!(w > 0.0) || !std::isfinite(w)) return false;
    if (verbose) std::fprintf(stderr, "dfx_scf purification: Gershgorin [%.3f, %.3f]\n", b[0], b[1]);
    const int64_t mm = (int64_t)m * m;
    hipLaunchKernelGGL(tc2_init_kernel, dim3(nblk(mm)), dim3(256), 0, st, F, m, b[1], 1.0 / w, P);
    int settled = 0;
    bool ok = false;
    for (steps = 0; steps < 100; ++steps) {
      square_sym(P, P2);
      hipLaunchKernelGGL(trace2_kernel, dim3(1), dim3(256), 0, st, P, P2, m, part.as<double>());
      DFX_HIP(hipMemcpyAsync(b, part.p, sizeof b, hipMemcpyDeviceToHost, st));
      DFX_HIP(hipStreamSynchronize(st));
      if (!std::isfinite(b[0]) || !std::isfinite(b[1])) return false;
      if (b[0] - b[1] < 1e-9 * nocc && ++settled > 3) {
        ok = std::fabs(b[0] - nocc) < 1e-6;
        why = "trace";
        break;
      }
      why = "not settled";
      if (std::fabs(b[1] - nocc) < std::fabs(2.0 * b[0] - b[1] - nocc))
        std::swap(P, P2);
      else
        hipLaunchKernelGGL(tc2_raise_kernel, dim3(nblk(mm)), dim3(256), 0, st, P, P2, mm);
    }
    if (!ok) return false;
    // Cholesky QR, twice, with the library's own factorisation: G = Z^T Z = L L^T,
    // Z <- Z L^-T (then Z^T Z = L^-1 G L^-T = I)
    const size_t mo = (size_t)m * nocc;
    if (qr_linv.n < sizeof(double) * (size_t)nocc * nocc) qr_linv.alloc(sizeof(double) * (size_t)nocc * nocc);
    if (qr_work.n < sizeof(double) * cholesky_work_elems(nocc))
      qr_work.alloc(sizeof(double) * cholesky_work_elems(nocc));
    if (qr_z.n < sizeof(double) * mo) qr_z.alloc(sizeof(double) * mo);
    if (!qr_info.p) qr_info.alloc(sizeof(int));
    double* Zc = Z;
    double* Zn = qr_z.as<double>();
    gemm(m, nocc, m, P, m, false, Y, nocc, false, Zc, nocc);  // Z = P Y
    for (int pass = 0; pass < 2; ++pass) {
      gemm(nocc, nocc, m, Zc, nocc, true, Zc, nocc, false, G, nocc);  // G = Z^T Z
      cholesky_inverse(G, nocc, qr_linv.as<double>(), qr_work.as<double>(), qr_info.as<int>(), st);
      hipLaunchKernelGGL(diag_minmax_kernel, dim3(1), dim3(256), 0, st, G, nocc, part.as<double>());  // diag of L
      int info = 0;
      DFX_HIP(hipMemcpyAsync(&info, qr_info.p, sizeof(int), hipMemcpyDeviceToHost, st));
      DFX_HIP(hipMemcpyAsync(b, part.p, sizeof b, hipMemcpyDeviceToHost, st));
      DFX_HIP(hipStreamSynchronize(st));
      why = "Cholesky QR";
      if (info != 0 || !(b[0] > 1e-4 * b[1])) return false;
      gemm(m, nocc, nocc, Zc, nocc, false, qr_linv.as<double>(), nocc, true, Zn, nocc);  // Z L^-T
      std::swap(Zc, Zn);
    }
    DFX_HIP(hipMemcpyAsync(Y, Zc, sizeof(double) * mo, hipMemcpyDeviceToDevice, st));
    return true;
  }
  // symmetric eigen-decomposition in place: A (k x k) -> rows are eigenvectors, w ascending
  // (the library's block Jacobi, eig.hip)
  void syevd(double* A, int k, double* w) {
    if (eig_spans) eig_spans->begin();
    sym_eig(A, k, w, st);
    if (eig_spans) eig_spans->end();
  }
};

// The orthogonaliser X (n x m, X^T S X = I) of the SCF's orthonormal basis.
// Loewdin's X = S^-1/2 (m = n) by Newton-Schulz when the smallest eigenvalue of
// S is at least 100 ortho_thresh: no function would be dropped, and the span is
// that of every other choice.  Otherwise canonical orthogonalisation, X = U
// s^-1/2 over the eigenvalues above ortho_thresh (the block Jacobi
// eigensolver); with want_u, U gets those eigenvectors (n x m).
struct Ortho {
  DevMem X, U;
  int m = 0;
  bool lowdin = false;
  double lmin = 0.0;
  int ns_steps = 0;
};

static Ortho make_orthogonalizer(Scf& S, const double* Sm, int n, double thresh, bool want_u) {
  Ortho r;
  hipStream_t st = S.st;
  const int64_t n2 = (int64_t)n * n;
  {
    DevMem b4[4];
    double* buf[4];
    for (int k = 0; k < 4; ++k) {
      b4[k].alloc(8 * (size_t)n2);
      buf[k] = b4[k].as<double>();
    }
    double *isq = nullptr, *sq = nullptr;
    if (S.inv_sqrt(Sm, n, buf, isq, sq, r.lmin, r.ns_steps) && r.lmin >= 100.0 * thresh) {
      for (int k = 0; k < 4; ++k)
        if (buf[k] == isq) r.X = std::move(b4[k]);
      r.m = n;
      r.lowdin = true;
      if (S.verbose)
        std::fprintf(stderr, "dfx_scf: Loewdin orthogonaliser, %d Newton-Schulz steps, lambda_min(S) ~ %.3e\n",
                     r.ns_steps, r.lmin);
      return r;
    }
  }
  DevMem W(8 * n2), sv(8 * (size_t)n);
  DFX_HIP(hipMemcpyAsync(W.p, Sm, 8 * n2, hipMemcpyDeviceToDevice, st));
  S.syevd(W.as<double>(), n, sv.as<double>());
  std::vector<double> s_h(n);
  DFX_HIP(hipMemcpyAsync(s_h.data(), sv.p, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
  DFX_HIP(hipStreamSynchronize(st));
  int ndrop = 0;
  while (ndrop < n && s_h[ndrop] < thresh) ++ndrop;
  r.m = n - ndrop;
  r.lmin = s_h.empty() ? 0.0 : s_h[0];
  if (r.m <= 0) return r;
  r.X.alloc(8 * (size_t)n * r.m);
  hipLaunchKernelGGL(build_x_kernel, dim3(nblk((int64_t)n * r.m)), dim3(256), 0, st, W.as<double>(),
                     sv.as<double>(), n, ndrop, r.m, r.X.as<double>());
  if (want_u) {
    r.U.alloc(8 * (size_t)n * r.m);
    hipLaunchKernelGGL(build_u_kernel, dim3(nblk((int64_t)n * r.m)), dim3(256), 0, st, W.as<double>(), n, ndrop,
                       r.m, r.U.as<double>());
  }
  if (S.verbose) std::fprintf(stderr, "dfx_scf: canonical orthogonaliser, %d of %d functions kept\n", r.m, n);
  return r;
}

// C_sel[mu][j] = W[idx[j]][mu] * scale[j]  (rows of W are eigenvectors)
__global__ void gather_evec_kernel(const double* __restrict__ W, int n, const int* __restrict__ idx,
                                   const double* __restrict__ scale, int r, double* __restrict__ Csel) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * r) return;
  const int mu = (int)(i / r), j = (int)(i % r);
  Csel[i] = W[(int64_t)idx[j] * n + mu] * scale[j];
}

// Solve the bordered DIIS system  [B -1; -1 0] [c; l] = [0; -1]  (Gaussian elimination
// with partial pivoting).  Returns false if it is singular to working precision.
static bool diis_solve(const std::vector<double>& Bm, int m, std::vector<double>& c) {
  const int N = m + 1;
  std::vector<double> A((size_t)N * N, 0.0), r(N, 0.0);
  // scale the error overlaps for conditioning
  double sc = 0.0;
  for (int i = 0; i < m; ++i) sc = std::max(sc, std::fabs(Bm[i * m + i]));
  if (!(sc > 0.0)) return false;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) A[i * N + j] = Bm[i * m + j] / sc;
  for (int i = 0; i < m; ++i) A[i * N + m] = A[m * N + i] = -1.0;
  r[m] = -1.0;
  double amax = 0.0, amin = 1e300;
  for (int k = 0; k < N; ++k) {
    int p = k;
    for (int i = k + 1; i < N; ++i)
      if (std::fabs(A[i * N + k]) > std::fabs(A[p * N + k])) p = i;
    if (p != k) {
      for (int j = 0; j < N; ++j) std::swap(A[k * N + j], A[p * N + j]);
      std::swap(r[k], r[p]);
    }
    const double piv = A[k * N + k];
    amax = std::max(amax, std::fabs(piv));
    amin = std::min(amin, std::fabs(piv));
    if (piv == 0.0) return false;
    for (int i = k + 1; i < N; ++i) {
      const double f = A[i * N + k] / piv;
      for (int j = k; j < N; ++j) A[i * N + j] -= f * A[k * N + j];
      r[i] -= f * r[k];
    }
  }
  if (amin < 1e-14 * amax) return false;
  std::vector<double> x(N);
  for (int k = N - 1; k >= 0; --k) {
    double s = r[k];
    for (int j = k + 1; j < N; ++j) s -= A[k * N + j] * x[j];
    x[k] = s / A[k * N + k];
  }
  c.assign(x.begin(), x.begin() + m);
  return true;
}

// K(D) = K(C+) - K(C-) with D = V diag(lambda) V^T, C+- = V_+- sqrt(|lambda_+-|);
// eigenvalues below 1e-14 max|lambda| are dropped.  Columns go to k_build in
// chunks of at most 512.  Synchronous.
void k_from_density(const JKArgs& a, const double* D, double* K, hipStream_t st) {
  const int n = a.nbf;
  const int64_t n2 = (int64_t)n * n;
  Scf S;
  S.st = st;
  DevMem W(8 * n2), lam(8 * (size_t)n);
  DFX_HIP(hipMemcpyAsync(W.p, D, 8 * n2, hipMemcpyDeviceToDevice, st));
  S.syevd(W.as<double>(), n, lam.as<double>());
  std::vector<double> l(n);
  DFX_HIP(hipMemcpyAsync(l.data(), lam.p, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
  DFX_HIP(hipStreamSynchronize(st));
  double lmax = 0.0;
  for (double x : l) lmax = std::max(lmax, std::fabs(x));
  std::vector<int> pos, neg;
  for (int k = 0; k < n; ++k) {
    if (l[k] > 1e-14 * lmax) pos.push_back(k);
    else if (l[k] < -1e-14 * lmax) neg.push_back(k);
  }
  constexpr int CH = 512;
  DevMem Cs(8 * (size_t)n * CH), Kt(8 * n2), idx_d(sizeof(int) * CH), sc_d(8 * CH);
  DevMem work(k_work_bytes(a, std::min(CH, std::max(1, (int)std::max(pos.size(), neg.size())))));
  fill_f64(K, (size_t)n2, 0.0, st);
  for (int sign = 1; sign >= -1; sign -= 2) {
    const std::vector<int>& sel = sign > 0 ? pos : neg;
    for (size_t c0 = 0; c0 < sel.size(); c0 += CH) {
      const int r = (int)std::min<size_t>(CH, sel.size() - c0);
      std::vector<int> id(sel.begin() + c0, sel.begin() + c0 + r);
      std::vector<double> sc(r);
      for (int j = 0; j < r; ++j) sc[j] = std::sqrt(std::fabs(l[id[j]]));
      DFX_HIP(hipMemcpyAsync(idx_d.p, id.data(), sizeof(int) * r, hipMemcpyHostToDevice, st));
      DFX_HIP(hipMemcpyAsync(sc_d.p, sc.data(), 8 * (size_t)r, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(gather_evec_kernel, dim3(nblk((int64_t)n * r)), dim3(256), 0, st, W.as<double>(), n,
                         idx_d.as<int>(), sc_d.as<double>(), r, Cs.as<double>());
      k_build(a, Cs.as<double>(), r, Kt.as<double>(), work.p, st);
      Comb cb{};
      cb.m = 2;
      cb.F[0] = K;
      cb.c[0] = 1.0;
      cb.F[1] = Kt.as<double>();
      cb.c[1] = (double)sign;
      hipLaunchKernelGGL(lincomb_kernel, dim3(nblk(n2)), dim3(256), 0, st, cb, K, n2);
      DFX_HIP(hipStreamSynchronize(st));  // host vectors of this chunk go out of scope
    }
  }
}

// The arena over opts.workspace (null without one).  The size is checked
// against scf_need before any device work.
static std::unique_ptr<Arena> scf_arena(const dfx_scf_opts& o, const HostShells& hb, const HostShells& ha, int natom,
                                        const char* fn) {
  if (!o.workspace) return nullptr;
  const int64_t need = scf_need(hb, ha, natom, o.diis_size);
  if ((int64_t)o.ws_bytes < need)
    throw Error(DFX_ENOMEM, std::string(fn) + ": workspace of " + std::to_string(o.ws_bytes) + " bytes, " +
                                std::to_string(need) + " needed (dfx_scf_plan)");
  return std::make_unique<Arena>(o.workspace, o.ws_bytes);
}

}  // namespace dfx

using namespace dfx;

extern "C" {

int dfx_scf_plan(const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh, int natom,
                 const dfx_scf_opts* opts, int64_t* bytes) {
  return guard([&] {
    if (!bytes || natom <= 0) throw Error(DFX_EINVAL, "dfx_scf_plan: bad argument");
    dfx_scf_opts o;
    dfx_scf_default_opts(&o);
    if (opts) o = *opts;
    if (o.diis_size < 1 || o.diis_size > 16) throw Error(DFX_EINVAL, "dfx_scf_plan: bad options");
    const HostShells hb = make_shells(shells, nsh, 3, "orbital basis");
    const HostShells ha = make_shells(aux, nauxsh, 4, "auxiliary basis");
    *bytes = scf_need(hb, ha, natom, o.diis_size);
  });
}

void dfx_scf_default_opts(dfx_scf_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tau = 1e-12;
  o->conv_dE = 1e-10;
  o->conv_err = 1e-7;
  o->ortho_thresh = 1e-8;
  o->switch_err = 1e-5;
  o->max_iter = 100;
  o->diis_size = 8;
  o->schedule = DFX_SCHED_FP64;
  o->mixed_prec = DFX_FP32;
  o->guess = DFX_GUESS_CORE;
  o->verbose = 0;
  o->switch_auto = 1;
  o->purify = 1;
}

int dfx_scf(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
            const dfx_scf_opts* opts_in, const double* init, double* E_out, double* C_out, double* eps_out,
            dfx_scf_info* info) {
  int status = DFX_OK;
  const int rc = guard([&] {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (!geom || !E_out) throw Error(DFX_EINVAL, "dfx_scf: NULL argument");
    if (geom->natom <= 0 || !geom->xyz || !geom->Z) throw Error(DFX_EINVAL, "dfx_scf: bad geometry");
    dfx_scf_opts o;
    dfx_scf_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.level_shift != 0.0) throw Error(DFX_EINVAL, "dfx_scf: level_shift applies to dfx_uhf / dfx_rohf only");
    if (o.diis_size < 1 || o.diis_size > 16 || o.max_iter < 1) throw Error(DFX_EINVAL, "dfx_scf: bad options");
    if ((o.guess == DFX_GUESS_CINIT || o.guess == DFX_GUESS_DENSITY) && !init)
      throw Error(DFX_EINVAL, "dfx_scf: guess needs init");
    if (o.guess == DFX_GUESS_LEARNED) {
      if (!o.model) throw Error(DFX_EINVAL, "dfx_scf: learned guess needs a model");
      guess_check_basis(o.model, geom, shells, nsh);
    }
    int nelec = -geom->charge;
    for (int a = 0; a < geom->natom; ++a) nelec += geom->Z[a];
    if (nelec <= 0 || nelec % 2) throw Error(DFX_EINVAL, "dfx_scf: closed shell needs an even, positive electron count");
    const int nocc = nelec / 2;
    HostShells hb = make_shells(shells, nsh, 3, "orbital basis");
    HostShells ha = make_shells(aux, nauxsh, 4, "auxiliary basis");
    const int n = hb.nbf;
    if (nocc > n) throw Error(DFX_EINVAL, "dfx_scf: more occupied orbitals than basis functions");

    // with a caller's workspace every device buffer of the call lives in it
    std::unique_ptr<Arena> arena = scf_arena(o, hb, ha, geom->natom, "dfx_scf");
    ArenaScope scope(arena.get());
    Scf S;
    {
      DevCtx& ctx = thread_ctx();
      S.st = ctx.st;
    }
    hipStream_t st = S.st;
    S.n = n;
    S.nocc = nocc;
    S.part.alloc(sizeof(double) * 512);
    S.gw.alloc(sizeof(double) * std::max<size_t>(4 * (size_t)n * n, syrk_f64_work_elems(n)));
    S.verbose = o.verbose;
    EventSpans sp_eig_all, sp_pur;
    sp_eig_all.st = sp_pur.st = S.st;
    S.eig_spans = &sp_eig_all;
    const int64_t n2 = (int64_t)n * n;

    // ---- setup: fitted integrals, one-electron matrices, E_nn, orthogonaliser
    std::unique_ptr<dfx_B> B = build_B(std::move(hb), std::move(ha), o.tau, 0, st);
    DevMem Sm(8 * n2), Tm(8 * n2), Vm(8 * n2), h(8 * n2);
    int1e_build(B->bas, geom, Sm.as<double>(), Tm.as<double>(), Vm.as<double>(), st);
    hipLaunchKernelGGL(add_kernel, dim3(nblk(n2)), dim3(256), 0, st, Tm.as<double>(), Vm.as<double>(),
                       h.as<double>(), n2);
    Tm.release();
    Vm.release();
    double Enuc = 0.0;
    for (int a = 0; a < geom->natom; ++a)
      for (int b = 0; b < a; ++b) {
        const double* A = geom->xyz + 3 * a;
        const double* Bx = geom->xyz + 3 * b;
        const double r = std::sqrt((A[0] - Bx[0]) * (A[0] - Bx[0]) + (A[1] - Bx[1]) * (A[1] - Bx[1]) +
                                   (A[2] - Bx[2]) * (A[2] - Bx[2]));
        Enuc += (double)geom->Z[a] * geom->Z[b] / r;
      }
    Ortho orth = make_orthogonalizer(S, Sm.as<double>(), n, o.ortho_thresh, o.guess == DFX_GUESS_LEARNED);
    const int m = orth.m;
    if (m < nocc) throw Error(DFX_EINVAL, "dfx_scf: basis too linearly dependent");
    S.m = m;
    DevMem X = std::move(orth.X), Uk = std::move(orth.U);
    const bool lowdin = orth.lowdin;

    DevMem F(8 * n2), D(8 * n2), Jm(8 * n2), Km(8 * n2), t1(8 * n2), t2(8 * n2);
    DevMem Fp(8 * (size_t)m * m), eps(8 * (size_t)m), Cm(8 * (size_t)n * m), Cocc(8 * (size_t)n * nocc);
    const int dsz = o.diis_size;
    std::vector<DevMem> Fh(dsz), Eh(dsz);
    for (int k = 0; k < dsz; ++k) {
      Fh[k].alloc(8 * n2);
      Eh[k].alloc(8 * (size_t)m * m);
    }

    // occupied orbitals of a Fock-like matrix F: Cocc = X Y with Y the nocc lowest
    // levels of F' = X^T F X (kept in Fq), D = Cocc Cocc^T.  Purification when a
    // previous Y exists, else (or if it fails) the full eigen-decomposition, which also gives C and eps.
    DevMem Fq(8 * (size_t)m * m), Yo(8 * (size_t)m * nocc), Zo(8 * (size_t)m * nocc),
        Go(8 * (size_t)nocc * nocc), lohi(16 * (size_t)m);
    bool have_y = false, cm_valid = false, fq_valid = false;
    int n_purified = 0, n_eigh = 0, purify_steps = 0;
    auto diag = [&](const double* Fx) {
      S.eig_spans = nullptr;
      sp_eig_all.begin();
      S.gemm(m, n, n, X.as<double>(), m, true, Fx, n, false, t1.as<double>(), n);        // X^T F
      S.gemm(m, m, n, t1.as<double>(), n, false, X.as<double>(), m, false, Fq.as<double>(), m);
      fq_valid = true;
      int steps = 0;
      const char* why = "";
      const bool tried = o.purify && have_y;
      bool purified = false;
      if (tried) {
        sp_pur.begin();
        purified = S.purify_occ(Fq.as<double>(), t1.as<double>(), t2.as<double>(), Yo.as<double>(), Zo.as<double>(),
                                Go.as<double>(), lohi.as<double>(), steps, why);
        sp_pur.end();
      }
      if (purified) {
        if (o.verbose) std::fprintf(stderr, "dfx_scf purification: %d steps\n", steps);
        S.gemm(n, nocc, m, X.as<double>(), m, false, Yo.as<double>(), nocc, false, Cocc.as<double>(), nocc);
        cm_valid = false;
        ++n_purified;
        purify_steps += steps;
      } else {
        if (tried && o.verbose) std::fprintf(stderr, "dfx_scf purification failed (%s), eigen-decomposition\n", why);
        DFX_HIP(hipMemcpyAsync(Fp.p, Fq.p, 8 * (size_t)m * m, hipMemcpyDeviceToDevice, st));
        S.syevd(Fp.as<double>(), m, eps.as<double>());
        S.gemm(n, m, m, X.as<double>(), m, false, Fp.as<double>(), m, true, Cm.as<double>(), m);  // X V
        hipLaunchKernelGGL(copy_cols_kernel, dim3(nblk((int64_t)n * nocc)), dim3(256), 0, st, Cm.as<double>(), m,
                           n, nocc, Cocc.as<double>(), nocc);
        hipLaunchKernelGGL(rows_to_cols_kernel, dim3(nblk((int64_t)m * nocc)), dim3(256), 0, st, Fp.as<double>(), m,
                           0, nocc, Yo.as<double>());
        have_y = cm_valid = true;
        ++n_eigh;
      }
      S.gemm(n, n, nocc, Cocc.as<double>(), nocc, false, Cocc.as<double>(), nocc, true, D.as<double>(), n);
      sp_eig_all.end();
      S.eig_spans = &sp_eig_all;
    };

    // ---- guess
    const auto tg0 = clk::now();
    int fallback = 0;  // 1: non-finite learned prediction, 2: learned start did not converge
    std::vector<double> Dl;
    if (o.guess == DFX_GUESS_LEARNED) {
      Dl.resize(n2);
      guess_predict_density(o.model, geom, Dl.data(), st);
      for (double x : Dl)
        if (!std::isfinite(x)) {
          fallback = 1;
          break;
        }
    }
    if (o.guess == DFX_GUESS_CORE || fallback) {
      diag(h.as<double>());
    } else if (o.guess == DFX_GUESS_CINIT) {
      DevMem Ci(8 * n2);
      DFX_HIP(hipMemcpyAsync(Ci.p, init, 8 * n2, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(copy_cols_kernel, dim3(nblk((int64_t)n * nocc)), dim3(256), 0, st, Ci.as<double>(), n, n,
                         nocc, Cocc.as<double>(), nocc);
      S.gemm(n, n, nocc, Cocc.as<double>(), nocc, false, Cocc.as<double>(), nocc, true, D.as<double>(), n);
    } else if (o.guess == DFX_GUESS_DENSITY || o.guess == DFX_GUESS_LEARNED) {
      // the density in the orthonormal basis of X; its top nocc eigenvectors give C_occ
      DevMem Di(8 * n2);
      DFX_HIP(hipMemcpyAsync(Di.p, Dl.empty() ? init : Dl.data(), 8 * n2, hipMemcpyHostToDevice, st));
      if (o.guess == DFX_GUESS_DENSITY) {
        // AO density: X^T S D S X
        S.gemm(n, n, n, Sm.as<double>(), n, false, Di.as<double>(), n, false, t1.as<double>(), n);   // S D
        S.gemm(n, n, n, t1.as<double>(), n, false, Sm.as<double>(), n, false, t2.as<double>(), n);   // S D S
        S.gemm(m, n, n, X.as<double>(), m, true, t2.as<double>(), n, false, t1.as<double>(), n);     // X^T SDS
        S.gemm(m, m, n, t1.as<double>(), n, false, X.as<double>(), m, false, Fp.as<double>(), m);
      } else if (lowdin) {
        // Loewdin density P = S^1/2 D S^1/2: with X = S^-1/2, X^T S D S X = P itself
        DFX_HIP(hipMemcpyAsync(Fp.p, Di.p, 8 * n2, hipMemcpyDeviceToDevice, st));
      } else {
        // Loewdin density P = S^1/2 D S^1/2: X^T S D S X = U^T P U with X^T S^1/2 = U^T
        S.gemm(m, n, n, Uk.as<double>(), m, true, Di.as<double>(), n, false, t1.as<double>(), n);    // U^T P
        S.gemm(m, m, n, t1.as<double>(), n, false, Uk.as<double>(), m, false, Fp.as<double>(), m);
      }
      // the top nocc eigenvectors span the occupied space of the lowest levels of
      // -P': purified from a seeded random start, else the full eigen-decomposition
      bool done = false;
      if (o.purify) {
        const int64_t mm = (int64_t)m * m, mo = (int64_t)m * nocc;
        DFX_HIP(hipMemcpyAsync(Fq.p, Fp.p, 8 * (size_t)mm, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(negate_kernel, dim3(nblk(mm)), dim3(256), 0, st, Fq.as<double>(), mm);
        hipLaunchKernelGGL(rand_fill_kernel, dim3(nblk(mo)), dim3(256), 0, st, Yo.as<double>(), mo,
                           (uint64_t)0x5DEECE66Dull);
        int steps = 0;
        const char* why = "";
        done = S.purify_occ(Fq.as<double>(), t1.as<double>(), t2.as<double>(), Yo.as<double>(), Zo.as<double>(),
                            Go.as<double>(), lohi.as<double>(), steps, why);
        if (o.verbose) {
          if (done)
            std::fprintf(stderr, "dfx_scf guess purification: %d steps\n", steps);
          else
            std::fprintf(stderr, "dfx_scf guess purification failed (%s)\n", why);
        }
        if (done)
          S.gemm(n, nocc, m, X.as<double>(), m, false, Yo.as<double>(), nocc, false, Cocc.as<double>(), nocc);
      }
      if (!done) {
        S.syevd(Fp.as<double>(), m, eps.as<double>());
        // eigenvectors of the largest nocc eigenvalues are the last nocc rows
        S.gemm(n, m, m, X.as<double>(), m, false, Fp.as<double>(), m, true, Cm.as<double>(), m);
        hipLaunchKernelGGL(copy_cols_kernel, dim3(nblk((int64_t)n * nocc)), dim3(256), 0, st,
                           Cm.as<double>() + (m - nocc), m, n, nocc, Cocc.as<double>(), nocc);
        hipLaunchKernelGGL(rows_to_cols_kernel, dim3(nblk((int64_t)m * nocc)), dim3(256), 0, st, Fp.as<double>(),
                           m, m - nocc, nocc, Yo.as<double>());
      }
      have_y = true;
      S.gemm(n, n, nocc, Cocc.as<double>(), nocc, false, Cocc.as<double>(), nocc, true, D.as<double>(), n);
    } else {
      throw Error(DFX_EINVAL, "dfx_scf: unknown guess");
    }
    Uk.release();
    DFX_HIP(hipStreamSynchronize(st));
    const auto t1c = clk::now();
    const double t_guess = std::chrono::duration<double>(t1c - tg0).count();

    // ---- iterations
    EventSpans sp_j, sp_kx[3], sp_ks[3];
    sp_j.st = st;
    for (int k = 0; k < 3; ++k) sp_kx[k].st = sp_ks[k].st = st;
    struct Timer : KTimer {
      EventSpans *x, *s;
      void begin_x() override { x->begin(); }
      void end_x() override { x->end(); }
      void begin_syrk() override { s->begin(); }
      void end_syrk() override { s->end(); }
    } ktimer;
    int n_jk_p[3] = {0, 0, 0};
    JKArgs ja{B->hi.as<float>(), B->lo.as<float>(), B->naux, n, B->ncols_t, PREC_FP64};
    const bool mixed = (o.schedule == DFX_SCHED_MIXED);
    int nfp64 = 0, it = 0, n_mixed = 0, it_done = 0;
    double floor_est[3] = {0.0, 0.0, 0.0};
    double E = 0.0, Eold = 0.0, emax = 0.0;
    bool converged = false;
    dfx_scf_info inf{};
    for (int pass = 0; pass < 2; ++pass) {
    // precision stages: reduced precision first, FP64 last.  A stage ends when the
    // DIIS error falls below its threshold or stops improving.
    std::vector<int> stages;
    std::vector<double> stage_thr;
    if (mixed && o.mixed_prec == DFX_BF16) {
      stages = {DFX_BF16, DFX_FP32, DFX_FP64};
      stage_thr = {std::max(o.switch_err, 1e-2), o.switch_err, 0.0};
    } else if (mixed) {
      stages = {DFX_FP32, DFX_FP64};
      stage_thr = {o.switch_err, 0.0};
    } else {
      stages = {DFX_FP64};
      stage_thr = {0.0};
    }
    int stage = 0, stage_it = 0;
    std::vector<double> stage_errs;
    int prec = stages[0];
    int hcount = 0, hpos = 0;
    bool stage_estimated = false;
    nfp64 = 0;
    std::vector<double> Bdiis((size_t)dsz * dsz, 0.0);
    for (it = 1; it <= o.max_iter; ++it) {
      const int ih = it_done + it;  // iteration number over both passes
      // the floor of reduced precision p at the current density: how far its K
      // moves the DIIS error, measured on every S-th auxiliary function (rows S q
      // of B, a tensor with row stride S ncols) and scaled to all of them
      // (independent rounding errors add in quadrature)
      auto estimate_floor = [&](int p) {
        JKArgs sub = ja;
        sub.prec = p;
        const int Sg = std::max(1, std::min(16, B->naux / 64));
        sub.naux = (B->naux + Sg - 1) / Sg;
        sub.ncols = ja.ncols * Sg;
        JKArgs s64 = sub;
        s64.prec = PREC_FP64;
        void* ws = B->ensure_work(std::max(k_work_bytes(sub, nocc), k_work_bytes(s64, nocc)));
        k_build(sub, Cocc.as<double>(), nocc, Km.as<double>(), ws, st, nullptr);
        k_build(s64, Cocc.as<double>(), nocc, Jm.as<double>(), ws, st, nullptr);
        Comb cd{};
        cd.m = 2;
        cd.F[0] = Km.as<double>();
        cd.c[0] = 1.0;
        cd.F[1] = Jm.as<double>();
        cd.c[1] = -1.0;
        hipLaunchKernelGGL(lincomb_kernel, dim3(nblk(n2)), dim3(256), 0, st, cd, F.as<double>(), n2);
        S.gemm(n, n, n, F.as<double>(), n, false, D.as<double>(), n, false, t1.as<double>(), n);
        S.gemm(n, n, n, t1.as<double>(), n, false, Sm.as<double>(), n, false, t2.as<double>(), n);
        hipLaunchKernelGGL(antisym_kernel, dim3(nblk(n2)), dim3(256), 0, st, t2.as<double>(), t1.as<double>(), n);
        S.gemm(m, n, n, X.as<double>(), m, true, t1.as<double>(), n, false, t2.as<double>(), n);
        S.gemm(m, m, n, t2.as<double>(), n, false, X.as<double>(), m, false, Fp.as<double>(), m);
        return S.reduce_max(Fp.as<double>(), (int64_t)m * m) * std::sqrt((double)B->naux / sub.naux);
      };
      // a BF16 stage is checked on entry: where the basis is nearly linearly
      // dependent, X^T (.) X amplifies BF16's rounding of K beyond the stage's own
      // threshold, and its Fock matrices would lead the SCF away (measured on
      // (H2O)64: DIIS errors of 10 and more).  Such a stage is skipped.
      if (mixed && o.switch_auto && prec == DFX_BF16 && stage_it == 0) {
        const double est = estimate_floor(DFX_BF16);
        floor_est[DFX_BF16] = est;
        if (o.verbose) std::fprintf(stderr, "dfx_scf BF16 stage: estimated floor %.3e on entry\n", est);
        if (est > stage_thr[stage]) {
          if (o.verbose) std::fprintf(stderr, "dfx_scf BF16 stage skipped\n");
          ++stage;
          prec = stages[stage];
        }
      }
      ja.prec = prec;
      size_t need = std::max(sizeof(double) * (2 * (size_t)B->ncols_t + B->naux + 8), k_work_bytes(ja, nocc));
      // the floor is estimated once per stage, at the first iteration after the
      // stage's error fell below 1e-2: by then DIIS converges steadily and the
      // density is close enough to the solution for the estimate to be the floor
      // (at a poor starting density it overshoots and would end the stage early)
      const bool estimate = mixed && o.switch_auto && prec != DFX_FP64 && !stage_estimated && !stage_errs.empty() &&
                            stage_errs.back() < 1e-2;
      if (estimate) {
        const double est = estimate_floor(prec);
        floor_est[prec] = est;
        stage_thr[stage] = std::max(stage_thr[stage], est);
        stage_estimated = true;
        if (o.verbose) std::fprintf(stderr, "dfx_scf stage %d: estimated floor %.3e\n", stage, est);
      }
      void* w = B->ensure_work(need);
      sp_j.begin();
      j_build(ja, D.as<double>(), Jm.as<double>(), reinterpret_cast<double*>(w), st);
      sp_j.end();
      ktimer.x = &sp_kx[prec];
      ktimer.s = &sp_ks[prec];
      ++n_jk_p[prec];
      k_build(ja, Cocc.as<double>(), nocc, Km.as<double>(), w, st, &ktimer);
      hipLaunchKernelGGL(fock_kernel, dim3(nblk(n2)), dim3(256), 0, st, h.as<double>(), Jm.as<double>(),
                         Km.as<double>(), F.as<double>(), n2);
      E = S.reduce_sum(D.as<double>(), h.as<double>(), F.as<double>(), n2) + Enuc;
      // e = X^T (F D S - S D F) X
      S.gemm(n, n, n, F.as<double>(), n, false, D.as<double>(), n, false, t1.as<double>(), n);
      S.gemm(n, n, n, t1.as<double>(), n, false, Sm.as<double>(), n, false, t2.as<double>(), n);
      hipLaunchKernelGGL(antisym_kernel, dim3(nblk(n2)), dim3(256), 0, st, t2.as<double>(), t1.as<double>(), n);
      S.gemm(m, n, n, X.as<double>(), m, true, t1.as<double>(), n, false, t2.as<double>(), n);
      double* e_new = Eh[hpos].as<double>();
      S.gemm(m, m, n, t2.as<double>(), n, false, X.as<double>(), m, false, e_new, m);
      emax = S.reduce_max(e_new, (int64_t)m * m);
      if (ih <= DFX_MAXHIST) {
        inf.E_hist[ih - 1] = E;
        inf.err_hist[ih - 1] = emax;
        inf.prec_hist[ih - 1] = (int8_t)prec;
      }
      if (o.verbose)
        std::fprintf(stderr, "dfx_scf it %3d  %s  E = %.12f  dE = %.3e  err = %.3e\n", ih,
                     prec == DFX_FP64 ? "fp64" : (prec == DFX_FP32 ? "fp32" : "bf16"), E, E - Eold, emax);
      ++stage_it;
      if (prec == DFX_FP64) {
        ++nfp64;
        // after a reduced-precision stage the first FP64 build has no FP64 predecessor
        // to difference against; its commutator with the exact Fock matrix decides
        const bool dE_ok = mixed ? (nfp64 == 1 || std::fabs(E - Eold) < o.conv_dE)
                                 : (it >= 2 && std::fabs(E - Eold) < o.conv_dE);
        if (dE_ok && emax < o.conv_err) {
          converged = true;
          break;
        }
      } else {
        ++n_mixed;
      }
      Eold = E;
      // next precision stage once the error is below the stage threshold, or the
      // stage has stalled: no factor-2 gain of its best error over the last WIN
      // iterations.  WIN = 4 once the error is below 1e-2, where the reduced-precision
      // floors lie.  Above it a stall is the erratic start from a poor guess, which
      // FP64 would not cure: WIN = 16 in FP32 (its floor is far lower), 8 in BF16.
      // Into FP64 from a stage whose floor was measured at or below 1e-3, the DIIS
      // history carries over: those Fock matrices are good enough to extrapolate
      // with, and the FP64 entries take over as their errors fall below the floor.
      // Otherwise (BF16, or a stage that stalled before its floor was measured) the
      // history restarts from a plain diagonalisation, since the coarse Fock
      // matrices would pin the extrapolation at their own error level.
      stage_errs.push_back(emax);
      bool stalled = false;
      const int WIN = *std::min_element(stage_errs.begin(), stage_errs.end()) < 1e-2 ? 4
                      : prec == DFX_BF16                                              ? 8
                                                                                      : 16;
      if (stage_it > WIN) {
        const double recent = *std::min_element(stage_errs.end() - WIN, stage_errs.end());
        const double before = *std::min_element(stage_errs.begin(), stage_errs.end() - WIN);
        stalled = recent > 0.5 * before;
      }
      if (prec != DFX_FP64 && (emax < stage_thr[stage] || stalled)) {
        ++stage;
        prec = stages[stage];
        stage_it = 0;
        stage_errs.clear();
        stage_estimated = false;
        const double fl = floor_est[stages[stage - 1]];
        if (prec != DFX_FP64 || !(fl > 0.0 && fl <= 1e-3)) {
          hcount = 0;
          hpos = 0;
          diag(F.as<double>());
          continue;
        }
      }
      // DIIS history (ring buffer)
      DFX_HIP(hipMemcpyAsync(Fh[hpos].p, F.p, 8 * n2, hipMemcpyDeviceToDevice, st));
      hcount = std::min(hcount + 1, dsz);
      // overlaps of the new error with every stored one
      std::vector<double> Bn(dsz, 0.0);
      for (int k = 0; k < hcount; ++k) Bn[k] = S.reduce_sum(Eh[k].as<double>(), e_new, nullptr, (int64_t)m * m);
      for (int k = 0; k < hcount; ++k) Bdiis[(size_t)hpos * dsz + k] = Bdiis[(size_t)k * dsz + hpos] = Bn[k];
      const double* Fuse = F.as<double>();
      if (hcount > 1) {
        // slots in age order (oldest first) for dropping when ill-conditioned
        std::vector<int> slots;
        for (int k = 0; k < hcount; ++k) slots.push_back((hpos + 1 + k + (dsz - hcount)) % dsz);
        while (slots.size() > 1) {
          const int mm = (int)slots.size();
          std::vector<double> Bm((size_t)mm * mm), c;
          for (int i = 0; i < mm; ++i)
            for (int j = 0; j < mm; ++j) Bm[i * mm + j] = Bdiis[(size_t)slots[i] * dsz + slots[j]];
          if (diis_solve(Bm, mm, c)) {
            Comb cb{};
            cb.m = mm;
            for (int i = 0; i < mm; ++i) {
              cb.F[i] = Fh[slots[i]].as<double>();
              cb.c[i] = c[i];
            }
            hipLaunchKernelGGL(lincomb_kernel, dim3(nblk(n2)), dim3(256), 0, st, cb, t2.as<double>(), n2);
            Fuse = t2.as<double>();
            break;
          }
          slots.erase(slots.begin());
        }
      }
      hpos = (hpos + 1) % dsz;
      diag(Fuse);
    }
    it_done += std::min(it, o.max_iter);
    // a learned start that does not converge is retried once from the core guess
    if (converged || o.guess != DFX_GUESS_LEARNED || fallback) break;
    fallback = 2;
    Eold = 0.0;
    diag(h.as<double>());
    }
    DFX_HIP(hipStreamSynchronize(st));
    const auto t2c = clk::now();

    *E_out = E;
    if ((C_out || eps_out) && !cm_valid && fq_valid) {
      // orbitals and energies of the Fock matrix whose occupied space gave D
      DFX_HIP(hipMemcpyAsync(Fp.p, Fq.p, 8 * (size_t)m * m, hipMemcpyDeviceToDevice, st));
      S.eig_spans = nullptr;
      S.syevd(Fp.as<double>(), m, eps.as<double>());
      S.gemm(n, m, m, X.as<double>(), m, false, Fp.as<double>(), m, true, Cm.as<double>(), m);
      DFX_HIP(hipStreamSynchronize(st));
    }
    if (C_out) {
      // full C (n x n): the first m columns from X C', the rest zero
      std::vector<double> Ch((size_t)n * m), Cf((size_t)n * n, 0.0);
      DFX_HIP(hipMemcpy(Ch.data(), Cm.p, 8 * (size_t)n * m, hipMemcpyDeviceToHost));
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < m; ++c) Cf[(size_t)r * n + c] = Ch[(size_t)r * m + c];
      std::memcpy(C_out, Cf.data(), 8 * n2);
    }
    if (eps_out) {
      std::vector<double> e(m);
      DFX_HIP(hipMemcpy(e.data(), eps.p, 8 * (size_t)m, hipMemcpyDeviceToHost));
      for (int i = 0; i < n; ++i) eps_out[i] = i < m ? e[i] : 0.0;
    }
    inf.niter = it_done;
    inf.guess_fallback = fallback;
    inf.n_purified = n_purified;
    inf.n_eigh = n_eigh;
    inf.purify_steps = purify_steps;
    inf.converged = converged ? 1 : 0;
    inf.n_mixed = n_mixed;
    inf.ndropped = n - m;
    inf.nbf = n;
    inf.naux = B->naux;
    inf.nocc = nocc;
    inf.E_nuc = Enuc;
    inf.err_max = emax;
    inf.t_setup = std::chrono::duration<double>(t1c - t0).count();
    inf.t_guess = t_guess;
    for (int k = 0; k < 3; ++k) inf.floor_est[k] = floor_est[k];
    inf.t_scf = std::chrono::duration<double>(t2c - t1c).count();
    inf.t_total = std::chrono::duration<double>(clk::now() - t0).count();
    inf.t_eri = B->info.eri_seconds;
    inf.t_metric = B->info.metric_seconds;
    inf.t_trsm = B->info.trsm_seconds;
    inf.t_trsm_update = B->info.trsm_update_seconds;
    inf.trsm_update_flops = B->info.trsm_update_flops;
    inf.n_trsm_update = B->info.trsm_update_launches;
    inf.t_j = sp_j.seconds();
    inf.t_kx = inf.t_ksyrk = 0.0;
    inf.n_kx_launch = 0;
    for (int k = 0; k < 3; ++k) {
      inf.t_kx_p[k] = sp_kx[k].seconds();
      inf.t_ksyrk_p[k] = sp_ks[k].seconds();
      inf.n_jk_p[k] = n_jk_p[k];
      inf.n_kx_launch_p[k] = sp_kx[k].count();
      inf.t_kx += inf.t_kx_p[k];
      inf.t_ksyrk += inf.t_ksyrk_p[k];
      inf.n_kx_launch += inf.n_kx_launch_p[k];
    }
    inf.t_eig = S.eig_spans ? S.eig_spans->seconds() : 0.0;
    inf.t_purify = sp_pur.seconds();
    inf.n_jk = sp_j.count();
    inf.nintegrals = B->info.nintegrals;
    inf.ncols = B->info.ncols;
    if (info) *info = inf;
    if (!converged) {
      status = DFX_ENOCONV;
      set_last_error("dfx_scf: not converged in " + std::to_string(o.max_iter) + " iterations");
    }
  });
  return rc != DFX_OK ? rc : status;
}

// Open-shell SCF on the fitted J and K.  restricted = false: UHF, one orbital set
// per spin, each diagonalising its own Fock matrix.  restricted = true: ROHF, one
// orbital set whose n_beta lowest are doubly and the next n_alpha - n_beta singly
// occupied, the eigenvectors of Roothaan's effective Fock matrix (the diagonal
// blocks take (F_alpha + F_beta) / 2; core-open F_beta, open-virtual F_alpha),
// formed and extrapolated in the orthonormal basis of X.
static int open_shell_scf(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux,
                          int nauxsh, const dfx_scf_opts* opts_in, int multiplicity, double* E_out,
                          double* C_out, double* eps_out, dfx_scf_info* info, bool restricted) {
  const std::string fn = restricted ? "dfx_rohf" : "dfx_uhf";
  int status = DFX_OK;
  const int rc = guard([&] {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    if (!geom || !E_out) throw Error(DFX_EINVAL, fn + ": NULL argument");
    if (geom->natom <= 0 || !geom->xyz || !geom->Z) throw Error(DFX_EINVAL, fn + ": bad geometry");
    dfx_scf_opts o;
    dfx_scf_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.diis_size < 1 || o.diis_size > 16 || o.max_iter < 1) throw Error(DFX_EINVAL, fn + ": bad options");
    if (o.guess != DFX_GUESS_CORE || o.schedule != DFX_SCHED_FP64)
      throw Error(DFX_EINVAL, fn + ": core guess and FP64 schedule only");
    if (!(o.level_shift >= 0.0) || !std::isfinite(o.level_shift))
      throw Error(DFX_EINVAL, fn + ": level_shift must be finite and >= 0");
    int nelec = -geom->charge;
    for (int a = 0; a < geom->natom; ++a) nelec += geom->Z[a];
    if (multiplicity < 1 || nelec <= 0 || (nelec + multiplicity - 1) % 2 || multiplicity - 1 > nelec)
      throw Error(DFX_EINVAL, fn + ": electron count and multiplicity do not match");
    const int na = (nelec + multiplicity - 1) / 2, nb = nelec - na;
    HostShells hb = make_shells(shells, nsh, 3, "orbital basis");
    HostShells ha = make_shells(aux, nauxsh, 4, "auxiliary basis");
    const int n = hb.nbf;
    if (na > n) throw Error(DFX_EINVAL, fn + ": more occupied orbitals than basis functions");

    std::unique_ptr<Arena> arena = scf_arena(o, hb, ha, geom->natom, fn.c_str());
    ArenaScope scope(arena.get());
    Scf S;
    {
      DevCtx& ctx = thread_ctx();
      S.st = ctx.st;
    }
    hipStream_t st = S.st;
    S.n = n;
    S.nocc = na;
    S.part.alloc(sizeof(double) * 512);
    S.gw.alloc(sizeof(double) * std::max<size_t>(4 * (size_t)n * n, syrk_f64_work_elems(n)));
    const int64_t n2 = (int64_t)n * n;

    // setup: fitted integrals, one-electron matrices, E_nn, canonical orthogonaliser
    std::unique_ptr<dfx_B> B = build_B(std::move(hb), std::move(ha), o.tau, 0, st);
    DevMem Sm(8 * n2), Tm(8 * n2), Vm(8 * n2), h(8 * n2);
    int1e_build(B->bas, geom, Sm.as<double>(), Tm.as<double>(), Vm.as<double>(), st);
    hipLaunchKernelGGL(add_kernel, dim3(nblk(n2)), dim3(256), 0, st, Tm.as<double>(), Vm.as<double>(),
                       h.as<double>(), n2);
    Tm.release();
    Vm.release();
    double Enuc = 0.0;
    for (int a = 0; a < geom->natom; ++a)
      for (int b = 0; b < a; ++b) {
        const double* A = geom->xyz + 3 * a;
        const double* Bx = geom->xyz + 3 * b;
        const double r = std::sqrt((A[0] - Bx[0]) * (A[0] - Bx[0]) + (A[1] - Bx[1]) * (A[1] - Bx[1]) +
                                   (A[2] - Bx[2]) * (A[2] - Bx[2]));
        Enuc += (double)geom->Z[a] * geom->Z[b] / r;
      }
    Ortho orth = make_orthogonalizer(S, Sm.as<double>(), n, o.ortho_thresh, false);
    const int m = orth.m;
    if (m < na) throw Error(DFX_EINVAL, fn + ": basis too linearly dependent");
    S.m = m;
    DevMem X = std::move(orth.X);

    // per spin: occupied orbitals, density, K, Fock matrix, DIIS error
    const int nocc_s[2] = {na, nb};
    DevMem J(8 * n2), Dt(8 * n2), t1(8 * n2), t2(8 * n2), Fp(8 * (size_t)m * m);
    // orbitals (n x m, C = X V^T) and levels of the last solve: one per spin (UHF),
    // one set (ROHF)
    DevMem Cm[2], eps[2], Cocc[2], D[2], K[2], F[2];
    for (int s2 = 0; s2 < 2; ++s2) {
      Cm[s2].alloc(8 * (size_t)n * m);
      eps[s2].alloc(8 * (size_t)m);
      Cocc[s2].alloc(8 * (size_t)n * std::max(1, nocc_s[s2]));
      D[s2].alloc(8 * n2);
      K[s2].alloc(8 * n2);
      F[s2].alloc(8 * n2);
    }
    const int dsz = o.diis_size;
    std::vector<DevMem> Fh(2 * dsz), Eh(2 * dsz);
    for (int k = 0; k < 2 * dsz; ++k) {
      Fh[k].alloc(8 * n2);
      Eh[k].alloc(8 * (size_t)m * m);
    }
    // occupied orbitals of spin s2 from a Fock-like matrix F: the nocc lowest levels
    // of F' = X^T F X (kept in Fq[s2]; for ROHF the one effective matrix, both
    // counts).  They come by purification, as for RHF, once a previous occupied
    // space Y of that spin exists (every iteration after the first); otherwise,
    // or if it fails, by the full eigen-decomposition, which also gives the
    // orbitals and levels C, eps.
    DevMem Fq[2], Yo[2], Zo, Go, lohi;
    bool have_y[2] = {false, false}, cm_valid[2] = {false, false};
    int n_purified = 0, n_eigh = 0, purify_steps = 0;
    {
      const int nmax = std::max(1, std::max(na, nb));
      for (int s2 = 0; s2 < 2; ++s2) {
        if (!restricted || s2 == 0) Fq[s2].alloc(8 * (size_t)m * m);
        Yo[s2].alloc(8 * (size_t)m * std::max(1, nocc_s[s2]));
      }
      Zo.alloc(8 * (size_t)m * nmax);
      Go.alloc(8 * (size_t)nmax * nmax);
      lohi.alloc(16 * (size_t)m);
    }
    auto diag = [&](int s2, const double* Fx) {
      const int no = nocc_s[s2];
      S.gemm(m, n, n, X.as<double>(), m, true, Fx, n, false, t1.as<double>(), n);
      S.gemm(m, m, n, t1.as<double>(), n, false, X.as<double>(), m, false, Fq[s2].as<double>(), m);
      if (no == 0) {
        DFX_HIP(hipMemsetAsync(D[s2].p, 0, 8 * n2, st));
        cm_valid[s2] = false;
        return;
      }
      if (o.purify && have_y[s2]) {
        int steps = 0;
        const char* why = "";
        S.nocc = no;
        if (S.purify_occ(Fq[s2].as<double>(), t1.as<double>(), t2.as<double>(), Yo[s2].as<double>(),
                         Zo.as<double>(), Go.as<double>(), lohi.as<double>(), steps, why)) {
          S.gemm(n, no, m, X.as<double>(), m, false, Yo[s2].as<double>(), no, false, Cocc[s2].as<double>(), no);
          S.gemm(n, n, no, Cocc[s2].as<double>(), no, false, Cocc[s2].as<double>(), no, true, D[s2].as<double>(), n);
          cm_valid[s2] = false;
          ++n_purified;
          purify_steps += steps;
          return;
        }
        if (o.verbose) std::fprintf(stderr, "%s purification failed (%s), eigen-decomposition\n", fn.c_str(), why);
      }
      DFX_HIP(hipMemcpyAsync(Fp.p, Fq[s2].p, 8 * (size_t)m * m, hipMemcpyDeviceToDevice, st));
      S.syevd(Fp.as<double>(), m, eps[s2].as<double>());
      S.gemm(n, m, m, X.as<double>(), m, false, Fp.as<double>(), m, true, Cm[s2].as<double>(), m);
      hipLaunchKernelGGL(copy_cols_kernel, dim3(nblk((int64_t)n * no)), dim3(256), 0, st, Cm[s2].as<double>(), m, n,
                         no, Cocc[s2].as<double>(), no);
      hipLaunchKernelGGL(rows_to_cols_kernel, dim3(nblk((int64_t)m * no)), dim3(256), 0, st, Fp.as<double>(), m, 0, no,
                         Yo[s2].as<double>());
      S.gemm(n, n, no, Cocc[s2].as<double>(), no, false, Cocc[s2].as<double>(), no, true, D[s2].as<double>(), n);
      have_y[s2] = cm_valid[s2] = true;
      ++n_eigh;
    };
    // ROHF: the occupied spaces of one m x m matrix of the orthonormal basis, the
    // na and nb lowest levels, kept as the projectors P_a, P_b (m x m); C = X V^T
    // when the matrix was diagonalised
    const int64_t m2 = (int64_t)m * m;
    DevMem Fo[2], tm, Rm, Feff, Dp, Pp[2];
    if (restricted) {
      for (auto& f : Fo) f.alloc(8 * m2);
      for (auto& f : Pp) f.alloc(8 * m2);
      tm.alloc(8 * m2);
      Rm.alloc(8 * m2);
      Feff.alloc(8 * m2);
      Dp.alloc(8 * m2);
    }
    // densities, occupied orbitals and projectors from the columns Yo[s2]
    auto from_y = [&]() {
      for (int s2 = 0; s2 < 2; ++s2) {
        const int no = nocc_s[s2];
        if (no == 0) {
          DFX_HIP(hipMemsetAsync(D[s2].p, 0, 8 * n2, st));
          DFX_HIP(hipMemsetAsync(Pp[s2].p, 0, 8 * m2, st));
          continue;
        }
        S.gemm(n, no, m, X.as<double>(), m, false, Yo[s2].as<double>(), no, false, Cocc[s2].as<double>(), no);
        S.gemm(n, n, no, Cocc[s2].as<double>(), no, false, Cocc[s2].as<double>(), no, true, D[s2].as<double>(), n);
        S.gemm(m, m, no, Yo[s2].as<double>(), no, false, Yo[s2].as<double>(), no, true, Pp[s2].as<double>(), m);
      }
    };
    auto update_orth = [&](const double* Fm) {
      DFX_HIP(hipMemcpyAsync(Fq[0].p, Fm, 8 * m2, hipMemcpyDeviceToDevice, st));
      if (o.purify && have_y[0]) {
        bool ok = true;
        int steps_all = 0;
        const char* why = "";
        for (int s2 = 0; s2 < 2 && ok; ++s2) {
          if (nocc_s[s2] == 0) continue;
          int steps = 0;
          S.nocc = nocc_s[s2];
          ok = S.purify_occ(Fq[0].as<double>(), t1.as<double>(), t2.as<double>(), Yo[s2].as<double>(),
                            Zo.as<double>(), Go.as<double>(), lohi.as<double>(), steps, why);
          steps_all += steps;
        }
        if (ok) {
          from_y();
          cm_valid[0] = false;
          ++n_purified;
          purify_steps += steps_all;
          return;
        }
        if (o.verbose) std::fprintf(stderr, "%s purification failed (%s), eigen-decomposition\n", fn.c_str(), why);
      }
      DFX_HIP(hipMemcpyAsync(Fp.p, Fq[0].p, 8 * m2, hipMemcpyDeviceToDevice, st));
      S.syevd(Fp.as<double>(), m, eps[0].as<double>());
      S.gemm(n, m, m, X.as<double>(), m, false, Fp.as<double>(), m, true, Cm[0].as<double>(), m);
      for (int s2 = 0; s2 < 2; ++s2)
        if (nocc_s[s2] > 0)
          hipLaunchKernelGGL(rows_to_cols_kernel, dim3(nblk((int64_t)m * nocc_s[s2])), dim3(256), 0, st,
                             Fp.as<double>(), m, 0, nocc_s[s2], Yo[s2].as<double>());
      from_y();
      have_y[0] = cm_valid[0] = true;
      ++n_eigh;
    };
    if (restricted) {
      S.gemm(m, n, n, X.as<double>(), m, true, h.as<double>(), n, false, t1.as<double>(), n);
      S.gemm(m, m, n, t1.as<double>(), n, false, X.as<double>(), m, false, Feff.as<double>(), m);
      update_orth(Feff.as<double>());
    } else {
      diag(0, h.as<double>());
      diag(1, h.as<double>());
    }
    DFX_HIP(hipStreamSynchronize(st));
    const auto t1c = clk::now();

    JKArgs ja{B->hi.as<float>(), B->lo.as<float>(), B->naux, n, B->ncols_t, PREC_FP64};
    dfx_scf_info inf{};
    std::vector<double> Bdiis((size_t)dsz * dsz, 0.0);
    int hcount = 0, hpos = 0, it = 0;
    double E = 0.0, Eold = 0.0, emax = 0.0;
    bool converged = false;
    for (it = 1; it <= o.max_iter; ++it) {
      // the K plan chunks Q by the occupied count, so size the work for both spins
      void* w = B->ensure_work(std::max({sizeof(double) * (2 * (size_t)B->ncols_t + B->naux + 8),
                                         k_work_bytes(ja, std::max(1, na)), k_work_bytes(ja, std::max(1, nb))}));
      hipLaunchKernelGGL(add_kernel, dim3(nblk(n2)), dim3(256), 0, st, D[0].as<double>(), D[1].as<double>(),
                         Dt.as<double>(), n2);
      j_build(ja, Dt.as<double>(), J.as<double>(), reinterpret_cast<double*>(w), st);
      double sum = 0.0;
      for (int s2 = 0; s2 < 2; ++s2) {
        if (nocc_s[s2] > 0)
          k_build(ja, Cocc[s2].as<double>(), nocc_s[s2], K[s2].as<double>(), w, st, nullptr);
        else
          DFX_HIP(hipMemsetAsync(K[s2].p, 0, 8 * n2, st));
        hipLaunchKernelGGL(uhf_fock_kernel, dim3(nblk(n2)), dim3(256), 0, st, h.as<double>(), J.as<double>(),
                           K[s2].as<double>(), F[s2].as<double>(), n2);
        sum += S.reduce_sum(D[s2].as<double>(), h.as<double>(), F[s2].as<double>(), n2);
      }
      E = 0.5 * sum + Enuc;
      emax = 0.0;
      if (restricted) {
        // F_s' = X^T F_s X; F_eff' = A + Z + Z^T with Z = P_o Delta (P_v - P_c)
        for (int s2 = 0; s2 < 2; ++s2) {
          S.gemm(m, n, n, X.as<double>(), m, true, F[s2].as<double>(), n, false, t1.as<double>(), n);
          S.gemm(m, m, n, t1.as<double>(), n, false, X.as<double>(), m, false, Fo[s2].as<double>(), m);
        }
        hipLaunchKernelGGL(rohf_delta_kernel, dim3(nblk(m2)), dim3(256), 0, st, Fo[0].as<double>(),
                           Fo[1].as<double>(), Pp[0].as<double>(), Pp[1].as<double>(), Rm.as<double>(),
                           tm.as<double>(), m2);
        S.gemm(m, m, m, tm.as<double>(), m, false, Rm.as<double>(), m, false, Feff.as<double>(), m);
        hipLaunchKernelGGL(rohf_vc_kernel, dim3(nblk(m2)), dim3(256), 0, st, Pp[0].as<double>(),
                           Pp[1].as<double>(), tm.as<double>(), m);
        S.gemm(m, m, m, Feff.as<double>(), m, false, tm.as<double>(), m, false, Rm.as<double>(), m);
        hipLaunchKernelGGL(rohf_feff_kernel, dim3(nblk(m2)), dim3(256), 0, st, Fo[0].as<double>(),
                           Fo[1].as<double>(), Rm.as<double>(), Feff.as<double>(), m);
        // D' = P_a + P_b; e = F_eff' D' - D' F_eff'
        hipLaunchKernelGGL(add_kernel, dim3(nblk(m2)), dim3(256), 0, st, Pp[0].as<double>(), Pp[1].as<double>(),
                           Dp.as<double>(), m2);
        S.gemm(m, m, m, Feff.as<double>(), m, false, Dp.as<double>(), m, false, tm.as<double>(), m);
        hipLaunchKernelGGL(antisym_kernel, dim3(nblk(m2)), dim3(256), 0, st, tm.as<double>(),
                           Eh[2 * hpos].as<double>(), m);
        emax = S.reduce_max(Eh[2 * hpos].as<double>(), m2);
      }
      // UHF: e_s = X^T (F_s D_s S - S D_s F_s) X into the ring slot of each spin
      for (int s2 = 0; s2 < 2 && !restricted; ++s2) {
        S.gemm(n, n, n, F[s2].as<double>(), n, false, D[s2].as<double>(), n, false, t1.as<double>(), n);
        S.gemm(n, n, n, t1.as<double>(), n, false, Sm.as<double>(), n, false, t2.as<double>(), n);
        hipLaunchKernelGGL(antisym_kernel, dim3(nblk(n2)), dim3(256), 0, st, t2.as<double>(), t1.as<double>(), n);
        S.gemm(m, n, n, X.as<double>(), m, true, t1.as<double>(), n, false, t2.as<double>(), n);
        S.gemm(m, m, n, t2.as<double>(), n, false, X.as<double>(), m, false, Eh[2 * hpos + s2].as<double>(), m);
        emax = std::max(emax, S.reduce_max(Eh[2 * hpos + s2].as<double>(), (int64_t)m * m));
      }
      if (it <= DFX_MAXHIST) {
        inf.E_hist[it - 1] = E;
        inf.err_hist[it - 1] = emax;
        inf.prec_hist[it - 1] = (int8_t)DFX_FP64;
      }
      if (o.verbose)
        std::fprintf(stderr, "%s it %3d  E = %.12f  dE = %.3e  err = %.3e\n", fn.c_str(), it, E, E - Eold, emax);
      if (it >= 2 && std::fabs(E - Eold) < o.conv_dE && emax < o.conv_err) {
        converged = true;
        break;
      }
      Eold = E;
      // DIIS over both spins: one set of coefficients from the summed error overlaps
      const int nsp = restricted ? 1 : 2;
      const int64_t fsz = restricted ? m2 : n2;
      if (restricted)
        DFX_HIP(hipMemcpyAsync(Fh[2 * hpos].p, Feff.p, 8 * m2, hipMemcpyDeviceToDevice, st));
      else
        for (int s2 = 0; s2 < 2; ++s2)
          DFX_HIP(hipMemcpyAsync(Fh[2 * hpos + s2].p, F[s2].p, 8 * n2, hipMemcpyDeviceToDevice, st));
      hcount = std::min(hcount + 1, dsz);
      for (int k = 0; k < hcount; ++k) {
        double b = 0.0;
        for (int s2 = 0; s2 < nsp; ++s2)
          b += S.reduce_sum(Eh[2 * k + s2].as<double>(), Eh[2 * hpos + s2].as<double>(), nullptr, m2);
        Bdiis[(size_t)hpos * dsz + k] = Bdiis[(size_t)k * dsz + hpos] = b;
      }
      const double* Fuse[2] = {restricted ? Feff.as<double>() : F[0].as<double>(), F[1].as<double>()};
      DevMem* Fext[2] = {&t1, &t2};
      if (hcount > 1) {
        std::vector<int> slots;
        for (int k = 0; k < hcount; ++k) slots.push_back((hpos + 1 + k + (dsz - hcount)) % dsz);
        while (slots.size() > 1) {
          const int mm = (int)slots.size();
          std::vector<double> Bm((size_t)mm * mm), c;
          for (int i = 0; i < mm; ++i)
            for (int j = 0; j < mm; ++j) Bm[i * mm + j] = Bdiis[(size_t)slots[i] * dsz + slots[j]];
          if (diis_solve(Bm, mm, c)) {
            for (int s2 = 0; s2 < nsp; ++s2) {
              Comb cb{};
              cb.m = mm;
              for (int i = 0; i < mm; ++i) {
                cb.F[i] = Fh[2 * slots[i] + s2].as<double>();
                cb.c[i] = c[i];
              }
              hipLaunchKernelGGL(lincomb_kernel, dim3(nblk(fsz)), dim3(256), 0, st, cb, Fext[s2]->as<double>(), fsz);
              Fuse[s2] = Fext[s2]->as<double>();
            }
            break;
          }
          slots.erase(slots.begin());
        }
      }
      hpos = (hpos + 1) % dsz;
      if (restricted) {
        if (o.level_shift > 0.0) {
          // Dp still holds the density of the current orbitals in the orthonormal basis
          if (Fuse[0] != t1.as<double>())
            DFX_HIP(hipMemcpyAsync(t1.p, Fuse[0], 8 * m2, hipMemcpyDeviceToDevice, st));
          hipLaunchKernelGGL(shift_orth_kernel, dim3(nblk(m2)), dim3(256), 0, st, t1.as<double>(), Dp.as<double>(),
                             o.level_shift, m);
          Fuse[0] = t1.as<double>();
        }
        update_orth(Fuse[0]);
        continue;
      }
      // diag overwrites t1 (X^T F): extrapolated alpha Fock matrix goes to F[0] first
      if (Fuse[0] != F[0].as<double>())
        DFX_HIP(hipMemcpyAsync(F[0].p, Fuse[0], 8 * n2, hipMemcpyDeviceToDevice, st));
      if (Fuse[1] != F[1].as<double>())
        DFX_HIP(hipMemcpyAsync(F[1].p, Fuse[1], 8 * n2, hipMemcpyDeviceToDevice, st));
      if (o.level_shift > 0.0)
        for (int s2 = 0; s2 < 2; ++s2) {
          S.gemm(n, n, n, Sm.as<double>(), n, false, D[s2].as<double>(), n, false, t1.as<double>(), n);
          S.gemm(n, n, n, t1.as<double>(), n, false, Sm.as<double>(), n, false, t2.as<double>(), n);
          hipLaunchKernelGGL(shift_ao_kernel, dim3(nblk(n2)), dim3(256), 0, st, F[s2].as<double>(), Sm.as<double>(),
                             t2.as<double>(), o.level_shift, n2);
        }
      diag(0, F[0].as<double>());
      diag(1, F[1].as<double>());
    }
    DFX_HIP(hipStreamSynchronize(st));
    const auto t2c = clk::now();
    *E_out = E;
    // spins (UHF) or the one set (ROHF) whose last occupied space came from
    // purification: orbitals and levels from one eigen-decomposition of the same F'
    for (int s2 = 0; s2 < (restricted ? 1 : 2) && (C_out || eps_out); ++s2)
      if (!cm_valid[s2]) {
        DFX_HIP(hipMemcpyAsync(Fp.p, Fq[s2].p, 8 * (size_t)m * m, hipMemcpyDeviceToDevice, st));
        S.syevd(Fp.as<double>(), m, eps[s2].as<double>());
        S.gemm(n, m, m, X.as<double>(), m, false, Fp.as<double>(), m, true, Cm[s2].as<double>(), m);
        DFX_HIP(hipStreamSynchronize(st));
      }
    // the orbitals whose densities gave E: [nbf][nbf] per set, the first m columns
    // X V^T and the rest zero; levels [nbf], zero beyond m
    const int nset = restricted ? 1 : 2;
    for (int s2 = 0; s2 < nset; ++s2) {
      if (C_out) {
        std::vector<double> Ch((size_t)n * m);
        DFX_HIP(hipMemcpy(Ch.data(), Cm[s2].p, 8 * (size_t)n * m, hipMemcpyDeviceToHost));
        double* Co = C_out + (size_t)s2 * n2;
        for (int r = 0; r < n; ++r)
          for (int c = 0; c < n; ++c) Co[(size_t)r * n + c] = c < m ? Ch[(size_t)r * m + c] : 0.0;
      }
      if (eps_out) {
        std::vector<double> e(m);
        DFX_HIP(hipMemcpy(e.data(), eps[s2].p, 8 * (size_t)m, hipMemcpyDeviceToHost));
        for (int i = 0; i < n; ++i) eps_out[(size_t)s2 * n + i] = i < m ? e[i] : 0.0;
      }
    }
    inf.niter = std::min(it, o.max_iter);
    inf.converged = converged ? 1 : 0;
    inf.n_purified = n_purified;
    inf.n_eigh = n_eigh;
    inf.purify_steps = purify_steps;
    inf.ndropped = n - m;
    inf.nbf = n;
    inf.naux = B->naux;
    inf.nocc = na;
    inf.E_nuc = Enuc;
    inf.err_max = emax;
    inf.t_setup = std::chrono::duration<double>(t1c - t0).count();
    inf.t_scf = std::chrono::duration<double>(t2c - t1c).count();
    inf.t_total = std::chrono::duration<double>(clk::now() - t0).count();
    inf.t_eri = B->info.eri_seconds;
    inf.t_metric = B->info.metric_seconds;
    inf.t_trsm = B->info.trsm_seconds;
    inf.t_trsm_update = B->info.trsm_update_seconds;
    inf.trsm_update_flops = B->info.trsm_update_flops;
    inf.n_trsm_update = B->info.trsm_update_launches;
    inf.nintegrals = B->info.nintegrals;
    inf.ncols = B->info.ncols;
    if (info) *info = inf;
    if (!converged) {
      status = DFX_ENOCONV;
      set_last_error(fn + ": not converged in " + std::to_string(o.max_iter) + " iterations");
    }
  });
  return rc != DFX_OK ? rc : status;
}

int dfx_uhf(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
            const dfx_scf_opts* opts, int multiplicity, double* E, double* C, double* eps, dfx_scf_info* info) {
  return open_shell_scf(geom, shells, nsh, aux, nauxsh, opts, multiplicity, E, C, eps, info, false);
}

int dfx_rohf(const dfx_geom* geom, const dfx_shell* shells, int nsh, const dfx_shell* aux, int nauxsh,
             const dfx_scf_opts* opts, int multiplicity, double* E, double* C, double* eps, dfx_scf_info* info) {
  return open_shell_scf(geom, shells, nsh, aux, nauxsh, opts, multiplicity, E, C, eps, info, true);
}

int dfx_lowdin(const dfx_geom* geom, const dfx_shell* shells, int nsh, const double* D, double* P, void* stream) {
  return guard([&] {
    if (!geom || !shells || !D || !P) throw Error(DFX_EINVAL, "dfx_lowdin: NULL argument");
    HostShells hb = make_shells(shells, nsh, 3, "orbital basis");
    const int n = hb.nbf;
    const int64_t n2 = (int64_t)n * n;
    Scf S;
    S.st = (hipStream_t)stream;
    hipStream_t st = S.st;
    S.part.alloc(sizeof(double) * 512);
    DevMem W(8 * n2), Tm(8 * n2), Vm(8 * n2), sv(8 * (size_t)n);
    int1e_build(hb, geom, W.as<double>(), Tm.as<double>(), Vm.as<double>(), st);
    // S^1/2 by Newton-Schulz; by the eigen-decomposition where S is too close to singular for it
    bool done = false;
    {
      DevMem b4[4];
      double* buf[4];
      for (int k = 0; k < 4; ++k) {
        b4[k].alloc(8 * (size_t)n2);
        buf[k] = b4[k].as<double>();
      }
      double *isq = nullptr, *sq = nullptr, lmin = 0.0;
      int steps = 0;
      if (S.inv_sqrt(W.as<double>(), n, buf, isq, sq, lmin, steps)) {
        DFX_HIP(hipMemcpyAsync(Vm.p, sq, 8 * n2, hipMemcpyDeviceToDevice, st));
        done = true;
      }
    }
    if (!done) {
      S.syevd(W.as<double>(), n, sv.as<double>());  // rows of W: eigenvectors
      hipLaunchKernelGGL(scale_rows_sqrt_kernel, dim3(nblk(n2)), dim3(256), 0, st, W.as<double>(),
                         sv.as<double>(), n, Tm.as<double>());
      S.gemm(n, n, n, W.as<double>(), n, true, Tm.as<double>(), n, false, Vm.as<double>(), n);  // S^1/2
    }
    DFX_HIP(hipMemcpyAsync(W.p, D, 8 * n2, hipMemcpyHostToDevice, st));
    S.gemm(n, n, n, Vm.as<double>(), n, false, W.as<double>(), n, false, Tm.as<double>(), n);  // S^1/2 D
    S.gemm(n, n, n, Tm.as<double>(), n, false, Vm.as<double>(), n, false, W.as<double>(), n);  // ... S^1/2
    DFX_HIP(hipMemcpyAsync(P, W.p, 8 * n2, hipMemcpyDeviceToHost, st));
    DFX_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
