// DF-MP2 correlation energy of a closed-shell RHF reference (section "Standard
// algorithms": MP2 as a post-HF method, built on the density-fitting
// operations of Eqs. (1) and (2)):
//
//   (ia|Q)  = sum_{mu nu} C_mu,i B_Q,mu nu C_nu,a     two index transformations, Eq. (1)
//   (ia|jb) = sum_Q (ia|Q)(jb|Q)                       contraction of two tensors, Eq. (2)
//   E2      = sum_{ij,ab} (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b)
//
// The first transformation is the exchange build's FP64 half transform
// (X_Q = B_Q C_occ); the second is a DGEMM with C_vir.  The three-index tensor
// is kept as A[i][a][Q], so that for each i one DGEMM gives (ia|jb) for all
// j <= i and all a, b; a reduction kernel applies the denominators.  All FP64.
#include <algorithm>
#include <vector>

#include "host.h"

namespace dfx {

// dst[r][c] = src[r][c0 + c], r < rows, c < cols
__global__ void mp2_cols_kernel(const double* __restrict__ src, int lds, int c0, int rows, int cols,
                                double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int r = (int)(i / cols), c = (int)(i % cols);
  dst[i] = src[(int64_t)r * lds + c0 + c];
}

// A[i][a][q0 + q] = T[a][q no + i]: (ia|Q) of one chunk of Q into the [i][a][Q] layout
__global__ void mp2_scatter_kernel(const double* __restrict__ T, int nv, int no, int nq, int naux, int q0,
                                   double* __restrict__ A) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nv * nq * no;
  if (idx >= tot) return;
  const int a = (int)(idx / ((int64_t)nq * no));
  const int64_t r = idx % ((int64_t)nq * no);
  const int q = (int)(r / no), i = (int)(r % no);
  A[((int64_t)i * nv + a) * naux + q0 + q] = T[idx];
}

// partial sums over (j <= i, a, b) of M[a][j nv + b] (2 M[a][j nv + b] - M[b][j nv + a]) /
// (e_i + e_j - e_a - e_b), weight 2 for j < i; M = (ia|jb) for one i.  Fixed grid and
// tree order: out[blockIdx.x]
constexpr int MP2_RB = 1024;
constexpr int MP2_T = 32;
// Work item (j, A <= B): the 32 x 32 tiles X = M_j[A][B] and Y = M_j[B][A] of the
// nv x nv block M_j[a][b] = (ia|jb), both read as rows (coalesced) into padded
// LDS.  Off the tile diagonal the item adds the (a, b) and (b, a) terms of the
// pair at once: x (2x - y) + y (2y - x) = 2 (x^2 - x y + y^2), x = (ia|jb),
// y = (ib|ja), over the common denominator.  Blocks take items blockIdx.x,
// blockIdx.x + MP2_RB, ... so the order of every sum is fixed.
__global__ void __launch_bounds__(256) mp2_pair_kernel(const double* __restrict__ M, int nv, int i,
                                                       const double* __restrict__ eo, const double* __restrict__ ev,
                                                       double* __restrict__ out) {
  __shared__ double X[MP2_T][MP2_T + 1], Y[MP2_T][MP2_T + 1];
  __shared__ double red[256];
  const int nt = (nv + MP2_T - 1) / MP2_T;
  const int64_t ntp = (int64_t)nt * (nt + 1) / 2;
  const int64_t nwork = ntp * (i + 1);
  const int64_t ld = (int64_t)(i + 1) * nv;
  const double ei = eo[i];
  double s = 0.0;
  for (int64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int j = (int)(w / ntp);
    const int tp = (int)(w % ntp);
    int Bt = (int)((sqrt(8.0 * tp + 1.0) - 1.0) * 0.5);
    while ((Bt + 1) * (Bt + 2) / 2 <= tp) ++Bt;
    while (Bt * (Bt + 1) / 2 > tp) --Bt;
    const int At = tp - Bt * (Bt + 1) / 2;  // At <= Bt
    const int a0 = At * MP2_T, b0 = Bt * MP2_T;
    const double* Mj = M + (int64_t)j * nv;
    for (int e = threadIdx.x; e < MP2_T * MP2_T; e += blockDim.x) {
      const int r = e / MP2_T, c = e % MP2_T;
      X[r][c] = (a0 + r < nv && b0 + c < nv) ? Mj[(int64_t)(a0 + r) * ld + b0 + c] : 0.0;
      if (At != Bt) Y[r][c] = (b0 + r < nv && a0 + c < nv) ? Mj[(int64_t)(b0 + r) * ld + a0 + c] : 0.0;
    }
    __syncthreads();
    const double eij = ei + eo[j], wj = j < i ? 2.0 : 1.0;
    for (int e = threadIdx.x; e < MP2_T * MP2_T; e += blockDim.x) {
      const int r = e / MP2_T, c = e % MP2_T;
      const int aa = a0 + r, bb = b0 + c;
      if (aa < nv && bb < nv) {
        const double d = eij - ev[aa] - ev[bb];
        const double x = X[r][c];
        if (At == Bt) {
          const double y = X[c][r];
          s += wj * x * (2.0 * x - y) / d;
        } else {
          const double y = Y[c][r];
          s += wj * 2.0 * (x * x - x * y + y * y) / d;
        }
      }
    }
    __syncthreads();
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

static unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

double mp2_energy(const JKArgs& a, const double* C, int nmo, const double* eps, int nocc, int nfrozen,
                  hipStream_t st) {
  const int nbf = a.nbf, naux = a.naux;
  const int no = nocc - nfrozen, nv = nmo - nocc;
  if (nfrozen < 0 || no <= 0 || nv <= 0 || nmo > nbf) throw Error(DFX_EINVAL, "dfx_mp2: bad orbital counts");
  if (no > 512) throw Error(DFX_EUNSUPPORTED, "dfx_mp2: more than 512 correlated occupied orbitals");
  JKArgs a64 = a;
  a64.prec = PREC_FP64;
  // orbital blocks, energies
  DevMem Co(sizeof(double) * (size_t)nbf * no), Cv(sizeof(double) * (size_t)nbf * nv);
  hipLaunchKernelGGL(mp2_cols_kernel, dim3(nb256((int64_t)nbf * no)), dim3(256), 0, st, C, nmo, nfrozen, nbf, no,
                     Co.as<double>());
  hipLaunchKernelGGL(mp2_cols_kernel, dim3(nb256((int64_t)nbf * nv)), dim3(256), 0, st, C, nmo, nocc, nbf, nv,
                     Cv.as<double>());
  std::vector<double> eo_h(eps + nfrozen, eps + nocc), ev_h(eps + nocc, eps + nmo);
  DevMem eo = upload(eo_h, st), ev = upload(ev_h, st);
  // (ia|Q) in chunks of Q: X = B_Q C_occ, then T = C_vir^T X
  const size_t per_q = (size_t)(nbf + nv) * no * sizeof(double);
  const int qc = (int)std::max<size_t>(1, std::min<size_t>(naux, ((size_t)4 << 30) / per_q));
  DevMem X(sizeof(double) * (size_t)nbf * qc * no), T(sizeof(double) * (size_t)nv * qc * no);
  DevMem hw(half_transform_f64_work(a64, no));
  DevMem A(sizeof(double) * (size_t)no * nv * naux);
  for (int q0 = 0; q0 < naux; q0 += qc) {
    const int nq = std::min(qc, naux - q0);
    const int64_t w = (int64_t)nq * no;
    half_transform_f64(a64, Co.as<double>(), no, q0, nq, X.as<double>(), w, hw.p, st);
    GemmF64 g{};
    g.M = nv; g.N = (int)w; g.K = nbf;
    g.A = Cv.as<double>(); g.lda = nv; g.ta = true;
    g.B = X.as<double>(); g.ldb = w;
    g.C = T.as<double>(); g.ldc = w;
    g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
    dgemm(g, st);
    hipLaunchKernelGGL(mp2_scatter_kernel, dim3(nb256((int64_t)nv * w)), dim3(256), 0, st, T.as<double>(), nv, no,
                       nq, naux, q0, A.as<double>());
  }
  X.release();
  T.release();
  // per i: M = A_i A_{0..i}^T = (ia|jb) for j <= i, then the energy terms
  DevMem M(sizeof(double) * (size_t)nv * no * nv);
  const int64_t sk_elems = (int64_t)64 << 20;  // split-K partial products for the small first products
  DevMem sk(sizeof(double) * (size_t)sk_elems);
  DevMem part(sizeof(double) * (size_t)no * MP2_RB);
  for (int i = 0; i < no; ++i) {
    GemmF64 g{};
    g.M = nv; g.N = (i + 1) * nv; g.K = naux;
    g.A = A.as<double>() + (int64_t)i * nv * naux; g.lda = naux;
    g.B = A.as<double>(); g.ldb = naux; g.tb = true;
    g.C = M.as<double>(); g.ldc = (int64_t)(i + 1) * nv;
    g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
    dgemm_sk(g, sk.as<double>(), sk_elems, st);
    hipLaunchKernelGGL(mp2_pair_kernel, dim3(MP2_RB), dim3(256), 0, st, M.as<double>(), nv, i, eo.as<double>(),
                       ev.as<double>(), part.as<double>() + (int64_t)i * MP2_RB);
  }
  std::vector<double> ph((size_t)no * MP2_RB);
  DFX_HIP(hipMemcpyAsync(ph.data(), part.p, sizeof(double) * ph.size(), hipMemcpyDeviceToHost, st));
  DFX_HIP(hipStreamSynchronize(st));
  double E = 0.0;
  for (double v : ph) E += v;
  return E;
}

}  // namespace dfx
