// Internal launch interface of the dfx kernels (not part of the C-ABI).
#pragma once
#include "common.h"
#include "dfx.h"  // status codes
#include "eri_args.h"

namespace dfx {

struct SchwarzArgs {
  DevShells sh;
  const int* pf;   // [npairs] shell with the larger l
  const int* ps;   // [npairs] shell with the smaller l
  int npairs;
  double* q;       // [npairs] out: sqrt(max (mu nu|mu nu))
  const double* rys;
};

struct OneEArgs {
  DevShells sh;
  const int* pf;
  const int* ps;
  int npairs;
  int n;           // nbf (row stride of S, T, V)
  double *S, *T, *V;
  const double* xyz;  // [natom][3]
  const double* Z;    // [natom]
  int natom;
  const double* rys;
};

void eri3_dispatch(int LA, int LB, int LC, bool unitb, int mode, Eri3Args a, hipStream_t st);
void metric_dispatch(int LA, int LC, Eri3Args a, hipStream_t st);
void schwarz_dispatch(int LA, int LB, SchwarzArgs a, hipStream_t st);
void onee_dispatch(int LA, int LB, OneEArgs a, hipStream_t st);
void aux_schwarz(const double* J, int64_t ld, DevShells aux, double* q, hipStream_t st);

// ---- dense FP64 linear algebra (linalg.hip) --------------------------------
// C = alpha op(A) op(B) + beta C, row-major, strided batch over blockIdx.z.
struct GemmF64 {
  int M, N, K;
  const double* A; int64_t lda; int64_t sA;
  const double* B; int64_t ldb; int64_t sB;
  double* C; int64_t ldc; int64_t sC;
  double alpha, beta;
  int batch;
  bool ta, tb;     // op(A) = A^T, op(B) = B^T
  bool lowerA;     // A is lower triangular (skip zero k-blocks)
  bool lowerC;     // only the lower triangle of C is needed (skip blocks above)
};
void dgemm(const GemmF64& g, hipStream_t st);
// dgemm, with the k-range split over up to 8 partial products (work: ns M N
// doubles, work_elems available) when C alone has too few 128 x 128 tiles to
// fill the chip; the partials are summed in a fixed order
void dgemm_sk(const GemmF64& g, double* work, int64_t work_elems, hipStream_t st);


// B = L^-1 raw in place over raw (n x ncols, FP64, row stride ncols), by
// blocked forward substitution with the lower-triangular L (n x n): backward
// stable, unlike a product with an explicit inverse.  work: trsm_work_elems(n)
// doubles (packed copies of L's 64 x 64 diagonal blocks), free once the last
// launch on st has run.
struct TrsmStats {
  double update_flops = 0.0;  // 2 M K N of every update product
  int update_launches = 0;
};
// optional GPU timer around each update product (events recorded on st)
struct TrsmTimer {
  virtual void begin() = 0;
  virtual void end() = 0;
  virtual ~TrsmTimer() = default;
};
size_t trsm_work_elems(int n);
TrsmStats trsm_solve(const double* L, int n, double* raw, int64_t ncols, double* work, hipStream_t st,
                     TrsmTimer* timer = nullptr);
// X = L^-T X in place (n x ncols, row stride ncols) by blocked back
// substitution with the lower-triangular L: the transpose of trsm_solve.
void trsm_solve_t(const double* L, int n, double* X, int64_t ncols, hipStream_t st);
// hi = fl32(B), lo = fl32(B - hi) of B (n x ncols) into rows of length ld_out (whole
// 32 x 32 tiles): element t of each row from column src[t] of B, zero where src[t] < 0
void tile_split(const double* B, int n, int64_t ncols, const int64_t* src, float* hi, float* lo, int64_t ld_out,
                hipStream_t st);

// Blocked Cholesky J = L L^T in place (lower), then Linv = L^-1.  Returns via
// *info (device int) the first non-positive pivot + 1, or 0; a pivot below
// 1e-14 of its original diagonal element counts as non-positive.
// work: cholesky_work_elems(n) doubles.
void cholesky_inverse(double* J, int n, double* Linv, double* work, int* info, hipStream_t st);
// the factor alone (no L^-1), same work and error reporting
void cholesky_factor(double* J, int n, double* work, int* info, hipStream_t st);
size_t cholesky_work_elems(int n);

// Symmetric eigen-decomposition by the two-sided block Jacobi method (eig.hip):
// A (n x n, row-major; the symmetric part is used) is overwritten with the
// orthonormal eigenvectors as rows, w (device, n) gets the eigenvalues in
// ascending order.  Every off-diagonal element of the final rotated matrix is
// below 1e-15 sqrt(|a_ii a_jj|).  Synchronous; returns the number of sweeps;
// throws after 40 sweeps.  Device memory: sym_eig_work_bytes(n).
int sym_eig(double* A, int n, double* w, hipStream_t st);
size_t sym_eig_work_bytes(int n);

// ---- J / K (jk.hip) ----------------------------------------------------------
enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2 };
struct JKArgs {
  const float* hi;
  const float* lo;
  int naux, nbf;
  int64_t ncols;   // tiled columns
  int prec;
  // K work cap in bytes (0: the default chunk sizes).  With a cap the
  // auxiliary index is cut into as many chunks as it takes for k_work_bytes to
  // stay within it, and the SYRK keeps eight partial-sum slices; DFX_ENOMEM if
  // even one auxiliary function per chunk does not fit.
  size_t ws_cap = 0;
};
void j_build(const JKArgs& a, const double* D, double* J, double* work, hipStream_t st);
// gamma_Q = sum B_Q,mu nu D_mu nu alone (Eq. 3a); dvec: ncols doubles of work
void j_gamma(const JKArgs& a, const double* D, double* gam, double* dvec, hipStream_t st);
// K from the occupied block C [nbf][nocc] (row-major); work >= k_work_bytes
size_t k_work_bytes(const JKArgs& a, int nocc);
// optional GPU timers around the two K phases (events are recorded on st)
struct KTimer {
  virtual void begin_x() = 0;
  virtual void end_x() = 0;
  virtual void begin_syrk() = 0;
  virtual void end_syrk() = 0;
  virtual ~KTimer() = default;
};
void k_build(const JKArgs& a, const double* C, int nocc, double* K, void* work, hipStream_t st,
             KTimer* timer = nullptr);
// FP64 K (jk_f64.hip), dispatched by k_build for PREC_FP64
size_t k_work_bytes_f64(const JKArgs& a, int nocc);
// X[mu][(Q - q0) nocc + i] = sum_nu B_Q[mu][nu] C[nu][i], Q in [q0, q0 + nq): the FP64
// half transform of the exchange build on its own (work: half_transform_f64_work bytes)
size_t half_transform_f64_work(const JKArgs& a, int nocc);
void half_transform_f64(const JKArgs& a, const double* C, int nocc, int q0, int nq, double* X, int64_t ldx,
                        void* work, hipStream_t st);
// DF-MP2 correlation energy from B and canonical orbitals (mp2.hip)
double mp2_energy(const JKArgs& a, const double* C, int nmo, const double* eps, int nocc, int nfrozen,
                  hipStream_t st);
void k_build_f64(const JKArgs& a, const double* C, int nocc, double* K, void* work, hipStream_t st,
                 KTimer* timer);
// C = A A^T (both triangles) for a row-major n x k A, even row stride lda,
// 16-byte aligned (jk_f64.hip); work: syrk_f64_work_elems(n) doubles
size_t syrk_f64_work_elems(int n);
void syrk_f64(const double* A, int64_t lda, int n, int64_t k, double* C, double* work, hipStream_t st);
// reduced-precision K (jk_mixed.hip), dispatched by k_build for PREC_FP32 / PREC_BF16
size_t k_work_bytes_mixed(const JKArgs& a, int nocc);
void k_build_mixed(const JKArgs& a, const double* C, int nocc, double* K, void* work, hipStream_t st,
                   KTimer* timer);
// canonical packed rows [q1 - q0][ncols_p] (FP64) from the tiled storage;
// toff[c] is the tile offset of packed column c
// dense rows out[q1 - q0][nbf][nbf] (FP64 = hi + lo) from the tiled storage
void unpack_rows(const float* hi, const float* lo, int64_t ncols_t, int nbf, int q0, int q1, double* out,
                 hipStream_t st);
void export_rows(const float* hi, const float* lo, const double* raw, int64_t ncols_t, int q0, int q1,
                 const int64_t* toff, int64_t ncols_p, double* out, hipStream_t st);

// ---- small dense helpers (linalg.hip) ----------------------------------------
void fill_f64(double* p, size_t n, double v, hipStream_t st);
void sym_from_lower(double* A, int n, hipStream_t st);

}  // namespace dfx
