// Dense FP64 linear algebra on gfx950 MFMA: a tiled DGEMM (v_mfma_f64_16x16x4),
// the blocked Cholesky factorisation of the fitting metric J_PQ = L L^T (and
// L^-1 where asked), and the transform B = L^-1 (mu nu|P) of Eq. (1c) with
// M' = L^-1 by blocked forward substitution, then split into two FP32 words.
#include <algorithm>

#include "kernels.h"

namespace dfx {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GM = 128, GN = 128, GK = 16, GT = 256;
// k-major LDS rows of GM + 16 doubles: the four k rows a fragment read touches
// fall on alternate halves of the 64 banks (2 passes per read, the minimum)
constexpr int LDS_PAD = 16;
enum { EPI_F64 = 0, EPI_SUB = 1 };  // EPI_SUB: C -= A B (the B transform's updates)

// Workgroup -> tile map.  Workgroups are dealt round-robin to the 8 XCDs; give
// each XCD a contiguous range of tiles (M-block fastest) so that the tiles that
// share a B panel also share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int tiles) {
  const int q = tiles >> 3, r = tiles & 7;
  const int x = bid & 7, slot = bid >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + slot;
}

// 8 consecutive doubles from p (16-byte aligned) as four 16-byte loads
__device__ __forceinline__ void ld8d(const double* __restrict__ p, double* v) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const double2 x = q[e];
    v[2 * e] = x.x;
    v[2 * e + 1] = x.y;
  }
}

// C = alpha op(A) op(B) + beta C (EPI_F64), or C -= op(A) op(B) (EPI_SUB).
// Each k-stage is loaded into registers while the MFMAs of the previous stage run.
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(GT, 2) dgemm_kernel(GemmF64 g) {
  __shared__ double As[GK][GM + LDS_PAD];
  __shared__ double Bs[GK][GN + LDS_PAD];
  const int MB = (g.M + GM - 1) / GM, NB = (g.N + GN - 1) / GN;
  const int t = xcd_tile(blockIdx.x, MB * NB);
  const int m0 = (t % MB) * GM, n0 = (t / MB) * GN;
  if (g.lowerC && n0 > m0 + GM - 1) return;
  const int z = blockIdx.z;
  const double* __restrict__ A = g.A + z * g.sA;
  const double* __restrict__ B = g.B + z * g.sB;
  double* __restrict__ C = g.C + z * g.sC;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
  const int li = lane & 15, lk = lane >> 4;
  // vector loads need even leading dimensions and 16-byte aligned bases
  const bool va = (g.lda % 2 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const bool vb = (g.ldb % 2 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  int kmax = g.K;
  if (g.lowerA && m0 + GM < kmax) kmax = m0 + GM;

  double ra[8], rb[8];
  auto load = [&](int k0) {
    if (!TA) {  // row m, 8 consecutive k
      const int m = m0 + (tid >> 1), k = k0 + (tid & 1) * 8;
      if (va && m < g.M && k + 8 <= kmax) {
        ld8d(A + (int64_t)m * g.lda + k, ra);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) ra[j] = (m < g.M && k + j < kmax) ? A[(int64_t)m * g.lda + k + j] : 0.0;
      }
    } else {    // row k, 8 consecutive m
      const int k = k0 + (tid >> 4), m = m0 + (tid & 15) * 8;
      if (va && k < kmax && m + 8 <= g.M) {
        ld8d(A + (int64_t)k * g.lda + m, ra);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) ra[j] = (m + j < g.M && k < kmax) ? A[(int64_t)k * g.lda + m + j] : 0.0;
      }
    }
    if (!TB) {  // row k, 8 consecutive n
      const int k = k0 + (tid >> 4), n = n0 + (tid & 15) * 8;
      if (vb && k < kmax && n + 8 <= g.N) {
        ld8d(B + (int64_t)k * g.ldb + n, rb);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) rb[j] = (n + j < g.N && k < kmax) ? B[(int64_t)k * g.ldb + n + j] : 0.0;
      }
    } else {    // row n, 8 consecutive k
      const int n = n0 + (tid >> 1), k = k0 + (tid & 1) * 8;
      if (vb && n < g.N && k + 8 <= kmax) {
        ld8d(B + (int64_t)n * g.ldb + k, rb);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) rb[j] = (n < g.N && k + j < kmax) ? B[(int64_t)n * g.ldb + k + j] : 0.0;
      }
    }
  };
  auto store = [&]() {  // registers -> LDS, k-major
    if (!TA) {
      const int i = tid >> 1, kb = (tid & 1) * 8;
#pragma unroll
      for (int j = 0; j < 8; ++j) As[kb + j][i] = ra[j];
    } else {
      const int k = tid >> 4, mb = (tid & 15) * 8;
#pragma unroll
      for (int j = 0; j < 8; ++j) As[k][mb + j] = ra[j];
    }
    if (!TB) {
      const int k = tid >> 4, nb = (tid & 15) * 8;
#pragma unroll
      for (int j = 0; j < 8; ++j) Bs[k][nb + j] = rb[j];
    } else {
      const int n = tid >> 1, kb = (tid & 1) * 8;
#pragma unroll
      for (int j = 0; j < 8; ++j) Bs[kb + j][n] = rb[j];
    }
  };

  if (kmax > 0) load(0);
  for (int k0 = 0; k0 < kmax; k0 += GK) {
    __syncthreads();  // the previous stage's fragments have been read
    store();
    __syncthreads();
    if (k0 + GK < kmax) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      double fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) fa[i] = As[kk + lk][wm + i * 16 + li];
#pragma unroll
      for (int j = 0; j < 4; ++j) fb[j] = Bs[kk + lk][wn + j * 16 + li];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
  }

  // ---- epilogue.  v_mfma_f64_16x16x4 leaves element (row, col) of its 16x16
  // block in lane col + 16 (row % 4), register row / 4, so
  // acc[i][j][r] is C[wm + 16 i + 4 r + lk][wn + 16 j + li]
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + r * 4 + lk;
        const int n = n0 + wn + j * 16 + li;
        if (m < g.M && n < g.N) {
          const int64_t o = (int64_t)m * g.ldc + n;
          if (EPI == EPI_F64) {
            double v = g.alpha * acc[i][j][r];
            if (g.beta != 0.0) v = fma(g.beta, C[o], v);
            C[o] = v;
          } else {
            C[o] = C[o] - acc[i][j][r];
          }
        }
      }
}

static int gemm_tiles(int M, int N) { return ((M + GM - 1) / GM) * ((N + GN - 1) / GN); }

void dgemm(const GemmF64& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  const dim3 grid(gemm_tiles(g.M, g.N), 1, g.batch > 0 ? g.batch : 1);
  GemmF64 a = g;
  if (g.K <= 0) {  // C = beta C
    a.K = 0;
  }
#define L(TA_, TB_) \
  hipLaunchKernelGGL((dgemm_kernel<TA_, TB_, EPI_F64>), grid, dim3(GT), 0, st, a)
  if (!g.ta && !g.tb) L(false, false);
  else if (!g.ta && g.tb) L(false, true);
  else if (g.ta && !g.tb) L(true, false);
  else L(true, true);
#undef L
}

// C = alpha sum_s W_s + beta C, partials W_s [M][N] contiguous, summed in order
__global__ void sk_reduce_kernel(const double* __restrict__ W, int ns, int M, int N, double alpha, double beta,
                                 double* __restrict__ C, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mn = (int64_t)M * N;
  if (i >= mn) return;
  double s = 0.0;
  for (int z = 0; z < ns; ++z) s += W[z * mn + i];
  double* c = C + (i / N) * ldc + (i % N);
  *c = beta != 0.0 ? alpha * s + beta * *c : alpha * s;
}

void dgemm_sk(const GemmF64& g, double* work, int64_t work_elems, hipStream_t st) {
  const int tiles = gemm_tiles(g.M, g.N);
  const int64_t mn = (int64_t)g.M * g.N;
  int ns = 1;
  while (ns < 8 && tiles * ns < 512 && g.K / (2 * ns) >= 128 && 2 * ns * mn <= work_elems) ns *= 2;
  if (ns == 1 || g.batch > 1 || g.lowerA || g.lowerC || !work) {
    dgemm(g, st);
    return;
  }
  const int klen = ((g.K + ns - 1) / ns + GK - 1) / GK * GK;
  GemmF64 a = g;
  a.ldc = g.N;
  a.alpha = 1.0;
  a.beta = 0.0;
  a.batch = 1;
  auto launch = [&](const GemmF64& x, int nz) {
    const dim3 grid(tiles, 1, nz);
#define L(TA_, TB_) \
  hipLaunchKernelGGL((dgemm_kernel<TA_, TB_, EPI_F64>), grid, dim3(GT), 0, st, x)
    if (!x.ta && !x.tb) L(false, false);
    else if (!x.ta && x.tb) L(false, true);
    else if (x.ta && !x.tb) L(true, false);
    else L(true, true);
#undef L
  };
  if ((int64_t)klen * ns == g.K) {  // equal k-ranges: one batched launch
    a.K = klen;
    a.sA = g.ta ? (int64_t)klen * g.lda : klen;
    a.sB = g.tb ? klen : (int64_t)klen * g.ldb;
    a.sC = mn;
    a.C = work;
    launch(a, ns);
  } else {
    int z = 0;
    for (int k0 = 0; k0 < g.K; k0 += klen, ++z) {
      a.K = std::min(klen, g.K - k0);
      a.A = g.ta ? g.A + (int64_t)k0 * g.lda : g.A + k0;
      a.B = g.tb ? g.B + k0 : g.B + (int64_t)k0 * g.ldb;
      a.C = work + z * mn;
      a.sA = a.sB = a.sC = 0;
      launch(a, 1);
    }
    ns = z;
  }
  hipLaunchKernelGGL(sk_reduce_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, work, ns, g.M, g.N,
                     g.alpha, g.beta, g.C, g.ldc);
}

// ---------------------------------------------------------------------------
// B = L^-1 raw by blocked forward substitution, in place over raw (n x ncols,
// row stride ncols).  Left-looking over blocks of TB = 128 rows: the block's
// rows take R_i -= L_i,0:i B_0:i as one DGEMM (MFMA, the rows before it are
// already B), then the 128 x 128 diagonal block is solved by substitution, in
// two halves of 64 rows with the DGEMM R_2 -= L_21 B_1 between them.  Unlike a
// product with an explicitly formed L^-1, whose rounding errors are amplified
// by cond(L), this is backward stable: the result is the exact transform with
// a metric perturbed at the rounding level.
constexpr int TS_T = 256;   // columns per workgroup of the substitution
constexpr int TS_R = 64;    // rows solved in registers

// L x = b for the nr <= 64 rows r0.. of every column c of X: one column per
// thread, its 64 unknowns in registers.  Rows go in groups of 8: the group's
// right-hand sides take s_r -= L_rk x_k for every earlier unknown k (one step
// per k reads the 8 entries L_(g..g+7),k, stored k-major in LDS so that they are
// consecutive), then the 8 x 8 triangle is solved, x_r = s_r / L_rr.  The block
// of L is staged in LDS and every lane reads the same address.
constexpr int TS_G = 8;
template <bool FULL>  // FULL: nr == 64
__global__ void __launch_bounds__(TS_T) trsv64_cols_kernel(const double* __restrict__ L, int64_t ldl, int nr,
                                                           double* __restrict__ X, int64_t ldx, int ncols) {
  __shared__ double Lt[TS_R][TS_R];  // Lt[k][i] = L_ik
  for (int e = threadIdx.x; e < TS_R * TS_R; e += TS_T) {
    const int k = e / TS_R, i = e % TS_R;
    // rows beyond nr: the identity, so their (zero) unknowns stay zero
    Lt[k][i] = (i < nr && k < nr) ? (k <= i ? L[(int64_t)i * ldl + k] : 0.0) : (i == k ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = blockIdx.x * TS_T + threadIdx.x;
  if (c >= ncols) return;
  double x[TS_R];
#pragma unroll
  for (int g = 0; g < TS_R; g += TS_G) {
    double s[TS_G];
#pragma unroll
    for (int r = 0; r < TS_G; ++r) {
      // the row base is wave-uniform; rows past nr read row nr - 1 and drop it
      const int row = FULL ? g + r : min(g + r, nr - 1);
      const double v = X[(int64_t)row * ldx + c];
      s[r] = (FULL || g + r < nr) ? v : 0.0;
    }
#pragma unroll
    for (int k = 0; k < g; ++k) {
      double l[TS_G];
#pragma unroll
      for (int r = 0; r < TS_G; ++r) l[r] = Lt[k][g + r];
#pragma unroll
      for (int r = 0; r < TS_G; ++r) s[r] = fma(-l[r], x[k], s[r]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < TS_G; ++r) {
#pragma unroll
      for (int k = 0; k < r; ++k) s[r] = fma(-Lt[g + k][g + r], x[g + k], s[r]);
      x[g + r] = s[r] / Lt[g + r][g + r];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // without branches: rows past nr store to row nr - 1, in descending order so
  // that the last store there (program order, one thread) is x[nr - 1]
#pragma unroll
  for (int i = TS_R - 1; i >= 0; --i) X[(int64_t)(FULL ? i : min(i, nr - 1)) * ldx + c] = x[i];
}

// The same substitution for a full 64-row block, L given as a packed k-major
// copy of the block (pack_diag_kernel: row k holds L_ik, i >= k, zeros before).
// Every lane needs the same L_ik at the same step: read from global memory at
// wave-uniform addresses (one base, constant offsets), they come through the
// scalar cache into SGPRs, which the FMAs take directly, instead of every lane
// reading them from LDS (whose return bandwidth bounds the kernel above).  Same
// operations in the same order, so the same results bit for bit.
__global__ void __launch_bounds__(TS_T) trsv64_sym_kernel(const double* __restrict__ Lk, double* __restrict__ X,
                                                          int64_t ldx, int ncols) {
  const int c = blockIdx.x * TS_T + threadIdx.x;
  const bool own = c < ncols;
  const int cc = own ? c : ncols - 1;  // lanes past the end repeat the last column and store nothing
  double x[TS_R];
#pragma unroll
  for (int g = 0; g < TS_R; g += TS_G) {
    double s[TS_G];
#pragma unroll
    for (int r = 0; r < TS_G; ++r) s[r] = X[(int64_t)(g + r) * ldx + cc];
#pragma unroll
    for (int k = 0; k < g; ++k) {
      double l[TS_G];
#pragma unroll
      for (int r = 0; r < TS_G; ++r) l[r] = Lk[k * TS_R + g + r];
#pragma unroll
      for (int r = 0; r < TS_G; ++r) s[r] = fma(-l[r], x[k], s[r]);
      // a compiler-only fence: the loads of L are invariant and would otherwise all be
      // hoisted to the top, far beyond the SGPR budget
      asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int r = 0; r < TS_G; ++r) {
#pragma unroll
      for (int k = 0; k < r; ++k) s[r] = fma(-Lk[(g + k) * TS_R + g + r], x[g + k], s[r]);
      x[g + r] = s[r] / Lk[(g + r) * TS_R + g + r];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (own) {
#pragma unroll
    for (int i = 0; i < TS_R; ++i) X[(int64_t)i * ldx + c] = x[i];
  }
}

// Packed k-major copies of the full 64 x 64 diagonal blocks of L (row stride n),
// one workgroup per block: P[b][k][i] = L_(64b + i),(64b + k) for i >= k, else 0.
__global__ void pack_diag_kernel(const double* __restrict__ L, int n, double* __restrict__ P) {
  const int64_t o = (int64_t)blockIdx.x * TS_R * n + (int64_t)blockIdx.x * TS_R;
  double* __restrict__ Pb = P + (int64_t)blockIdx.x * TS_R * TS_R;
  for (int e = threadIdx.x; e < TS_R * TS_R; e += blockDim.x) {
    const int k = e / TS_R, i = e % TS_R;
    Pb[e] = i >= k ? L[o + (int64_t)i * n + k] : 0.0;
  }
}

// L^T x = b for the nr <= 64 rows of every column of X (the diagonal block L of
// the back substitution B = L^-T R): x_i = (b_i - sum_k>i L_ki x_k) / L_ii,
// rows from the last, in groups of 8 as in trsv64_cols_kernel.  Rows beyond nr
// are the identity with zero right-hand sides.
template <bool FULL>
__global__ void __launch_bounds__(TS_T) trsv64t_cols_kernel(const double* __restrict__ L, int64_t ldl, int nr,
                                                            double* __restrict__ X, int64_t ldx, int ncols) {
  __shared__ double Lr[TS_R][TS_R];  // Lr[k][i] = L_ki
  for (int e = threadIdx.x; e < TS_R * TS_R; e += TS_T) {
    const int k = e / TS_R, i = e % TS_R;
    Lr[k][i] = (i < nr && k < nr) ? (i <= k ? L[(int64_t)k * ldl + i] : 0.0) : (i == k ? 1.0 : 0.0);
  }
  __syncthreads();
  const int c = blockIdx.x * TS_T + threadIdx.x;
  if (c >= ncols) return;
  double x[TS_R];
#pragma unroll
  for (int g = TS_R - TS_G; g >= 0; g -= TS_G) {
    double s[TS_G];
#pragma unroll
    for (int r = 0; r < TS_G; ++r) {
      const int row = FULL ? g + r : min(g + r, nr - 1);
      const double v = X[(int64_t)row * ldx + c];
      s[r] = (FULL || g + r < nr) ? v : 0.0;
    }
#pragma unroll
    for (int k = TS_R - 1; k >= g + TS_G; --k) {
      double l[TS_G];
#pragma unroll
      for (int r = 0; r < TS_G; ++r) l[r] = Lr[k][g + r];
#pragma unroll
      for (int r = 0; r < TS_G; ++r) s[r] = fma(-l[r], x[k], s[r]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = TS_G - 1; r >= 0; --r) {
#pragma unroll
      for (int k = r + 1; k < TS_G; ++k) s[r] = fma(-Lr[g + k][g + r], x[g + k], s[r]);
      x[g + r] = s[r] / Lr[g + r][g + r];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = TS_R - 1; i >= 0; --i) X[(int64_t)(FULL ? i : min(i, nr - 1)) * ldx + c] = x[i];
}

// hi = fl32(B), lo = fl32(B - hi) in the tile layout, gathered: element t of a
// tiled row takes packed column src[t] of the same row of B, or zero where
// src[t] < 0 (tile padding, screened pairs), so every element of the tiled rows
// is written.  One workgroup per 32 x 32 tile and SPLIT_Q rows: thread i takes
// tile elements i, i + 256, i + 512, i + 768, so a wave writes two whole tile
// rows (coalesced), while the workgroup reads the few contiguous pair blocks of
// B the tile draws on, with their reuse in one XCD's L2.
constexpr int SPLIT_Q = 4;
__global__ void __launch_bounds__(256) tile_split_kernel(const double* __restrict__ B, int64_t ncols, int nrows,
                                                         const int64_t* __restrict__ src, float* __restrict__ hi,
                                                         float* __restrict__ lo, int64_t ld_out) {
  const int64_t t0 = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  int64_t s[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) s[j] = src[t0 + 256 * j];
  const int q0 = blockIdx.y * SPLIT_Q;
  double v[SPLIT_Q][4];
#pragma unroll
  for (int k = 0; k < SPLIT_Q; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v[k][j] = (q0 + k < nrows && s[j] >= 0) ? B[(int64_t)(q0 + k) * ncols + s[j]] : 0.0;
#pragma unroll
  for (int k = 0; k < SPLIT_Q; ++k) {
    if (q0 + k >= nrows) break;
    const int64_t o = (int64_t)(q0 + k) * ld_out + t0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float h = (float)v[k][j];
      hi[o + 256 * j] = h;
      lo[o + 256 * j] = (float)(v[k][j] - (double)h);
    }
  }
}

// Lk: for a full block (nr == 64), its packed k-major copy (pack_diag_kernel)
static void trsv64_cols(const double* L, int64_t ldl, int nr, double* X, int64_t ldx, int64_t ncols,
                        hipStream_t st, const double* Lk = nullptr) {
  // columns in slabs whose indices fit the kernel's 32-bit column offsets
  const int64_t slab = (int64_t)TS_T * 1048576;
  for (int64_t c0 = 0; c0 < ncols; c0 += slab) {
    const int nc = (int)std::min<int64_t>(slab, ncols - c0);
    const dim3 g((unsigned)((nc + TS_T - 1) / TS_T));
    if (Lk && nr == TS_R)
      hipLaunchKernelGGL(trsv64_sym_kernel, g, dim3(TS_T), 0, st, Lk, X + c0, ldx, nc);
    else if (nr == TS_R)
      hipLaunchKernelGGL(trsv64_cols_kernel<true>, g, dim3(TS_T), 0, st, L, ldl, nr, X + c0, ldx, nc);
    else
      hipLaunchKernelGGL(trsv64_cols_kernel<false>, g, dim3(TS_T), 0, st, L, ldl, nr, X + c0, ldx, nc);
  }
}

// X[rows] -= A X[krows]: R_i -= L_i,0:k B_0:k over all columns, in slabs that
// keep each launch's grid within range
static void trsv64t_cols(const double* L, int64_t ldl, int nr, double* X, int64_t ldx, int64_t ncols,
                         hipStream_t st) {
  const int64_t slab = (int64_t)TS_T * 1048576;
  for (int64_t c0 = 0; c0 < ncols; c0 += slab) {
    const int nc = (int)std::min<int64_t>(slab, ncols - c0);
    const dim3 g((unsigned)((nc + TS_T - 1) / TS_T));
    if (nr == TS_R)
      hipLaunchKernelGGL(trsv64t_cols_kernel<true>, g, dim3(TS_T), 0, st, L, ldl, nr, X + c0, ldx, nc);
    else
      hipLaunchKernelGGL(trsv64t_cols_kernel<false>, g, dim3(TS_T), 0, st, L, ldl, nr, X + c0, ldx, nc);
  }
}

// C -= A^T X over all columns: A stored K x M (lda), the transposed blocks of L
static void trsm_update_t(const double* A, int64_t lda, int M, int K, const double* Bsrc, double* C, int64_t ncols,
                          hipStream_t st) {
  const int64_t slab = (int64_t)GN * 65536;
  for (int64_t c0 = 0; c0 < ncols; c0 += slab) {
    GemmF64 g{};
    g.M = M; g.N = (int)std::min<int64_t>(slab, ncols - c0); g.K = K;
    g.A = A; g.lda = lda; g.ta = true;
    g.B = Bsrc + c0; g.ldb = ncols;
    g.C = C + c0; g.ldc = ncols;
    g.alpha = -1.0; g.beta = 1.0; g.batch = 1;
    hipLaunchKernelGGL((dgemm_kernel<true, false, EPI_SUB>), dim3(gemm_tiles(g.M, g.N)), dim3(GT), 0, st, g);
  }
}

void trsm_solve_t(const double* L, int n, double* X, int64_t ncols, hipStream_t st) {
  if (ncols <= 0 || n <= 0) return;
  constexpr int TB = 2 * TS_R;
  const int nb = (n + TB - 1) / TB;
  for (int bi = nb - 1; bi >= 0; --bi) {
    const int r0 = bi * TB, rb = std::min(TB, n - r0), r1 = r0 + rb;
    // rows r0.. of the block: R -= (L_k,block)^T X_k over the solved rows k >= r1
    if (r1 < n) trsm_update_t(L + (int64_t)r1 * n + r0, n, rb, n - r1, X + (int64_t)r1 * ncols,
                              X + (int64_t)r0 * ncols, ncols, st);
    const int h1 = std::min(TS_R, rb);
    if (rb > TS_R) {  // lower half of the block first, then the upper one
      const int rm = r0 + TS_R;
      trsv64t_cols(L + (int64_t)rm * n + rm, n, rb - TS_R, X + (int64_t)rm * ncols, ncols, ncols, st);
      trsm_update_t(L + (int64_t)rm * n + r0, n, TS_R, rb - TS_R, X + (int64_t)rm * ncols, X + (int64_t)r0 * ncols,
                    ncols, st);
    }
    trsv64t_cols(L + (int64_t)r0 * n + r0, n, h1, X + (int64_t)r0 * ncols, ncols, ncols, st);
  }
}

static double trsm_update(const double* A, int64_t lda, int M, int K, const double* Bsrc, double* C, int64_t ncols,
                          hipStream_t st) {
  const int64_t slab = (int64_t)GN * 65536;
  for (int64_t c0 = 0; c0 < ncols; c0 += slab) {
    GemmF64 g{};
    g.M = M; g.N = (int)std::min<int64_t>(slab, ncols - c0); g.K = K;
    g.A = A; g.lda = lda;
    g.B = Bsrc + c0; g.ldb = ncols;
    g.C = C + c0; g.ldc = ncols;
    g.alpha = -1.0; g.beta = 1.0; g.batch = 1;
    hipLaunchKernelGGL((dgemm_kernel<false, false, EPI_SUB>), dim3(gemm_tiles(g.M, g.N)), dim3(GT), 0, st, g);
  }
  return 2.0 * M * (double)K * (double)ncols;
}

size_t trsm_work_elems(int n) { return (size_t)(n / TS_R) * TS_R * TS_R; }

TrsmStats trsm_solve(const double* L, int n, double* raw, int64_t ncols, double* work, hipStream_t st,
                     TrsmTimer* timer) {
  TrsmStats z{};
  if (ncols <= 0) return z;
  constexpr int TB = 2 * TS_R;
  // packed copies of the full diagonal blocks for the scalar-load substitution
  const int nfull = n / TS_R;
  if (nfull > 0) hipLaunchKernelGGL(pack_diag_kernel, dim3((unsigned)nfull), dim3(256), 0, st, L, n, work);
  auto packed = [&](int r) { return r + TS_R <= nfull * TS_R ? work + (int64_t)(r / TS_R) * TS_R * TS_R : nullptr; };
  for (int r0 = 0; r0 < n; r0 += TB) {
    const int rb = std::min(TB, n - r0);
    if (r0 > 0) {
      if (timer) timer->begin();
      z.update_flops += trsm_update(L + (int64_t)r0 * n, n, rb, r0, raw, raw + (int64_t)r0 * ncols, ncols, st);
      if (timer) timer->end();
      ++z.update_launches;
    }
    const int h1 = std::min(TS_R, rb);
    trsv64_cols(L + (int64_t)r0 * n + r0, n, h1, raw + (int64_t)r0 * ncols, ncols, ncols, st, packed(r0));
    if (rb > TS_R) {
      const int r1 = r0 + TS_R;
      if (timer) timer->begin();
      z.update_flops += trsm_update(L + (int64_t)r1 * n + r0, n, rb - TS_R, TS_R, raw + (int64_t)r0 * ncols,
                                    raw + (int64_t)r1 * ncols, ncols, st);
      if (timer) timer->end();
      ++z.update_launches;
      trsv64_cols(L + (int64_t)r1 * n + r1, n, rb - TS_R, raw + (int64_t)r1 * ncols, ncols, ncols, st, packed(r1));
    }
  }
  return z;
}

void tile_split(const double* B, int n, int64_t ncols, const int64_t* src, float* hi, float* lo, int64_t ld_out,
                hipStream_t st) {
  if (n <= 0 || ld_out <= 0) return;
  if (ld_out % 1024) throw Error(-1, "tile_split: the tiled row length must be whole 32 x 32 tiles");
  for (int q0 = 0; q0 < n; q0 += 65535 * SPLIT_Q) {
    const int nq = std::min(65535 * SPLIT_Q, n - q0);
    const dim3 g((unsigned)(ld_out / 1024), (unsigned)((nq + SPLIT_Q - 1) / SPLIT_Q));
    hipLaunchKernelGGL(tile_split_kernel, g, dim3(256), 0, st, B + (int64_t)q0 * ncols, ncols, nq, src,
                       hi + (int64_t)q0 * ld_out, lo + (int64_t)q0 * ld_out, ld_out);
  }
}

// ---------------------------------------------------------------------------
// Cholesky of one diagonal block (nb <= 64) in LDS, plus its lower-triangular
// inverse.  A non-positive pivot records its global index + 1 in *info.
constexpr int CB = 64;
__global__ void __launch_bounds__(64) potrf_diag_kernel(double* J, int n, int k0, int kb,
                                                        double* Linv, int64_t ldx, int* info,
                                                        const double* __restrict__ diag0) {
  __shared__ double a[CB][CB + 1];
  __shared__ double x[CB][CB + 1];
  const int t = threadIdx.x;
  for (int i = 0; i < kb; ++i)
    if (t < kb) a[i][t] = (t <= i) ? J[(int64_t)(k0 + i) * n + k0 + t] : 0.0;
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (t == 0) {
      // a pivot that lost all but rounding noise of the original diagonal
      // counts as non-positive: the metric is not numerically positive definite
      const double d = a[j][j];
      if (!(d > 1e-14 * diag0[k0 + j])) {
        if (*info == 0) *info = k0 + j + 1;
        a[j][j] = __builtin_nan("");
      } else {
        a[j][j] = sqrt(d);
      }
    }
    __syncthreads();
    if (t > j && t < kb) a[t][j] /= a[j][j];
    __syncthreads();
    if (t > j && t < kb)
      for (int c = j + 1; c <= t; ++c) a[t][c] -= a[t][j] * a[c][j];
    __syncthreads();
  }
  // inverse, one column per thread: X[c][c] = 1/L[c][c],
  // X[i][c] = -(sum_{k=c}^{i-1} L[i][k] X[k][c]) / L[i][i]
  if (t < kb) {
    const int c = t;
    for (int i = 0; i < kb; ++i) x[i][c] = 0.0;
    x[c][c] = 1.0 / a[c][c];
    for (int i = c + 1; i < kb; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += a[i][k] * x[k][c];
      x[i][c] = -s / a[i][i];
    }
  }
  __syncthreads();
  for (int i = 0; i < kb; ++i)
    if (t < kb) {
      J[(int64_t)(k0 + i) * n + k0 + t] = (t <= i) ? a[i][t] : 0.0;
      Linv[(int64_t)i * ldx + t] = x[i][t];
    }
}

__global__ void copy2d_kernel(const double* src, int64_t lds, double* dst, int64_t ldd, int rows,
                              int cols) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)rows * cols) return;
  const int r = (int)(idx / cols), c = (int)(idx % cols);
  dst[r * ldd + c] = src[r * lds + c];
}
static void copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int rows, int cols,
                   hipStream_t st) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return;
  hipLaunchKernelGGL(copy2d_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, lds, dst,
                     ldd, rows, cols);
}

__global__ void fill_kernel(double* p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
void fill_f64(double* p, size_t n, double v, hipStream_t st) {
  if (!n) return;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

__global__ void sym_lower_kernel(double* A, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int r = (int)(idx / n), c = (int)(idx % n);
  if (c > r) A[idx] = A[(int64_t)c * n + r];
}
void sym_from_lower(double* A, int n, hipStream_t st) {
  const int64_t t = (int64_t)n * n;
  hipLaunchKernelGGL(sym_lower_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, A, n);
}

__global__ void zero_upper_kernel(double* A, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  if ((int)(idx % n) > (int)(idx / n)) A[idx] = 0.0;
}

__global__ void diag_kernel(const double* A, int n, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[(int64_t)i * n + i];
}

// J (n x n, lower part used) -> L in place (upper zeroed), Linv = L^-1.
// work: at least n * (CB + 1) doubles.
// work: the panel (n x CB), the original diagonal (n), and the split-K partial
// products of the inverse's block rows (8 x CB x n)
size_t cholesky_work_elems(int n) { return (size_t)n * (CB + 1) + std::max((size_t)8 * CB * n, (size_t)CB * CB); }

// J = L L^T in place; with Linv, the inverses of the diagonal blocks go there
// (the rest of Linv is then formed by cholesky_inverse), else to work.
static void cholesky_factor_impl(double* J, int n, double* Linv, double* work, int* info, hipStream_t st) {
  DFX_HIP(hipMemsetAsync(info, 0, sizeof(int), st));
  double* diag0 = work + (size_t)n * CB;
  double* xblk = work + (size_t)n * (CB + 1);  // CB x CB when there is no Linv
  hipLaunchKernelGGL(diag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, J, n, diag0);
  for (int k0 = 0; k0 < n; k0 += CB) {
    const int kb = std::min(CB, n - k0);
    double* X = Linv ? Linv + (int64_t)k0 * n + k0 : xblk;
    const int64_t ldx = Linv ? n : CB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(64), 0, st, J, n, k0, kb, X, ldx, info, diag0);
    const int r0 = k0 + kb, rows = n - r0;
    if (rows <= 0) break;
    // panel: L21 = A21 inv(L11)^T
    GemmF64 g{};
    g.M = rows; g.N = kb; g.K = kb;
    g.A = J + (int64_t)r0 * n + k0; g.lda = n;
    g.B = X; g.ldb = ldx; g.tb = true;
    g.C = work; g.ldc = kb;
    g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
    dgemm(g, st);
    copy2d(work, kb, J + (int64_t)r0 * n + k0, n, rows, kb, st);
    // trailing update of the lower triangle: A22 -= L21 L21^T
    GemmF64 u{};
    u.M = rows; u.N = rows; u.K = kb;
    u.A = work; u.lda = kb;
    u.B = work; u.ldb = kb; u.tb = true;
    u.C = J + (int64_t)r0 * n + r0; u.ldc = n;
    u.alpha = -1.0; u.beta = 1.0; u.batch = 1; u.lowerC = true;
    dgemm(u, st);
  }
  {
    const int64_t t = (int64_t)n * n;
    hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, J, n);
  }
}

void cholesky_factor(double* J, int n, double* work, int* info, hipStream_t st) {
  cholesky_factor_impl(J, n, nullptr, work, info, st);
}

void cholesky_inverse(double* J, int n, double* Linv, double* work, int* info, hipStream_t st) {
  fill_f64(Linv, (size_t)n * n, 0.0, st);
  cholesky_factor_impl(J, n, Linv, work, info, st);
  // off-diagonal blocks of L^-1, block row by block row (row-wise substitution,
  // which keeps the inverse accurate for an ill-conditioned metric; a recursive
  // X21 = -X22 L21 X11 lost two to three digits on kappa = 8.6e9):
  // X_i,0:i = -inv(L_ii) (L_i,0:i X_0:i,0:i).  The first product is thin (64
  // rows) but long: its k-range is split over up to 8 partial products.
  double* part = work + (size_t)n * (CB + 1);
  const int64_t part_elems = (int64_t)8 * CB * n;
  for (int i0 = CB; i0 < n; i0 += CB) {
    const int ib = std::min(CB, n - i0);
    GemmF64 g{};
    g.M = ib; g.N = i0; g.K = i0;
    g.A = J + (int64_t)i0 * n; g.lda = n;
    g.B = Linv; g.ldb = n;
    g.C = work; g.ldc = i0;
    g.alpha = 1.0; g.beta = 0.0; g.batch = 1;
    dgemm_sk(g, part, part_elems, st);
    GemmF64 h{};
    h.M = ib; h.N = i0; h.K = ib;
    h.A = Linv + (int64_t)i0 * n + i0; h.lda = n;
    h.B = work; h.ldb = i0;
    h.C = Linv + (int64_t)i0 * n; h.ldc = n;
    h.alpha = -1.0; h.beta = 0.0; h.batch = 1;
    dgemm(h, st);
  }
}

}  // namespace dfx
