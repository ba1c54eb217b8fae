// Exchange build K = sum_Q (B_Q C)(B_Q C)^T (Eqs. 1a, 2a) in FP64 on gfx950
// v_mfma_f64_16x16x4f64, with B_Q = hi + lo (two FP32 words per element).
// Phase 1 (half transform) streams each packed 32x32 tile of B_Q once per
// block of 64 or 128 rows as vector loads, transposing tiles of the upper
// triangle in LDS, and multiplies it by all occupied columns of C at once.
// Phase 2 is a split-K SYRK over the (Q, i) index into FP64 partial sums with
// an XCD-aware tile map, reduced in a fixed order.  Both phases issue the
// global loads of the next k-stage before the MFMAs of the current one.
#include <algorithm>

#include <string>
#include <type_traits>

#include "kernels.h"

namespace dfx {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int S64 = 16;   // k-width of one LDS stage (half a tile column of B_Q)
constexpr int PA = 1;     // row padding (doubles) of [row][k] tiles: odd row strides keep the
                          // fragment reads of 16 consecutive rows on distinct banks
constexpr int PB = 16;    // row padding (doubles) of the [k][i] C stage

// C_occ zero-padded to Cp[nbfp][np] (np = 64 NCB, nbfp = 32 ntiles), so that a
// k-stage of C is one contiguous, aligned block
__global__ void cpad_kernel(const double* __restrict__ C, int nbf, int nocc, int nbfp, int np,
                            double* __restrict__ Cp) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nbfp * np) return;
  const int nu = (int)(idx / np), i = (int)(idx % np);
  Cp[idx] = (nu < nbf && i < nocc) ? C[(int64_t)nu * nocc + i] : 0.0;
}

// ---- phase 1: X_Q[mu][i] = sum_nu B_Q[mu][nu] C[nu][i] for a block of MR = 64 RB
// rows of mu and all occupied columns (padded to NP = 64 NCB).  Eight waves in
// a 2 x 4 grid: wave w owns rows [(w & 1) MR / 2, +MR / 2) and columns
// [(w >> 1) NCB 16, +NCB 16), i.e. 2 RB x NCB accumulator blocks.
constexpr int KX_T = 512;
// Rows per block in units of 64.  128 rows halve the L2 reads of C per flop,
// which pays from 256 occupied columns on (measured); beyond 320 columns the
// 128-row accumulators no longer fit in 256 registers.
constexpr int kx_rb(int ncb) { return (ncb >= 4 && ncb <= 5) ? 2 : 1; }
template <int NCB, int RB>
__global__ void __launch_bounds__(KX_T) kx64_kernel(const float* __restrict__ hi, const float* __restrict__ lo,
                                                    int64_t ncols, int nbf, int q0, const double* __restrict__ Cp,
                                                    int nocc, double* __restrict__ X, int64_t ldx) {
  constexpr int NP = 64 * NCB;
  constexpr int MR = 64 * RB;
  constexpr int WA = 2 * RB;                  // 16-row fragments per wave
  constexpr int EP = 2 * RB;                  // consecutive A elements per thread per stage
  constexpr int TPR = KX_T / (MR / 32);       // threads per 32-row tile row
  constexpr int NCL = S64 * NP / (2 * KX_T);  // 16-byte pairs of C per thread per stage
  static_assert(NCL * 2 * KX_T == S64 * NP, "C stage must split evenly");
  static_assert(TPR * EP == 32 * S64, "A stage must split evenly");
  typedef float vfa __attribute__((ext_vector_type(EP)));
  __shared__ double As[2][MR][S64 + PA];
  __shared__ double Bs[2][S64][NP + PB];
  const int Q = q0 + blockIdx.y;
  const int m0 = blockIdx.x * MR;
  const int I0 = m0 >> 5;
  const int nt = ntiles_for(nbf);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w & 1) * (MR / 2), wc = (w >> 1) * NCB * 16;
  const float* __restrict__ rh = hi + (int64_t)Q * ncols;
  const float* __restrict__ rl = lo + (int64_t)Q * ncols;
  // A loader: thread group `half` serves tile row I0 + half, EP consecutive
  // elements per thread (along nu in a direct tile, along mu in a mirrored one)
  const int half = tid / TPR, t = tid % TPR;
  const int I = I0 + half;
  constexpr int DK = S64 / EP;  // threads per row of a direct stage
  constexpr int TM = 32 / EP;   // threads per row of a mirrored stage

  vfa ah, al;
  double2 cr[NCL];
  auto load = [&](int stage) {
    const int J = stage >> 1, h = stage & 1;
    ah = al = vfa(0.f);
    if (I < nt) {
      int64_t off;
      if (I >= J)  // direct tile (I, J): row mu = t / DK, nu = 16 h + EP (t % DK) ..
        off = tile_base(I, J) + (t / DK) * 32 + 16 * h + (t % DK) * EP;
      else         // tile (J, I): row nu = 16 h + t / TM, mu = EP (t % TM) ..
        off = tile_base(J, I) + (16 * h + t / TM) * 32 + (t % TM) * EP;
      ah = *reinterpret_cast<const vfa*>(rh + off);
      al = *reinterpret_cast<const vfa*>(rl + off);
    }
    const double2* __restrict__ cs = reinterpret_cast<const double2*>(Cp + (int64_t)stage * S64 * NP);
#pragma unroll
    for (int c = 0; c < NCL; ++c) cr[c] = cs[tid + KX_T * c];
  };
  // stage s goes to LDS buffer s & 1: one barrier per stage, since stage s's
  // buffer was last read in stage s - 2, which every wave finished before the
  // barrier of stage s - 1
  auto store = [&](int stage) {
    const int J = stage >> 1, b = stage & 1;
    if (I >= J) {
      const int r = half * 32 + t / DK, k0 = (t % DK) * EP;
#pragma unroll
      for (int e = 0; e < EP; ++e) As[b][r][k0 + e] = (double)ah[e] + (double)al[e];
    } else {
      const int k = t / TM, r0 = half * 32 + (t % TM) * EP;
#pragma unroll
      for (int e = 0; e < EP; ++e) As[b][r0 + e][k] = (double)ah[e] + (double)al[e];
    }
#pragma unroll
    for (int c = 0; c < NCL; ++c) {
      const int e = 2 * (tid + KX_T * c);  // NP is even: a pair never straddles rows
      Bs[b][e / NP][e % NP] = cr[c].x;
      Bs[b][e / NP][e % NP + 1] = cr[c].y;
    }
  };

  v4d acc[WA][NCB];
#pragma unroll
  for (int a = 0; a < WA; ++a)
#pragma unroll
    for (int b = 0; b < NCB; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

  auto mma = [&](auto bufc) {
    constexpr int BUF = decltype(bufc)::value;
#pragma unroll
    for (int kk = 0; kk < S64; kk += 4) {
      double fa[WA];
#pragma unroll
      for (int a = 0; a < WA; ++a) fa[a] = As[BUF][wr + a * 16 + li][kk + lk];
#pragma unroll
      for (int b = 0; b < NCB; ++b) {
        const double fb = Bs[BUF][kk + lk][wc + b * 16 + li];
#pragma unroll
        for (int a = 0; a < WA; ++a) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb, acc[a][b], 0, 0, 0);
      }
    }
  };
  const int nstage = 2 * nt;  // even: the stages pair up over the two buffers
  load(0);
  for (int s = 0; s < nstage; s += 2) {
    store(s);
    __syncthreads();
    load(s + 1);  // in flight during the MFMAs below
    mma(std::integral_constant<int, 0>{});
    store(s + 1);
    __syncthreads();
    if (s + 2 < nstage) load(s + 2);
    mma(std::integral_constant<int, 1>{});
  }
  // f64 MFMA output: element r of lane (li, lk) is row 4 r + lk, column li
#pragma unroll
  for (int a = 0; a < WA; ++a)
#pragma unroll
    for (int b = 0; b < NCB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = m0 + wr + a * 16 + 4 * r + lk;
        const int i = wc + b * 16 + li;
        if (mu < nbf && i < nocc) X[(int64_t)mu * ldx + (int64_t)blockIdx.y * nocc + i] = acc[a][b][r];
      }
}

// ---- phase 2: P_s = X_s X_s^T (lower 128x128 tiles) for k-slices s of X.
// Workgroups are dealt round-robin to the 8 XCDs; every tile of a slice goes to
// one XCD so that the slice of X is fetched from HBM once per XCD L2.  Eight
// waves in a 2 x 4 grid of 64 x 32 sub-tiles; on a diagonal tile the two waves
// whose sub-tiles lie wholly above the diagonal load and synchronise but skip
// their MFMAs.  Two LDS buffers alternate, so each stage needs one barrier:
// stage t's buffer was last read in stage t - 2, which every wave finished
// before the barrier of stage t - 1.
constexpr int SY_T = 512;
__global__ void __launch_bounds__(SY_T) syrk64_kernel(const double* __restrict__ X, int64_t ldx, int nbf,
                                                      int64_t kslice, int64_t kdim, int nslices, int ntl,
                                                      double* __restrict__ P) {
  __shared__ double As[2][128][S64 + PA];
  __shared__ double Bs[2][128][S64 + PA];
  const int bid = blockIdx.x;
  const int xcd = bid & 7, local = bid >> 3;
  const int s = xcd + 8 * (local / ntl);
  const int tl = local % ntl;
  if (s >= nslices) return;
  int ti = (int)((sqrt(8.0 * tl + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= tl) ++ti;
  while (ti * (ti + 1) / 2 > tl) --ti;
  const int tj = tl - ti * (ti + 1) / 2;
  const int m0 = ti * 128, n0 = tj * 128;
  const int64_t k0s = (int64_t)s * kslice;
  const int64_t k1s = k0s + kslice < kdim ? k0s + kslice : kdim;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 64, wn = (w >> 1) * 32;
  const bool active = !(ti == tj && wn >= wm + 64);
  const int li = lane & 15, lk = lane >> 4;
  // loader: row r = tid / 4 of both operands, 4 consecutive k from kq
  const int r = tid >> 2, kq = (tid & 3) * 4;
  const int ma = m0 + r, nb = n0 + r;

  double va[4], vb[4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) va[e] = vb[e] = 0.0;
    if (k0 + S64 <= k1s) {
      if (ma < nbf) {
        const double2* p = reinterpret_cast<const double2*>(X + (int64_t)ma * ldx + k0 + kq);
        const double2 v0 = p[0], v1 = p[1];
        va[0] = v0.x, va[1] = v0.y, va[2] = v1.x, va[3] = v1.y;
      }
      if (nb < nbf) {
        const double2* p = reinterpret_cast<const double2*>(X + (int64_t)nb * ldx + k0 + kq);
        const double2 v0 = p[0], v1 = p[1];
        vb[0] = v0.x, vb[1] = v0.y, vb[2] = v1.x, vb[3] = v1.y;
      }
    } else {  // ragged end of the slice
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t k = k0 + kq + e;
        if (k < k1s) {
          if (ma < nbf) va[e] = X[(int64_t)ma * ldx + k];
          if (nb < nbf) vb[e] = X[(int64_t)nb * ldx + k];
        }
      }
    }
  };

  v4d acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

  auto stage = [&](auto bufc) {
    constexpr int BUF = decltype(bufc)::value;
#pragma unroll
    for (int kk = 0; kk < S64; kk += 4) {
      double fa[4], fb[2];
#pragma unroll
      for (int a = 0; a < 4; ++a) fa[a] = As[BUF][wm + a * 16 + li][kk + lk];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = Bs[BUF][wn + b * 16 + li][kk + lk];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      As[buf][r][kq + e] = va[e];
      Bs[buf][r][kq + e] = vb[e];
    }
  };

  if (k0s < k1s) load(k0s);
  for (int64_t k0 = k0s; k0 < k1s; k0 += 2 * S64) {
    put(0);
    __syncthreads();
    if (k0 + S64 < k1s) load(k0 + S64);
    if (active) stage(std::integral_constant<int, 0>{});
    if (k0 + S64 < k1s) {
      put(1);
      __syncthreads();
      if (k0 + 2 * S64 < k1s) load(k0 + 2 * S64);
      if (active) stage(std::integral_constant<int, 1>{});
    }
  }
  if (!active) return;
  double* __restrict__ Ps = P + (int64_t)s * nbf * nbf;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + a * 16 + 4 * q + lk;
        const int n = n0 + wn + b * 16 + li;
        if (m < nbf && n <= m) Ps[(int64_t)m * nbf + n] = acc[a][b][q];
      }
}

// K (lower) = sum_s P_s, fixed order
__global__ void k_reduce64_kernel(const double* __restrict__ P, int ns, int nbf, double* __restrict__ K,
                                  int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n2 = (int64_t)nbf * nbf;
  if (idx >= n2) return;
  const int r = (int)(idx / nbf), c = (int)(idx % nbf);
  if (c > r) return;
  double s = accumulate ? K[idx] : 0.0;
  for (int k = 0; k < ns; ++k) s += P[k * n2 + idx];
  K[idx] = s;
}

struct F64Plan {
  int qc, ns, ntl, np, nbfp;
  int64_t ldx;
  size_t x_bytes, p_bytes, c_bytes;
};

static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

// X chunks of at most 8 GiB, balanced over the chunks; enough SYRK slices (a
// multiple of 8) to give the chip ~2048 workgroups, partial sums within 2 GiB.
// Under a work cap: eight slices and X in what the cap leaves.
static F64Plan f64_plan(const JKArgs& a, int nocc) {
  F64Plan p{};
  const size_t per_q = (size_t)a.nbf * nocc * sizeof(double);
  p.np = 64 * ((nocc + 63) / 64);
  p.nbfp = ntiles_for(a.nbf) * TILE;
  p.c_bytes = (size_t)p.nbfp * p.np * sizeof(double);
  size_t xbytes = (size_t)8 << 30;
  int64_t by_mem = ((int64_t)2 << 30) / ((int64_t)a.nbf * a.nbf * 8);
  if (a.ws_cap) {
    // eight slices, C, the row padding of X (7 doubles per row) and alignment
    const size_t fixed = a256((size_t)8 * a.nbf * a.nbf * 8) + p.c_bytes + (size_t)a.nbf * 56 + 1024;
    if (a.ws_cap < fixed + per_q)
      throw Error(DFX_ENOMEM, "K work: " + std::to_string(a.ws_cap) + " bytes hold no chunk (" +
                                  std::to_string(fixed + per_q) + " needed)");
    xbytes = a.ws_cap - fixed;
    by_mem = 8;
  }
  size_t cap = xbytes / per_q;
  if (cap < 1) cap = 1;
  const int nchunks = (int)((a.naux + cap - 1) / cap);
  p.qc = (a.naux + nchunks - 1) / nchunks;
  const int64_t kdim = (int64_t)p.qc * nocc;
  p.ldx = (kdim + 7) / 8 * 8;
  const int mt = (a.nbf + 127) / 128;
  p.ntl = mt * (mt + 1) / 2;
  int64_t ns = (2048 + p.ntl - 1) / p.ntl;
  const int64_t by_len = (kdim + S64 - 1) / S64;  // at least one stage per slice
  ns = std::min(ns, std::max<int64_t>(1, std::min(by_mem, by_len)));
  p.ns = (int)(((ns + 7) / 8) * 8);
  p.x_bytes = (size_t)a.nbf * p.ldx * sizeof(double);
  p.p_bytes = (size_t)p.ns * a.nbf * a.nbf * sizeof(double);
  return p;
}

size_t half_transform_f64_work(const JKArgs& a, int nocc) {
  const F64Plan p = f64_plan(a, nocc);
  return p.c_bytes;
}

void half_transform_f64(const JKArgs& a, const double* C, int nocc, int q0, int nq, double* X, int64_t ldx,
                        void* work, hipStream_t st) {
  const F64Plan p = f64_plan(a, nocc);
  const int ncb = (nocc + 63) / 64;
  if (ncb > 8) throw Error(-6, "half transform: more than 512 columns");
  if (q0 < 0 || nq <= 0 || q0 + nq > a.naux || ldx < (int64_t)nq * nocc) throw Error(-1, "half transform: bad range");
  double* Cp = reinterpret_cast<double*>(work);
  const int64_t ncp = (int64_t)p.nbfp * p.np;
  hipLaunchKernelGGL(cpad_kernel, dim3((unsigned)((ncp + 255) / 256)), dim3(256), 0, st, C, a.nbf, nocc, p.nbfp,
                     p.np, Cp);
  const int mr = 64 * kx_rb(ncb);
  const dim3 g1((a.nbf + mr - 1) / mr, nq);
  switch (ncb) {
#define KX64(N)                                                                                                   \
  case N:                                                                                                         \
    hipLaunchKernelGGL((kx64_kernel<N, kx_rb(N)>), g1, dim3(KX_T), 0, st, a.hi, a.lo, a.ncols, a.nbf, q0, Cp, nocc, \
                       X, ldx);                                                                                   \
    break;
    KX64(1) KX64(2) KX64(3) KX64(4) KX64(5) KX64(6) KX64(7) KX64(8)
#undef KX64
  }
}

size_t k_work_bytes_f64(const JKArgs& a, int nocc) {
  const F64Plan p = f64_plan(a, nocc);
  return a256(p.x_bytes) + a256(p.p_bytes) + p.c_bytes + 256;
}

void k_build_f64(const JKArgs& a, const double* C, int nocc, double* K, void* work, hipStream_t st,
                 KTimer* timer) {
  const F64Plan p = f64_plan(a, nocc);
  const int ncb = (nocc + 63) / 64;
  if (ncb > 8) throw Error(-6, "k_build: more than 512 occupied orbitals");
  char* w = reinterpret_cast<char*>(work);
  double* X = reinterpret_cast<double*>(w);
  double* P = reinterpret_cast<double*>(w + a256(p.x_bytes));
  double* Cp = reinterpret_cast<double*>(w + a256(p.x_bytes) + a256(p.p_bytes));
  const int64_t n2 = (int64_t)a.nbf * a.nbf;
  const int64_t ncp = (int64_t)p.nbfp * p.np;
  hipLaunchKernelGGL(cpad_kernel, dim3((unsigned)((ncp + 255) / 256)), dim3(256), 0, st, C, a.nbf, nocc, p.nbfp,
                     p.np, Cp);
  for (int q0 = 0; q0 < a.naux; q0 += p.qc) {
    const int nq = std::min(p.qc, a.naux - q0);
    const int64_t kdim = (int64_t)nq * nocc;
    const int mr = 64 * kx_rb(ncb);
    const dim3 g1((a.nbf + mr - 1) / mr, nq);
    if (timer) timer->begin_x();
    switch (ncb) {
#define KX64(N)                                                                                                   \
  case N:                                                                                                         \
    hipLaunchKernelGGL((kx64_kernel<N, kx_rb(N)>), g1, dim3(KX_T), 0, st, a.hi, a.lo, a.ncols, a.nbf, q0, Cp, nocc, \
                       X, p.ldx);                                                                                 \
    break;
      KX64(1) KX64(2) KX64(3) KX64(4) KX64(5) KX64(6) KX64(7) KX64(8)
#undef KX64
    }
    if (timer) timer->end_x();
    if (timer) timer->begin_syrk();
    const int64_t kslice = ((kdim + p.ns - 1) / p.ns + S64 - 1) / S64 * S64;
    hipLaunchKernelGGL(syrk64_kernel, dim3((unsigned)(p.ns * p.ntl)), dim3(SY_T), 0, st, X, p.ldx, a.nbf, kslice,
                       kdim, p.ns, p.ntl, P);
    hipLaunchKernelGGL(k_reduce64_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, P, p.ns, a.nbf, K,
                       q0 > 0 ? 1 : 0);
    if (timer) timer->end_syrk();
  }
  sym_from_lower(K, a.nbf, st);
}

// C = A A^T (n x n, both triangles) for a row-major n x k matrix A with an even
// row stride lda, on the exchange build's SYRK: lower 128 x 128 tiles, eight
// k-slices (one per XCD), summed in FP64 in a fixed order, then mirrored.
// For a symmetric A this is A^2 at half the FLOPs of a general product.
// work: syrk_f64_work_elems(n) doubles.
size_t syrk_f64_work_elems(int n) { return (size_t)8 * n * n; }

void syrk_f64(const double* A, int64_t lda, int n, int64_t k, double* C, double* work, hipStream_t st) {
  if (n <= 0) return;
  if ((lda & 1) || lda < k || (reinterpret_cast<uintptr_t>(A) & 15))
    throw Error(-1, "syrk_f64: A needs an even row stride >= k and 16-byte alignment");
  const int mt = (n + 127) / 128;
  const int ntl = mt * (mt + 1) / 2;
  const int ns = 8;
  const int64_t kslice = ((k + ns - 1) / ns + S64 - 1) / S64 * S64;
  const int64_t n2 = (int64_t)n * n;
  hipLaunchKernelGGL(syrk64_kernel, dim3((unsigned)(ns * ntl)), dim3(SY_T), 0, st, A, lda, n, kslice, k, ns, ntl,
                     work);
  hipLaunchKernelGGL(k_reduce64_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, work, ns, n, C, 0);
  sym_from_lower(C, n, st);
}

}  // namespace dfx
