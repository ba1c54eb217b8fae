// Exchange build K = sum_Q (B_Q C)(B_Q C)^T (Eqs. 1a, 2a) in FP64 on gfx950
// v_mfma_f64_16x16x4f64, with B_Q = hi + lo (two FP32 words per element).
// Phase 1 (half transform) streams each packed 32x32 tile of B_Q once per
// 64-row block as 16-byte vector loads, transposing tiles of the upper
// triangle in LDS, and multiplies it by all occupied columns of C at once.
// Phase 2 is a split-K SYRK over the (Q, i) index into FP64 partial sums with
// an XCD-aware tile map, reduced in a fixed order.  Both phases issue the
// global loads of the next k-stage before the MFMAs of the current one.
#include <algorithm>

#include "kernels.h"

namespace dfx {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int S64 = 16;   // k-width of one LDS stage (half a tile column of B_Q)
constexpr int PA = 2;     // row padding (doubles) of [row][k] tiles: conflict-free A/B fragments
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

// ---- phase 1: X_Q[mu][i] = sum_nu B_Q[mu][nu] C[nu][i] for a 64-row block of mu
// and all occupied columns (padded to NP = 64 NCB).  Wave w owns columns
// [w NCB 16, (w + 1) NCB 16) of all four 16-row blocks.
template <int NCB>
__global__ void __launch_bounds__(256) kx64_kernel(const float* __restrict__ hi, const float* __restrict__ lo,
                                                   int64_t ncols, int nbf, int q0, const double* __restrict__ Cp,
                                                   int nocc, double* __restrict__ X, int64_t ldx) {
  constexpr int NP = 64 * NCB;
  constexpr int NCL = S64 * NP / 512;  // 16-byte pairs of C per thread per stage
  __shared__ double As[64][S64 + PA];
  __shared__ double Bs[S64][NP + PB];
  const int Q = q0 + blockIdx.y;
  const int m0 = blockIdx.x * 64;
  const int I0 = m0 >> 5;
  const int nt = ntiles_for(nbf);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const float* __restrict__ rh = hi + (int64_t)Q * ncols;
  const float* __restrict__ rl = lo + (int64_t)Q * ncols;
  // A loader: threads 0..127 serve tile row I0, 128..255 tile row I0 + 1
  const int half = tid >> 7, t = tid & 127;
  const int I = I0 + half;

  float4 ah, al;
  double2 cr[NCL];
  auto load = [&](int stage) {
    const int J = stage >> 1, h = stage & 1;
    ah = al = make_float4(0.f, 0.f, 0.f, 0.f);
    if (I < nt) {
      int64_t off;
      if (I >= J)  // direct tile (I, J): row mu = t / 4, nu = 16 h + 4 (t % 4) ..
        off = tile_base(I, J) + (t >> 2) * 32 + 16 * h + (t & 3) * 4;
      else         // tile (J, I): row nu = 16 h + t / 8, mu = 4 (t % 8) ..
        off = tile_base(J, I) + (16 * h + (t >> 3)) * 32 + (t & 7) * 4;
      ah = *reinterpret_cast<const float4*>(rh + off);
      al = *reinterpret_cast<const float4*>(rl + off);
    }
    const double2* __restrict__ cs = reinterpret_cast<const double2*>(Cp + (int64_t)stage * S64 * NP);
#pragma unroll
    for (int c = 0; c < NCL; ++c) cr[c] = cs[tid + 256 * c];
  };
  auto store = [&](int stage) {
    const int J = stage >> 1;
    const double v[4] = {(double)ah.x + (double)al.x, (double)ah.y + (double)al.y, (double)ah.z + (double)al.z,
                         (double)ah.w + (double)al.w};
    if (I >= J) {
      const int r = half * 32 + (t >> 2), k0 = (t & 3) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[r][k0 + e] = v[e];
    } else {
      const int k = t >> 3, r0 = half * 32 + (t & 7) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[r0 + e][k] = v[e];
    }
#pragma unroll
    for (int c = 0; c < NCL; ++c) {
      const int e = 2 * (tid + 256 * c);  // NP is even: a pair never straddles rows
      Bs[e / NP][e % NP] = cr[c].x;
      Bs[e / NP][e % NP + 1] = cr[c].y;
    }
  };

  v4d acc[4][NCB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NCB; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

  const int nstage = 2 * nt;
  load(0);
  for (int s = 0; s < nstage; ++s) {
    __syncthreads();  // every wave is done with the previous stage
    store(s);
    __syncthreads();
    if (s + 1 < nstage) load(s + 1);  // in flight during the MFMAs below
#pragma unroll
    for (int kk = 0; kk < S64; kk += 4) {
      double fa[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) fa[a] = As[a * 16 + li][kk + lk];
#pragma unroll
      for (int b = 0; b < NCB; ++b) {
        const double fb = Bs[kk + lk][w * NCB * 16 + b * 16 + li];
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb, acc[a][b], 0, 0, 0);
      }
    }
  }
  // f64 MFMA output: element r of lane (li, lk) is row 4 r + lk, column li
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NCB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = m0 + a * 16 + 4 * r + lk;
        const int i = w * NCB * 16 + b * 16 + li;
        if (mu < nbf && i < nocc) X[(int64_t)mu * ldx + (int64_t)blockIdx.y * nocc + i] = acc[a][b][r];
      }
}

// ---- phase 2: P_s = X_s X_s^T (lower 128x128 tiles) for k-slices s of X.
// Workgroups are dealt round-robin to the 8 XCDs; every tile of a slice goes to
// one XCD so that the slice of X is fetched from HBM once per XCD L2.
__global__ void __launch_bounds__(256) syrk64_kernel(const double* __restrict__ X, int64_t ldx, int nbf,
                                                     int64_t kslice, int64_t kdim, int nslices, int ntl,
                                                     double* __restrict__ P) {
  __shared__ double As[128][S64 + PA];
  __shared__ double Bs[128][S64 + PA];
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
  const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
  const int li = lane & 15, lk = lane >> 4;
  // loader: row r = tid / 2 of both operands, 8 consecutive k from kh
  const int r = tid >> 1, kh = (tid & 1) * 8;
  const int ma = m0 + r, nb = n0 + r;

  double va[8], vb[8];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) va[e] = vb[e] = 0.0;
    if (k0 + S64 <= k1s) {
      if (ma < nbf) {
        const double2* p = reinterpret_cast<const double2*>(X + (int64_t)ma * ldx + k0 + kh);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double2 v = p[e];
          va[2 * e] = v.x;
          va[2 * e + 1] = v.y;
        }
      }
      if (nb < nbf) {
        const double2* p = reinterpret_cast<const double2*>(X + (int64_t)nb * ldx + k0 + kh);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double2 v = p[e];
          vb[2 * e] = v.x;
          vb[2 * e + 1] = v.y;
        }
      }
    } else {  // ragged end of the slice
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + kh + e;
        if (k < k1s) {
          if (ma < nbf) va[e] = X[(int64_t)ma * ldx + k];
          if (nb < nbf) vb[e] = X[(int64_t)nb * ldx + k];
        }
      }
    }
  };

  v4d acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

  if (k0s < k1s) load(k0s);
  for (int64_t k0 = k0s; k0 < k1s; k0 += S64) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[r][kh + e] = va[e];
      Bs[r][kh + e] = vb[e];
    }
    __syncthreads();
    if (k0 + S64 < k1s) load(k0 + S64);
#pragma unroll
    for (int kk = 0; kk < S64; kk += 4) {
      double fa[4], fb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) fa[a] = As[wm + a * 16 + li][kk + lk];
#pragma unroll
      for (int b = 0; b < 4; ++b) fb[b] = Bs[wn + b * 16 + li][kk + lk];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
  }
  double* __restrict__ Ps = P + (int64_t)s * nbf * nbf;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
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

// X chunks of at most 8 GiB, balanced over the chunks; enough SYRK slices (a
// multiple of 8) to give the chip ~2048 workgroups, partial sums within 2 GiB
static F64Plan f64_plan(const JKArgs& a, int nocc) {
  F64Plan p{};
  const size_t per_q = (size_t)a.nbf * nocc * sizeof(double);
  size_t cap = ((size_t)8 << 30) / per_q;
  if (cap < 1) cap = 1;
  const int nchunks = (int)((a.naux + cap - 1) / cap);
  p.qc = (a.naux + nchunks - 1) / nchunks;
  const int64_t kdim = (int64_t)p.qc * nocc;
  p.ldx = (kdim + 7) / 8 * 8;
  const int mt = (a.nbf + 127) / 128;
  p.ntl = mt * (mt + 1) / 2;
  int64_t ns = (2048 + p.ntl - 1) / p.ntl;
  const int64_t by_mem = ((int64_t)2 << 30) / ((int64_t)a.nbf * a.nbf * 8);
  const int64_t by_len = (kdim + S64 - 1) / S64;  // at least one stage per slice
  ns = std::min(ns, std::max<int64_t>(1, std::min(by_mem, by_len)));
  p.ns = (int)(((ns + 7) / 8) * 8);
  p.x_bytes = (size_t)a.nbf * p.ldx * sizeof(double);
  p.p_bytes = (size_t)p.ns * a.nbf * a.nbf * sizeof(double);
  p.np = 64 * ((nocc + 63) / 64);
  p.nbfp = ntiles_for(a.nbf) * TILE;
  p.c_bytes = (size_t)p.nbfp * p.np * sizeof(double);
  return p;
}

static size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

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
    const dim3 g1((a.nbf + 63) / 64, nq);
    if (timer) timer->begin_x();
    switch (ncb) {
#define KX64(N)                                                                                            \
  case N:                                                                                                  \
    hipLaunchKernelGGL((kx64_kernel<N>), g1, dim3(256), 0, st, a.hi, a.lo, a.ncols, a.nbf, q0, Cp, nocc, X, \
                       p.ldx);                                                                             \
    break;
      KX64(1) KX64(2) KX64(3) KX64(4) KX64(5) KX64(6) KX64(7) KX64(8)
#undef KX64
    }
    if (timer) timer->end_x();
    if (timer) timer->begin_syrk();
    const int64_t kslice = ((kdim + p.ns - 1) / p.ns + S64 - 1) / S64 * S64;
    hipLaunchKernelGGL(syrk64_kernel, dim3((unsigned)(p.ns * p.ntl)), dim3(256), 0, st, X, p.ldx, a.nbf, kslice,
                       kdim, p.ns, p.ntl, P);
    hipLaunchKernelGGL(k_reduce64_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, P, p.ns, a.nbf, K,
                       q0 > 0 ? 1 : 0);
    if (timer) timer->end_syrk();
  }
  sym_from_lower(K, a.nbf, st);
}

}  // namespace dfx
