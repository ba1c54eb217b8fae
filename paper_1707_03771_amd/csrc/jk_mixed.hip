// Exchange build K = sum_Q (B_Q C)(B_Q C)^T (Eqs. 1a, 2a) in reduced precision
// on gfx950 MFMA, FP32 accumulation:
//   FP32: B hi word and C in FP32, v_mfma_f32_16x16x4_f32;
//   BF16: B hi word and C rounded to BF16 (nearest even), v_mfma_f32_16x16x32_bf16.
// Phase 1 (half transform) reads each packed 32x32 tile of B_Q from HBM and
// multiplies it by all occupied columns at once, so B is streamed once per use;
// X is written in the compute precision.  Phase 2 is a split-K SYRK over the
// (Q, i) index: FP32 MFMA sums of KT products, added up in FP64, reduced over
// the slices in FP64 in a fixed order.
#include <string>
#include <type_traits>

#include "kernels.h"

namespace dfx {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

// ---- precision traits --------------------------------------------------------
struct Bf16Tr {
  using E = __bf16;
  static constexpr int KM = 32;
  __device__ __forceinline__ static v4f mma(const E* a, const E* b, v4f c) {
    const v8bf av = *reinterpret_cast<const v8bf*>(a);
    const v8bf bv = *reinterpret_cast<const v8bf*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
  // lane's A/B fragment start within a [row][k] LDS tile: 8 consecutive k
  __device__ __forceinline__ static int koff(int lk) { return 8 * lk; }
};
struct F32Tr {
  using E = float;
  static constexpr int KM = 4;
  __device__ __forceinline__ static v4f mma(const E* a, const E* b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(*a, *b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int koff(int lk) { return lk; }
};

constexpr int KT = 32;       // k-width of one LDS stage (one tile column of B_Q)
// LDS row padding: 16 bytes, so that rows stay 16-byte aligned for vector stores
// while the FP32 fragment reads of 16 consecutive rows spread over the banks
template <class E> constexpr int lpad() { return 16 / (int)sizeof(E); }

template <class E> __device__ __forceinline__ E cvt(float x) { return (E)x; }

// 8 consecutive elements as raw 128-bit words (one word for BF16, two for FP32)
template <class E> struct W8 { static constexpr int N = sizeof(E) * 8 / 16; uint4 w[N]; };
template <class E>
__device__ __forceinline__ W8<E> ld8(const E* __restrict__ p) {
  W8<E> r;
#pragma unroll
  for (int i = 0; i < W8<E>::N; ++i) r.w[i] = reinterpret_cast<const uint4*>(p)[i];
  return r;
}
template <class E>
__device__ __forceinline__ void st8(E* p, const W8<E>& v) {
#pragma unroll
  for (int i = 0; i < W8<E>::N; ++i) reinterpret_cast<uint4*>(p)[i] = v.w[i];
}
// 8 floats -> 8 elements of E, packed
template <class E>
__device__ __forceinline__ W8<E> pack8(float4 a, float4 b) {
  W8<E> r;
  if constexpr (sizeof(E) == 2) {
    v8bf v = {(E)a.x, (E)a.y, (E)a.z, (E)a.w, (E)b.x, (E)b.y, (E)b.z, (E)b.w};
    r.w[0] = *reinterpret_cast<uint4*>(&v);
  } else {
    r.w[0] = *reinterpret_cast<uint4*>(&a);
    r.w[1] = *reinterpret_cast<uint4*>(&b);
  }
  return r;
}

// ---- C_occ^T in the compute precision, zero padded: Ct[i][nu], i < npad, nu < nbfp
template <class E>
__global__ void ct_kernel(const double* __restrict__ C, int nbf, int nocc, int npad, int nbfp, E* Ct) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)npad * nbfp) return;
  const int i = (int)(idx / nbfp), nu = (int)(idx % nbfp);
  Ct[idx] = cvt<E>((i < nocc && nu < nbf) ? (float)C[(int64_t)nu * nocc + i] : 0.0f);
}

// ---- phase 1: X_Q[mu][i] for a 64-row block of mu and all (padded) i columns.
// Wave w owns columns [w NCB 16, (w + 1) NCB 16); all four 16-row blocks.
template <class Tr, int NCB>
__global__ void __launch_bounds__(256) kx_mixed_kernel(const float* __restrict__ hi, int64_t ncols,
                                                       int nbf, int q0, const typename Tr::E* __restrict__ Ct,
                                                       int nbfp, int nocc, typename Tr::E* __restrict__ X,
                                                       int64_t ldx) {
  using E = typename Tr::E;
  constexpr int NP = 64 * NCB;  // padded occupied columns
  __shared__ __align__(16) E As[64][KT + lpad<E>()];
  __shared__ __align__(16) E Bs[NP][KT + lpad<E>()];
  const int Q = q0 + blockIdx.y;
  const int m0 = blockIdx.x * 64;
  const int I0 = m0 >> 5;
  const int nt = ntiles_for(nbf);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const float* __restrict__ row = hi + (int64_t)Q * ncols;
  v4f acc[4][NCB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NCB; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

  // tile J's operands are loaded into registers while the MFMAs of tile J - 1 run
  const int half = tid >> 7, t = tid & 127;
  const int I = I0 + half;
  constexpr int NCH = NP * KT / 8;  // 8-element chunks of Ct's stage
  constexpr int NCV = (NCH + 255) / 256;
  float4 va0, va1;
  W8<E> vb[NCV];
  bool direct = false;
  auto load = [&](int J) {
    // A: rows m0..m0+63 = row tiles I0 and I0 + 1, columns of tile J
    va0 = make_float4(0.f, 0.f, 0.f, 0.f);
    va1 = va0;
    direct = I >= J;
    if (I < nt) {
      const float4* src = reinterpret_cast<const float4*>(
          row + (direct ? tile_base(I, J) : tile_base(J, I)) + (t >> 2) * 32 + (t & 3) * 8);
      va0 = src[0];
      va1 = src[1];
    }
    // B: Ct[:, 32J .. 32J+31], 8 elements per chunk
#pragma unroll
    for (int c = 0; c < NCV; ++c) {
      const int ch = tid + c * 256;
      if (ch < NCH) vb[c] = ld8(Ct + (int64_t)(ch >> 2) * nbfp + J * KT + (ch & 3) * 8);
    }
  };

  if (nt > 0) load(0);
  for (int J = 0; J < nt; ++J) {
    __syncthreads();  // the MFMAs of tile J - 1 have read their operands
    if (direct) {  // tile row (t >> 2) is mu, elements are nu
      const int r = half * 32 + (t >> 2), k0 = (t & 3) * 8;
      st8(&As[r][k0], pack8<E>(va0, va1));
    } else {       // tile row (t >> 2) is nu, elements are mu
      const int k = t >> 2, r0 = half * 32 + (t & 3) * 8;
      As[r0 + 0][k] = cvt<E>(va0.x);
      As[r0 + 1][k] = cvt<E>(va0.y);
      As[r0 + 2][k] = cvt<E>(va0.z);
      As[r0 + 3][k] = cvt<E>(va0.w);
      As[r0 + 4][k] = cvt<E>(va1.x);
      As[r0 + 5][k] = cvt<E>(va1.y);
      As[r0 + 6][k] = cvt<E>(va1.z);
      As[r0 + 7][k] = cvt<E>(va1.w);
    }
#pragma unroll
    for (int c = 0; c < NCV; ++c) {
      const int ch = tid + c * 256;
      if (ch < NCH) st8(&Bs[ch >> 2][(ch & 3) * 8], vb[c]);
    }
    __syncthreads();
    if (J + 1 < nt) load(J + 1);
#pragma unroll
    for (int kk = 0; kk < KT; kk += Tr::KM) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const E* pa = &As[a * 16 + li][kk + Tr::koff(lk)];
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
          const E* pb = &Bs[w * NCB * 16 + b * 16 + li][kk + Tr::koff(lk)];
          acc[a][b] = Tr::mma(pa, pb, acc[a][b]);
        }
      }
    }
  }
  // store: element (4 lk + r, li) of each 16x16 block
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NCB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mu = m0 + a * 16 + lk * 4 + r;
        const int i = w * NCB * 16 + b * 16 + li;
        if (mu < nbf && i < nocc) X[(int64_t)mu * ldx + (int64_t)blockIdx.y * nocc + i] = cvt<E>(acc[a][b][r]);
      }
}

// ---- phase 2: P_s = X_s X_s^T (lower 128x128 tiles) for k-slices s of X.
// Workgroups are dealt round-robin to the 8 XCDs; the map sends every tile of a
// slice to one XCD so that the slice of X is fetched from HBM once per XCD L2.
// Eight waves in a 2 x 4 grid of 64 x 32 sub-tiles.  The MFMAs accumulate one
// k-stage (KT products) in FP32; each stage's sums are added into FP64
// registers, so no FP32 accumulator sums more than KT products.  A block's sums
// are added at the start of the next stage, just before its first MFMA (which
// starts from zero), so the additions overlap the other blocks' MFMAs.  Two LDS
// buffers alternate, one barrier per stage: stage t's buffer was last read in
// stage t - 2, which every wave finished before the barrier of stage t - 1.  On
// a diagonal tile the two waves whose sub-tiles lie above the diagonal skip
// their MFMAs.
constexpr int SYM_T = 512;
template <class Tr>
__global__ void __launch_bounds__(SYM_T) syrk_mixed_kernel(const typename Tr::E* __restrict__ X, int64_t ldx,
                                                           int nbf, int64_t kslice, int64_t kdim, int nslices,
                                                           int ntl, double* __restrict__ P) {
  using E = typename Tr::E;
  __shared__ __align__(16) E As[2][128][KT + lpad<E>()];
  __shared__ __align__(16) E Bs[2][128][KT + lpad<E>()];
  // blockIdx.x -> (slice, lower tile)
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
  // loader: row r of both operands, 8 consecutive k from k8
  const int r = tid >> 2, k8 = (tid & 3) * 8;
  const int ma = m0 + r, nb = n0 + r;

  W8<E> va, vb;
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < W8<E>::N; ++i) va.w[i] = vb.w[i] = make_uint4(0, 0, 0, 0);
    if (k0 + KT <= k1s) {
      if (ma < nbf) va = ld8(X + (int64_t)ma * ldx + k0 + k8);
      if (nb < nbf) vb = ld8(X + (int64_t)nb * ldx + k0 + k8);
    } else {  // ragged end of the slice: element by element
      E ea[8], eb[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + k8 + e;
        ea[e] = (ma < nbf && k < k1s) ? X[(int64_t)ma * ldx + k] : cvt<E>(0.0f);
        eb[e] = (nb < nbf && k < k1s) ? X[(int64_t)nb * ldx + k] : cvt<E>(0.0f);
      }
      __builtin_memcpy(&va, ea, sizeof ea);
      __builtin_memcpy(&vb, eb, sizeof eb);
    }
  };

  double sum[4][2][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) sum[a][b][q] = 0.0;

  // acc starts at zero, so adding it before the first stage changes nothing
  v4f acc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  auto stage = [&](auto bufc) {
    constexpr int BUF = decltype(bufc)::value;
#pragma unroll
    for (int kk = 0; kk < KT; kk += Tr::KM)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          v4f c = acc[a][b];
          if (kk == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[a][b][q] += (double)acc[a][b][q];
            c = v4f{0.f, 0.f, 0.f, 0.f};
          }
          acc[a][b] = Tr::mma(&As[BUF][wm + a * 16 + li][kk + Tr::koff(lk)],
                              &Bs[BUF][wn + b * 16 + li][kk + Tr::koff(lk)], c);
        }
  };
  auto put = [&](int buf) {
    st8(&As[buf][r][k8], va);
    st8(&Bs[buf][r][k8], vb);
  };

  if (k0s < k1s) load(k0s);
  for (int64_t k0 = k0s; k0 < k1s; k0 += 2 * KT) {
    put(0);
    __syncthreads();
    if (k0 + KT < k1s) load(k0 + KT);  // in flight during the MFMAs below
    if (active) stage(std::integral_constant<int, 0>{});
    if (k0 + KT < k1s) {
      put(1);
      __syncthreads();
      if (k0 + 2 * KT < k1s) load(k0 + 2 * KT);
      if (active) stage(std::integral_constant<int, 1>{});
    }
  }
  if (!active) return;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) sum[a][b][q] += (double)acc[a][b][q];
  double* __restrict__ Ps = P + (int64_t)s * nbf * nbf;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + a * 16 + lk * 4 + q;
        const int n = n0 + wn + b * 16 + li;
        if (m < nbf && n <= m) Ps[(int64_t)m * nbf + n] = sum[a][b][q];
      }
}

// K (lower) = sum_s P_s in FP64, fixed order; then mirrored by the caller
__global__ void k_reduce_mixed_kernel(const double* __restrict__ P, int ns, int nbf, double* __restrict__ K,
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

struct MixedPlan {
  int ncb, npad, nbfp, qc, ns, ntl;
  int64_t kslice, kdim;
  size_t ct_bytes, x_bytes, p_bytes;
};

static MixedPlan mixed_plan(const JKArgs& a, int nocc, size_t esize) {
  MixedPlan p{};
  p.ncb = (nocc + 63) / 64;
  p.npad = 64 * p.ncb;
  p.nbfp = ntiles_for(a.nbf) * TILE;
  const size_t per_q = (size_t)a.nbf * nocc * esize;
  size_t xbytes = (size_t)2 << 30;
  if (a.ws_cap) {
    // C, eight partial-sum slices, the row padding of X and alignment
    const size_t fixed = (size_t)p.npad * p.nbfp * esize + (size_t)8 * a.nbf * a.nbf * 8 + (size_t)a.nbf * 8 * esize +
                         1024 + 512;
    if (a.ws_cap < fixed + per_q)
      throw Error(DFX_ENOMEM, "K work: " + std::to_string(a.ws_cap) + " bytes hold no chunk (" +
                                  std::to_string(fixed + per_q) + " needed)");
    xbytes = a.ws_cap - fixed;
  }
  size_t cap = xbytes / per_q;
  if (cap < 1) cap = 1;
  p.qc = (int)std::min<size_t>(cap, (size_t)a.naux);
  p.kdim = (int64_t)p.qc * nocc;
  const int mt = (a.nbf + 127) / 128;
  p.ntl = mt * (mt + 1) / 2;
  // enough slices to fill the chip several times over, a multiple of 8 (the FP32
  // sums are already flushed to FP64 every KT products inside the kernel)
  int ns = (2048 + p.ntl - 1) / p.ntl;
  ns = ((ns + 7) / 8) * 8;
  const int64_t maxs = (p.kdim + KT - 1) / KT;
  if (ns > maxs) ns = (int)(((maxs + 7) / 8) * 8);
  if (ns < 8 || a.ws_cap) ns = 8;
  p.ns = ns;
  p.kslice = ((p.kdim + ns - 1) / ns + KT - 1) / KT * KT;
  p.ct_bytes = (size_t)p.npad * p.nbfp * esize;
  p.x_bytes = (size_t)a.nbf * ((p.kdim + 7) / 8 * 8) * esize;
  p.p_bytes = (size_t)ns * a.nbf * a.nbf * sizeof(double);
  return p;
}

size_t k_work_bytes_mixed(const JKArgs& a, int nocc) {
  const size_t es = a.prec == PREC_BF16 ? 2 : 4;
  const MixedPlan p = mixed_plan(a, nocc, es);
  return p.ct_bytes + p.x_bytes + p.p_bytes + 1024;
}

template <class Tr>
static void k_build_tr(const JKArgs& a, const double* C, int nocc, double* K, void* work, hipStream_t st,
                       KTimer* timer) {
  using E = typename Tr::E;
  const MixedPlan p = mixed_plan(a, nocc, sizeof(E));
  if (p.ncb > 8) throw Error(-6, "k_build: more than 512 occupied orbitals in reduced precision");
  char* w = reinterpret_cast<char*>(work);
  E* Ct = reinterpret_cast<E*>(w);
  E* X = reinterpret_cast<E*>(w + ((p.ct_bytes + 255) & ~(size_t)255));
  double* P = reinterpret_cast<double*>(w + ((p.ct_bytes + 255) & ~(size_t)255) + ((p.x_bytes + 255) & ~(size_t)255));
  const int64_t ctn = (int64_t)p.npad * p.nbfp;
  hipLaunchKernelGGL(ct_kernel<E>, dim3((unsigned)((ctn + 255) / 256)), dim3(256), 0, st, C, a.nbf, nocc, p.npad,
                     p.nbfp, Ct);
  const int64_t n2 = (int64_t)a.nbf * a.nbf;
  for (int q0 = 0; q0 < a.naux; q0 += p.qc) {
    const int nq = std::min(p.qc, a.naux - q0);
    const int64_t kdim = (int64_t)nq * nocc;
    const int64_t ldx = (kdim + 7) / 8 * 8;  // rows of X start 16-byte aligned
    const dim3 g1((a.nbf + 63) / 64, nq);
    if (timer) timer->begin_x();
    switch (p.ncb) {
#define KXC(N)                                                                                   \
  case N:                                                                                        \
    hipLaunchKernelGGL((kx_mixed_kernel<Tr, N>), g1, dim3(256), 0, st, a.hi, a.ncols, a.nbf, q0, Ct, \
                       p.nbfp, nocc, X, ldx);                                                    \
    break;
      KXC(1) KXC(2) KXC(3) KXC(4) KXC(5) KXC(6) KXC(7) KXC(8)
#undef KXC
    }
    if (timer) timer->end_x();
    if (timer) timer->begin_syrk();
    int ns = p.ns;
    int64_t kslice = ((kdim + ns - 1) / ns + KT - 1) / KT * KT;
    const int nblocks = ((ns + 7) / 8) * 8 * p.ntl;
    hipLaunchKernelGGL(syrk_mixed_kernel<Tr>, dim3(nblocks), dim3(SYM_T), 0, st, X, ldx, a.nbf, kslice, kdim, ns,
                       p.ntl, P);
    hipLaunchKernelGGL(k_reduce_mixed_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, P, ns, a.nbf,
                       K, q0 > 0 ? 1 : 0);
    if (timer) timer->end_syrk();
  }
  sym_from_lower(K, a.nbf, st);
}

void k_build_mixed(const JKArgs& a, const double* C, int nocc, double* K, void* work, hipStream_t st,
                   KTimer* timer) {
  if (a.prec == PREC_BF16)
    k_build_tr<Bf16Tr>(a, C, nocc, K, work, st, timer);
  else
    k_build_tr<F32Tr>(a, C, nocc, K, work, st, timer);
}

}  // namespace dfx
