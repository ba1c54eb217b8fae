// Coulomb and exchange builds from the fitted tensor B (section "Density
// fitting utilities"):
//   J: gamma_Q = sum_{mu nu} B_Q,mu nu D_mu nu       (Eq. 3a)
//      J_mu nu = sum_Q gamma_Q B_Q,mu nu             (Eq. 3b)
//   K: X_Q = B_Q C                                   (Eq. 1a, half transform)
//      K_mu nu = sum_Q sum_i X_Q,mu i X_Q,nu i       (Eq. 2a)
// B is stored as two FP32 words (hi, lo) per element in the packed 32x32 tile
// layout (common.h).  The FP64 path reads hi + lo; the mixed path reads hi.
#include "kernels.h"

namespace dfx {

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// tile index -> (I, J), I >= J
__device__ __forceinline__ void tile_ij(int t, int& I, int& J) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// weighted density in the tile layout: off-diagonal tiles count twice
__global__ void pack_density_kernel(const double* __restrict__ D, int nbf, double* __restrict__ d) {
  const int t = blockIdx.x;
  int I, J;
  tile_ij(t, I, J);
  const double w = (I == J) ? 1.0 : 2.0;
  for (int e = threadIdx.x; e < TILE2; e += blockDim.x) {
    const int r = I * TILE + (e >> 5), c = J * TILE + (e & 31);
    d[(int64_t)t * TILE2 + e] = (r < nbf && c < nbf) ? w * D[(int64_t)r * nbf + c] : 0.0;
  }
}

// gamma_Q = sum_c B[Q][c] d[c], B = hi + lo, FP64 accumulation.  A workgroup
// takes JG_Q consecutive Q, so each element of d is fetched once per JG_Q rows
// of B (d is as long as a row of B: read once per Q it doubled the kernel's
// traffic).  Every Q keeps the same per-thread column order and tree, so the
// result does not depend on JG_Q.
constexpr int JG_Q = 4;
__global__ void __launch_bounds__(256) j_gamma_kernel(const float* __restrict__ hi,
                                                      const float* __restrict__ lo, int64_t ncols, int naux,
                                                      const double* __restrict__ d, double* gam) {
  const int Q0 = blockIdx.x * JG_Q;
  const int nq = min(JG_Q, naux - Q0);
  const double4* d4 = reinterpret_cast<const double4*>(d);
  const int64_t n4 = ncols >> 2;
  double s[JG_Q];
#pragma unroll
  for (int k = 0; k < JG_Q; ++k) s[k] = 0.0;
  for (int64_t i = threadIdx.x; i < n4; i += blockDim.x) {
    const double4 dd = d4[i];
#pragma unroll
    for (int k = 0; k < JG_Q; ++k) {
      if (k < nq) {
        const float4 h = reinterpret_cast<const float4*>(hi + (int64_t)(Q0 + k) * ncols)[i];
        const float4 l = reinterpret_cast<const float4*>(lo + (int64_t)(Q0 + k) * ncols)[i];
        s[k] += ((double)h.x + (double)l.x) * dd.x + ((double)h.y + (double)l.y) * dd.y +
                ((double)h.z + (double)l.z) * dd.z + ((double)h.w + (double)l.w) * dd.w;
      }
    }
  }
  __shared__ double red[JG_Q][256];
#pragma unroll
  for (int k = 0; k < JG_Q; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
#pragma unroll
      for (int k = 0; k < JG_Q; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < nq) gam[Q0 + threadIdx.x] = red[threadIdx.x][0];
}

// Jvec[c] = sum_Q B[Q][c] gamma_Q, B = hi + lo, four columns per thread, fixed Q order
__global__ void __launch_bounds__(256) j_back_kernel(const float* __restrict__ hi,
                                                     const float* __restrict__ lo, int64_t ncols,
                                                     int naux, const double* __restrict__ gam,
                                                     double* __restrict__ jv) {
  const int64_t c4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c4 >= (ncols >> 2)) return;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  const float4* h4 = reinterpret_cast<const float4*>(hi) + c4;
  const float4* l4 = reinterpret_cast<const float4*>(lo) + c4;
  const int64_t stride = ncols >> 2;
  for (int Q = 0; Q < naux; ++Q) {
    const double g = gam[Q];
    const float4 h = h4[Q * stride], l = l4[Q * stride];
    a0 = fma((double)h.x + (double)l.x, g, a0);
    a1 = fma((double)h.y + (double)l.y, g, a1);
    a2 = fma((double)h.z + (double)l.z, g, a2);
    a3 = fma((double)h.w + (double)l.w, g, a3);
  }
  reinterpret_cast<double4*>(jv)[c4] = double4{a0, a1, a2, a3};
}

// tile layout -> dense symmetric matrix
__global__ void unpack_sym_kernel(const double* __restrict__ v, int nbf, double* __restrict__ M) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nbf * nbf) return;
  int r = (int)(idx / nbf), c = (int)(idx % nbf);
  if (r < c) {
    const int t = r;
    r = c;
    c = t;
  }
  M[idx] = v[tile_base(r >> 5, c >> 5) + ((r & 31) << 5) + (c & 31)];
}

void j_gamma(const JKArgs& a, const double* D, double* gam, double* dvec, hipStream_t st) {
  const int nt = ntiles_for(a.nbf);
  hipLaunchKernelGGL(pack_density_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, st, D, a.nbf, dvec);
  // both words of B in every precision: J is bandwidth-bound, and with the hi
  // word alone its error (amplified by the conditioning of the metric) exceeds
  // that of a reduced-precision K
  hipLaunchKernelGGL(j_gamma_kernel, dim3((a.naux + JG_Q - 1) / JG_Q), dim3(256), 0, st, a.hi, a.lo, a.ncols, a.naux,
                     dvec, gam);
}

void j_build(const JKArgs& a, const double* D, double* J, double* work, hipStream_t st) {
  double* dvec = work;                       // ncols
  double* gam = work + a.ncols;              // naux
  double* jv = gam + ((a.naux + 3) & ~3);    // ncols
  j_gamma(a, D, gam, dvec, st);
  const unsigned gb = (unsigned)(((a.ncols >> 2) + 255) / 256);
  hipLaunchKernelGGL(j_back_kernel, dim3(gb), dim3(256), 0, st, a.hi, a.lo, a.ncols, a.naux, gam, jv);
  const int64_t n2 = (int64_t)a.nbf * a.nbf;
  hipLaunchKernelGGL(unpack_sym_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, jv, a.nbf, J);
}

// ---------------------------------------------------------------------------
// K: FP64 in jk_f64.hip, FP32 / BF16 in jk_mixed.hip
size_t k_work_bytes(const JKArgs& a, int nocc) {
  return a.prec == PREC_FP64 ? k_work_bytes_f64(a, nocc) : k_work_bytes_mixed(a, nocc);
}

void k_build(const JKArgs& a, const double* C, int nocc, double* K, void* work, hipStream_t st,
             KTimer* timer) {
  if (a.prec == PREC_FP64)
    k_build_f64(a, C, nocc, K, work, st, timer);
  else
    k_build_mixed(a, C, nocc, K, work, st, timer);
}

// ---------------------------------------------------------------------------
// canonical packed export: out[q - q0][c] = B[q][toff[c]] (hi + lo), or raw[q][toff[c]]
__global__ void export_kernel(const float* __restrict__ hi, const float* __restrict__ lo,
                              const double* __restrict__ raw, int64_t ncols_t,
                              const int64_t* __restrict__ toff, int64_t ncols_p, int q0,
                              double* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols_p) return;
  const int q = q0 + blockIdx.y;
  // toff[c]: the tile offset of canonical column c in B's rows, or its raw column
  out[(int64_t)blockIdx.y * ncols_p + c] =
      raw ? raw[(int64_t)q * ncols_p + toff[c]]
          : (double)hi[(int64_t)q * ncols_t + toff[c]] + (lo ? (double)lo[(int64_t)q * ncols_t + toff[c]] : 0.0);
}

// out[q - q0][mu][nu] = B_q (mu, nu) = hi + lo at the packed tile position
__global__ void unpack_rows_kernel(const float* __restrict__ hi, const float* __restrict__ lo, int64_t ncols_t,
                                   int nbf, int q0, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n2 = (int64_t)nbf * nbf;
  if (i >= n2) return;
  const int mu = (int)(i / nbf), nu = (int)(i % nbf);
  const int r = mu > nu ? mu : nu, c = mu > nu ? nu : mu;
  const int64_t o = (int64_t)(q0 + blockIdx.y) * ncols_t + tile_base(r >> 5, c >> 5) + ((r & 31) << 5) + (c & 31);
  out[(int64_t)blockIdx.y * n2 + i] = (double)hi[o] + (double)lo[o];
}

void unpack_rows(const float* hi, const float* lo, int64_t ncols_t, int nbf, int q0, int q1, double* out,
                 hipStream_t st) {
  if (q1 <= q0) return;
  const int64_t n2 = (int64_t)nbf * nbf;
  const dim3 g((unsigned)((n2 + 255) / 256), q1 - q0);
  hipLaunchKernelGGL(unpack_rows_kernel, g, dim3(256), 0, st, hi, lo, ncols_t, nbf, q0, out);
}

void export_rows(const float* hi, const float* lo, const double* raw, int64_t ncols_t, int q0, int q1,
                 const int64_t* toff, int64_t ncols_p, double* out, hipStream_t st) {
  if (q1 <= q0 || ncols_p <= 0) return;
  const dim3 g((unsigned)((ncols_p + 255) / 256), q1 - q0);
  hipLaunchKernelGGL(export_kernel, g, dim3(256), 0, st, hi, lo, raw, ncols_t, toff, ncols_p, q0, out);
}

}  // namespace dfx
