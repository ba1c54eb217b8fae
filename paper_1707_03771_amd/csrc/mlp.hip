// FP32 multilayer perceptron on gfx950 for the learned starting guess:
// Linear -> SiLU -> ... -> Linear, mean-squared-error loss, hand-written
// backward pass and Adam.  Parameters theta are one flat array: for each layer
// W (out x in, row-major) then b (out).
#include <cmath>

#include "host.h"
#include "mlp.h"

namespace dfx {

// ---- tiled SGEMM on FP32 matrix cores: C = op(A) op(B) (+ C), row-major.
// A workgroup owns a 64 x 64 tile of C; its four waves own 32 x 32 quarters,
// each as 2 x 2 tiles of v_mfma_f32_16x16x4f32 (FP32 products, FP32 sums).
// K goes through LDS in slices of 16.  MFMA operands: lane (li, lk) = (lane %
// 16, lane / 16) gives A[row li][k lk] and B[k lk][col li]; the result's
// element r of that lane is C[row 4 lk + r][col li].
constexpr int SG = 64, SK = 16;
typedef float v4f __attribute__((ext_vector_type(4)));
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) sgemm_kernel(int M, int N, int K, const float* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb, float* __restrict__ C,
                                                   int ldc, int accumulate) {
  __shared__ float As[SG][SK + 1];  // As[m][k]
  __shared__ float Bs[SK][SG + 1];  // Bs[k][n]
  const int m0 = blockIdx.y * SG, n0 = blockIdx.x * SG;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += SK) {
    for (int e = threadIdx.x; e < SG * SK; e += 256) {
      const int mm = e / SK, kk = e % SK;
      const int m = m0 + mm, k = k0 + kk;
      As[mm][kk] = (m < M && k < K) ? (TA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k]) : 0.0f;
      const int nn = e / SK, n = n0 + nn;
      Bs[kk][nn] = (n < N && k < K) ? (TB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n]) : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < SK; kk += 4) {
      float fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = As[wm + a * 16 + li][kk + lk];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = Bs[kk + lk][wn + b * 16 + li];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + a * 16 + 4 * lk + r, n = n0 + wn + b * 16 + li;
        if (m < M && n < N) {
          float* c = C + (int64_t)m * ldc + n;
          *c = accumulate ? *c + acc[a][b][r] : acc[a][b][r];
        }
      }
}

static void sgemm(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C,
                  int ldc, bool accumulate, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  const dim3 g((N + SG - 1) / SG, (M + SG - 1) / SG);
#define SGL(X, Y) hipLaunchKernelGGL((sgemm_kernel<X, Y>), g, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, accumulate ? 1 : 0)
  if (!ta && !tb) SGL(false, false);
  else if (!ta && tb) SGL(false, true);
  else if (ta && !tb) SGL(true, false);
  else SGL(true, true);
#undef SGL
}

// Z = Z + b (per column); A = silu(Z) (or A = Z for the output layer)
__global__ void bias_act_kernel(float* Z, float* Aout, const float* __restrict__ b, int rows, int cols, int act) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const float z = Z[i] + b[i % cols];
  Z[i] = z;
  Aout[i] = act ? z / (1.0f + expf(-z)) : z;
}

// G *= silu'(Z)
__global__ void dsilu_kernel(float* G, const float* __restrict__ Z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float z = Z[i];
  const float s = 1.0f / (1.0f + expf(-z));
  G[i] *= s * (1.0f + z * (1.0f - s));
}

// db[c] = sum_r G[r][c], fixed order
__global__ void colsum_kernel(const float* __restrict__ G, int rows, int cols, float* db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; ++r) s += G[(int64_t)r * cols + c];
  db[c] = s;
}

// G = 2 (Y - T) / n ; per-block partial sums of (Y - T)^2
__global__ void mse_kernel(const float* __restrict__ Y, const float* __restrict__ T, float* G, int64_t n,
                           double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    G[i] = 2.0f * d / (float)n;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void adam_kernel(float* theta, const float* __restrict__ g, float* m, float* v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// out[r][:] = src[idx[r]][:]
__global__ void gather_rows_kernel(const float* __restrict__ src, const int* __restrict__ idx, int rows, int cols,
                                   float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * cols) return;
  const int r = (int)(i / cols), c = (int)(i % cols);
  out[i] = src[(int64_t)idx[r] * cols + c];
}

static unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

int64_t mlp_nparams(const std::vector<int>& w) {
  int64_t n = 0;
  for (size_t i = 0; i + 1 < w.size(); ++i) n += (int64_t)w[i] * w[i + 1] + w[i + 1];
  return n;
}

size_t mlp_work_floats(const std::vector<int>& w, int batch) {
  size_t s = 0;
  for (size_t i = 1; i < w.size(); ++i) s += 2 * (size_t)batch * w[i];  // Z and A per layer
  int mx = 0;
  for (int x : w) mx = std::max(mx, x);
  return s + 2 * (size_t)batch * mx + 1024;                           // two gradient buffers + partials
}

// forward: A_L = network(X); Z/A of every layer kept in work for the backward pass
static const float* forward_impl(const std::vector<int>& w, const float* theta, const float* X, int batch,
                                 float* work, hipStream_t st) {
  const int nl = (int)w.size() - 1;
  const float* a = X;
  const float* p = theta;
  float* wp = work;
  for (int l = 0; l < nl; ++l) {
    const int ni = w[l], no = w[l + 1];
    float* Z = wp;
    float* A = wp + (size_t)batch * no;
    wp += 2 * (size_t)batch * no;
    sgemm(false, true, batch, no, ni, a, ni, p, ni, Z, no, false, st);  // Z = a W^T
    hipLaunchKernelGGL(bias_act_kernel, dim3(nb((int64_t)batch * no)), dim3(256), 0, st, Z, A,
                       p + (size_t)ni * no, batch, no, l < nl - 1 ? 1 : 0);
    p += (size_t)ni * no + no;
    a = A;
  }
  return a;
}

void mlp_forward(const std::vector<int>& w, const float* theta, const float* X, int batch, float* Y, float* work,
                 hipStream_t st) {
  const float* out = forward_impl(w, theta, X, batch, work, st);
  DFX_HIP(hipMemcpyAsync(Y, out, sizeof(float) * (size_t)batch * w.back(), hipMemcpyDeviceToDevice, st));
}

// acc[0] += sum of the 64 partial sums / n  (one thread, fixed order)
__global__ void loss_accumulate_kernel(const double* __restrict__ part, int64_t n, double* acc) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < 64; ++i) s += part[i];
  acc[0] += s / (double)n;
}

static void loss_grad_impl(const std::vector<int>& w, const float* theta, const float* X, const float* T, int batch,
                           float* grad, float* work, double*& part_out, int64_t& nout_out, hipStream_t st);

double mlp_loss_grad(const std::vector<int>& w, const float* theta, const float* X, const float* T, int batch,
                     float* grad, float* work, hipStream_t st) {
  double* part = nullptr;
  int64_t nout = 0;
  loss_grad_impl(w, theta, X, T, batch, grad, work, part, nout, st);
  std::vector<double> hp(64);
  DFX_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * 64, hipMemcpyDeviceToHost, st));
  DFX_HIP(hipStreamSynchronize(st));
  double s = 0.0;
  for (double v : hp) s += v;
  return s / (double)nout;
}

void mlp_loss_grad_acc(const std::vector<int>& w, const float* theta, const float* X, const float* T, int batch,
                       float* grad, float* work, double* loss_acc, hipStream_t st) {
  double* part = nullptr;
  int64_t nout = 0;
  loss_grad_impl(w, theta, X, T, batch, grad, work, part, nout, st);
  hipLaunchKernelGGL(loss_accumulate_kernel, dim3(1), dim3(64), 0, st, part, nout, loss_acc);
}

static void loss_grad_impl(const std::vector<int>& w, const float* theta, const float* X, const float* T, int batch,
                           float* grad, float* work, double*& part_out, int64_t& nout_out, hipStream_t st) {
  const int nl = (int)w.size() - 1;
  const float* Y = forward_impl(w, theta, X, batch, work, st);
  size_t act = 0;
  for (int l = 1; l <= nl; ++l) act += 2 * (size_t)batch * w[l];
  int mx = 0;
  for (int x : w) mx = std::max(mx, x);
  float* G = work + act;
  float* G2 = G + (size_t)batch * mx;
  double* part = reinterpret_cast<double*>(work + ((act + 2 * (size_t)batch * mx + 1) & ~(size_t)1));
  const int64_t nout = (int64_t)batch * w.back();
  hipLaunchKernelGGL(mse_kernel, dim3(64), dim3(256), 0, st, Y, T, G, nout, part);
  // parameter offsets
  std::vector<size_t> off(nl);
  size_t o = 0;
  for (int l = 0; l < nl; ++l) {
    off[l] = o;
    o += (size_t)w[l] * w[l + 1] + w[l + 1];
  }
  // layer activations: Z_l at zofs[l], A_l at zofs[l] + batch * w[l+1]
  std::vector<size_t> zofs(nl);
  size_t zo = 0;
  for (int l = 0; l < nl; ++l) {
    zofs[l] = zo;
    zo += 2 * (size_t)batch * w[l + 1];
  }
  for (int l = nl - 1; l >= 0; --l) {
    const int ni = w[l], no = w[l + 1];
    if (l < nl - 1)
      hipLaunchKernelGGL(dsilu_kernel, dim3(nb((int64_t)batch * no)), dim3(256), 0, st, G, work + zofs[l],
                         (int64_t)batch * no);
    const float* a_in = (l == 0) ? X : work + zofs[l - 1] + (size_t)batch * w[l];
    sgemm(true, false, no, ni, batch, G, no, a_in, ni, grad + off[l], ni, false, st);  // dW = G^T a
    hipLaunchKernelGGL(colsum_kernel, dim3((no + 255) / 256), dim3(256), 0, st, G, batch, no,
                       grad + off[l] + (size_t)ni * no);
    if (l > 0) {
      sgemm(false, false, batch, ni, no, G, no, theta + off[l], ni, G2, ni, false, st);  // dA_in = G W
      std::swap(G, G2);
    }
  }
  part_out = part;
  nout_out = nout;
}

void mlp_adam(float* theta, const float* grad, float* m, float* v, int64_t n, int step, float lr, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(nb(n)), dim3(256), 0, st, theta, grad, m, v, n, lr, b1, b2, eps, c1, c2);
}

void gather_rows(const float* src, const int* idx, int rows, int cols, float* out, hipStream_t st) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(nb((int64_t)rows * cols)), dim3(256), 0, st, src, idx, rows, cols, out);
}

}  // namespace dfx

using namespace dfx;

extern "C" {

int dfx_mlp_forward(const int32_t* widths, int nlayers, const float* theta, const float* X, int batch, float* Y,
                    void* stream) {
  return guard([&] {
    if (!widths || nlayers < 1 || !theta || !X || !Y || batch <= 0) throw Error(DFX_EINVAL, "dfx_mlp_forward: bad argument");
    std::vector<int> w(widths, widths + nlayers + 1);
    DevMem work(sizeof(float) * mlp_work_floats(w, batch));
    mlp_forward(w, theta, X, batch, Y, work.as<float>(), (hipStream_t)stream);
    DFX_HIP(hipStreamSynchronize((hipStream_t)stream));
  });
}

int dfx_mlp_loss_grad(const int32_t* widths, int nlayers, const float* theta, const float* X, const float* T, int batch,
                      float* grad, double* loss, void* stream) {
  return guard([&] {
    if (!widths || nlayers < 1 || !theta || !X || !T || !grad || batch <= 0)
      throw Error(DFX_EINVAL, "dfx_mlp_loss_grad: bad argument");
    std::vector<int> w(widths, widths + nlayers + 1);
    DevMem work(sizeof(float) * mlp_work_floats(w, batch));
    const double L = mlp_loss_grad(w, theta, X, T, batch, grad, work.as<float>(), (hipStream_t)stream);
    if (loss) *loss = L;
  });
}

int dfx_mlp_adam(float* theta, const float* grad, float* m, float* v, int64_t n, int step, float lr, void* stream) {
  return guard([&] {
    if (!theta || !grad || !m || !v || n <= 0 || step < 1) throw Error(DFX_EINVAL, "dfx_mlp_adam: bad argument");
    mlp_adam(theta, grad, m, v, n, step, lr, (hipStream_t)stream);
  });
}

}  // extern "C"
