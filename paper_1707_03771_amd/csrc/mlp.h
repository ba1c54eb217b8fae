// FP32 MLP kernels for the learned starting guess (mlp.hip).
#pragma once
#include <vector>

#include "common.h"

namespace dfx {

int64_t mlp_nparams(const std::vector<int>& widths);
size_t mlp_work_floats(const std::vector<int>& widths, int batch);
void mlp_forward(const std::vector<int>& widths, const float* theta, const float* X, int batch, float* Y,
                 float* work, hipStream_t st);
// mean squared error over all outputs and its gradient in theta (synchronises st)
double mlp_loss_grad(const std::vector<int>& widths, const float* theta, const float* X, const float* T, int batch,
                     float* grad, float* work, hipStream_t st);
// the same without synchronising: the batch's mean squared error is added to *loss_acc (device)
void mlp_loss_grad_acc(const std::vector<int>& widths, const float* theta, const float* X, const float* T, int batch,
                       float* grad, float* work, double* loss_acc, hipStream_t st);
void mlp_adam(float* theta, const float* grad, float* m, float* v, int64_t n, int step, float lr, hipStream_t st);
void gather_rows(const float* src, const int* idx, int rows, int cols, float* out, hipStream_t st);

}  // namespace dfx
