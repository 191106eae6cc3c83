// Learned step-cost model: network kernels (mlp.hip) and the planner hook
// (costmodel.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lf {

constexpr int N_FEATURES = 14;

int64_t mlp_param_count(int n_in, int H);
uint64_t mlp_workspace_bytes(int H, int64_t batch);
hipError_t mlp_forward(const float* params, int n_in, int H, const float* X, int64_t batch, float* Y,
                       float* ws, hipStream_t s, bool keep);
hipError_t mlp_gradients(const float* params, int n_in, int H, const float* X, const float* T,
                         int64_t batch, float* grads, float* loss, float* ws, hipStream_t s);
hipError_t mlp_adam(float* p, float* m, float* v, const float* g, int64_t n, int step, float lr,
                    float b1, float b2, float eps, hipStream_t s);

// Features of a step C[z,m,n] = sum_k A[z,m,k] B[z,n,k] with 2^nz x 2^nm x
// 2^nn x 2^nk and compute type dtype (0 complex64, 1 complex-half).
void step_features(int nz, int nm, int nn, int nk, int dtype, float* out);

}  // namespace lf
