// Kernels of the learned step-cost model: a three-layer perceptron
// in -> H -> H -> 1 (ReLU on the hidden layers) in float32, trained by mean
// squared error with Adam.  Parameters are one float32 array:
//   W1 [in][H], b1 [H], W2 [H][H], b2 [H], W3 [H] (column), b3 [1].
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/leapfrog.h"
#include "mlp.h"

namespace lf {

// C[i][j] = sum_k A(i,k) B(k,j) (+ bias[j]) (relu), 32x32 tiles staged in
// LDS.  A(i,k) = A[i*lda + k] or, transposed, A[k*lda + i]; same for B.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) sgemm_kernel(const float* A, const float* B, float* C,
                                                    const float* bias, int M, int N, int K,
                                                    int lda, int ldb, int ldc, int relu) {
  __shared__ float sA[32][33];
  __shared__ float sB[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  float acc[4] = {0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += 32) {
    for (int r = ty; r < 32; r += 8) {
      int i = i0 + r, k = k0 + tx;
      float av = 0.f;
      if (i < M && k < K) av = TA ? A[int64_t(k) * lda + i] : A[int64_t(i) * lda + k];
      sA[r][tx] = av;
      int kk = k0 + r, j = j0 + tx;
      float bv = 0.f;
      if (kk < K && j < N) bv = TB ? B[int64_t(j) * ldb + kk] : B[int64_t(kk) * ldb + j];
      sB[r][tx] = bv;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      const float b = sB[k][tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += sA[ty + 8 * q][k] * b;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + ty + 8 * q, j = j0 + tx;
    if (i < M && j < N) {
      float v = acc[q] + (bias ? bias[j] : 0.f);
      if (relu) v = v > 0.f ? v : 0.f;
      C[int64_t(i) * ldc + j] = v;
    }
  }
}

static hipError_t sgemm(bool ta, bool tb, const float* A, const float* B, float* C,
                        const float* bias, int M, int N, int K, int lda, int ldb, int ldc, int relu,
                        hipStream_t s) {
  dim3 grid((N + 31) / 32, (M + 31) / 32);
  if (!ta && !tb) hipLaunchKernelGGL((sgemm_kernel<false, false>), grid, dim3(256), 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc, relu);
  else if (ta && !tb) hipLaunchKernelGGL((sgemm_kernel<true, false>), grid, dim3(256), 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc, relu);
  else if (!ta && tb) hipLaunchKernelGGL((sgemm_kernel<false, true>), grid, dim3(256), 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc, relu);
  else hipLaunchKernelGGL((sgemm_kernel<true, true>), grid, dim3(256), 0, s, A, B, C, bias, M, N, K, lda, ldb, ldc, relu);
  return hipGetLastError();
}

// dy = 2 (y - t) / n, and per-block partial sums of (y - t)^2
__global__ void __launch_bounds__(256) mse_grad_kernel(const float* y, const float* t, float* dy,
                                                       float* partial, int64_t n) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d / float(n);
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// loss = sum(partial) / n (one block), fixed order
__global__ void finish_loss_kernel(const float* partial, int nparts, int64_t n, float* loss) {
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < nparts; ++i) s += partial[i];
    *loss = s / float(n);
  }
}

// column sums of a [rows][cols] matrix (bias gradients), fixed order
__global__ void __launch_bounds__(256) colsum_kernel(const float* a, float* out, int64_t rows,
                                                     int cols) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int64_t r = 0; r < rows; ++r) s += a[r * cols + j];
  out[j] = s;
}

// d *= (z > 0)
__global__ void __launch_bounds__(256) relu_mask_kernel(float* d, const float* z, int64_t n) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    if (!(z[i] > 0.f)) d[i] = 0.f;
}

__global__ void __launch_bounds__(256) adam_kernel(float* p, float* m, float* v, const float* g,
                                                   int64_t n, float lr, float b1, float b2, float eps,
                                                   float c1, float c2) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

int64_t mlp_param_count(int n_in, int H) { return int64_t(n_in) * H + H + int64_t(H) * H + H + H + 1; }

uint64_t mlp_workspace_bytes(int H, int64_t batch) {
  // z1, h1, z2, h2 [batch][H]; y, dy [batch]; partial sums
  return uint64_t(4 * batch * H + 2 * batch + 1024) * sizeof(float);
}

struct MlpView {
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
static MlpView view(const float* p, int n_in, int H) {
  MlpView v;
  v.W1 = p;
  v.b1 = v.W1 + int64_t(n_in) * H;
  v.W2 = v.b1 + H;
  v.b2 = v.W2 + int64_t(H) * H;
  v.W3 = v.b2 + H;
  v.b3 = v.W3 + H;
  return v;
}

hipError_t mlp_forward(const float* params, int n_in, int H, const float* X, int64_t batch, float* Y,
                       float* ws, hipStream_t s, bool keep) {
  MlpView w = view(params, n_in, H);
  float* z1 = ws;
  float* h1 = z1 + batch * H;
  float* z2 = h1 + batch * H;
  float* h2 = z2 + batch * H;
  const int M = int(batch);
  hipError_t e;
  if (keep) {
    if ((e = sgemm(false, false, X, w.W1, z1, w.b1, M, H, n_in, n_in, H, H, 0, s))) return e;
    if ((e = sgemm(false, false, X, w.W1, h1, w.b1, M, H, n_in, n_in, H, H, 1, s))) return e;
    if ((e = sgemm(false, false, h1, w.W2, z2, w.b2, M, H, H, H, H, H, 0, s))) return e;
    if ((e = sgemm(false, false, h1, w.W2, h2, w.b2, M, H, H, H, H, H, 1, s))) return e;
  } else {
    if ((e = sgemm(false, false, X, w.W1, h1, w.b1, M, H, n_in, n_in, H, H, 1, s))) return e;
    if ((e = sgemm(false, false, h1, w.W2, h2, w.b2, M, H, H, H, H, H, 1, s))) return e;
  }
  return sgemm(false, false, h2, w.W3, Y, w.b3, M, 1, H, H, 1, 1, 0, s);
}

hipError_t mlp_gradients(const float* params, int n_in, int H, const float* X, const float* T,
                         int64_t batch, float* grads, float* loss, float* ws, hipStream_t s) {
  MlpView w = view(params, n_in, H);
  float* z1 = ws;
  float* h1 = z1 + batch * H;
  float* z2 = h1 + batch * H;
  float* h2 = z2 + batch * H;
  float* y = h2 + batch * H;
  float* dy = y + batch;
  float* partial = dy + batch;
  float* gW1 = grads;
  float* gb1 = gW1 + int64_t(n_in) * H;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + int64_t(H) * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H;
  const int M = int(batch);
  hipError_t e;
  if ((e = mlp_forward(params, n_in, H, X, batch, y, ws, s, true))) return e;
  int nparts = int((batch + 255) / 256);
  if (nparts > 512) nparts = 512;
  hipLaunchKernelGGL(mse_grad_kernel, dim3(nparts), dim3(256), 0, s, y, T, dy, partial, batch);
  hipLaunchKernelGGL(finish_loss_kernel, dim3(1), dim3(64), 0, s, partial, nparts, batch, loss);
  // layer 3: gW3 = h2^T dy, gb3 = sum dy, dh2 = dy W3^T (stored in z... reuse h2 buffer after)
  if ((e = sgemm(true, false, h2, dy, gW3, nullptr, H, 1, M, H, 1, 1, 0, s))) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, s, dy, gb3, batch, 1);
  // dz2 = (dy W3^T) * (z2 > 0), written over h2
  if ((e = sgemm(false, true, dy, w.W3, h2, nullptr, M, H, 1, 1, 1, H, 0, s))) return e;
  hipLaunchKernelGGL(relu_mask_kernel, dim3(256), dim3(256), 0, s, h2, z2, batch * H);
  if ((e = sgemm(true, false, h1, h2, gW2, nullptr, H, H, M, H, H, H, 0, s))) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, h2, gb2, batch, H);
  // dz1 = (dz2 W2^T) * (z1 > 0), written over h1 (h1 no longer needed)
  if ((e = sgemm(false, true, h2, w.W2, z2, nullptr, M, H, H, H, H, H, 0, s))) return e;
  hipLaunchKernelGGL(relu_mask_kernel, dim3(256), dim3(256), 0, s, z2, z1, batch * H);
  if ((e = sgemm(true, false, X, z2, gW1, nullptr, n_in, H, M, n_in, H, H, 0, s))) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, z2, gb1, batch, H);
  return hipGetLastError();
}

hipError_t mlp_adam(float* p, float* m, float* v, const float* g, int64_t n, int step, float lr,
                    float b1, float b2, float eps, hipStream_t s) {
  const float c1 = 1.f - powf(b1, float(step)), c2 = 1.f - powf(b2, float(step));
  hipLaunchKernelGGL(adam_kernel, dim3(256), dim3(256), 0, s, p, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lf
