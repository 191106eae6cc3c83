// Learned step-cost model used by the path search (extension of Methods C's
// cost-driven search): a small network predicts the log of a step's run
// time from the step's features; the planner then sums predicted times
// instead of FLOP and byte counts.  The network is evaluated on the GPU by
// the library's own forward kernel, in one batch over every step shape the
// search can meet for a given batch size, and the predictions are kept in a
// table the search reads.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <random>
#include <unordered_map>
#include <vector>

#include "../../include/leapfrog.h"
#include "mlp.h"
#include "plan.h"

namespace lf {

void step_features(int nz, int nm, int nn, int nk, int dtype, float* f) {
  const double es = dtype ? 4.0 : 8.0;
  const double macs = std::ldexp(1.0, nz + nm + nn + nk);
  const double bytes = es * (std::ldexp(1.0, nz + nm + nk) + std::ldexp(1.0, nz + nn + nk) +
                             std::ldexp(1.0, nz + nm + nn));
  const double peak = dtype ? 2.5e15 : 157.3e12;
  const double roof_us = std::max(8.0 * macs / peak, bytes / 8.0e12) * 1e6;
  f[0] = float(nz);
  f[1] = float(nm);
  f[2] = float(nn);
  f[3] = float(nk);
  f[4] = float(nz + nm + nn + nk);
  f[5] = float(nz + nm + nk);
  f[6] = float(nz + nn + nk);
  f[7] = float(nz + nm + nn);
  f[8] = float(std::log2(bytes));
  f[9] = float(std::log2(8.0 * macs / bytes));
  f[10] = float(dtype);
  f[11] = float(nm >= 5 && nn >= 4 && nk >= 2);
  f[12] = float(nz > 0);
  f[13] = float(std::log2(roof_us));
}

namespace {

struct Model {
  bool loaded = false;
  int n_in = N_FEATURES, H = 128;
  std::vector<float> params;         // host copy
  std::vector<float> xm, xs;         // feature normalisation
  float ym = 0, ys = 1;              // target normalisation (log seconds)
  // predicted seconds, keyed by (nz, nm, nn, nk, dtype)
  std::unordered_map<uint64_t, double> table;
  std::vector<char> nz_done;         // nz values whose shapes are tabulated
};
Model g_model;
std::mutex g_mu;

uint64_t key(int nz, int nm, int nn, int nk, int dt) {
  return (uint64_t(nz) << 40) | (uint64_t(nm) << 30) | (uint64_t(nn) << 20) | (uint64_t(nk) << 10) | uint64_t(dt);
}

constexpr int SHAPE_MAX = 34;

// Tabulates every shape with the given nz on the GPU (one batched forward).
hipError_t tabulate(Model& m, int nz) {
  std::vector<float> X;
  std::vector<uint64_t> keys;
  float f[N_FEATURES];
  for (int dt = 0; dt < 2; ++dt)
    for (int nm = 0; nm <= SHAPE_MAX; ++nm)
      for (int nn = 0; nn <= SHAPE_MAX; ++nn)
        for (int nk = 0; nk <= SHAPE_MAX; ++nk) {
          if (nz + nm + nk > 40 || nz + nn + nk > 40 || nz + nm + nn > 40) continue;
          step_features(nz, nm, nn, nk, dt, f);
          for (int i = 0; i < N_FEATURES; ++i) X.push_back((f[i] - m.xm[i]) / m.xs[i]);
          keys.push_back(key(nz, nm, nn, nk, dt));
        }
  const int64_t B = int64_t(keys.size());
  float *dP = nullptr, *dX = nullptr, *dY = nullptr, *dW = nullptr;
  hipError_t e;
  const size_t wsb = mlp_workspace_bytes(m.H, B);
  if ((e = hipMalloc(&dP, m.params.size() * sizeof(float)))) return e;
  if ((e = hipMalloc(&dX, X.size() * sizeof(float)))) { (void)hipFree(dP); return e; }
  if ((e = hipMalloc(&dY, B * sizeof(float)))) { (void)hipFree(dP); (void)hipFree(dX); return e; }
  if ((e = hipMalloc(&dW, wsb))) { (void)hipFree(dP); (void)hipFree(dX); (void)hipFree(dY); return e; }
  std::vector<float> Y(B);
  e = hipMemcpy(dP, m.params.data(), m.params.size() * sizeof(float), hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(dX, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice);
  if (!e) e = mlp_forward(dP, m.n_in, m.H, dX, B, dY, dW, nullptr, false);
  if (!e) e = hipMemcpy(Y.data(), dY, B * sizeof(float), hipMemcpyDeviceToHost);
  (void)hipFree(dP);
  (void)hipFree(dX);
  (void)hipFree(dY);
  (void)hipFree(dW);
  if (e) return e;
  for (int64_t i = 0; i < B; ++i) m.table[keys[i]] = std::exp(double(Y[i]) * m.ys + m.ym);
  if (int(m.nz_done.size()) <= nz) m.nz_done.resize(nz + 1, 0);
  m.nz_done[nz] = 1;
  return hipSuccess;
}

struct MlpCost : CostFn {
  double step(int nz, int nm, int nn, int nk, int dtype) const override {
    auto it = g_model.table.find(key(nz, nm, nn, nk, dtype));
    if (it != g_model.table.end()) return it->second;
    // outside the tabulated range: plain roofline time plus launch cost
    double macs = std::ldexp(1.0, nz + nm + nn + nk);
    double es = dtype ? 4.0 : 8.0;
    double bytes = es * (std::ldexp(1.0, nz + nm + nk) + std::ldexp(1.0, nz + nn + nk) +
                         std::ldexp(1.0, nz + nm + nn));
    return 8.0 * macs / (dtype ? 2.5e15 : 157.3e12) + bytes / 8.0e12 + 3e-6;
  }
};
MlpCost g_cost;

}  // namespace

// Planner hook: the loaded model, tabulated for batch exponents 0 and nb.
const CostFn* mlp_cost_fn_for(int nb, std::string* err) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_model.loaded) return nullptr;
  for (int nz : {0, nb}) {
    if (int(g_model.nz_done.size()) > nz && g_model.nz_done[nz]) continue;
    hipError_t e = tabulate(g_model, nz);
    if (e) {
      if (err) *err = std::string("cost model evaluation failed: ") + hipGetErrorString(e);
      return nullptr;
    }
  }
  return &g_cost;
}

}  // namespace lf

namespace {
thread_local std::string g_cm_err;
}

namespace {

__global__ void __launch_bounds__(256) gather_rows(const float* X, const float* T, const int* idx, int64_t rows,
                                                   int n_in, float* Xb, float* Tb) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= rows * n_in) return;
  const int64_t r = i / n_in, c = i - r * n_in;
  const int64_t src = idx[r];
  Xb[i] = X[src * n_in + c];
  if (c == 0) Tb[r] = T[src];
}

__global__ void add_into(float* acc, const float* x) {
  if (threadIdx.x == 0) acc[0] += x[0];
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

extern "C" {

lf_status lf_costmodel_train(const float* X, const float* T, int64_t n, int32_t n_in, int32_t hidden,
                             int32_t epochs, int32_t batch, float lr, uint64_t seed, float* params,
                             float* x_mean, float* x_std, float* y_mean, float* y_std, float* curve,
                             void* stream) {
  if (!X || !T || !params || !x_mean || !x_std || !y_mean || !y_std || n_in < 1 || hidden < 1 ||
      epochs < 1 || batch < 1 || n < batch || n > (int64_t(1) << 30) || !(lr > 0))
    return LF_INVALID_ARGUMENT;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // standardisation of features and targets (population mean and deviation)
  std::vector<double> xm(n_in, 0.0), xs(n_in, 0.0);
  double ym = 0.0, ys = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < n_in; ++c) xm[c] += X[i * n_in + c];
    ym += T[i];
  }
  for (int c = 0; c < n_in; ++c) xm[c] /= double(n);
  ym /= double(n);
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < n_in; ++c) {
      const double d = X[i * n_in + c] - xm[c];
      xs[c] += d * d;
    }
    ys += (T[i] - ym) * (T[i] - ym);
  }
  std::vector<float> Xn(size_t(n) * n_in), Tn(n);
  for (int c = 0; c < n_in; ++c) {
    xs[c] = std::sqrt(xs[c] / double(n));
    x_mean[c] = float(xm[c]);
    x_std[c] = xs[c] > 0 ? float(xs[c]) : 1.0f;
  }
  ys = std::sqrt(ys / double(n));
  *y_mean = float(ym);
  *y_std = ys > 0 ? float(ys) : 1.0f;
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < n_in; ++c) Xn[i * n_in + c] = (X[i * n_in + c] - x_mean[c]) / x_std[c];
    Tn[i] = (T[i] - *y_mean) / *y_std;
  }
  // device buffers for one training run
  const int64_t np = lf::mlp_param_count(n_in, hidden);
  const uint64_t wsb = lf::mlp_workspace_bytes(hidden, batch);
  DevBuf dX, dT, dIdx, dXb, dTb, dM, dV, dG, dLoss, dWs;
  if (hipMalloc(&dX.p, sizeof(float) * Xn.size()) || hipMalloc(&dT.p, sizeof(float) * n) ||
      hipMalloc(&dIdx.p, sizeof(int) * n) || hipMalloc(&dXb.p, sizeof(float) * batch * n_in) ||
      hipMalloc(&dTb.p, sizeof(float) * batch) || hipMalloc(&dM.p, sizeof(float) * np) ||
      hipMalloc(&dV.p, sizeof(float) * np) || hipMalloc(&dG.p, sizeof(float) * np) ||
      hipMalloc(&dLoss.p, sizeof(float) * 2) || hipMalloc(&dWs.p, wsb))
    return LF_HIP_ERROR;
  float* fX = static_cast<float*>(dX.p);
  float* fT = static_cast<float*>(dT.p);
  int* iIdx = static_cast<int*>(dIdx.p);
  float* fXb = static_cast<float*>(dXb.p);
  float* fTb = static_cast<float*>(dTb.p);
  float* fLoss = static_cast<float*>(dLoss.p);   // [0] batch loss, [1] epoch sum
  if (hipMemcpyAsync(fX, Xn.data(), sizeof(float) * Xn.size(), hipMemcpyHostToDevice, st) ||
      hipMemcpyAsync(fT, Tn.data(), sizeof(float) * n, hipMemcpyHostToDevice, st) ||
      hipMemsetAsync(dM.p, 0, sizeof(float) * np, st) || hipMemsetAsync(dV.p, 0, sizeof(float) * np, st))
    return LF_HIP_ERROR;
  std::mt19937_64 rng(seed);
  std::vector<int> perm(n);
  int step = 0;
  const int64_t nb = n / batch;
  const int64_t rows = int64_t(batch) * n_in;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) perm[i] = int(i);
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[std::uniform_int_distribution<int64_t>(0, i)(rng)]);
    // cosine schedule over the epochs
    const float lr_ep = float(lr * 0.5 * (1.0 + std::cos(M_PI * double(ep) / double(epochs))));
    if (hipMemcpyAsync(iIdx, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, st) ||
        hipMemsetAsync(fLoss + 1, 0, sizeof(float), st))
      return LF_HIP_ERROR;
    for (int64_t b = 0; b < nb; ++b) {
      hipLaunchKernelGGL(gather_rows, dim3(unsigned((rows + 255) / 256)), dim3(256), 0, st, fX, fT,
                         iIdx + b * batch, int64_t(batch), n_in, fXb, fTb);
      hipError_t e = lf::mlp_gradients(params, n_in, hidden, fXb, fTb, batch, static_cast<float*>(dG.p), fLoss,
                                   static_cast<float*>(dWs.p), st);
      if (e) return LF_HIP_ERROR;
      hipLaunchKernelGGL(add_into, dim3(1), dim3(64), 0, st, fLoss + 1, fLoss);
      e = lf::mlp_adam(params, static_cast<float*>(dM.p), static_cast<float*>(dV.p), static_cast<float*>(dG.p), np,
                   ++step, lr_ep, 0.9f, 0.999f, 1e-8f, st);
      if (e) return LF_HIP_ERROR;
    }
    if (curve) {
      float sum = 0;
      if (hipMemcpyAsync(&sum, fLoss + 1, sizeof(float), hipMemcpyDeviceToHost, st) || hipStreamSynchronize(st))
        return LF_HIP_ERROR;
      curve[ep] = sum / float(nb);
    }
  }
  if (hipStreamSynchronize(st) || hipGetLastError()) return LF_HIP_ERROR;
  return LF_OK;
}

lf_status lf_step_features(int32_t nz, int32_t nm, int32_t nn, int32_t nk, int32_t dtype, float* out) {
  if (!out || nz < 0 || nm < 0 || nn < 0 || nk < 0 || (dtype != 0 && dtype != 1)) return LF_INVALID_ARGUMENT;
  lf::step_features(nz, nm, nn, nk, dtype, out);
  return LF_OK;
}

lf_status lf_mlp_sizes(int32_t n_in, int32_t hidden, int64_t max_batch, int64_t* n_params,
                       uint64_t* workspace_bytes) {
  if (n_in < 1 || hidden < 1 || max_batch < 1 || !n_params || !workspace_bytes) return LF_INVALID_ARGUMENT;
  *n_params = lf::mlp_param_count(n_in, hidden);
  *workspace_bytes = lf::mlp_workspace_bytes(hidden, max_batch);
  return LF_OK;
}

lf_status lf_mlp_forward(const float* params, int32_t n_in, int32_t hidden, const float* X,
                         int64_t batch, float* Y, void* ws, uint64_t ws_bytes, void* stream) {
  if (!params || !X || !Y || !ws || n_in < 1 || hidden < 1 || batch < 1 || batch > (int64_t(1) << 31))
    return LF_INVALID_ARGUMENT;
  if (ws_bytes < lf::mlp_workspace_bytes(hidden, batch)) return LF_OUT_OF_WORKSPACE;
  hipError_t e = lf::mlp_forward(params, n_in, hidden, X, batch, Y, static_cast<float*>(ws),
                                 static_cast<hipStream_t>(stream), false);
  return e ? LF_HIP_ERROR : LF_OK;
}

lf_status lf_mlp_gradients(const float* params, int32_t n_in, int32_t hidden, const float* X,
                           const float* T, int64_t batch, float* grads, float* loss, void* ws,
                           uint64_t ws_bytes, void* stream) {
  if (!params || !X || !T || !grads || !loss || !ws || n_in < 1 || hidden < 1 || batch < 1 ||
      batch > (int64_t(1) << 31))
    return LF_INVALID_ARGUMENT;
  if (ws_bytes < lf::mlp_workspace_bytes(hidden, batch)) return LF_OUT_OF_WORKSPACE;
  hipError_t e = lf::mlp_gradients(params, n_in, hidden, X, T, batch, grads, loss,
                                   static_cast<float*>(ws), static_cast<hipStream_t>(stream));
  return e ? LF_HIP_ERROR : LF_OK;
}

lf_status lf_mlp_adam_step(float* params, float* m, float* v, const float* grads, int64_t n_params,
                           int32_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (!params || !m || !v || !grads || n_params < 1 || step < 1) return LF_INVALID_ARGUMENT;
  hipError_t e = lf::mlp_adam(params, m, v, grads, n_params, step, lr, beta1, beta2, eps,
                              static_cast<hipStream_t>(stream));
  return e ? LF_HIP_ERROR : LF_OK;
}

lf_status lf_costmodel_load(const float* params, int32_t n_in, int32_t hidden, const float* x_mean,
                            const float* x_std, float y_mean, float y_std) {
  if (!params || !x_mean || !x_std || n_in != lf::N_FEATURES || hidden < 1 || !(y_std > 0))
    return LF_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(lf::g_mu);
  lf::Model m;
  m.loaded = true;
  m.n_in = n_in;
  m.H = hidden;
  m.params.assign(params, params + lf::mlp_param_count(n_in, hidden));
  m.xm.assign(x_mean, x_mean + n_in);
  m.xs.assign(x_std, x_std + n_in);
  for (auto& s : m.xs) if (!(s > 0)) s = 1.0f;
  m.ym = y_mean;
  m.ys = y_std;
  lf::g_model = std::move(m);
  return LF_OK;
}

lf_status lf_costmodel_clear(void) {
  std::lock_guard<std::mutex> lk(lf::g_mu);
  lf::g_model = lf::Model();
  return LF_OK;
}

lf_status lf_costmodel_predict(int32_t nz, int32_t nm, int32_t nn, int32_t nk, int32_t dtype,
                               double* seconds) {
  if (!seconds) return LF_INVALID_ARGUMENT;
  std::string err;
  const lf::CostFn* cf = lf::mlp_cost_fn_for(nz, &err);
  if (!cf) return err.empty() ? LF_INVALID_ARGUMENT : LF_HIP_ERROR;
  *seconds = cf->step(nz, nm, nn, nk, dtype);
  return LF_OK;
}

}  // extern "C"
