// C ABI of the learned coarse-correction network: create, parameters,
// forward, loss gradient and the training loop (Adam on mini-batches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "learned.h"

using namespace fc;

namespace {

void destroy_model(fc_model_s* m) {
  if (!m) return;
  m->ws.release();
  for (void* p : {(void*)m->net.p, (void*)m->net.wpk, (void*)m->net.g, (void*)m->net.m,
                  (void*)m->net.v})
    if (p) (void)hipFree(p);
  delete m;
}

bool valid_arch(const int32_t* ch, int32_t in_ch) {
  if (!ch || in_ch < 1 || in_ch > 8) return false;
  for (int i = 0; i < 4; ++i)
    if (ch[i] < 1 || ch[i] > 128) return false;
  return true;
}

double sum_partials_host(const double* d_partial, hipStream_t s) {
  double h[1024];
  if (hipMemcpyAsync(h, d_partial, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return NAN;
  if (hipStreamSynchronize(s) != hipSuccess) return NAN;
  double t = 0.0;
  for (double v : h) t += v;
  return t;
}

}  // namespace

#define FC_TRY_M(x)                 \
  do {                              \
    fc_status s_ = (x);             \
    if (s_ != FC_OK) return s_;     \
  } while (0)

extern "C" {

fc_status fc_model_param_count(const int32_t* ch, int32_t in_ch, int64_t* n) {
  if (!valid_arch(ch, in_ch) || !n) {
    set_error("fc_model_param_count: invalid architecture");
    return FC_E_ARG;
  }
  *n = net_param_count(ch, in_ch);
  return FC_OK;
}

fc_status fc_model_create(const int32_t* ch, int32_t in_ch, const float* params, fc_model* out) {
  if (!valid_arch(ch, in_ch) || !params || !out) {
    set_error("fc_model_create: invalid arguments");
    return FC_E_ARG;
  }
  *out = nullptr;
  std::unique_ptr<fc_model_s, void (*)(fc_model_s*)> m(new (std::nothrow) fc_model_s(),
                                                       destroy_model);
  if (!m) return FC_E_NOMEM;
  Net& net = m->net;
  net.init(ch, in_ch);
  const size_t n = (size_t)net.nparam;
  FC_HIP(hipMalloc(&net.p, n * sizeof(float)));
  FC_HIP(hipMalloc(&net.wpk, (size_t)net.nwpk * sizeof(uint16_t)));
  FC_HIP(hipMalloc(&net.g, n * sizeof(float)));
  FC_HIP(hipMalloc(&net.m, n * sizeof(float)));
  FC_HIP(hipMalloc(&net.v, n * sizeof(float)));
  FC_HIP(hipMemcpy(net.p, params, n * sizeof(float), hipMemcpyHostToDevice));
  FC_HIP(hipMemset(net.m, 0, n * sizeof(float)));
  FC_HIP(hipMemset(net.v, 0, n * sizeof(float)));
  FC_HIP(net_sync_bf16(net, nullptr));
  FC_HIP(hipDeviceSynchronize());
  *out = m.release();
  return FC_OK;
}

fc_status fc_model_get_params(fc_model m, float* params) {
  if (!m || !params) return FC_E_ARG;
  FC_HIP(hipMemcpy(params, m->net.p, m->net.nparam * sizeof(float), hipMemcpyDeviceToHost));
  return FC_OK;
}

fc_status fc_model_set_params(fc_model m, const float* params) {
  if (!m || !params) return FC_E_ARG;
  FC_HIP(hipMemcpy(m->net.p, params, m->net.nparam * sizeof(float), hipMemcpyHostToDevice));
  FC_HIP(net_sync_bf16(m->net, nullptr));
  FC_HIP(hipDeviceSynchronize());
  return FC_OK;
}

fc_status fc_model_forward(fc_model m, int32_t batch, int32_t grid, const float* x_dev,
                           float* y_dev, void* stream) {
  if (!m || batch < 1 || grid < 2 || !x_dev || !y_dev) {
    set_error("fc_model_forward: invalid arguments");
    return FC_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  FC_TRY_M(m->ws.ensure(m->net, batch, grid));
  FC_HIP(net_forward(m->net, m->ws, x_dev, batch, s));
  const int64_t n = (int64_t)batch * grid * grid * grid;
  FC_HIP(hipMemcpyAsync(y_dev, m->ws.y(), n * sizeof(float), hipMemcpyDeviceToDevice, s));
  return FC_OK;
}

fc_status fc_model_loss_grad(fc_model m, int32_t batch, int32_t grid, const float* x_dev,
                             const float* t_dev, double* loss, float* grad_host, void* stream) {
  if (!m || batch < 1 || grid < 2 || !x_dev || !t_dev) {
    set_error("fc_model_loss_grad: invalid arguments");
    return FC_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  FC_TRY_M(m->ws.ensure(m->net, batch, grid));
  const int64_t n = (int64_t)batch * grid * grid * grid;
  FC_HIP(net_forward(m->net, m->ws, x_dev, batch, s));
  FC_HIP(net_mse(m->ws, t_dev, m->ws.gy(), n, s));
  FC_HIP(net_backward(m->net, m->ws, x_dev, m->ws.gy(), batch, s));
  const double l = sum_partials_host(m->ws.partial, s) / (double)n;
  if (loss) *loss = l;
  if (grad_host)
    FC_HIP(hipMemcpy(grad_host, m->net.g, m->net.nparam * sizeof(float), hipMemcpyDeviceToHost));
  return FC_OK;
}

fc_status fc_model_train(fc_model m, int64_t n_samples, int32_t grid, const float* x_dev,
                         const float* t_dev, const fc_train_opts* opts, double* history,
                         void* stream) {
  if (!m || n_samples < 1 || grid < 2 || !x_dev || !t_dev || !opts || opts->epochs < 1 ||
      opts->batch < 1 || !(opts->lr > 0.f)) {
    set_error("fc_model_train: invalid arguments");
    return FC_E_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)std::min<int64_t>(opts->batch, n_samples);
  FC_TRY_M(m->ws.ensure(m->net, B, grid));
  const int64_t vox = (int64_t)grid * grid * grid;
  const int in_ch = m->net.in_ch;
  float* xb = nullptr;
  float* tb = nullptr;
  FC_HIP(hipMalloc(&xb, (size_t)B * in_ch * vox * sizeof(float)));
  FC_HIP(hipMalloc(&tb, (size_t)B * vox * sizeof(float)));
  const int64_t steps_per_epoch = n_samples / B;
  fc_status st = FC_OK;
  for (int ep = 0; ep < opts->epochs && st == FC_OK; ++ep) {
    double acc = 0.0;
    for (int64_t it = 0; it < steps_per_epoch; ++it) {
      // deterministic interleaved mini-batches: sample (it + j*steps) % n,
      // shifted by the epoch so batches differ between epochs
      for (int j = 0; j < B; ++j) {
        const int64_t k = (it + j * steps_per_epoch + ep) % n_samples;
        if (hipMemcpyAsync(xb + (int64_t)j * in_ch * vox, x_dev + k * in_ch * vox,
                           in_ch * vox * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(tb + (int64_t)j * vox, t_dev + k * vox, vox * sizeof(float),
                           hipMemcpyDeviceToDevice, s) != hipSuccess) {
          st = FC_E_DEVICE;
          break;
        }
      }
      if (st != FC_OK) break;
      const int64_t n = (int64_t)B * vox;
      if (net_forward(m->net, m->ws, xb, B, s) != hipSuccess ||
          net_mse(m->ws, tb, m->ws.gy(), n, s) != hipSuccess ||
          net_backward(m->net, m->ws, xb, m->ws.gy(), B, s) != hipSuccess ||
          net_adam(m->net, opts->lr, ++m->net.step, s) != hipSuccess) {
        st = FC_E_DEVICE;
        break;
      }
      if (history) acc += sum_partials_host(m->ws.partial, s) / (double)n;
    }
    if (history) history[ep] = acc / std::max<int64_t>(1, steps_per_epoch);
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(xb);
  (void)hipFree(tb);
  if (st != FC_OK) set_error("fc_model_train: a kernel launch failed");
  return st;
}

void fc_model_destroy(fc_model m) { destroy_model(m); }

}  // extern "C"
