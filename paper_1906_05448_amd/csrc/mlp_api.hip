// mlp_api.hip - C ABI of the gradient-corrector network: parameters in a
// caller-allocated device workspace, forward pass, gradient, Adam.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>

#include "internal.hpp"
#include "mlp_device.hpp"

namespace {

constexpr size_t kAlignM = 256;
size_t up(size_t b) { return (b + kAlignM - 1) / kAlignM * kAlignM; }

struct MlpPlan {
  size_t theta, m, v, grad, part, lpart, loss, total;
};

MlpPlan mlp_plan() {
  MlpPlan p{};
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += up(b);
    return o;
  };
  const size_t P = (size_t)lbm::kMlpParams * sizeof(float);
  p.theta = take(P);
  p.m = take(P);
  p.v = take(P);
  p.grad = take(P);
  p.part = take((size_t)lbm::kMlpGrid * P);
  p.lpart = take((size_t)lbm::kMlpGrid * sizeof(double));
  p.loss = take(sizeof(double));
  p.total = off;
  return p;
}

// ---- gradient without allocation -------------------------------------------
// The per-workgroup partial sums of the gradient live in this file-scope
// device array instead of a network workspace: every GPU the library runs on
// holds one copy of it (10.5 MB) until the process ends. Host code must not
// pass the array's name to a kernel (on the host it is only a stand-in for
// the symbol): its device address is looked up once per device with
// hipGetSymbolAddress and kept in scratch_addr.
constexpr size_t kScratchPartBytes = (size_t)lbm::kMlpGrid * lbm::kMlpParams * sizeof(float);
constexpr size_t kScratchBytes = kScratchPartBytes + (size_t)lbm::kMlpGrid * sizeof(double);
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices] = {};

// Device address of this GPU's scratch array (the current device).
hipError_t scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_addr[dev] = p;
  }
  *out = scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

struct lbm_mlp {
  hipStream_t stream;
  float *theta, *m, *v, *grad, *part;
  double *lpart, *loss;
  int64_t t;       // Adam steps taken
  bool has_grad;   // a gradient is ready for lbm_mlp_adam_step
};

extern "C" {

size_t lbm_mlp_workspace_size(void) { return mlp_plan().total; }

int lbm_mlp_set_params(lbm_mlp* h, const float* params) {
  if (!h || !params) return LBM_E_ARG;
  const size_t P = (size_t)lbm::kMlpParams * sizeof(float);
  if (hipMemcpyAsync(h->theta, params, P, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipMemsetAsync(h->m, 0, P, h->stream) != hipSuccess || hipMemsetAsync(h->v, 0, P, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return LBM_E_HIP;
  h->t = 0;
  h->has_grad = false;
  return LBM_OK;
}

int lbm_mlp_init(void* workspace, size_t bytes, const float* params, void* stream, lbm_mlp** out) {
  if (!out) return LBM_E_ARG;
  *out = nullptr;
  if (!workspace || !params) return LBM_E_ARG;
  const MlpPlan p = mlp_plan();
  if (bytes < p.total) return LBM_E_SIZE;
  if (((uintptr_t)workspace) % kAlignM) return LBM_E_ARG;
  lbm_mlp* h = new (std::nothrow) lbm_mlp{};
  if (!h) return LBM_E_SIZE;
  char* b = (char*)workspace;
  h->stream = (hipStream_t)stream;
  h->theta = (float*)(b + p.theta);
  h->m = (float*)(b + p.m);
  h->v = (float*)(b + p.v);
  h->grad = (float*)(b + p.grad);
  h->part = (float*)(b + p.part);
  h->lpart = (double*)(b + p.lpart);
  h->loss = (double*)(b + p.loss);
  const int st = lbm_mlp_set_params(h, params);
  if (st != LBM_OK) {
    delete h;
    return st;
  }
  *out = h;
  return LBM_OK;
}

int lbm_mlp_get_params(lbm_mlp* h, float* params) {
  if (!h || !params) return LBM_E_ARG;
  if (hipMemcpyAsync(params, h->theta, (size_t)lbm::kMlpParams * sizeof(float), hipMemcpyDeviceToHost, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return LBM_E_HIP;
  return LBM_OK;
}

const float* lbm_mlp_device_params(const lbm_mlp* h) { return h ? h->theta : nullptr; }

int lbm_mlp_forward(lbm_mlp* h, const uint16_t* x, int64_t n, float* y) {
  if (!h || n < 0 || (n > 0 && (!x || !y))) return LBM_E_ARG;
  // rows move as 16-byte vectors
  if (n > 0 && (((uintptr_t)x | (uintptr_t)y) & 15u)) return LBM_E_ARG;
  return lbm::launch_mlp_forward(h->stream, h->theta, x, n, y) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_mlp_gradient(lbm_mlp* h, const uint16_t* x, const float* t, int64_t n, double* loss, float* grad) {
  if (!h || n <= 0 || !x || !t) return LBM_E_ARG;
  if (lbm::launch_mlp_gradient(h->stream, h->theta, x, t, n, h->part, h->lpart, h->grad, h->loss) != hipSuccess)
    return LBM_E_HIP;
  h->has_grad = true;
  if (loss || grad) {
    double l = 0.0;
    if (hipMemcpyAsync(&l, h->loss, sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess) return LBM_E_HIP;
    if (grad && hipMemcpyAsync(grad, h->grad, (size_t)lbm::kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                               h->stream) != hipSuccess)
      return LBM_E_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_E_HIP;
    if (loss) *loss = l / (9.0 * (double)n);
  }
  return LBM_OK;
}

int lbm_mlp_gradient_noalloc(const float* theta, const uint16_t* x, const float* t, int64_t n, float* grad,
                             double* loss_sum, void* stream) {
  if (!theta || !x || !t || !grad || !loss_sum || n <= 0) return LBM_E_ARG;
  if (n > LBM_MLP_NOALLOC_MAX_SAMPLES) return LBM_E_SIZE;
  void* sp = nullptr;
  if (scratch_for_current_device(&sp) != hipSuccess) return LBM_E_HIP;
  float* part = (float*)sp;
  double* lpart = (double*)((char*)sp + kScratchPartBytes);
  return lbm::launch_mlp_gradient((hipStream_t)stream, theta, x, t, n, part, lpart, grad, loss_sum) == hipSuccess
             ? LBM_OK
             : LBM_E_HIP;
}

int lbm_mlp_adam_step(lbm_mlp* h, double lr, double beta1, double beta2, double eps) {
  if (!h || !h->has_grad || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) ||
      !(eps > 0.0))
    return LBM_E_ARG;
  h->t += 1;
  const double c1 = 1.0 / (1.0 - pow(beta1, (double)h->t));
  const double c2 = 1.0 / (1.0 - pow(beta2, (double)h->t));
  return lbm::launch_mlp_adam(h->stream, h->theta, h->m, h->v, h->grad, (float)lr, (float)beta1, (float)beta2,
                              (float)eps, (float)c1, (float)c2) == hipSuccess
             ? LBM_OK
             : LBM_E_HIP;
}

int lbm_mlp_sync(lbm_mlp* h) {
  if (!h) return LBM_E_ARG;
  return hipStreamSynchronize(h->stream) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

void lbm_mlp_destroy(lbm_mlp* h) { delete h; }

}  // extern "C"
