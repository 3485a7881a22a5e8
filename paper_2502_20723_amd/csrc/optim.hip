// First-order parameter updates of the training loop (App. C, optimisation
// procedure: hybrid update with SGD or Adam, and the learning-rate schedule).
//
// SGD:  theta <- theta - eta g.
// Adam (Kingma and Ba, "Adam: a method for stochastic optimization", ICLR 2015,
// Algorithm 1): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// theta <- theta - eta m_hat / (sqrt(v_hat) + eps) with m_hat = m / (1 - b1^t),
// v_hat = v / (1 - b2^t), t = 1, 2, ...  The moments stay in FP64; the update
// is formed in FP64 and the FP32 parameters are rounded once.  The bias
// corrections are computed on the host and passed in.
//
// Both are one pass over P parameters (HBM-bound: SGD reads 12 and writes 4
// bytes per parameter, Adam reads 28 and writes 20).
#include <cmath>

#include "common.h"

namespace tdo {

// Contraction into fused multiply-adds is off in both kernels: each operation
// rounds once, in the order written, as the definitions state.
__global__ void k_sgd(int64_t P, float* __restrict__ theta, const double* __restrict__ g, double lr) {
#pragma clang fp contract(off)
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x)
    theta[k] = (float)((double)theta[k] - lr * g[k]);
}

__global__ void k_adam(int64_t P, float* __restrict__ theta, const double* __restrict__ g, double* __restrict__ m,
                       double* __restrict__ v, double lr, double b1, double b2, double c1, double c2, double eps) {
#pragma clang fp contract(off)
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
    const double gk = g[k];
    const double mk = b1 * m[k] + (1.0 - b1) * gk;
    const double vk = b2 * v[k] + (1.0 - b2) * (gk * gk);
    m[k] = mk;
    v[k] = vk;
    const double mh = mk / c1, vh = vk / c2;
    theta[k] = (float)((double)theta[k] - lr * mh / (sqrt(vh) + eps));
  }
}

}  // namespace tdo

using namespace tdo;

namespace {

unsigned grid_of(int64_t P) {
  const int64_t b = (P + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

extern "C" {

double tdo_lr_schedule(int64_t step, double eta0, int64_t i_switch, int64_t i_decay, double alpha) {
  if (step < i_switch) return eta0;
  const double x = i_decay > 0 ? std::fmin(1.0, (double)(step - i_switch) / (double)i_decay) : 1.0;
  return eta0 * (1.0 + std::cos(M_PI * x)) / 2.0 + alpha * eta0;
}

int32_t tdo_sgd_step(int64_t P, float* params, const double* grad, double lr, hipStream_t stream) {
  clear_error();
  TDO_CHECK(P >= 0, TDO_EINVAL, "P=%lld < 0", (long long)P);
  if (P == 0) return TDO_OK;
  TDO_CHECK(params && grad, TDO_EINVAL, "NULL buffer");
  TDO_CHECK(std::isfinite(lr), TDO_EINVAL, "learning rate %g is not finite", lr);
  hipLaunchKernelGGL(k_sgd, dim3(grid_of(P)), dim3(256), 0, stream, P, params, grad, lr);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t tdo_adam_step(int64_t P, float* params, const double* grad, double* m, double* v, int64_t t, double lr,
                      double beta1, double beta2, double eps, hipStream_t stream) {
  clear_error();
  TDO_CHECK(P >= 0, TDO_EINVAL, "P=%lld < 0", (long long)P);
  TDO_CHECK(t >= 1, TDO_EINVAL, "step t=%lld: Adam counts steps from 1", (long long)t);
  TDO_CHECK(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0, TDO_EINVAL,
            "betas (%g, %g) outside [0, 1)", beta1, beta2);
  TDO_CHECK(eps > 0.0 && std::isfinite(lr), TDO_EINVAL, "eps=%g must be positive and lr=%g finite", eps, lr);
  if (P == 0) return TDO_OK;
  TDO_CHECK(params && grad && m && v, TDO_EINVAL, "NULL buffer");
  const double c1 = 1.0 - std::pow(beta1, (double)t), c2 = 1.0 - std::pow(beta2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_of(P)), dim3(256), 0, stream, P, params, grad, m, v, lr, beta1, beta2, c1,
                     c2, eps);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // extern "C"
