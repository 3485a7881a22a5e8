// Stochastic reconfiguration (App. C, metric tensor and hybrid update):
// solve (S + lambda I) x = g with
//   S_kl = Re sum_b w_b conj(dO_k(x_b)) dO_l(x_b),  dO = O - sum_b w_b O(x_b),
// O_k(x) = d log rho(x) / d theta_k, w normalised to sum 1, for the real
// parameters theta.  With J the 2B x P matrix of rows sqrt(w_b) dRe O(x_b) and
// sqrt(w_b) dIm O(x_b), S = J^T J, so S is never formed: conjugate gradients
// on (J^T J + lambda I) x = g take two passes over J per iteration (rows
// u = J p in segments, the segment sums, then columns J^T u).
//
// The Jacobian comes from tdo_log_rho_jacobian; this call centres and scales
// it in place.  Dot products are two-stage FP64 sums in a fixed order (slices,
// then one workgroup over the slices) and CG's scalars stay on the device, so the iteration count is fixed by the
// caller and the result does not depend on scheduling.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "netapi.h"
#include "train.h"

namespace tdo {

namespace {

constexpr int kT = 256;

__device__ double block_reduce(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = kT / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

}  // namespace

// sc[0] = sum of the weights (B when w is NULL).
__global__ void __launch_bounds__(kT) k_sr_wsum(const double* __restrict__ w, int64_t B, double* __restrict__ sc) {
  __shared__ double red[kT];
  double a = 0.0;
  for (int64_t b = threadIdx.x; b < B; b += kT) a += w ? w[b] : 1.0;
  a = block_reduce(a, red);
  if (threadIdx.x == 0) sc[0] = a;
}

// Column k: subtract the weighted mean of each part and scale row b by sqrt(w_b / sum w).
__global__ void k_sr_center(double* __restrict__ J, int64_t B, int64_t P, const double* __restrict__ w,
                            const double* __restrict__ sc) {
  const double inv = 1.0 / sc[0];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
    for (int part = 0; part < 2; ++part) {
      double mean = 0.0;
      for (int64_t b = 0; b < B; ++b) mean += (w ? w[b] : 1.0) * inv * J[(2 * b + part) * P + k];
      for (int64_t b = 0; b < B; ++b) {
        double* e = J + (2 * b + part) * P + k;
        *e = sqrt((w ? w[b] : 1.0) * inv) * (*e - mean);
      }
    }
  }
}

// Partial row dots: workgroup (r, s) forms J[r] . p over segment s of kSeg equal
// segments, into up[r][s] (summed in segment order by the column pass).
constexpr int kSeg = 8;
__global__ void __launch_bounds__(kT) k_sr_rows(const double* __restrict__ J, int64_t R, int64_t P,
                                                const double* __restrict__ p, double* __restrict__ up) {
  __shared__ double red[kT];
  const int64_t seg = (P + kSeg - 1) / kSeg;
  for (int64_t rs = blockIdx.x; rs < R * kSeg; rs += gridDim.x) {
    const int64_t r = rs / kSeg, s = rs % kSeg;
    const double* row = J + r * P;
    const int64_t k1 = std::min<int64_t>(P, (s + 1) * seg);
    double a = 0.0;
    for (int64_t k = s * seg + threadIdx.x; k < k1; k += kT) a += row[k] * p[k];
    a = block_reduce(a, red);
    if (threadIdx.x == 0) up[rs] = a;
  }
}

// u[r] = sum over s of up[r][s], in segment order.
__global__ void k_sr_usum(const double* __restrict__ up, int64_t R, double* __restrict__ u) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += (int64_t)gridDim.x * blockDim.x) {
    double a = 0.0;
#pragma unroll
    for (int s = 0; s < kSeg; ++s) a += up[r * kSeg + s];
    u[r] = a;
  }
}

// Ap[k] = sum_r J[r][k] u[r] + lambda p[k], one thread per column; four
// accumulators over r mod 4 (summed in that order) keep four loads in flight.
__global__ void k_sr_cols(const double* __restrict__ J, int64_t R, int64_t P, const double* __restrict__ u,
                          const double* __restrict__ p, double lambda, double* __restrict__ Ap) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t r = 0;
    for (; r + 4 <= R; r += 4) {
      a0 += J[r * P + k] * u[r];
      a1 += J[(r + 1) * P + k] * u[r + 1];
      a2 += J[(r + 2) * P + k] * u[r + 2];
      a3 += J[(r + 3) * P + k] * u[r + 3];
    }
    for (; r < R; ++r) a0 += J[r * P + k] * u[r];
    Ap[k] = ((a0 + a1) + (a2 + a3)) + lambda * p[k];
  }
}

// a . b in a fixed order: kDotParts workgroups sum contiguous slices into part[],
// then one workgroup sums the parts (k_sr_dot_fin).
constexpr int kDotParts = 256;
__global__ void __launch_bounds__(kT) k_sr_dot(const double* __restrict__ a, const double* __restrict__ b,
                                               int64_t P, double* __restrict__ part) {
  __shared__ double red[kT];
  const int64_t slice = (P + kDotParts - 1) / kDotParts;
  const int64_t k0 = blockIdx.x * slice, k1 = std::min<int64_t>(P, k0 + slice);
  double s = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kT) s += a[k] * b[k];
  s = block_reduce(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kT) k_sr_dot_fin(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double red[kT];
  double s = 0.0;
  for (int i = threadIdx.x; i < kDotParts; i += kT) s += part[i];
  s = block_reduce(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

// x <- 0, r <- g, p <- g.
__global__ void k_sr_init(const double* __restrict__ g, int64_t P, double* __restrict__ x, double* __restrict__ r,
                          double* __restrict__ p) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
    x[k] = 0.0;
    r[k] = g[k];
    p[k] = g[k];
  }
}

// alpha = rs / (p . Ap) (0 when p . Ap = 0); x += alpha p; r -= alpha Ap.
__global__ void k_sr_step(int64_t P, const double* __restrict__ sc, const double* __restrict__ p,
                          const double* __restrict__ Ap, double* __restrict__ x, double* __restrict__ r) {
  const double pAp = sc[2], rs = sc[1];
  const double alpha = pAp != 0.0 ? rs / pAp : 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
    x[k] += alpha * p[k];
    r[k] -= alpha * Ap[k];
  }
}

// beta = rs_new / rs (0 when rs = 0); p = r + beta p.
__global__ void k_sr_dir(int64_t P, const double* __restrict__ sc, const double* __restrict__ r,
                         double* __restrict__ p) {
  const double rs = sc[1], rn = sc[3];
  const double beta = rs != 0.0 ? rn / rs : 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = r[k] + beta * p[k];
}

// rs <- rs_new.
__global__ void k_sr_roll(double* __restrict__ sc) {
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[1] = sc[3];
}

// info[0] = |r| / |g| from the recurrence, info[1] = |g|.
__global__ void k_sr_info(const double* __restrict__ sc, double* __restrict__ info) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double gn = sqrt(sc[4]);
    info[0] = gn > 0.0 ? sqrt(sc[1]) / gn : 0.0;
    info[1] = gn;
  }
}

// --- the matrix-free form: S p = J^T (J p) from one forward-mode and one reverse-mode pass

// sc[0..2] = sum w, sum w Re t, sum w Im t over the samples (one workgroup, fixed order).
__global__ void __launch_bounds__(kT) k_mf_mean(const float* __restrict__ t, const double* __restrict__ w, int64_t B,
                                                double* __restrict__ sc) {
  __shared__ double red[kT];
  double a = 0.0, re = 0.0, im = 0.0;
  for (int64_t b = threadIdx.x; b < B; b += kT) {
    const double wb = w ? w[b] : 1.0;
    a += wb;
    re += wb * t[2 * b];
    im += wb * t[2 * b + 1];
  }
  a = block_reduce(a, red);
  re = block_reduce(re, red);
  im = block_reduce(im, red);
  if (threadIdx.x == 0) {
    sc[0] = a;
    sc[1] = re;
    sc[2] = im;
  }
}

// seed_b = (w_b / W) (t_b - sum w t / W): the reverse-mode seeds of J^T (J p).
__global__ void k_mf_seeds(const float* __restrict__ t, const double* __restrict__ w, int64_t B,
                           const double* __restrict__ sc, float* __restrict__ seed) {
  const double W = sc[0], mr = sc[1] / W, mi = sc[2] / W;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < B; b += (int64_t)gridDim.x * blockDim.x) {
    const double f = (w ? w[b] : 1.0) / W;
    seed[2 * b] = (float)(f * (t[2 * b] - mr));
    seed[2 * b + 1] = (float)(f * (t[2 * b + 1] - mi));
  }
}

// Ap += lambda p
__global__ void k_mf_shift(int64_t P, double lambda, const double* __restrict__ p, double* __restrict__ Ap) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x)
    Ap[k] += lambda * p[k];
}

}  // namespace tdo

using namespace tdo;

extern "C" int32_t tdo_sr_solve(tdo_ctx_t* ctx, double* jac, int64_t B, int64_t P, const double* weights,
                                const double* grad, double lambda, int32_t iters, double* x, double* info,
                                hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(B >= 1 && P >= 1, TDO_EINVAL, "B=%lld, P=%lld: both must be >= 1", (long long)B, (long long)P);
  TDO_CHECK(lambda > 0.0 && std::isfinite(lambda), TDO_EINVAL, "diagonal shift lambda=%g must be positive", lambda);
  TDO_CHECK(iters >= 0, TDO_EINVAL, "iters=%d < 0", iters);
  TDO_CHECK(jac && grad && x, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  Arena ar;
  const size_t or_ = ar.take<double>((size_t)P), op = ar.take<double>((size_t)P), oap = ar.take<double>((size_t)P);
  const size_t oup = ar.take<double>(2 * (size_t)B * kSeg), ou = ar.take<double>(2 * (size_t)B);
  const size_t osc = ar.take<double>(8);
  const size_t opart = ar.take<double>(kDotParts);
  TDO_TRY(ensure_workspace(&c, ar.used));
  double* r = at<double>(c.ws, or_);
  double* p = at<double>(c.ws, op);
  double* Ap = at<double>(c.ws, oap);
  double* up = at<double>(c.ws, oup);
  double* u = at<double>(c.ws, ou);
  double* sc = at<double>(c.ws, osc);  // [0] sum w, [1] rs, [2] p.Ap, [3] rs_new, [4] g.g
  double* part = at<double>(c.ws, opart);
  auto dot = [&](const double* a, const double* b, double* out) -> int32_t {
    hipLaunchKernelGGL(k_sr_dot, dim3(kDotParts), dim3(kT), 0, stream, a, b, P, part);
    hipLaunchKernelGGL(k_sr_dot_fin, dim3(1), dim3(kT), 0, stream, part, out);
    TDO_HIP(hipGetLastError());
    return TDO_OK;
  };
  const int64_t R = 2 * B;
  const unsigned gp = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(P, 256), 4096));
  const unsigned gr = (unsigned)std::min<int64_t>(R * kSeg, 16384);
  hipLaunchKernelGGL(k_sr_wsum, dim3(1), dim3(kT), 0, stream, weights, B, sc);
  hipLaunchKernelGGL(k_sr_center, dim3(gp), dim3(256), 0, stream, jac, B, P, weights, sc);
  hipLaunchKernelGGL(k_sr_init, dim3(gp), dim3(256), 0, stream, grad, P, x, r, p);
  TDO_HIP(hipGetLastError());
  TDO_TRY(dot(grad, grad, sc + 1));
  TDO_TRY(dot(grad, grad, sc + 4));
  for (int32_t it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_sr_rows, dim3(gr), dim3(kT), 0, stream, jac, R, P, p, up);
    hipLaunchKernelGGL(k_sr_usum, dim3((unsigned)std::min<int64_t>(ceil_div(R, 256), 1024)), dim3(256), 0, stream,
                       up, R, u);
    hipLaunchKernelGGL(k_sr_cols, dim3(gp), dim3(256), 0, stream, jac, R, P, u, p, lambda, Ap);
    TDO_TRY(dot(p, Ap, sc + 2));
    hipLaunchKernelGGL(k_sr_step, dim3(gp), dim3(256), 0, stream, P, sc, p, Ap, x, r);
    TDO_TRY(dot(r, r, sc + 3));
    hipLaunchKernelGGL(k_sr_dir, dim3(gp), dim3(256), 0, stream, P, sc, r, p);
    hipLaunchKernelGGL(k_sr_roll, dim3(1), dim3(64), 0, stream, sc);
    TDO_HIP(hipGetLastError());
  }
  if (info) {
    hipLaunchKernelGGL(k_sr_info, dim3(1), dim3(64), 0, stream, sc, info);
    TDO_HIP(hipGetLastError());
  }
  return TDO_OK;
}

// S p = Re sum_b w_b conj(dO_b) (dO_b . p) with t_b = O_b . p from the forward-mode pass:
// sum_b w_b t_b conj... = J^T J p is the reverse-mode product with the seeds w_b (t_b - mean_w t)
// (the mean term vanishes against the centring of O).
extern "C" int32_t tdo_sr_solve_matfree(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n,
                                        const uint64_t* cfg, int64_t B, const double* weights, tdo_prec_t prec,
                                        const double* grad, double lambda, int32_t iters, double* x, double* info,
                                        hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan npj, npv;
  TDO_TRY(jvp_check(ctx->c, arch, n, B, &npj));
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &npv));
  TDO_CHECK(B >= 1, TDO_EINVAL, "B=%lld < 1", (long long)B);
  TDO_CHECK(lambda > 0.0 && std::isfinite(lambda), TDO_EINVAL, "diagonal shift lambda=%g must be positive", lambda);
  TDO_CHECK(iters >= 0, TDO_EINVAL, "iters=%d < 0", iters);
  TDO_CHECK(params && cfg && grad && x, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, npj.pp.nparams, stream));
  const int64_t P = npj.pp.nparams;
  // CG vectors and scalars, the per-sample tangents and seeds, the forward-mode buffers (at
  // most a third of the rest of the budget), then the reverse-mode plan in what remains
  Arena ar;
  const size_t or_ = ar.take<double>((size_t)P), op = ar.take<double>((size_t)P), oap = ar.take<double>((size_t)P);
  const size_t osc = ar.take<double>(16), opart = ar.take<double>(kDotParts);
  const size_t ot = ar.take<float>(2 * (size_t)B), oseed = ar.take<float>(2 * (size_t)B);
  TDO_CHECK(c.budget > ar.used + 4096, TDO_ENOMEM, "workspace budget %zu too small", c.budget);
  JvpWs j;
  TDO_TRY(plan_jvp(npj, B, (c.budget - ar.used) / 3, ar, &j));
  TrainWs t;
  TDO_TRY(plan_train_at(c, npv, B, 1, ar.used, c.budget, &t));
  TDO_TRY(ensure_workspace(&c, t.total));
  void* ws = c.ws;
  double *r = at<double>(ws, or_), *p = at<double>(ws, op), *Ap = at<double>(ws, oap), *sc = at<double>(ws, osc);
  double* part = at<double>(ws, opart);
  float *tv = at<float>(ws, ot), *seed = at<float>(ws, oseed), *tanf = at<float>(ws, j.tanf);
  const unsigned gp = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(P, 256), 4096));
  const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(B, 256), 4096));
  auto dot = [&](const double* a, const double* b, double* out) -> int32_t {
    hipLaunchKernelGGL(k_sr_dot, dim3(kDotParts), dim3(kT), 0, stream, a, b, P, part);
    hipLaunchKernelGGL(k_sr_dot_fin, dim3(1), dim3(kT), 0, stream, part, out);
    TDO_HIP(hipGetLastError());
    return TDO_OK;
  };
  {  // the reverse-mode weight fragments, packed once
    NetWeights w = weights_at(ws, t.woff);
    TDO_TRY(pack_weights(npv, params, &w, stream));
    TDO_TRY(launch_pack_backward(npv.pp, params, npv.bf16, at<char>(ws, t.wback), stream));
  }
  // sc: [1] rs, [2] p.Ap, [3] rs_new, [4] g.g, [8..10] weight sum and weighted tangent sums
  hipLaunchKernelGGL(k_sr_init, dim3(gp), dim3(256), 0, stream, grad, P, x, r, p);
  TDO_HIP(hipGetLastError());
  TDO_TRY(dot(grad, grad, sc + 1));
  TDO_TRY(dot(grad, grad, sc + 4));
  for (int32_t it = 0; it < iters; ++it) {
    TDO_TRY(jvp_tangent_f32(p, P, tanf, stream));
    TDO_TRY(run_jvp(npj, ws, j, params, cfg, B, tv, stream));
    hipLaunchKernelGGL(k_mf_mean, dim3(1), dim3(kT), 0, stream, tv, weights, B, sc + 8);
    hipLaunchKernelGGL(k_mf_seeds, dim3(gb), dim3(256), 0, stream, tv, weights, B, sc + 8, seed);
    TDO_HIP(hipGetLastError());
    TDO_TRY(vjp_run(c, npv, t, params, cfg, B, seed, Ap, true, stream));
    hipLaunchKernelGGL(k_mf_shift, dim3(gp), dim3(256), 0, stream, P, lambda, p, Ap);
    TDO_HIP(hipGetLastError());
    TDO_TRY(dot(p, Ap, sc + 2));
    hipLaunchKernelGGL(k_sr_step, dim3(gp), dim3(256), 0, stream, P, sc, p, Ap, x, r);
    TDO_TRY(dot(r, r, sc + 3));
    hipLaunchKernelGGL(k_sr_dir, dim3(gp), dim3(256), 0, stream, P, sc, r, p);
    hipLaunchKernelGGL(k_sr_roll, dim3(1), dim3(64), 0, stream, sc);
    TDO_HIP(hipGetLastError());
  }
  if (info) {
    hipLaunchKernelGGL(k_sr_info, dim3(1), dim3(64), 0, stream, sc, info);
    TDO_HIP(hipGetLastError());
  }
  return TDO_OK;
}
