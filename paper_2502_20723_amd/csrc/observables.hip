// Mixed-state observables and purity of the ansatz.
//
// Observables (supplementary section on mixed-state observables; App. C,
// evaluation of local observables): <A> = sum_alpha P(alpha) A~(alpha) with
// P(alpha) = rho(alpha, alpha) / Tr rho and
// A~(alpha) = sum_beta rho(alpha, beta) / rho(alpha, alpha) <beta|A|alpha>.
// For the Pauli operators at site i (bit 0 = spin up, s_i = 1 - 2 bit_i) the
// only beta with a nonzero element are alpha itself and alpha^(i), alpha with
// site i flipped:
//   sigma^z_i: A~ = s_i;
//   sigma^x_i: A~ = r_i = rho(alpha, alpha^(i)) / rho(alpha, alpha);
//   sigma^y_i: A~ = i s_i r_i  (<down|sigma^y|up> = i, <up|sigma^y|down> = -i).
// One sample therefore needs n + 1 network evaluations: the rows
// (alpha, alpha), (alpha, alpha^(0)), ..., (alpha, alpha^(n-1)), evaluated by
// the same forward kernels as tdo_log_rho, then combined per sample.
//
// The ansatz is Hermitian but not forced positive, so rho(alpha, alpha) is real
// with either sign.  Samples are taken from |rho(alpha, alpha)| and the sign s
// is carried as a weight: <A> = sum s A~ / sum s.  A sample with
// rho(alpha, alpha) = 0 has sign 0; its r_i are read as 0.
//
// Purity (Ising section): Tr rho^2 / (Tr rho)^2 = E[t] / E[s]^2 over
// independent pairs (alpha, beta) from |rho(alpha, alpha)|, with
// t = |rho(alpha, beta)|^2 / (|rho(alpha, alpha)| |rho(beta, beta)|), by
// Hermiticity rho(beta, alpha) = conj rho(alpha, beta).  Three rows per pair.
//
// Sums over samples are in FP64, by one workgroup in a fixed order, so that
// results do not depend on scheduling.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "netapi.h"
#include "train.h"

namespace tdo {

namespace {

constexpr int kRedThreads = 256;

__device__ __forceinline__ float diag_sign(float re, float im) {
  // log rho(alpha, alpha) = log|rho| + i pi when rho(alpha, alpha) < 0
  return (re == -INFINITY) ? 0.f : (fabsf(im) > 1.5707964f ? -1.f : 1.f);
}

template <int K>
__device__ void block_sum(double (&acc)[K], double* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < K; ++k) red[k * kRedThreads + t] = acc[k];
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int k = 0; k < K; ++k) red[k * kRedThreads + t] += red[k * kRedThreads + t + h];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = red[k * kRedThreads];
}

}  // namespace

// Rows of S samples: row s (n + 1) + j is (alpha_s, alpha_s) for j = 0 and
// (alpha_s, alpha_s with site j - 1 flipped) otherwise.
__global__ void k_obs_rows(const uint64_t* __restrict__ alpha, int64_t S, int n, uint64_t* __restrict__ cfg) {
  const int64_t E = S * (n + 1);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / (n + 1);
    const int j = (int)(e - s * (n + 1));
    const uint64_t a = alpha[s];
    cfg[2 * e] = a;
    cfg[2 * e + 1] = j ? (a ^ (1ull << (j - 1))) : a;
  }
}

// One thread per sample: the site averages (1/n) sum_i of the local estimators,
// local[s] = (x re, x im, y re, y im, z re, z im), log rho(alpha, alpha), and
// optionally the estimators of every site, site[s][i] in the same layout.
__global__ void k_obs_local(const float* __restrict__ lr, const uint64_t* __restrict__ alpha, int64_t S, int n,
                            float* __restrict__ lrd, float* __restrict__ local, float* __restrict__ site) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
    const float* l = lr + 2 * s * (n + 1);
    const float d_re = l[0], d_im = l[1];
    const bool zero = d_re == -INFINITY;
    const uint64_t a = alpha[s];
    double xr = 0, xi = 0, yr = 0, yi = 0;
    int z = 0;
    for (int i = 0; i < n; ++i) {
      const int si = ((a >> i) & 1ull) ? -1 : 1;
      z += si;
      const float o_re = l[2 + 2 * i], o_im = l[3 + 2 * i];
      double rr = 0.0, ri = 0.0;
      if (!zero && o_re != -INFINITY) {
        const double m = exp((double)o_re - (double)d_re);
        double sn, cs;
        sincos((double)o_im - (double)d_im, &sn, &cs);
        rr = m * cs;
        ri = m * sn;
      }
      xr += rr;
      xi += ri;
      yr -= si * ri;  // i s_i (rr + i ri)
      yi += si * rr;
      if (site) {  // per site: (x, y, z) as (re, im)
        float* q = site + (s * n + i) * 6;
        q[0] = (float)rr;
        q[1] = (float)ri;
        q[2] = (float)(-si * ri);
        q[3] = (float)(si * rr);
        q[4] = (float)si;
        q[5] = 0.f;
      }
    }
    const double inv = 1.0 / n;
    lrd[2 * s] = d_re;
    lrd[2 * s + 1] = d_im;
    float* o = local + 6 * s;
    o[0] = (float)(xr * inv);
    o[1] = (float)(xi * inv);
    o[2] = (float)(yr * inv);
    o[3] = (float)(yi * inv);
    o[4] = (float)((double)z / n);  // correctly rounded: exact up to the FP32 store
    o[5] = 0.f;
  }
}

// One workgroup: mean[0..5] = sum s local / sum s (x, y, z as re, im),
// mean[6] = sum s / B.
__global__ void __launch_bounds__(kRedThreads) k_obs_mean(const float* __restrict__ lrd,
                                                          const float* __restrict__ local, int64_t B,
                                                          double* __restrict__ mean) {
  __shared__ double red[7 * kRedThreads];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < B; b += kRedThreads) {
    const float sg = diag_sign(lrd[2 * b], lrd[2 * b + 1]);
    if (sg == 0.f) continue;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += (double)sg * (double)local[6 * b + k];
    acc[6] += sg;
  }
  block_sum(acc, red);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 6; ++k) mean[k] = acc[k] / acc[6];
    mean[6] = acc[6] / (double)B;
  }
}

// Rows of P pairs: (alpha, beta), (alpha, alpha), (beta, beta).
__global__ void k_pur_rows(const uint64_t* __restrict__ alpha, const uint64_t* __restrict__ beta, int64_t P,
                           uint64_t* __restrict__ cfg) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t a = alpha[p], b = beta[p];
    cfg[6 * p] = a;
    cfg[6 * p + 1] = b;
    cfg[6 * p + 2] = a;
    cfg[6 * p + 3] = a;
    cfg[6 * p + 4] = b;
    cfg[6 * p + 5] = b;
  }
}

// t = |rho(a,b)|^2 / (|rho(a,a)| |rho(b,b)|) (0 when either diagonal vanishes)
// and s(a) + s(b).
__global__ void k_pur_terms(const float* __restrict__ lr, int64_t P, double* __restrict__ term,
                            float* __restrict__ sgn) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
    const float* l = lr + 6 * p;
    const float sa = diag_sign(l[2], l[3]), sb = diag_sign(l[4], l[5]);
    const bool vanish = sa == 0.f || sb == 0.f || l[0] == -INFINITY;
    term[p] = vanish ? 0.0 : exp(2.0 * (double)l[0] - (double)l[2] - (double)l[4]);
    sgn[p] = sa + sb;
  }
}

// out[0] = (sum t / P) / (sum s / 2P)^2, out[1] = sum s / 2P.
__global__ void __launch_bounds__(kRedThreads) k_pur_mean(const double* __restrict__ term,
                                                          const float* __restrict__ sgn, int64_t P,
                                                          double* __restrict__ out) {
  __shared__ double red[2 * kRedThreads];
  double acc[2] = {0, 0};
  for (int64_t p = threadIdx.x; p < P; p += kRedThreads) {
    acc[0] += term[p];
    acc[1] += sgn[p];
  }
  block_sum(acc, red);
  if (threadIdx.x == 0) {
    const double ms = acc[1] / (2.0 * (double)P);
    out[0] = (acc[0] / (double)P) / (ms * ms);
    out[1] = ms;
  }
}

namespace {

// Workspace of a chunked evaluation of `rows` network rows per item: packed
// weights, then per chunk the row configurations, residuals, z and log rho.
struct RowPlan {
  size_t woff[4], ocfg, oxa, oxb, oz, olr, tail;
  int64_t chunk;  // items per chunk
};

int32_t plan_rows(Context& c, const NetPlan& np, int64_t items, int rows, size_t tail_bytes, RowPlan* rp) {
  Arena ar;
  carve_weights(np, ar, rp->woff);
  rp->tail = ar.take<char>(tail_bytes);
  const size_t fixed = ar.used + 4096;
  const size_t per_block = 32 * (size_t)np.D * 4;
  const double per_row = 2.0 * per_block * (np.span ? 4.0 : 2.0 / np.cpb) + 16.0 + 16.0 + 8.0 + 64.0;
  const double per_item = per_row * rows;
  TDO_CHECK(c.budget > fixed + 8 * per_block + 64 * per_item, TDO_ENOMEM, "workspace budget %zu too small",
            c.budget);
  int64_t chunk = (int64_t)((double)(c.budget - fixed - 8 * per_block) / per_item);
  chunk = std::max<int64_t>(1, std::min<int64_t>(chunk, items));
  rp->chunk = chunk;
  const int64_t E = chunk * rows;
  rp->ocfg = ar.take<uint64_t>(2 * (size_t)E);
  const int64_t nblk = blocks_for(np, E);
  rp->oxa = ar.take<float>((size_t)nblk * 32 * np.D);
  rp->oxb = ar.take<float>((size_t)nblk * 32 * np.D);
  rp->oz = ar.take<float>(4 * (size_t)E);
  rp->olr = ar.take<float>(2 * (size_t)E);
  TDO_TRY(ensure_workspace(&c, ar.used));
  return TDO_OK;
}

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), 4096)); }

}  // namespace

}  // namespace tdo

using namespace tdo;

extern "C" {

int32_t tdo_observables(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n,
                        const uint64_t* alpha, int64_t B, tdo_prec_t prec, float* log_rho_diag, float* local,
                        float* local_site, double* mean, hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  TDO_CHECK(B >= 0, TDO_EINVAL, "B=%lld < 0", (long long)B);
  TDO_CHECK(B > 0 || mean == nullptr, TDO_EINVAL, "a mean over no samples");
  if (B == 0) return TDO_OK;
  TDO_CHECK(params && alpha && log_rho_diag && local, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  RowPlan rp;
  TDO_TRY(plan_rows(c, np, B, n + 1, 0, &rp));
  void* ws = c.ws;
  NetWeights w = weights_at(ws, rp.woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  uint64_t* cfg = at<uint64_t>(ws, rp.ocfg);
  float* lr = at<float>(ws, rp.olr);
  for (int64_t s0 = 0; s0 < B; s0 += rp.chunk) {
    const int64_t S = std::min(rp.chunk, B - s0);
    const int64_t E = S * (n + 1);
    hipLaunchKernelGGL(k_obs_rows, dim3(grid_for(E)), dim3(256), 0, stream, alpha + s0, S, (int)n, cfg);
    TDO_HIP(hipGetLastError());
    TDO_TRY(run_forward(np, w, cfg, E, nullptr, at<float>(ws, rp.oxa), at<float>(ws, rp.oxb), nullptr,
                        at<float>(ws, rp.oz), stream));
    TDO_TRY(launch_symmetrise(nullptr, E, at<float>(ws, rp.oz), lr, stream));
    hipLaunchKernelGGL(k_obs_local, dim3(grid_for(S)), dim3(256), 0, stream, lr, alpha + s0, S, (int)n,
                       log_rho_diag + 2 * s0, local + 6 * s0, local_site ? local_site + 6 * s0 * n : nullptr);
    TDO_HIP(hipGetLastError());
  }
  if (mean) {
    hipLaunchKernelGGL(k_obs_mean, dim3(1), dim3(kRedThreads), 0, stream, log_rho_diag, local, B, mean);
    TDO_HIP(hipGetLastError());
  }
  return TDO_OK;
}

int32_t tdo_purity(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n, const uint64_t* alpha,
                   const uint64_t* beta, int64_t P, tdo_prec_t prec, double* out, hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  TDO_CHECK(P >= 1, TDO_EINVAL, "P=%lld: a mean over no pairs", (long long)P);
  TDO_CHECK(params && alpha && beta && out, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  RowPlan rp;
  const size_t tail = (size_t)P * (sizeof(double) + sizeof(float)) + 256;
  TDO_TRY(plan_rows(c, np, P, 3, tail, &rp));
  void* ws = c.ws;
  NetWeights w = weights_at(ws, rp.woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  double* term = at<double>(ws, rp.tail);
  float* sgn = reinterpret_cast<float*>(term + P);
  uint64_t* cfg = at<uint64_t>(ws, rp.ocfg);
  float* lr = at<float>(ws, rp.olr);
  for (int64_t p0 = 0; p0 < P; p0 += rp.chunk) {
    const int64_t Q = std::min(rp.chunk, P - p0);
    const int64_t E = 3 * Q;
    hipLaunchKernelGGL(k_pur_rows, dim3(grid_for(Q)), dim3(256), 0, stream, alpha + p0, beta + p0, Q, cfg);
    TDO_HIP(hipGetLastError());
    TDO_TRY(run_forward(np, w, cfg, E, nullptr, at<float>(ws, rp.oxa), at<float>(ws, rp.oxb), nullptr,
                        at<float>(ws, rp.oz), stream));
    TDO_TRY(launch_symmetrise(nullptr, E, at<float>(ws, rp.oz), lr, stream));
    hipLaunchKernelGGL(k_pur_terms, dim3(grid_for(Q)), dim3(256), 0, stream, lr, Q, term + p0, sgn + p0);
    TDO_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_pur_mean, dim3(1), dim3(kRedThreads), 0, stream, term, sgn, P, out);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // extern "C"
