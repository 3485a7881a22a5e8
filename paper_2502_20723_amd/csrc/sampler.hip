// Metropolis-Hastings sampling of configurations x = (alpha, beta) from
// P(x) ~ |rho(x)|^2 (App. C, "Efficient Sampling Strategy"): a local move of
// the doubled configuration is proposed and accepted with probability
// min(1, |rho(x')|^2 / |rho(x)|^2) = min(1, exp(2 Re(log rho(x') - log rho(x)))).
//
// Moves (symmetric, each its own inverse): with probability p_pair flip alpha_i
// and beta_i together at a uniform site i; otherwise flip one uniform bit of
// the 2n bits (alpha first).  The pair move keeps parity(alpha) -
// parity(beta), which single flips cannot do in one step.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), one block per proposal and
// chain, counter (t mod 2^32, t >> 32, chain, 0), key (seed mod 2^32,
// seed >> 32); words r0 (move kind), r1 (site or bit), r2 (acceptance).
//
// One proposal for all chains of a chunk is: propose (one thread per chain),
// the forward pass of the network over the proposed configurations (the same
// layer kernels as tdo_log_rho), and accept (one thread per chain).
//
// The diagonal chain samples alpha from P(alpha) ~ |rho(alpha, alpha)|, the
// distribution of the mixed-state observable estimators (supplementary section
// on mixed-state observables).  A proposal flips one uniform site of alpha,
// i = (r1 n) >> 32, in both halves of (alpha, alpha), and is accepted iff
// (r2 + 0.5) 2^-32 < exp(Re log rho(alpha', alpha') - Re log rho(alpha, alpha)).
// Its Philox counter is (t mod 2^32, t >> 32, chain, 1): word 3 = 1 keeps it
// apart from the doubled-space chain's stream.  One sweep is n proposals.
#include <algorithm>

#include "common.h"
#include "netapi.h"
#include "train.h"

namespace tdo {

namespace {

struct Philox4x32 {
  uint32_t c[4];
};

// Philox4x32 with 10 rounds: each round forms the 64-bit products of counter
// words 0 and 2 with the two round multipliers, then mixes their high halves
// with counter words 1 and 3 and the round key; the key is bumped by the two
// Weyl increments between rounds.
__device__ __forceinline__ Philox4x32 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
  constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
  constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kMul0 * c0, p1 = (uint64_t)kMul1 * c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  return Philox4x32{{c0, c1, c2, c3}};
}

}  // namespace

__global__ void k_propose(const uint64_t* __restrict__ state, int64_t C, int64_t chain0, int n, uint64_t t,
                          uint64_t seed, uint64_t pair_thr, uint64_t* __restrict__ prop, double* __restrict__ u) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x) {
    const Philox4x32 r = philox10((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)(chain0 + c), 0u, (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    uint64_t a = state[2 * c], b = state[2 * c + 1];
    if ((uint64_t)r.c[0] < pair_thr) {
      const int i = (int)(((uint64_t)r.c[1] * (uint64_t)n) >> 32);
      a ^= 1ull << i;
      b ^= 1ull << i;
    } else {
      const int j = (int)(((uint64_t)r.c[1] * (uint64_t)(2 * n)) >> 32);
      if (j < n) a ^= 1ull << j;
      else b ^= 1ull << (j - n);
    }
    prop[2 * c] = a;
    prop[2 * c + 1] = b;
    u[c] = ((double)r.c[2] + 0.5) * 0x1p-32;
  }
}

// Accept iff u < exp(2 Re(log rho(x') - log rho(x))), compared in FP64; after the
// last proposal of a sweep the state is recorded.
__global__ void k_accept(int64_t C, const uint64_t* __restrict__ prop, const double* __restrict__ u,
                         const float* __restrict__ lrp, uint64_t* __restrict__ state, float* __restrict__ state_lr,
                         uint64_t* __restrict__ record) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x) {
    const double ratio = exp(2.0 * ((double)lrp[2 * c] - (double)state_lr[2 * c]));
    if (u[c] < ratio) {
      state[2 * c] = prop[2 * c];
      state[2 * c + 1] = prop[2 * c + 1];
      state_lr[2 * c] = lrp[2 * c];
      state_lr[2 * c + 1] = lrp[2 * c + 1];
    }
    if (record) {
      record[2 * c] = state[2 * c];
      record[2 * c + 1] = state[2 * c + 1];
    }
  }
}

__global__ void k_propose_diag(const uint64_t* __restrict__ state, int64_t C, int64_t chain0, int n, uint64_t t,
                               uint64_t seed, uint64_t* __restrict__ prop, double* __restrict__ u) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x) {
    const Philox4x32 r = philox10((uint32_t)t, (uint32_t)(t >> 32), (uint32_t)(chain0 + c), 1u, (uint32_t)seed,
                                  (uint32_t)(seed >> 32));
    const int i = (int)(((uint64_t)r.c[1] * (uint64_t)n) >> 32);
    const uint64_t a = state[c] ^ (1ull << i);
    prop[2 * c] = a;
    prop[2 * c + 1] = a;
    u[c] = ((double)r.c[2] + 0.5) * 0x1p-32;
  }
}

// Accept iff u < |rho(alpha')| / |rho(alpha)| = exp(Re log rho' - Re log rho), in FP64.
__global__ void k_accept_diag(int64_t C, const uint64_t* __restrict__ prop, const double* __restrict__ u,
                              const float* __restrict__ lrp, uint64_t* __restrict__ state,
                              float* __restrict__ state_lr, uint64_t* __restrict__ record) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x) {
    const double ratio = exp((double)lrp[2 * c] - (double)state_lr[2 * c]);
    if (u[c] < ratio) {
      state[c] = prop[2 * c];
      state_lr[2 * c] = lrp[2 * c];
      state_lr[2 * c + 1] = lrp[2 * c + 1];
    }
    if (record) record[c] = state[c];
  }
}

namespace {

// Workspace of a chain driver: packed weights, then per chain chunk the
// proposals, uniforms, z, log rho and residuals.
struct ChainWs {
  size_t woff[4], oprop, ou, oz, olr, oxa, oxb;
  int64_t chunk;
};

int32_t plan_chains(Context& c, const NetPlan& np, int64_t chains, ChainWs* cw) {
  Arena ar;
  carve_weights(np, ar, cw->woff);
  const size_t fixed = ar.used + 4096;
  const double per_chain = 16.0 + 8.0 + 16.0 + 8.0 + 2.0 * 32.0 * np.D * 4.0 * (np.span ? 4.0 : 2.0 / np.cpb) + 64.0;
  TDO_CHECK(c.budget > fixed + 64 * per_chain, TDO_ENOMEM, "workspace budget %zu too small", c.budget);
  int64_t chunk = std::min<int64_t>(chains, (int64_t)((double)(c.budget - fixed) / per_chain));
  cw->chunk = chunk = std::max<int64_t>(1, chunk);
  cw->oprop = ar.take<uint64_t>(2 * (size_t)chunk);
  cw->ou = ar.take<double>((size_t)chunk);
  cw->oz = ar.take<float>(4 * (size_t)chunk);
  cw->olr = ar.take<float>(2 * (size_t)chunk);
  const int64_t nblk = blocks_for(np, chunk);
  cw->oxa = ar.take<float>((size_t)nblk * 32 * np.D);
  cw->oxb = ar.take<float>((size_t)nblk * 32 * np.D);
  TDO_TRY(ensure_workspace(&c, ar.used));
  return TDO_OK;
}

}  // namespace

}  // namespace tdo

using namespace tdo;

extern "C" int32_t tdo_sample(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n, int64_t chains,
                              uint64_t* state, float* state_log_rho, uint64_t seed, uint64_t* counter, int32_t sweeps,
                              float p_pair, tdo_prec_t prec, uint64_t* samples, hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  TDO_CHECK(chains >= 0 && sweeps >= 0, TDO_EINVAL, "chains=%lld, sweeps=%d", (long long)chains, sweeps);
  TDO_CHECK(counter != nullptr, TDO_EINVAL, "counter is NULL");
  TDO_CHECK(p_pair >= 0.f && p_pair <= 1.f, TDO_EINVAL, "p_pair=%g outside [0, 1]", (double)p_pair);
  TDO_CHECK(chains < (int64_t(1) << 32), TDO_EINVAL, "chains=%lld: the chain index is one 32-bit counter word",
            (long long)chains);
  const uint64_t per_call = (uint64_t)sweeps * 2u * (uint64_t)n;
  if (chains == 0 || sweeps == 0) {
    *counter += per_call;
    return TDO_OK;
  }
  TDO_CHECK(params && state && state_log_rho && samples, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  ChainWs cw;
  TDO_TRY(plan_chains(c, np, chains, &cw));
  const int64_t chunk = cw.chunk;
  const size_t oprop = cw.oprop, ou = cw.ou, oz = cw.oz, olr = cw.olr, oxa = cw.oxa, oxb = cw.oxb;
  void* ws = c.ws;
  NetWeights w = weights_at(ws, cw.woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  const double thr_d = std::floor((double)p_pair * 4294967296.0);
  const uint64_t pair_thr = (uint64_t)std::min(thr_d, 4294967296.0);
  uint64_t* prop = at<uint64_t>(ws, oprop);
  double* u = at<double>(ws, ou);
  float* lrp = at<float>(ws, olr);
  for (int64_t c0 = 0; c0 < chains; c0 += chunk) {
    const int64_t Cc = std::min(chunk, chains - c0);
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(Cc, 256), 4096);
    uint64_t t = *counter;
    for (int32_t s = 0; s < sweeps; ++s) {
      for (int p = 0; p < 2 * n; ++p, ++t) {
        hipLaunchKernelGGL(k_propose, dim3(grid), dim3(256), 0, stream, state + 2 * c0, Cc, c0, n, t, seed, pair_thr,
                           prop, u);
        TDO_HIP(hipGetLastError());
        TDO_TRY(run_forward(np, w, prop, Cc, nullptr, at<float>(ws, oxa), at<float>(ws, oxb), nullptr,
                            at<float>(ws, oz), stream));
        TDO_TRY(launch_symmetrise(nullptr, Cc, at<float>(ws, oz), lrp, stream));
        uint64_t* rec = (p == 2 * n - 1) ? samples + ((size_t)s * chains + c0) * 2 : nullptr;
        hipLaunchKernelGGL(k_accept, dim3(grid), dim3(256), 0, stream, Cc, prop, u, lrp, state + 2 * c0,
                           state_log_rho + 2 * c0, rec);
        TDO_HIP(hipGetLastError());
      }
    }
  }
  *counter += per_call;
  return TDO_OK;
}

extern "C" int32_t tdo_sample_diag(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n,
                                   int64_t chains, uint64_t* state, float* state_log_rho, uint64_t seed,
                                   uint64_t* counter, int32_t sweeps, tdo_prec_t prec, uint64_t* samples,
                                   hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  TDO_CHECK(chains >= 0 && sweeps >= 0, TDO_EINVAL, "chains=%lld, sweeps=%d", (long long)chains, sweeps);
  TDO_CHECK(counter != nullptr, TDO_EINVAL, "counter is NULL");
  TDO_CHECK(chains < (int64_t(1) << 32), TDO_EINVAL, "chains=%lld: the chain index is one 32-bit counter word",
            (long long)chains);
  const uint64_t per_call = (uint64_t)sweeps * (uint64_t)n;
  if (chains == 0 || sweeps == 0) {
    *counter += per_call;
    return TDO_OK;
  }
  TDO_CHECK(params && state && state_log_rho && samples, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  ChainWs cw;
  TDO_TRY(plan_chains(c, np, chains, &cw));
  void* ws = c.ws;
  NetWeights w = weights_at(ws, cw.woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  uint64_t* prop = at<uint64_t>(ws, cw.oprop);
  double* u = at<double>(ws, cw.ou);
  float* lrp = at<float>(ws, cw.olr);
  for (int64_t c0 = 0; c0 < chains; c0 += cw.chunk) {
    const int64_t Cc = std::min(cw.chunk, chains - c0);
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(Cc, 256), 4096);
    uint64_t t = *counter;
    for (int32_t s = 0; s < sweeps; ++s) {
      for (int p = 0; p < n; ++p, ++t) {
        hipLaunchKernelGGL(k_propose_diag, dim3(grid), dim3(256), 0, stream, state + c0, Cc, c0, n, t, seed, prop,
                           u);
        TDO_HIP(hipGetLastError());
        TDO_TRY(run_forward(np, w, prop, Cc, nullptr, at<float>(ws, cw.oxa), at<float>(ws, cw.oxb), nullptr,
                            at<float>(ws, cw.oz), stream));
        TDO_TRY(launch_symmetrise(nullptr, Cc, at<float>(ws, cw.oz), lrp, stream));
        uint64_t* rec = (p == n - 1) ? samples + (size_t)s * chains + c0 : nullptr;
        hipLaunchKernelGGL(k_accept_diag, dim3(grid), dim3(256), 0, stream, Cc, prop, u, lrp, state + c0,
                           state_log_rho + 2 * c0, rec);
        TDO_HIP(hipGetLastError());
      }
    }
  }
  *counter += per_call;
  return TDO_OK;
}
