// Cost and gradient of the samples (App. C, "Optimization Procedure";
// Eq. lossnetk), the vector-Jacobian product of log rho, and their drivers.
//
// Gradient estimator (the paper's printed gradient line is garbled; this is
// the gradient, at fixed samples, of the self-normalised reweighted cost):
//   grad_B = [ 2 Re sum_b w_b conj(L_b) sum_k c_k e^{lr(y_k) - lr(x_b)} O(y_k)
//              - 2 F sum_b w_b Re O(x_b) ] / W,      O = d log rho / d theta,
// F = sum_b w_b |L_b|^2 / W, W = sum_b w_b.  The fixed-weight gradient is
//   grad_A = [ same first sum - 2 sum_b w_b |L_b|^2 Re O(x_b) ] / W,
// and grad_B = grad_A + 2 sum_b w_b (|L_b|^2 - F) Re O(x_b) / W.  Both are
// computed in that form: one VJP of log rho over every evaluated
// configuration with complex seeds g_k (plus the real seed -2 w_b |L_b|^2 on
// the sample's own entry), and for mode B a second VJP over the samples with
// the centred real seeds 2 w_b (|L_b|^2 - F) once F is known.  Writing B as
// A plus a centred term avoids subtracting two nearly equal sums.
//
// Seeds on log rho = log(e^{z1} + conj e^{z2}) split over the two passes as
//   pass (alpha, beta): (dF0, dF1) = (Re(g s1), -Im(g s1)),
//   pass (beta, alpha): (dF0, dF1) = (Re(g s2), +Im(g s2)),
// s1 = e^{z1}/(e^{z1} + conj e^{z2}), s2 = 1 - s1, for the seed convention
// Re(g * d log rho).
#include <algorithm>

#include "common.h"
#include "lindblad.h"
#include "netapi.h"
#include "train.h"

namespace tdo {

__device__ __forceinline__ void lse_split(float gre, float gim, const float* __restrict__ z, float* __restrict__ out) {
  const float a1 = z[0], b1 = z[1], a2 = z[2], b2 = z[3];
  const float mx = fmaxf(a1, a2);
  float s, c;
  const float e1 = expf(a1 - mx), e2 = expf(a2 - mx);
  sincosf(b1, &s, &c);
  const float w1r = e1 * c, w1i = e1 * s;
  sincosf(-b2, &s, &c);  // conj(e^{z2})
  const float w2r = e2 * c, w2i = e2 * s;
  const float Sr = w1r + w2r, Si = w1i + w2i;
  const float nn = Sr * Sr + Si * Si;
  if (!(nn > 0.f) || !isfinite(nn)) { out[0] = out[1] = out[2] = out[3] = 0.f; return; }
  // s1 = w1 / S, s2 = w2 / S
  const float s1r = (w1r * Sr + w1i * Si) / nn, s1i = (w1i * Sr - w1r * Si) / nn;
  const float s2r = (w2r * Sr + w2i * Si) / nn, s2i = (w2i * Sr - w2r * Si) / nn;
  const float t1r = gre * s1r - gim * s1i, t1i = gre * s1i + gim * s1r;
  const float t2r = gre * s2r - gim * s2i, t2i = gre * s2i + gim * s2r;
  out[0] = t1r; out[1] = -t1i; out[2] = t2r; out[3] = t2i;
}

// VJP seeds: seed (dRe, dIm) on log rho -> g = dRe - i dIm.
// Seeds of one configuration for d(s_re Re log rho + s_im Im log rho) (the
// Jacobian rows).
__global__ void k_seeds_const(float s_re, float s_im, const float* __restrict__ z, float* __restrict__ dF) {
  if (blockIdx.x == 0 && threadIdx.x == 0) lse_split(s_re, -s_im, z, dF);
}

__global__ void k_seeds_vjp(const float* __restrict__ seed, const float* __restrict__ z, int64_t E, float* __restrict__ dF) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x)
    lse_split(seed[2 * e], -seed[2 * e + 1], z + 4 * e, dF + 4 * e);
}

// Seeds of the first sum: g_k = 2 w_b conj(L_b) c_k e^{lr_k - lr_x(b)}, plus
// -2 w_b |L_b|^2 on the sample's own entry (k = 0).
__global__ void k_seeds_loss(const int64_t* __restrict__ E_dev, const int32_t* __restrict__ owner,
                             const int64_t* __restrict__ off, const float* __restrict__ coef,
                             const float* __restrict__ lr, const float* __restrict__ L, const double* __restrict__ w,
                             int64_t w0, const float* __restrict__ z, float* __restrict__ dF) {
  const int64_t E = *E_dev;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = owner[e];
    const int64_t ex = off[b];
    const float xr = lr[2 * ex], xi = lr[2 * ex + 1];
    float gre = 0.f, gim = 0.f;
    if (!(isinf(xr) && xr < 0.f)) {
      const float wb = w ? (float)w[w0 + b] : 1.0f;
      const float Lr = L[2 * b], Li = L[2 * b + 1];
      const float er = expf(lr[2 * e] - xr);
      float sn, cs;
      sincosf(lr[2 * e + 1] - xi, &sn, &cs);
      const float cr = coef[2 * e], ci = coef[2 * e + 1];
      const float tr = (cr * cs - ci * sn) * er, ti = (cr * sn + ci * cs) * er;  // c e^{dlr}
      gre = 2.f * wb * (Lr * tr + Li * ti);  // 2 w conj(L) t
      gim = 2.f * wb * (Lr * ti - Li * tr);
      if (e == ex) gre -= 2.f * wb * (Lr * Lr + Li * Li);
    }
    lse_split(gre, gim, z + 4 * e, dF + 4 * e);
  }
}

// Centred real seeds 2 w_b (|L_b|^2 - F) on log rho(x_b), F = acc[0] / acc[1].
__global__ void k_seeds_centred(int64_t E, const double* __restrict__ w, int64_t w0, const float* __restrict__ L,
                                const double* __restrict__ acc, const float* __restrict__ z, float* __restrict__ dF) {
  const double F = acc[1] > 0 ? acc[0] / acc[1] : 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const double wb = w ? w[w0 + e] : 1.0;
    const double l2 = (double)L[2 * e] * L[2 * e] + (double)L[2 * e + 1] * L[2 * e + 1];
    lse_split((float)(2.0 * wb * (l2 - F)), 0.f, z + 4 * e, dF + 4 * e);
  }
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// loss = F, grad = g / W.
__global__ void k_finalize(const double* __restrict__ acc, const double* __restrict__ g, int64_t P,
                           double* __restrict__ loss, double* __restrict__ grad) {
  const double W = acc[1];
  if (blockIdx.x == 0 && threadIdx.x == 0) loss[0] = W > 0 ? acc[0] / W : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x)
    grad[i] = W > 0 ? g[i] / W : 0.0;
}

static int32_t fill(double* p, int64_t n, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 1024)), dim3(256), 0, st, p, n, v);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

// ------------------------------------------------------------------ backward driver
struct BwdBufs {
  void* wback;       // [L][layer_elems] transposed fragments
  float* ga;         // gradient ping-pong, [blocks][D/32][64][16]
  float* gb;
  float* partial;    // [nparts][maxlen]
  int nparts;
  double* mlp_acc;   // [2DM + M + D]
  double* attn_acc;  // [4 D^2]
  double* dT_acc;    // [64 D]
};

static int32_t run_backward(const NetPlan& np, const NetWeights& w, const BwdBufs& bb, const float* params,
                            const uint64_t* ecfg, int64_t E, const int64_t* E_dev, const Saves& sv, const float* dF,
                            double* gt, hipStream_t st) {
  const PackPlan& pp = np.pp;
  const int L = pp.layers, D = np.D, M = pp.M;
  const int64_t mlen = 2LL * D * M + M + D, alen = 4LL * D * D;
  for (int l = L - 1; l >= 0; --l) {
    BwdArgs a{};
    a.wf = static_cast<const char*>(w.wpack) + (size_t)l * pp.layer_elems * np.elem;
    a.wb = static_cast<const char*>(bb.wback) + (size_t)l * pp.layer_elems * np.elem;
    a.b1 = w.b1 + (size_t)l * M;
    a.save_x = static_cast<const char*>(sv.x) + (size_t)l * sv.layer_bytes;
    a.save_mid = static_cast<const char*>(sv.mid) + (size_t)l * sv.layer_bytes;
    a.lse = sv.lse ? sv.lse + (size_t)l * sv.lse_layer : nullptr;
    a.w1 = params + pp.off_layer0 + (int64_t)l * pp.layer_stride + 4LL * pp.d * pp.d;
    a.w2 = a.w1 + (int64_t)pp.d * pp.mlp + pp.mlp;
    a.head_w = w.head_w;
    a.partial = bb.partial;
    a.n_entries_dev = E_dev;
    a.n_entries = E;
    a.n = np.n;
    a.cpb = np.cpb;
    a.span = np.span;
    a.masked = np.masked;
    a.d_real = pp.d;
    a.M = M;
    a.score_scale = np.score_scale;
    a.inv_sqrt_dh = (float)(1.0 / std::sqrt((double)np.DH));
    a.mlp_waves = np.mlp_waves;
    // feed-forward sub-layer: gradient in ga (or from the seeds), out to gb
    a.g_in = (l == L - 1) ? nullptr : bb.ga;
    a.seeds = (l == L - 1) ? dF : nullptr;
    a.g_out = bb.gb;
    TDO_TRY(fill(bb.mlp_acc, mlen, 0.0, st));
    TDO_TRY(fill(bb.attn_acc, alen, 0.0, st));
    {
      ProfScope ps(np.prof, "bwd_mlp", st);
      if (np.bf16 && bwd_mlp_bf16_supported(pp.d, D, M))
        TDO_TRY(launch_bwd_mlp_bf16(a, bb.nparts, st));
      else
        TDO_TRY(launch_bwd_mlp(a, np.bf16, D, bb.nparts, st));
    }
    TDO_TRY(launch_reduce_partials(bb.partial, bb.nparts, mlen, bb.mlp_acc, st));
    // attention sub-layer: gb -> ga
    a.g_in = bb.gb;
    a.seeds = nullptr;
    a.g_out = bb.ga;
    int attn_parts = bb.nparts;
    {
      ProfScope ps(np.prof, "bwd_attn", st);
      if (np.bf16 && bwd_attn_bf16_supported(pp.d, D, np.DH, np.span)) {
        TDO_TRY(launch_bwd_attn_bf16(a, np.DH, bb.nparts, st));
        attn_parts = bwd_attn_bf16_parts(bb.nparts, np.span);
      } else {
        TDO_TRY(launch_bwd_attn(a, np.bf16, D, np.DH, bb.nparts, st));
      }
    }
    TDO_TRY(launch_reduce_partials(bb.partial, attn_parts, alen, bb.attn_acc, st));
    TDO_TRY(launch_scatter_layer(bb.mlp_acc, bb.attn_acc, pp.d, D, M, 1.0, gt + pp.off_layer0 + l * pp.layer_stride, st));
  }
  // the head kernel's workgroup slots reuse the partial buffer (free here; sized for them in plan_train)
  TDO_TRY(launch_bwd_head(np.bf16, D, sv.last, dF, E_dev, E, np.n, np.cpb, np.span, pp.d, gt + pp.off_head_w,
                          gt + pp.off_head_b, reinterpret_cast<double*>(bb.partial), st));
  // table gradient accumulated over every call of this entry point; the chain rule into the
  // convolution parameters (linear in it) runs once at the end (finish_backward)
  // two workgroups per CU (each wave a partial): the second one's waves hide the first's latencies
  TDO_TRY(launch_embed_scatter(D, bb.ga, ecfg, E_dev, E, np.n, np.cpb, np.span, bb.partial, 2 * bb.nparts, st));
  TDO_TRY(launch_reduce_partials(bb.partial, 8 * bb.nparts, 64LL * D, bb.dT_acc, st));
  return TDO_OK;
}

static int32_t finish_backward(const NetPlan& np, const BwdBufs& bb, const float* params, double* gt, hipStream_t st) {
  // the per-code slots reuse the partial buffer, idle at this point (sized for them in plan_train)
  return launch_embed_params(params, bb.dT_acc, np.pp.d, np.D, gt, reinterpret_cast<double*>(bb.partial), st);
}


int32_t plan_train_at(const Context& c, const NetPlan& np, int64_t B, int nslots, size_t base, size_t cap,
                      TrainWs* t) {
  const PackPlan& pp = np.pp;
  TDO_CHECK(bwd_mlp_lds(np.D, pp.M) <= 160 * 1024, TDO_EUNSUPPORTED,
            "backward of width %d with mlp %d exceeds the LDS of a workgroup", np.D, pp.M);
  Arena ar;
  ar.used = (base + 255) & ~size_t(255);
  carve_weights(np, ar, t->woff);
  t->wback = ar.take<char>((size_t)pp.layer_elems * pp.layers * np.elem);
  t->gA = ar.take<double>(pp.nparams);
  t->Lall = ar.take<float>(2 * B);
  t->acc = ar.take<double>(2);
  t->lpart = ar.take<double>(2 * LOSS_PARTS);
  const int64_t mlen = 2LL * np.D * pp.M + pp.M + np.D;
  t->mlp_acc = ar.take<double>(mlen);
  t->attn_acc = ar.take<double>(4LL * np.D * np.D);
  t->dT_acc = ar.take<double>(64LL * np.D);
  // per CU: the feed-forward weight partials, the attention weight partials of up to two workgroups,
  // or 8 wave partials of the table gradient; in all, at least the FP64 per-code slots of the
  // embedding chain rule and the head kernel's workgroup slots
  const int64_t maxlen = std::max<int64_t>(std::max<int64_t>(std::max<int64_t>(mlen, 2 * 4LL * np.D * np.D), 8 * 64LL * np.D),
                                           std::max<int64_t>(2 * 64 * (6LL * pp.d + 2LL * pp.d * pp.d),
                                                             2LL * HEAD_BLOCKS * (2 * pp.d + 2)) /
                                                   c.num_cus + 1);
  t->partial = ar.take<float>((size_t)c.num_cus * maxlen);
  const size_t fixed = ar.used + 64 * 256;  // includes the per-sample L buffer
  const int save = np.bf16 ? 2 : 4;
  const double blocks_per_entry = np.span ? 4.0 : 2.0 / np.cpb;
  const bool keep_lse = np.bf16;  // consumed by the BF16 attention backward
  const double per_block = 32.0 * np.D * (2 * 4 + (2 * pp.layers + 1) * save) +
                           (keep_lse ? (double)pp.layers * 32 * (np.D / np.DH) * 4 : 0.0);
  const double per_entry = blocks_per_entry * per_block + 80.0;
  const double per_sample = nslots * per_entry + 32.0;
  TDO_CHECK(cap > fixed + per_sample + 8 * per_block, TDO_ENOMEM,
            "workspace budget %zu bytes cannot hold one sample (%.0f bytes) and the fixed part (%zu bytes)", cap,
            per_sample, fixed);
  int64_t chunk = (int64_t)((double)(cap - fixed - 8 * per_block) / per_sample);
  chunk = std::max<int64_t>(1, std::min(chunk, B));
  t->chunk = chunk;
  t->emax = chunk * nslots;
  t->nblk = blocks_for(np, t->emax);
  t->cnt = ar.take<int32_t>(chunk);
  t->off = ar.take<int64_t>(chunk);
  t->etot = ar.take<int64_t>(1);
  t->ecfg = ar.take<uint64_t>(2 * t->emax);
  t->ecoef = ar.take<float>(2 * t->emax);
  t->eowner = ar.take<int32_t>(t->emax);
  t->lr = ar.take<float>(2 * t->emax);
  t->z = ar.take<float>(4 * t->emax);
  t->dF = ar.take<float>(4 * t->emax);
  const size_t xbytes = (size_t)t->nblk * 32 * np.D;
  t->xa = ar.take<float>(xbytes);
  t->xb = ar.take<float>(xbytes);
  t->layer_bytes = ((size_t)t->nblk * 32 * np.D * save + 255) & ~size_t(255);
  t->sx = ar.take<char>(t->layer_bytes * pp.layers);
  t->smid = ar.take<char>(t->layer_bytes * pp.layers);
  t->slast = ar.take<char>(t->layer_bytes);
  t->lse_layer = keep_lse ? (size_t)t->nblk * 32 * (np.D / np.DH) : 0;
  t->slse = ar.take<float>(t->lse_layer * pp.layers + 64);
  t->total = ar.used;
  return TDO_OK;
}

int32_t plan_train(const Context& c, const NetPlan& np, int64_t B, int nslots, TrainWs* t) {
  TDO_TRY(plan_train_at(c, np, B, nslots, 0, c.budget, t));
  return ensure_workspace(const_cast<Context*>(&c), t->total);
}

// The launch sequence of tdo_log_rho_vjp on a planned workspace: grad = sum_b seed_b . d log rho(x_b).
// With packed set, the forward and transposed weight fragments are taken as already packed.
int32_t vjp_run(Context& c, const NetPlan& np, const TrainWs& t, const float* params, const uint64_t* cfg, int64_t B,
                const float* seed, double* grad, bool packed, hipStream_t stream) {
  void* ws = c.ws;
  NetWeights w = weights_at(ws, t.woff);
  if (!packed) {
    TDO_TRY(pack_weights(np, params, &w, stream));
    TDO_TRY(launch_pack_backward(np.pp, params, np.bf16, at<char>(ws, t.wback), stream));
  } else {
    w.head_w = params + np.pp.off_head_w;
    w.head_b = params + np.pp.off_head_b;
  }
  TDO_TRY(fill(grad, np.pp.nparams, 0.0, stream));
  TDO_TRY(fill(at<double>(ws, t.dT_acc), 64LL * np.D, 0.0, stream));
  BwdBufs bb{at<char>(ws, t.wback), at<float>(ws, t.xa), at<float>(ws, t.xb), at<float>(ws, t.partial), c.num_cus,
             at<double>(ws, t.mlp_acc), at<double>(ws, t.attn_acc), at<double>(ws, t.dT_acc)};
  Saves sv{at<char>(ws, t.sx), at<char>(ws, t.smid), at<char>(ws, t.slast), t.layer_bytes,
           t.lse_layer ? at<float>(ws, t.slse) : nullptr, t.lse_layer};
  for (int64_t e0 = 0; e0 < B; e0 += t.chunk) {
    const int64_t E = std::min(t.chunk, B - e0);
    const uint64_t* ec = cfg + 2 * e0;
    TDO_TRY(run_forward(np, w, ec, E, nullptr, at<float>(ws, t.xa), at<float>(ws, t.xb), &sv, at<float>(ws, t.z), stream));
    hipLaunchKernelGGL(k_seeds_vjp, dim3(256), dim3(256), 0, stream, seed + 2 * e0, at<float>(ws, t.z), E, at<float>(ws, t.dF));
    TDO_HIP(hipGetLastError());
    TDO_TRY(run_backward(np, w, bb, params, ec, E, nullptr, sv, at<float>(ws, t.dF), grad, stream));
  }
  return finish_backward(np, bb, params, grad, stream);
}

}  // namespace tdo

using namespace tdo;

extern "C" int32_t tdo_log_rho_vjp(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n,
                                   const uint64_t* cfg, int64_t B, tdo_prec_t prec, const float* seed, double* grad,
                                   hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  TDO_CHECK(B >= 0, TDO_EINVAL, "B=%lld < 0", (long long)B);
  TDO_CHECK(params && grad && (B == 0 || (cfg && seed)), TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  TrainWs t;
  TDO_TRY(plan_train(c, np, std::max<int64_t>(B, 1), 1, &t));
  return vjp_run(c, np, t, params, cfg, B, seed, grad, false, stream);
}

// Per-sample log-derivatives: per configuration one forward, then one backward
// per part (Re, Im) with the launch sequence of tdo_log_rho_vjp on one
// configuration, on weights packed once.
extern "C" int32_t tdo_log_rho_jacobian(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n,
                                        const uint64_t* cfg, int64_t B, tdo_prec_t prec, double* jac,
                                        hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  TDO_CHECK(B >= 0, TDO_EINVAL, "B=%lld < 0", (long long)B);
  if (B == 0) return TDO_OK;
  TDO_CHECK(params && cfg && jac, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  TrainWs t;
  TDO_TRY(plan_train(c, np, 1, 1, &t));
  // kLanes independent copies of the one-configuration scratch, each driven on its
  // own stream (a single configuration occupies a few workgroups); the packed
  // weights of copy 0 are shared
  constexpr int kLanes = 4;
  const int lanes = (int)std::min<int64_t>(kLanes, B);
  const size_t stride = (t.total + 4095) & ~size_t(4095);
  TDO_TRY(ensure_workspace(&c, stride * lanes));
  char* ws0 = static_cast<char*>(c.ws);
  NetWeights w = weights_at(ws0, t.woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  TDO_TRY(launch_pack_backward(np.pp, params, np.bf16, at<char>(ws0, t.wback), stream));
  const int64_t P = np.pp.nparams;
  hipStream_t st[kLanes];
  hipEvent_t ev[kLanes + 1];
  int made_st = 0, made_ev = 0;
  int32_t rc = TDO_OK;
  auto cleanup = [&]() {
    for (int i = 0; i < made_st; ++i) (void)hipStreamDestroy(st[i]);
    for (int i = 0; i < made_ev; ++i) (void)hipEventDestroy(ev[i]);
  };
#define JAC_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      rc = set_error(TDO_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));                \
      cleanup();                                                                              \
      return rc;                                                                              \
    }                                                                                         \
  } while (0)
  for (int i = 0; i <= lanes; ++i, ++made_ev) JAC_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  for (int i = 0; i < lanes; ++i, ++made_st) JAC_HIP(hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking));
  JAC_HIP(hipEventRecord(ev[lanes], stream));  // packed weights ready
  for (int i = 0; i < lanes; ++i) JAC_HIP(hipStreamWaitEvent(st[i], ev[lanes], 0));
  for (int64_t b = 0; b < B && rc == TDO_OK; ++b) {
    const int lane = (int)(b % lanes);
    hipStream_t s = st[lane];
    char* ws = ws0 + stride * lane;
    BwdBufs bb{at<char>(ws0, t.wback), at<float>(ws, t.xa), at<float>(ws, t.xb), at<float>(ws, t.partial), c.num_cus,
               at<double>(ws, t.mlp_acc), at<double>(ws, t.attn_acc), at<double>(ws, t.dT_acc)};
    Saves sv{at<char>(ws, t.sx), at<char>(ws, t.smid), at<char>(ws, t.slast), t.layer_bytes,
             t.lse_layer ? at<float>(ws, t.slse) : nullptr, t.lse_layer};
    // one forward per configuration: the backward only reads the saved activations and z
    rc = run_forward(np, w, cfg + 2 * b, 1, nullptr, at<float>(ws, t.xa), at<float>(ws, t.xb), &sv,
                     at<float>(ws, t.z), s);
    for (int part = 0; part < 2 && rc == TDO_OK; ++part) {
      double* row = jac + (2 * b + part) * P;
      rc = fill(row, P, 0.0, s);
      if (rc == TDO_OK) rc = fill(at<double>(ws, t.dT_acc), 64LL * np.D, 0.0, s);
      if (rc == TDO_OK) {
        hipLaunchKernelGGL(k_seeds_const, dim3(1), dim3(64), 0, s, part == 0 ? 1.f : 0.f, part == 1 ? 1.f : 0.f,
                           at<float>(ws, t.z), at<float>(ws, t.dF));
        if (hipGetLastError() != hipSuccess) rc = set_error(TDO_EHIP, "k_seeds_const launch failed");
      }
      if (rc == TDO_OK) rc = run_backward(np, w, bb, params, cfg + 2 * b, 1, nullptr, sv, at<float>(ws, t.dF), row, s);
      if (rc == TDO_OK) rc = finish_backward(np, bb, params, row, s);
    }
  }
  // join: the caller's stream waits for every lane (also after an error, so that
  // nothing still runs on the scratch when the call returns)
  for (int i = 0; i < lanes; ++i) {
    if (hipEventRecord(ev[i], st[i]) == hipSuccess) (void)hipStreamWaitEvent(stream, ev[i], 0);
  }
  for (int i = 0; i < lanes; ++i) (void)hipStreamSynchronize(st[i]);
#undef JAC_HIP
  cleanup();
  return rc;
}

namespace tdo {

int32_t loss_grad_check(const Context& c, const tdo_arch_t* arch, const tdo_model_t* model, int64_t B, tdo_prec_t prec,
                        int32_t grad_mode, ModelDev* m, NetPlan* np, TrainWs* t) {
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  TDO_CHECK(grad_mode == 0 || grad_mode == 1, TDO_EINVAL, "grad_mode %d not 0 (B) or 1 (A)", grad_mode);
  TDO_CHECK(model != nullptr, TDO_EINVAL, "model is NULL");
  TDO_TRY(make_model(model, m));
  TDO_TRY(net_plan(&c, arch, model->n, prec == TDO_BF16, np));
  TDO_CHECK(B >= 1, TDO_EINVAL, "B=%lld < 1", (long long)B);
  return plan_train(c, *np, B, m->nslots, t);
}

int32_t loss_grad_run(Context& c, const NetPlan& np, const ModelDev& m, const TrainWs& t, const float* params,
                      const uint64_t* cfg, int64_t B, const double* weights, int32_t grad_mode, double* loss,
                      double* grad, float* lloc_out, hipStream_t stream) {
  void* ws = c.ws;
  NetWeights w = weights_at(ws, t.woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  TDO_TRY(launch_pack_backward(np.pp, params, np.bf16, at<char>(ws, t.wback), stream));
  const int64_t P = np.pp.nparams;
  double* gA = at<double>(ws, t.gA);
  double* acc = at<double>(ws, t.acc);
  float* Lall = lloc_out ? lloc_out : at<float>(ws, t.Lall);
  TDO_TRY(fill(gA, P, 0.0, stream));
  TDO_TRY(fill(at<double>(ws, t.dT_acc), 64LL * np.D, 0.0, stream));
  TDO_TRY(fill(acc, 2, 0.0, stream));
  BwdBufs bb{at<char>(ws, t.wback), at<float>(ws, t.xa), at<float>(ws, t.xb), at<float>(ws, t.partial), c.num_cus,
             at<double>(ws, t.mlp_acc), at<double>(ws, t.attn_acc), at<double>(ws, t.dT_acc)};
  Saves sv{at<char>(ws, t.sx), at<char>(ws, t.smid), at<char>(ws, t.slast), t.layer_bytes,
           t.lse_layer ? at<float>(ws, t.slse) : nullptr, t.lse_layer};
  const int64_t* Ed = at<int64_t>(ws, t.etot);
  for (int64_t b0 = 0; b0 < B; b0 += t.chunk) {
    const int64_t Bc = std::min(t.chunk, B - b0);
    TDO_TRY(launch_eval_list(m, cfg + 2 * b0, Bc, at<int32_t>(ws, t.cnt), at<int64_t>(ws, t.off), at<int64_t>(ws, t.etot),
                             at<uint64_t>(ws, t.ecfg), at<float>(ws, t.ecoef), at<int32_t>(ws, t.eowner), stream));
    const uint64_t* ec = at<uint64_t>(ws, t.ecfg);
    TDO_TRY(run_forward(np, w, ec, t.emax, Ed, at<float>(ws, t.xa), at<float>(ws, t.xb), &sv, at<float>(ws, t.z), stream));
    TDO_TRY(launch_symmetrise(Ed, 0, at<float>(ws, t.z), at<float>(ws, t.lr), stream));
    float* Lb = Lall + 2 * b0;
    TDO_TRY(launch_lloc_eval(Bc, at<int64_t>(ws, t.off), at<int32_t>(ws, t.cnt), at<float>(ws, t.ecoef), at<float>(ws, t.lr),
                             Lb, stream));
    TDO_TRY(launch_loss_accum(Bc, Lb, weights ? weights + b0 : nullptr, at<double>(ws, t.lpart), acc, stream));
    hipLaunchKernelGGL(k_seeds_loss, dim3(1024), dim3(256), 0, stream, Ed, at<int32_t>(ws, t.eowner), at<int64_t>(ws, t.off),
                       at<float>(ws, t.ecoef), at<float>(ws, t.lr), Lb, weights, b0, at<float>(ws, t.z), at<float>(ws, t.dF));
    TDO_HIP(hipGetLastError());
    TDO_TRY(run_backward(np, w, bb, params, ec, t.emax, Ed, sv, at<float>(ws, t.dF), gA, stream));
  }
  if (grad_mode == 0) {  // + 2 sum_b w_b (|L_b|^2 - F) Re O(x_b), F known from the first pass
    // one entry per sample here: the buffers sized for emax entries hold emax samples
    const int64_t chunk2 = std::max<int64_t>(1, std::min<int64_t>(B, t.emax));
    for (int64_t b0 = 0; b0 < B; b0 += chunk2) {
      const int64_t Bc = std::min(chunk2, B - b0);
      const uint64_t* ec = cfg + 2 * b0;
      TDO_TRY(run_forward(np, w, ec, Bc, nullptr, at<float>(ws, t.xa), at<float>(ws, t.xb), &sv, at<float>(ws, t.z), stream));
      hipLaunchKernelGGL(k_seeds_centred, dim3(256), dim3(256), 0, stream, Bc, weights, b0, Lall + 2 * b0, acc,
                         at<float>(ws, t.z), at<float>(ws, t.dF));
      TDO_HIP(hipGetLastError());
      TDO_TRY(run_backward(np, w, bb, params, ec, Bc, nullptr, sv, at<float>(ws, t.dF), gA, stream));
    }
  }
  TDO_TRY(finish_backward(np, bb, params, gA, stream));
  hipLaunchKernelGGL(k_finalize, dim3(256), dim3(256), 0, stream, acc, gA, P, loss, grad);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // namespace tdo

extern "C" int32_t tdo_loss_grad(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, const tdo_model_t* model,
                                 const uint64_t* cfg, int64_t B, const double* weights, tdo_prec_t prec,
                                 int32_t grad_mode, double* loss, double* grad, float* lloc_out, hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_HIP(hipSetDevice(ctx->c.device));
  ModelDev m;
  NetPlan np;
  TrainWs t;
  TDO_TRY(loss_grad_check(ctx->c, arch, model, B, prec, grad_mode, &m, &np, &t));
  TDO_CHECK(params && cfg && loss && grad, TDO_EINVAL, "NULL buffer");
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  return loss_grad_run(c, np, m, t, params, cfg, B, weights, grad_mode, loss, grad, lloc_out, stream);
}
