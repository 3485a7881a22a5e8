// Host-side plans shared by the forward, backward and sampling drivers.
#pragma once

#include <cmath>

#include "common.h"
#include "netapi.h"

namespace tdo {

struct NetPlan {
  PackPlan pp;
  bool bf16, span, masked;
  int D, DH, n, cpb, elem, num_cus;
  float score_scale;
  Profiler* prof;
  int fwd_wg_per_cu;  // workgroups per CU of the forward layer kernel (autotuned, default 1)
  int fwd_waves;      // waves per workgroup of the forward layer kernel: 8 (BF16, n <= 32) or 4 (autotuned)
  int mlp_waves;      // waves per workgroup of the BF16 feed-forward backward at mlp 256: 8 or 4 (autotuned)
};

inline uint64_t tune_key(const NetPlan& np) {
  return (uint64_t)np.n | ((uint64_t)np.bf16 << 8) | ((uint64_t)np.D << 16) | ((uint64_t)np.DH << 24) |
         ((uint64_t)np.pp.layers << 32) | ((uint64_t)np.pp.M << 40);
}

struct NetWeights {
  void* wpack;       // [L][layer_elems] forward fragments
  float* b1;         // [L][M]
  float* b2;         // [L][D]
  float* table;      // [64][D]
  const float* head_w;
  const float* head_b;
};

// Activations kept for the backward pass, block-major in the register layout.
struct Saves {
  void* x;            // [L] layer inputs
  void* mid;          // [L] feed-forward inputs
  void* last;         // output of the last layer
  size_t layer_bytes; // bytes of one layer's buffer
  float* lse;         // [L][blocks][32 rows][D/DH heads]: log2 of each attention row's softmax
                      // normaliser (BF16 path; NULL otherwise)
  size_t lse_layer;   // floats of one layer's part
};

// Workspace plan shared by the loss/gradient and VJP drivers.
struct TrainWs {
  size_t woff[4], wback, gA, Lall, acc, lpart, mlp_acc, attn_acc, dT_acc, partial;
  size_t cnt, off, etot, ecfg, ecoef, eowner, lr, z, dF, xa, xb, sx, smid, slast, slse;
  int64_t chunk, emax, nblk;
  size_t layer_bytes, lse_layer;
  size_t total;  // bytes of the whole plan
};

struct ModelDev;
int32_t plan_train(const Context& c, const NetPlan& np, int64_t B, int nslots, TrainWs* t);
// The same layout starting at byte offset base of the workspace, within cap bytes in all; allocates nothing.
int32_t plan_train_at(const Context& c, const NetPlan& np, int64_t B, int nslots, size_t base, size_t cap,
                      TrainWs* t);
// tdo_log_rho_vjp's launch sequence on a planned workspace (packed: weight fragments already packed).
int32_t vjp_run(Context& c, const NetPlan& np, const TrainWs& t, const float* params, const uint64_t* cfg, int64_t B,
                const float* seed, double* grad, bool packed, hipStream_t stream);
// Validation and workspace plan of one loss/gradient evaluation (grows the workspace).
int32_t loss_grad_check(const Context& c, const tdo_arch_t* arch, const tdo_model_t* model, int64_t B, tdo_prec_t prec,
                        int32_t grad_mode, ModelDev* m, NetPlan* np, TrainWs* t);
// The launch sequence of one loss/gradient evaluation on a planned workspace.
int32_t loss_grad_run(Context& c, const NetPlan& np, const ModelDev& m, const TrainWs& t, const float* params,
                      const uint64_t* cfg, int64_t B, const double* weights, int32_t grad_mode, double* loss,
                      double* grad, float* lloc_out, hipStream_t stream);

int32_t net_plan(const Context* c, const tdo_arch_t* arch, int n, bool bf16, NetPlan* np);

// Forward-mode pass (jvp.hip): buffers for chunks of ec configurations, laid out by plan_jvp
// from ar.used on within max_bytes (the FP32 tangent of the parameters first).
struct JvpWs {
  int64_t ec = 0;
  size_t tanf, T, Td, X, Xd, Y, Yd, Q, K, V, Qd, Kd, Vd, O, Od, H, Hd, z, zd;
};
int32_t plan_jvp(const NetPlan& np, int64_t B, size_t max_bytes, Arena& ar, JvpWs* j);
// out[e] (re, im) = d log rho(cfg[e]) along the tangent held at ws + j.tanf (FP32).
int32_t run_jvp(const NetPlan& np, void* ws, const JvpWs& j, const float* params, const uint64_t* cfg, int64_t B,
                float* out, hipStream_t st);
int32_t jvp_check(const Context& c, const tdo_arch_t* arch, int32_t n, int64_t B, NetPlan* np);
int32_t jvp_tangent_f32(const double* p, int64_t P, float* out, hipStream_t st);
int64_t blocks_for(const NetPlan& np, int64_t E);
int32_t pack_weights(const NetPlan& np, const float* params, NetWeights* w, hipStream_t st);
void carve_weights(const NetPlan& np, Arena& ar, size_t* offs);
NetWeights weights_at(void* ws, const size_t* offs);
int32_t run_forward(const NetPlan& np, const NetWeights& w, const uint64_t* ecfg, int64_t E, const int64_t* E_dev,
                    float* xa, float* xb, const Saves* sv, float* z, hipStream_t st);

}  // namespace tdo
