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
// Validation and workspace plan of one loss/gradient evaluation (grows the workspace).
int32_t loss_grad_check(const Context& c, const tdo_arch_t* arch, const tdo_model_t* model, int64_t B, tdo_prec_t prec,
                        int32_t grad_mode, ModelDev* m, NetPlan* np, TrainWs* t);
// The launch sequence of one loss/gradient evaluation on a planned workspace.
int32_t loss_grad_run(Context& c, const NetPlan& np, const ModelDev& m, const TrainWs& t, const float* params,
                      const uint64_t* cfg, int64_t B, const double* weights, int32_t grad_mode, double* loss,
                      double* grad, float* lloc_out, hipStream_t stream);

int32_t net_plan(const Context* c, const tdo_arch_t* arch, int n, bool bf16, NetPlan* np);
int64_t blocks_for(const NetPlan& np, int64_t E);
int32_t pack_weights(const NetPlan& np, const float* params, NetWeights* w, hipStream_t st);
void carve_weights(const NetPlan& np, Arena& ar, size_t* offs);
NetWeights weights_at(void* ws, const size_t* offs);
int32_t run_forward(const NetPlan& np, const NetWeights& w, const uint64_t* ecfg, int64_t E, const int64_t* E_dev,
                    float* xa, float* xb, const Saves* sv, float* z, hipStream_t st);

}  // namespace tdo
