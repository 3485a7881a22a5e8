// Host-visible argument blocks and launchers of the network kernels.
#pragma once

#include "common.h"

namespace tdo {

struct FwdArgs {
  const void* wpack;            // this layer's packed weights (BF16 or FP32 fragments)
  const float* b1;              // [M] (padded)
  const float* b2;              // [D] (padded)
  const float* table;           // first layer: embedding table [64][D]
  const uint64_t* ecfg;         // first layer: configurations [E][2]
  const int64_t* n_entries_dev; // E on the device, or NULL to use n_entries
  int64_t n_entries;
  const float* x_in;            // residual in, [blocks][D/32][64][16] (not first layer)
  float* x_out;                 // residual out (not last layer)
  void* save_x;                 // optional: layer input saved for the backward pass
  void* save_mid;               // optional: input of the feed-forward sub-layer
  void* save_last;              // optional (last layer): output x_L
  const float* head_w;          // last layer: [d][2]
  const float* head_b;          // last layer: [2]
  float* z;                     // last layer: [E][2 passes][2]
  int n, cpb, d_real, M;
  float score_scale;            // log2(e) / sqrt(d/heads)
  int first, last, masked, blocks_per_cu;
};

int32_t launch_fwd_layer(const FwdArgs& a, bool bf16, int D, int DH, bool span, int num_cus, hipStream_t st);
int32_t launch_embed_table(const float* params, int d, int D, float* table, hipStream_t st);
int32_t launch_symmetrise(const int64_t* E_dev, int64_t E_host, const float* z, float* lr, hipStream_t st);

// Packing of the flat parameter vector into per-layer MFMA fragments.
struct PackPlan {
  int d, D, heads, layers, mlp, M;
  int64_t off_conv1, off_conv2_b, off_layer0, layer_stride, off_head_w, off_head_b;
  int64_t nparams;
  int64_t layer_elems;  // packed elements per layer (forward fragments)
};
int32_t make_pack_plan(const tdo_arch_t* arch, PackPlan* pp);
// Writes L layers of forward fragments (elem = bf16 if bf16 else f32) and padded
// biases b1 [L][M], b2 [L][D].
int32_t launch_pack_forward(const PackPlan& pp, const float* params, bool bf16, void* wpack, float* b1,
                            float* b2, hipStream_t st);

}  // namespace tdo
