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
  float* save_lse;              // optional (BF16): [blocks][32 rows][D/DH heads] log2 of
                                // each attention row's softmax normaliser (+inf for a row with no key)
  void* save_last;              // optional (last layer): output x_L
  const float* head_w;          // last layer: [d][2]
  const float* head_b;          // last layer: [2]
  float* z;                     // last layer: [E][2 passes][2]
  int n, cpb, d_real, M;
  float score_scale;            // log2(e) / sqrt(d/heads)
  int first, last, masked, blocks_per_cu;
  int waves;                    // waves per workgroup (4, or 8 for BF16 with n <= 32)
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
// L layers of transposed fragments: Wq^T, Wk^T, Wv^T, Wo^T [D][D], then W2^T [D][M], W1^T [M][D].
int32_t launch_pack_backward(const PackPlan& pp, const float* params, bool bf16, void* wpack, hipStream_t st);

}  // namespace tdo

namespace tdo {

struct BwdArgs {
  const void* wf;               // this layer's forward fragments
  const void* wb;               // this layer's transposed fragments
  const float* b1;              // [M]
  const float* w1;              // this layer's W1 [d][mlp] and W2 [mlp][d] in the flat FP32 parameters
  const float* w2;
  const void* save_x;           // layer input
  const void* save_mid;         // feed-forward input
  const float* lse;             // attention row normalisers saved by the forward (or NULL)
  const float* g_in;            // incoming gradient [blocks][D/32][64][16] (NULL: from seeds)
  const float* seeds;           // last layer: per configuration-pass (dF0, dF1), [E][2][2]
  const float* head_w;          // [d][2]
  float* g_out;                 // outgoing gradient
  float* partial;               // per-workgroup FP32 weight-gradient accumulators
  const int64_t* n_entries_dev;
  int64_t n_entries;
  int n, cpb, span, masked, d_real, M;
  float score_scale, inv_sqrt_dh;
  int mlp_waves;                // BF16 feed-forward backward at mlp 256: 8 or 4 waves per workgroup
};

size_t bwd_mlp_lds(int D, int M);
// Feed-forward backward with BF16 operands and per-wave register gradients (width 64).
bool bwd_mlp_bf16_supported(int d, int D, int M);
int32_t launch_bwd_mlp_bf16(const BwdArgs& a, int blocks, hipStream_t st);
// Attention backward with BF16 operands and per-wave register gradients (width 64, n <= 32).
bool bwd_attn_bf16_supported(int d, int D, int DH, bool span);
int32_t launch_bwd_attn_bf16(const BwdArgs& a, int DH, int blocks, hipStream_t st);
// weight-gradient partial slots [4 D^2] that launch_bwd_attn_bf16 writes for `blocks` (one per CU)
int bwd_attn_bf16_parts(int blocks, bool span);
int32_t launch_bwd_mlp(const BwdArgs& a, bool bf16, int D, int blocks, hipStream_t st);
int32_t launch_bwd_attn(const BwdArgs& a, bool bf16, int D, int DH, int blocks, hipStream_t st);
// part: FP64 scratch of HEAD_BLOCKS * (2 d_real + 2) values (one slot per workgroup).
constexpr int HEAD_BLOCKS = 1024;
int32_t launch_bwd_head(bool bf16, int D, const void* save_last, const float* seeds, const int64_t* E_dev,
                        int64_t E_host, int n, int cpb, int span, int d_real, double* gw, double* gb, double* part,
                        hipStream_t st);
int32_t launch_embed_scatter(int D, const float* dx0, const uint64_t* ecfg, const int64_t* E_dev, int64_t E_host,
                             int n, int cpb, int span, float* partial, int blocks, hipStream_t st);
// part: FP64 scratch of 64 * (6 d + 2 d^2) values (one slot per window code).
int32_t launch_embed_params(const float* params, const double* dT, int d, int D, double* grad, double* part,
                            hipStream_t st);
int32_t launch_reduce_partials(const float* part, int nparts, int64_t len, double* out, hipStream_t st);
int32_t launch_scatter_layer(const double* mlp, const double* attn, int d, int D, int M, double scale, double* g,
                             hipStream_t st);

}  // namespace tdo
