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
};

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
};

int32_t net_plan(const Context* c, const tdo_arch_t* arch, int n, bool bf16, NetPlan* np);
int64_t blocks_for(const NetPlan& np, int64_t E);
int32_t pack_weights(const NetPlan& np, const float* params, NetWeights* w, hipStream_t st);
void carve_weights(const NetPlan& np, Arena& ar, size_t* offs);
NetWeights weights_at(void* ws, const size_t* offs);
int32_t run_forward(const NetPlan& np, const NetWeights& w, const uint64_t* ecfg, int64_t E, const int64_t* E_dev,
                    float* xa, float* xb, const Saves* sv, float* z, hipStream_t st);

}  // namespace tdo
