// Packing of the flat parameter vector (layout of tdo_num_params) into the
// per-layer MFMA fragment order of net.h, zero-padded to width D = max(32, d).
#include "common.h"
#include "net.h"
#include "netapi.h"

namespace tdo {

int32_t make_pack_plan(const tdo_arch_t* arch, PackPlan* pp) {
  TDO_CHECK(arch != nullptr, TDO_EINVAL, "arch is NULL");
  const int d = arch->d, H = arch->heads, L = arch->layers, m = arch->mlp;
  TDO_CHECK(d == 16 || d == 32 || d == 64, TDO_EUNSUPPORTED, "width d=%d not in {16, 32, 64}", d);
  TDO_CHECK(H >= 1 && d % H == 0, TDO_EINVAL, "heads=%d does not divide d=%d", H, d);
  TDO_CHECK(d / H == 8 || d / H == 16, TDO_EUNSUPPORTED, "head width d/heads=%d not in {8, 16}", d / H);
  TDO_CHECK(m >= 32 && m % 32 == 0 && m <= 512, TDO_EUNSUPPORTED, "mlp=%d must be a multiple of 32 in [32, 512]", m);
  TDO_CHECK(L >= 1 && L <= 16, TDO_EUNSUPPORTED, "layers=%d not in [1, 16]", L);
  TDO_CHECK(arch->c1 == 0 || arch->c1 == d, TDO_EUNSUPPORTED,
            "conv-1 width c1=%d: the kernels implement c1 = d (0 selects it)", arch->c1);
  TDO_CHECK(arch->act == TDO_ACT_RELU_FFN, TDO_EUNSUPPORTED,
            "activation set %d: the kernels implement TDO_ACT_RELU_FFN (0) only", arch->act);
  PackPlan p{};
  p.d = d;
  p.D = d < 32 ? 32 : d;
  p.heads = H;
  p.layers = L;
  p.mlp = m;
  p.M = m;
  p.off_conv1 = 0;
  p.off_conv2_b = 5LL * d + 2LL * d * d;
  p.off_layer0 = 6LL * d + 2LL * d * d;
  p.layer_stride = 4LL * d * d + 2LL * d * m + m + d;
  p.off_head_w = p.off_layer0 + (int64_t)L * p.layer_stride;
  p.off_head_b = p.off_head_w + 2LL * d;
  p.nparams = p.off_head_b + 2;
  p.layer_elems = 4LL * p.D * p.D + 2LL * p.D * p.M;
  *pp = p;
  return TDO_OK;
}

// Fragments of the layer matrices (bwd = false): Wq, Wk, Wv, Wo [D][D], W1 [D][M],
// W2 [M][D]; or of their transposes (bwd = true), used by the backward pass:
// Wq^T, Wk^T, Wv^T, Wo^T [D][D], W2^T [D][M], W1^T [M][D].
template <int KPL, class T>
__global__ void k_pack(const float* __restrict__ params, PackPlan pp, bool bwd, T* __restrict__ out,
                       float* __restrict__ b1o, float* __restrict__ b2o) {
  constexpr int ST = 32 / (2 * KPL);
  const int D = pp.D, M = pp.M, d = pp.d;
  const int64_t total = pp.layer_elems * pp.layers;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e / pp.layer_elems);
    int64_t k = e % pp.layer_elems;
    const float* lp = params + pp.off_layer0 + l * pp.layer_stride;
    // Packed matrix A[in][out], in < in_p (padded).  Forward: A = W, W[rows][cols]
    // row-major with rows = in, cols = out.  Backward: A = W^T, A[in][out] = W[out][in].
    const float* src;
    int in_p, wrows, wcols;
    if (k < 4LL * D * D) {
      const int mt = (int)(k / ((int64_t)D * D));
      k -= (int64_t)mt * D * D;
      src = lp + (int64_t)mt * d * d;
      in_p = D; wrows = d; wcols = d;
    } else if (k < 4LL * D * D + (int64_t)D * M) {
      k -= 4LL * D * D;
      if (!bwd) { src = lp + 4LL * d * d; in_p = D; wrows = d; wcols = M; }                      // W1 [d][M]
      else { src = lp + 4LL * d * d + (int64_t)d * M + M; in_p = D; wrows = M; wcols = d; }      // W2^T, W2 [M][d]
    } else {
      k -= 4LL * D * D + (int64_t)D * M;
      if (!bwd) { src = lp + 4LL * d * d + (int64_t)d * M + M; in_p = M; wrows = M; wcols = d; } // W2 [M][d]
      else { src = lp + 4LL * d * d; in_p = M; wrows = d; wcols = M; }                           // W1^T, W1 [d][M]
    }
    const int frag = (int)(k / (64 * KPL));
    const int rem = (int)(k % (64 * KPL));
    const int lane = rem / KPL, t = rem % KPL;
    const int s = frag % ST;
    const int ib = (frag / ST) % (in_p / 32);
    const int ob = frag / (ST * (in_p / 32));
    const int in = 32 * ib + tile_idx(s * KPL + t, lane >> 5);
    const int o = 32 * ob + (lane & 31);
    float v = 0.0f;
    if (!bwd) {
      if (in < wrows && o < wcols) v = src[(int64_t)in * wcols + o];
    } else {
      if (o < wrows && in < wcols) v = src[(int64_t)o * wcols + in];
    }
    out[e] = (T)v;
  }
  if (bwd) return;
  // biases (padded): b1 [L][M], b2 [L][D]
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)pp.layers * (M + D);
       e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e / (M + D));
    const int k = (int)(e % (M + D));
    const float* lp = params + pp.off_layer0 + l * pp.layer_stride;
    if (k < M) b1o[(int64_t)l * M + k] = lp[4LL * d * d + (int64_t)d * M + k];
    else {
      const int o = k - M;
      b2o[(int64_t)l * D + o] = o < d ? lp[4LL * d * d + 2LL * d * M + M + o] : 0.0f;
    }
  }
}

static int32_t launch_pack(const PackPlan& pp, const float* params, bool bf16, bool bwd, void* wpack, float* b1,
                           float* b2, hipStream_t st) {
  const int64_t total = pp.layer_elems * pp.layers;
  const int blocks = (int)std::min<int64_t>(ceil_div(total, 256), 4096);
  if (bf16)
    hipLaunchKernelGGL((k_pack<8, __bf16>), dim3(blocks), dim3(256), 0, st, params, pp, bwd, (__bf16*)wpack, b1, b2);
  else
    hipLaunchKernelGGL((k_pack<1, float>), dim3(blocks), dim3(256), 0, st, params, pp, bwd, (float*)wpack, b1, b2);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_pack_forward(const PackPlan& pp, const float* params, bool bf16, void* wpack, float* b1,
                            float* b2, hipStream_t st) {
  return launch_pack(pp, params, bf16, false, wpack, b1, b2, st);
}

int32_t launch_pack_backward(const PackPlan& pp, const float* params, bool bf16, void* wpack, hipStream_t st) {
  return launch_pack(pp, params, bf16, true, wpack, nullptr, nullptr, st);
}

}  // namespace tdo
