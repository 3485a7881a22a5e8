// Forward pass of the transformer density operator (main text "Transformer
// density operator ansatz"; App. B), one kernel launch per layer.
//
// Work decomposition.  The evaluation list holds E configurations, each
// evaluated in two passes: the direct channel order (alpha, beta) giving
// z(alpha, beta) and the swapped order (beta, alpha) giving z(beta, alpha)
// (Eq. log_sum_exp_conjugate).  For n <= 32 a 32-row block holds
// cpb = 32/n configurations of one pass (block g: pass g&1, configurations
// (g>>1)*cpb ...); attention is masked to rows of the same configuration.  For
// 32 < n <= 64 one configuration-pass spans two blocks (64 rows, rows >= n
// masked).  A wave owns a tile of NBR blocks and keeps its rows in registers
// through the whole layer: QKV projection, per-head softmax(QK^T/sqrt(dh))V,
// W_O and residual, then the ReLU feed-forward sub-layer and residual.
// The layer's packed weights are staged once per workgroup in LDS (BF16) or
// read through the caches (FP32); workgroups are persistent over tiles.
#include "common.h"
#include "net.h"
#include "netapi.h"

namespace tdo {

template <int D>
struct EmbedRow {
  // Window code of the two width-2 circular convolutions: x_i depends on
  // sites i, i+1, i+2; code = t_i + 4 t_{i+1} + 16 t_{i+2},
  // t = bit(channel 0) + 2 bit(channel 1).
  __device__ static __forceinline__ int code(uint64_t c0, uint64_t c1, int i, int n) {
    int cd = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int s = i + k;
      s = s >= n ? s - n : s;
      const int t = (int)((c0 >> s) & 1ull) + 2 * (int)((c1 >> s) & 1ull);
      cd += t << (2 * k);
    }
    return cd;
  }
};

// Table of the embedding: T[code][o] = act(b2 + e(t0,t1) W2[0] + e(t1,t2) W2[1]),
// e(ta,tb) = act(b1 + s(ta) W1[0] + s(tb) W1[1]), act = exact GELU (Eq. circ-conv).
__global__ void k_embed_table(const float* __restrict__ params, int d, int D, float* __restrict__ table) {
  __shared__ float e0[64], e1[64];
  const int code = blockIdx.x;
  const int t0 = code & 3, t1 = (code >> 2) & 3, t2 = (code >> 4) & 3;
  const float* w1 = params;            // [2 taps][2 ch][d]
  const float* b1 = params + 4 * d;    // [d]
  const float* w2 = b1 + d;            // [2 taps][d][d]
  const float* b2 = w2 + 2 * d * d;    // [d]
  auto spin = [](int t, int ch) { return 1.0f - 2.0f * (float)((t >> ch) & 1); };
  auto gelu = [](float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); };
  for (int c = threadIdx.x; c < d; c += blockDim.x) {
    float a = b1[c] + spin(t0, 0) * w1[0 * d + c] + spin(t0, 1) * w1[1 * d + c] + spin(t1, 0) * w1[2 * d + c] +
              spin(t1, 1) * w1[3 * d + c];
    float b = b1[c] + spin(t1, 0) * w1[0 * d + c] + spin(t1, 1) * w1[1 * d + c] + spin(t2, 0) * w1[2 * d + c] +
              spin(t2, 1) * w1[3 * d + c];
    e0[c] = gelu(a);
    e1[c] = gelu(b);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < D; o += blockDim.x) {
    float v = 0.f;
    if (o < d) {
      float acc = b2[o];
      for (int c = 0; c < d; ++c) acc += e0[c] * w2[c * d + o] + e1[c] * w2[d * d + c * d + o];
      v = gelu(acc);
    }
    table[code * D + o] = v;
  }
}

// Workgroup size NT: BF16 weights staged in LDS are shared by 8 waves (two per SIMD,
// so that one wave's latencies overlap the other's work) or by 4 waves (one per SIMD,
// with twice the registers); the choice is autotuned per shape.  Otherwise 4 waves.
// A wave of a spanning pass (two row blocks) needs more than half a SIMD's registers:
// with 8 waves it is held to 256 and spills a few values (24 at head width 16 with
// masking), which measured faster than one wave per SIMD.

// MBC: the feed-forward width in 32-column chunks when fixed at compile time (0: a.M / 32), so
// that the chunk loop unrolls and one chunk's LDS reads overlap the previous chunk's products.
// MASKED: some (query, key) pairs of a tile are invalid (several configurations per block, or
// padding rows); a compile-time choice, so that the unmasked kernel holds no mask registers.
template <class P, int D, int DH, bool SPAN, int MBC, bool MASKED, int NT>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu((SPAN && NT == 512) ? 2 : 1, (SPAN && NT == 512) ? 2 : 8))) k_fwd_layer(FwdArgs a) {
  constexpr int NB = D / 32;            // feature blocks
  constexpr int NBR = SPAN ? 2 : 1;     // row blocks per wave
  constexpr int HPB = 32 / DH;          // heads per 32-feature block
  constexpr int ST = P::STEPS;
  using elem_t = typename P::elem_t;
  using op_t = typename P::op_t;
  using save_t = typename P::save_t;
  constexpr bool WLDS = (P::KPL == 8);

  extern __shared__ __align__(16) char smem[];
  const int M = MBC ? 32 * MBC : a.M, MB = M / 32;
  const int wtotal = 4 * D * D + 2 * D * M;
  // LDS carve-up: [weights (BF16 only)] [b1 M] [b2 D] [table 64*D] [head weights: 64 float2]
  elem_t* wl = reinterpret_cast<elem_t*>(smem);
  float* b1s = reinterpret_cast<float*>(smem + (WLDS ? (size_t)wtotal * sizeof(elem_t) : 0));
  float* b2s = b1s + M;
  float* tabs = b2s + D;
  float2* hws = reinterpret_cast<float2*>(tabs + (a.first ? 64 * D : 0));  // last layer: (W_h[f][0], W_h[f][1]), 0 past d

  // ---- stage weights, biases and the embedding table
  const elem_t* wg = reinterpret_cast<const elem_t*>(a.wpack);
  if constexpr (WLDS) {
    const int n16 = wtotal * (int)sizeof(elem_t) / 16;
    const int4* src = reinterpret_cast<const int4*>(wg);
    int4* dst = reinterpret_cast<int4*>(wl);
    for (int i = threadIdx.x; i < n16; i += blockDim.x) dst[i] = src[i];
  }
  for (int i = threadIdx.x; i < M; i += blockDim.x) b1s[i] = a.b1[i];
  for (int i = threadIdx.x; i < D; i += blockDim.x) b2s[i] = a.b2[i];
  if (a.first)
    for (int i = threadIdx.x; i < 64 * D; i += blockDim.x) tabs[i] = a.table[i];
  if (a.last)
    for (int i = threadIdx.x; i < 64; i += blockDim.x)
      hws[i] = i < a.d_real ? make_float2(a.head_w[2 * i], a.head_w[2 * i + 1]) : make_float2(0.f, 0.f);
  __syncthreads();
  const elem_t* W = WLDS ? wl : wg;
  const elem_t* Wq = W + 0 * D * D;
  const elem_t* Wk = W + 1 * D * D;
  const elem_t* Wv = W + 2 * D * D;
  const elem_t* Wo = W + 3 * D * D;
  const elem_t* W1 = W + 4 * D * D;
  const elem_t* W2 = W + 4 * D * D + D * M;

  const int lane = threadIdx.x & 63, h = lane >> 5, lr = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int64_t E = a.n_entries_dev ? *a.n_entries_dev : a.n_entries;
  const int n = a.n, cpb = a.cpb;
  const int64_t ntiles = SPAN ? 2 * E : 2 * ((E + cpb - 1) / cpb);
  const float sc = a.score_scale;  // log2(e)/sqrt(dh)

  // valid (query row qb*32+lr, key row kb*32+tile_idx(r, h)) pairs as bit r of okbits[qb][kb]
  uint32_t okbits[NBR][NBR];
#pragma unroll
  for (int qb = 0; qb < NBR; ++qb)
#pragma unroll
    for (int kb = 0; kb < NBR; ++kb) {
      uint32_t bits = 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int key = kb * 32 + tile_idx(r, h);
        bool ok;
        if (SPAN) ok = key < n;
        else ok = a.masked ? ((key / n) == (SPAN ? 0 : lr / n) && (key / n) < cpb) : true;
        bits |= ok ? (1u << r) : 0u;
      }
      okbits[qb][kb] = bits;
    }

  // x of a layer after the first, for the wave's next tile: loaded one tile ahead (one row
  // block per tile; the two of a spanning tile would not fit in the registers), so that the
  // latency of the loads overlaps the current tile's work
  const int64_t tstride = (int64_t)gridDim.x * (blockDim.x >> 6);
  f32x16 xnext[NBR][NB];
  auto fetch_x = [&](int64_t tl) {
    if (a.first || tl >= ntiles) return;
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) {
        const float4* src = reinterpret_cast<const float4*>(a.x_in + (((tl * NBR + rb) * NB + ob) * 64 + lane) * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 v = src[q];
          xnext[rb][ob][4 * q + 0] = v.x; xnext[rb][ob][4 * q + 1] = v.y;
          xnext[rb][ob][4 * q + 2] = v.z; xnext[rb][ob][4 * q + 3] = v.w;
        }
      }
  };
  if (!SPAN) fetch_x((int64_t)blockIdx.x * (blockDim.x >> 6) + wave);

  for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; tile < ntiles; tile += tstride) {
    const int pass = (int)(tile & 1);
    // first entry of the tile and the slot/validity of this lane's rows
    const int64_t e0 = SPAN ? (tile >> 1) : (tile >> 1) * cpb;
    int rslot[NBR];
    bool rvalid[NBR];
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb) {
      const int row = rb * 32 + lr;
      if (SPAN) { rslot[rb] = 0; rvalid[rb] = row < n; }
      else { rslot[rb] = lr / n; rvalid[rb] = (lr / n) < cpb && (e0 + lr / n) < E; }
    }

    // ---- residual stream x (feature x row), FP32
    f32x16 x[NBR][NB];
    const int64_t gblk0 = tile * NBR;
    if (a.first) {
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb) {
        const int row = rb * 32 + lr;
        int code = 0;
        if (rvalid[rb]) {
          const int64_t e = e0 + rslot[rb];
          const uint64_t al = a.ecfg[2 * e], be = a.ecfg[2 * e + 1];
          const uint64_t c0 = pass ? be : al, c1 = pass ? al : be;
          code = EmbedRow<D>::code(c0, c1, SPAN ? row : (lr % n), n);
        }
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) {
          const float* tr = tabs + code * D + 32 * ob;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float4 v = *reinterpret_cast<const float4*>(tr + 8 * q + 4 * h);
            x[rb][ob][4 * q + 0] = v.x; x[rb][ob][4 * q + 1] = v.y;
            x[rb][ob][4 * q + 2] = v.z; x[rb][ob][4 * q + 3] = v.w;
          }
        }
      }
    } else {
      if (SPAN) fetch_x(tile);
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) x[rb][ob] = xnext[rb][ob];
    }
    if (!SPAN) fetch_x(tile + tstride);
    auto save = [&](void* dst, const f32x16 (&v)[NBR][NB]) {
      save_t* s = reinterpret_cast<save_t*>(dst);
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) {
          save_t* p = s + (((gblk0 + rb) * NB + ob) * 64 + lane) * 16;
#pragma unroll
          for (int r = 0; r < 16; ++r) p[r] = (save_t)v[rb][ob][r];
        }
    };
    if (a.save_x) save(a.save_x, x);

    // ---- attention: operands of x taken before the residual is updated
    op_t xo[NBR][NB][ST];
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int s = 0; s < ST; ++s) xo[rb][ib][s] = P::op(x[rb][ib], s);

#pragma unroll 1
    for (int hb = 0; hb < NB; ++hb) {
      f32x16 q[NBR], k[NBR], v[NBR];
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb) {
        q[rb] = f32x16{};
        k[rb] = f32x16{};
        v[rb] = f32x16{};
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            const int f = (hb * NB + ib) * ST + s;
            q[rb] = P::mma(ld_frag<P>(Wq, f, lane), xo[rb][ib][s], q[rb]);
            k[rb] = P::mma(ld_frag<P>(Wk, f, lane), xo[rb][ib][s], k[rb]);
            v[rb] = P::mma(xo[rb][ib][s], ld_frag<P>(Wv, f, lane), v[rb]);  // (row x feature)
          }
      }
      // score scale folded into q; per-head score operands of q and k packed once per head
      // block; V as operands (lane -> feature)
      using sop = typename P::template SOp<DH>;
      sop qp[NBR][HPB], kp[NBR][HPB];
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) q[rb][r] *= sc;
#pragma unroll
        for (int j = 0; j < HPB; ++j) {
          qp[rb][j] = P::template pack_head<DH>(q[rb], j);
          kp[rb][j] = P::template pack_head<DH>(k[rb], j);
        }
      }
      op_t vop[NBR][ST];
#pragma unroll
      for (int kb = 0; kb < NBR; ++kb)
#pragma unroll
        for (int s = 0; s < ST; ++s) vop[kb][s] = P::op(v[kb], s);
      // o = P V per head, row-major (lane -> row, values -> features).  Each head's product goes
      // into a fresh accumulator with the unmasked V operand (lane -> feature): only values
      // [VPH j, VPH (j + 1)) of each lane (the features of head j, see tile_idx) are head j's
      // output and are kept, normalised; the other values are dropped.
      constexpr int VPH = DH / 2;
      f32x16 o[NBR];
      float lsev[NBR][HPB];  // log2 softmax normalisers of this lane's row in each row block
#pragma unroll
      for (int j = 0; j < HPB; ++j) {
#pragma unroll
        for (int qb = 0; qb < NBR; ++qb) {
          f32x16 st[NBR];
          float m = -INFINITY;
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb) {
            st[kb] = P::template scores_packed<DH>(kp[kb][j], qp[qb][j], f32x16{});
            if constexpr (MASKED) {
#pragma unroll
              for (int r = 0; r < 16; ++r)
                if (!((okbits[qb][kb] >> r) & 1u)) st[kb][r] = -INFINITY;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) m = fmaxf(m, st[kb][r]);
          }
          m = xor32_max(m);
          const float mm = (m == -INFINITY) ? 0.f : m;  // a row with no key keeps P = 0
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb)
#pragma unroll
            for (int r = 0; r < 16; ++r) st[kb][r] = __builtin_amdgcn_exp2f(st[kb][r] - mm);
          // row sum as a pairwise tree (short dependency chains)
          float part[NBR * 8];
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb)
#pragma unroll
            for (int i = 0; i < 8; ++i) part[8 * kb + i] = st[kb][2 * i] + st[kb][2 * i + 1];
#pragma unroll
          for (int w = NBR * 4; w >= 1; w /= 2)
#pragma unroll
            for (int i = 0; i < w; ++i) part[i] += part[i + w];
          const float l = xor32_sum(part[0]);
          // l >= 1 when the row has a key (its maximum contributes exp2(0)): the hardware
          // reciprocal (1 ulp) replaces the division sequence
          const float invl = l > 0.f ? __builtin_amdgcn_rcpf(l) : 0.f;
          // for the backward: P = exp2(s - lse) (+inf for a row with no key, so that P = 0)
          lsev[qb][j] = l > 0.f ? mm + __builtin_amdgcn_logf(l) : INFINITY;
          f32x16 to = {};
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb)
#pragma unroll
            for (int s = 0; s < ST; ++s) to = P::mma(vop[kb][s], P::op(st[kb], s), to);
#pragma unroll
          for (int r = VPH * j; r < VPH * (j + 1); ++r) o[qb][r] = to[r] * invl;
        }
      }
      if constexpr (P::KPL == 8) {
        // the head block's normalisers are contiguous per row; one store per lane of the first
        // half (the second half's offset is out of range, and the resource is empty when nothing
        // is saved: no branch)
        const auto rl = rsrc(a.save_lse ? a.save_lse + gblk0 * 32 * (NB * HPB) : nullptr,
                             a.save_lse ? NBR * 32 * NB * HPB * 4 : 0);
#pragma unroll
        for (int qb = 0; qb < NBR; ++qb) {
          const int off = h == 0 ? ((qb * 32 + lr) * (NB * HPB) + hb * HPB) * 4 : 0x7ffffff0;
          if constexpr (HPB == 4) rst4(rl, off, make_float4(lsev[qb][0], lsev[qb][1], lsev[qb][2], lsev[qb][3]));
          else rst2(rl, off, make_float2(lsev[qb][0], lsev[qb][1]));
        }
      }
      // W_O into the residual
#pragma unroll
      for (int qb = 0; qb < NBR; ++qb) {
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
          for (int s = 0; s < ST; ++s)
            x[qb][ob] = P::mma(ld_frag<P>(Wo, (ob * NB + hb) * ST + s, lane), P::op(o[qb], s), x[qb][ob]);
      }
    }
    if (a.save_mid) save(a.save_mid, x);

    // ---- feed-forward sub-layer: x += relu(x W1 + b1) W2 + b2
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int s = 0; s < ST; ++s) xo[rb][ib][s] = P::op(x[rb][ib], s);
    // pre-activations of 32-unit chunk c: the products accumulate onto b1 (values
    // r = 4q .. 4q+3 hold 4 consecutive hidden units)
    auto ffn_pre = [&](int c, int rb) {
      f32x16 u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 b = *reinterpret_cast<const float4*>(b1s + 32 * c + 8 * q + 4 * h);
        u[4 * q] = b.x; u[4 * q + 1] = b.y; u[4 * q + 2] = b.z; u[4 * q + 3] = b.w;
      }
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int s = 0; s < ST; ++s) u = P::mma(ld_frag<P>(W1, (c * NB + ib) * ST + s, lane), xo[rb][ib][s], u);
      return u;
    };
    // One row block: software-pipelined over the chunks, chunk c+1's pre-activation products
    // issued before chunk c's ReLU and conversions, which then overlap them on the vector ALU
    // (two row blocks: chunk by chunk, a second chunk in flight would not fit in the
    // registers).  Each accumulator of x takes the chunks in order either way.
    if constexpr (SPAN) {
#pragma unroll
      for (int c = 0; c < MB; ++c)
#pragma unroll
        for (int rb = 0; rb < NBR; ++rb) {
          const f32x16 u = ffn_pre(c, rb);
#pragma unroll
          for (int ob = 0; ob < NB; ++ob)
#pragma unroll
            for (int s = 0; s < ST; ++s)
              x[rb][ob] = P::mma(ld_frag<P>(W2, (ob * MB + c) * ST + s, lane), P::relu_op(u, s), x[rb][ob]);
        }
    } else {
      constexpr int rb = 0;
      f32x16 un = ffn_pre(0, rb);
#pragma unroll
      for (int c = 0; c < MB; ++c) {
        const f32x16 u = un;
        if (c + 1 < MB) un = ffn_pre(c + 1, rb);
        op_t uo[ST];
#pragma unroll
        for (int s = 0; s < ST; ++s) uo[s] = P::relu_op(u, s);
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
          for (int s = 0; s < ST; ++s)
            x[rb][ob] = P::mma(ld_frag<P>(W2, (ob * MB + c) * ST + s, lane), uo[s], x[rb][ob]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
      for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int r = 0; r < 16; ++r) x[rb][ob][r] += b2s[32 * ob + tile_idx(r, h)];

    if (!a.last) {
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) {
          float4* dst = reinterpret_cast<float4*>(a.x_out + (((gblk0 + rb) * NB + ob) * 64 + lane) * 16);
#pragma unroll
          for (int qq = 0; qq < 4; ++qq)
            dst[qq] = make_float4(x[rb][ob][4 * qq], x[rb][ob][4 * qq + 1], x[rb][ob][4 * qq + 2], x[rb][ob][4 * qq + 3]);
        }
      continue;
    }
    // ---- last layer: save x_L, mean pooling over sites, dense head to z (Eq. global-pool-final)
    if (a.save_last) save(a.save_last, x);
    // per row: F = x_L W_h (features past d hold zero weights), summed over both lane halves
    float f0[NBR], f1[NBR];
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float2 hw = hws[32 * ob + tile_idx(r, h)];
          s0 += x[rb][ob][r] * hw.x;
          s1 += x[rb][ob][r] * hw.y;
        }
      f0[rb] = xor32_sum(s0);
      f1[rb] = xor32_sum(s1);
    }
    // mean over the n sites of each configuration: a segmented inclusive scan over the 32 row
    // lanes (segment = the configuration's rows; rows past the last configuration add nothing),
    // a fixed order of additions; the last row of each segment then holds its sum
    const int seg = SPAN ? 0 : lr / n, pos = SPAN ? lr : lr - seg * n;
    float v0 = 0.f, v1 = 0.f;
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
      if (rvalid[rb]) { v0 += f0[rb]; v1 += f1[rb]; }
#pragma unroll
    for (int dd = 1; dd < 32; dd <<= 1) {
      const float t0 = __shfl_up(v0, dd, 32), t1 = __shfl_up(v1, dd, 32);
      if (pos >= dd) { v0 += t0; v1 += t1; }
    }
    const int last = SPAN ? 31 : n - 1;  // in a spanning tile every lane's rows are one configuration
    if (h == 0 && pos == last && (SPAN || seg < cpb)) {
      const int64_t e = e0 + seg;
      if (e < E) {
        const float inv = 1.0f / (float)n;
        a.z[(e * 2 + pass) * 2 + 0] = v0 * inv + a.head_b[0];
        a.z[(e * 2 + pass) * 2 + 1] = v1 * inv + a.head_b[1];
      }
    }
  }
}

// log rho = log(e^{z1} + conj(e^{z2})) on the principal branch (Eq. log_sum_exp_conjugate).
__global__ void k_symmetrise(const int64_t* __restrict__ E_dev, int64_t E_host, const float* __restrict__ z,
                             float* __restrict__ lr) {
  const int64_t E = E_dev ? *E_dev : E_host;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const float a0 = z[4 * e], a1 = z[4 * e + 1];   // z(alpha, beta)
    const float b0 = z[4 * e + 2], b1 = z[4 * e + 3];  // z(beta, alpha), conjugated below
    const float mx = fmaxf(a0, b0);
    const float ea = expf(a0 - mx), eb = expf(b0 - mx);
    float sa, ca, sb, cb;
    sincosf(a1, &sa, &ca);
    sincosf(b1, &sb, &cb);
    const float sr = ea * ca + eb * cb, si = ea * sa - eb * sb;
    lr[2 * e] = mx + 0.5f * logf(sr * sr + si * si);
    lr[2 * e + 1] = atan2f(si, sr);
  }
}

// ------------------------------------------------------------------ dispatch
template <class P, int D, int DH, bool SPAN, int MBC, bool MASKED, int NT>
static int32_t launch_layer_nt(const FwdArgs& a, int num_cus, hipStream_t st) {
  const size_t wbytes = (P::KPL == 8) ? (size_t)(4 * D * D + 2 * D * a.M) * sizeof(typename P::elem_t) : 0;
  const size_t lds = wbytes + (size_t)(a.M + D) * 4 + (a.first ? 64 * D * 4 : 0) + 64 * sizeof(float2);
  auto kern = k_fwd_layer<P, D, DH, SPAN, MBC, MASKED, NT>;
  TDO_TRY(allow_full_lds((const void*)kern));
  const int blocks = num_cus * a.blocks_per_cu;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), lds, st, a);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

template <class P, int D, int DH, bool SPAN, int MBC, bool MASKED>
static int32_t launch_layer_m(const FwdArgs& a, int num_cus, hipStream_t st) {
  if constexpr (P::KPL == 8)
    if (a.waves == 8) return launch_layer_nt<P, D, DH, SPAN, MBC, MASKED, 512>(a, num_cus, st);
  return launch_layer_nt<P, D, DH, SPAN, MBC, MASKED, 256>(a, num_cus, st);
}

// the BF16 width-64 kernels with the feed-forward width 4 x 64 fixed at compile time
template <class P, int D, int DH, bool SPAN, bool MASKED>
static int32_t launch_layer_k(const FwdArgs& a, int num_cus, hipStream_t st) {
  if constexpr (P::KPL == 8 && D == 64)
    if (a.M == 256) return launch_layer_m<P, D, DH, SPAN, 8, MASKED>(a, num_cus, st);
  return launch_layer_m<P, D, DH, SPAN, 0, MASKED>(a, num_cus, st);
}

// masking is needed with several configurations per block, or padding rows of a spanning pass
template <class P, int D, int DH, bool SPAN>
static int32_t launch_layer_t(const FwdArgs& a, int num_cus, hipStream_t st) {
  const bool masked = SPAN ? (a.n < 64) : (a.masked != 0);
  return masked ? launch_layer_k<P, D, DH, SPAN, true>(a, num_cus, st) : launch_layer_k<P, D, DH, SPAN, false>(a, num_cus, st);
}

template <class P>
static int32_t launch_layer_p(const FwdArgs& a, int D, int DH, bool span, int num_cus, hipStream_t st) {
  if (D == 32 && DH == 8) return span ? launch_layer_t<P, 32, 8, true>(a, num_cus, st) : launch_layer_t<P, 32, 8, false>(a, num_cus, st);
  if (D == 64 && DH == 8) return span ? launch_layer_t<P, 64, 8, true>(a, num_cus, st) : launch_layer_t<P, 64, 8, false>(a, num_cus, st);
  if (D == 64 && DH == 16) return span ? launch_layer_t<P, 64, 16, true>(a, num_cus, st) : launch_layer_t<P, 64, 16, false>(a, num_cus, st);
  return set_error(TDO_EUNSUPPORTED, "no forward kernel for padded width %d, head width %d", D, DH);
}

int32_t launch_fwd_layer(const FwdArgs& a, bool bf16, int D, int DH, bool span, int num_cus, hipStream_t st) {
  return bf16 ? launch_layer_p<PBF16>(a, D, DH, span, num_cus, st) : launch_layer_p<PF32>(a, D, DH, span, num_cus, st);
}

int32_t launch_embed_table(const float* params, int d, int D, float* table, hipStream_t st) {
  hipLaunchKernelGGL(k_embed_table, dim3(64), dim3(64), 0, st, params, d, D, table);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_symmetrise(const int64_t* E_dev, int64_t E_host, const float* z, float* lr, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrise, dim3(1024), dim3(256), 0, st, E_dev, E_host, z, lr);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // namespace tdo
