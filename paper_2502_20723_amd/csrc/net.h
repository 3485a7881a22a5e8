// Device building blocks of the transformer density operator on CDNA4 MFMA.
//
// Register layout.  A wave owns blocks of 32 sequence rows (sites of one or
// more configurations).  Every activation lives in registers in the result
// layout of the 32x32 MFMA: for a 32x32 tile (feature x row), lane l holds row
// l%32 and the 16 features 8*(r/4) + 4*(l/32) + r%4, r = 0..15.  The same
// registers, taken KPL at a time, are a valid A or B operand for a contraction
// over those 32 features when the other operand enumerates features in the
// same order; the packed weights below are laid out in exactly that order,
// so GEMM chains (QKV, attention, W_O, MLP) never leave registers.
// Computing the product as (row x feature) instead (swapping the A and B
// operands) gives lane -> feature and r -> row, the layout used as operand of
// contractions over rows (attention P.V and the weight gradients).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <type_traits>

#include "common.h"

namespace tdo {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Feature (or row) index held by value r of lane half h in a 32x32 result tile.
__host__ __device__ constexpr int tile_idx(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Two FP32 values rounded to BF16 (round to nearest even) in one register, a in the low half.
// Written as one two-element conversion so that it is one v_cvt_pk_bf16_f32; element-wise
// conversions are sometimes emitted as one conversion per value plus a v_perm_b32.
__device__ __forceinline__ uint32_t pk2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
// BF16 operand of values 8s .. 8s+7 of a result tile (f32x16 or float[16]).
template <class V>
__device__ __forceinline__ bf16x8 cvt8(const V& v, int s) {
  u32x4 w;
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = pk2(v[8 * s + 2 * i], v[8 * s + 2 * i + 1]);
  return __builtin_bit_cast(bf16x8, w);
}

// ------------------------------------------------------------------ precisions
// BF16 operands, FP32 accumulation: v_mfma_f32_32x32x16_bf16 (8 values/lane).
struct PBF16 {
  static constexpr int KPL = 8;
  static constexpr int STEPS = 32 / (2 * KPL);  // k-steps per 32-feature block
  using elem_t = __bf16;                         // packed weight element
  using op_t = bf16x8;
  using save_t = __bf16;                         // saved activations for backward
  __device__ static __forceinline__ f32x16 mma(op_t a, op_t b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ op_t op(const f32x16& v, int s) { return cvt8(v, s); }
  // Operand s of relu(v).  Rounding to BF16 keeps the sign (a negative value rounds to a
  // negative value or -0), so the ReLU of the rounded pair is a signed 16-bit maximum with
  // 0 on the packed bits: one instruction per two values, the same bits as rounding relu(v).
  __device__ static __forceinline__ op_t relu_op(const f32x16& v, int s) {
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 t = __builtin_bit_cast(s16x8, cvt8(v, s));
    return __builtin_bit_cast(bf16x8, __builtin_elementwise_max(t, (s16x8){}));
  }
  // Score operand of one head: its DH features of a 32-feature result tile
  // (values [DH/2*j, DH/2*j + DH/2) of each lane), packed once and reused.
  template <int DH>
  struct SOp {
    typename std::conditional<DH == 8, s16x4, bf16x8>::type v;
  };
  template <int DH>
  __device__ static __forceinline__ SOp<DH> pack_head(const f32x16& x, int j) {
    SOp<DH> o;
    if constexpr (DH == 8) o.v = __builtin_bit_cast(s16x4, (u32x2){pk2(x[4 * j], x[4 * j + 1]), pk2(x[4 * j + 2], x[4 * j + 3])});
    else o.v = cvt8(x, j);
    return o;
  }
  template <int DH>
  __device__ static __forceinline__ f32x16 scores_packed(const SOp<DH>& a, const SOp<DH>& b, f32x16 c) {
    if constexpr (DH == 8) return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a.v, b.v, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, b.v, c, 0, 0, 0);
  }
  // Attention scores over DH features of head j (values [DH/2*j, DH/2*j + DH/2)).
  template <int DH>
  __device__ static __forceinline__ f32x16 scores(const f32x16& kv, const f32x16& qv, int j, f32x16 c) {
    static_assert(DH == 8 || DH == 16, "head width 8 or 16");
    return scores_packed<DH>(pack_head<DH>(kv, j), pack_head<DH>(qv, j), c);
  }
};

// FP32 operands: v_mfma_f32_32x32x2f32 (1 value/lane).
struct PF32 {
  static constexpr int KPL = 1;
  static constexpr int STEPS = 16;
  using elem_t = float;
  using op_t = float;
  using save_t = float;
  __device__ static __forceinline__ f32x16 mma(op_t a, op_t b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ op_t op(const f32x16& v, int s) { return v[s]; }
  __device__ static __forceinline__ op_t relu_op(const f32x16& v, int s);
  template <int DH>
  struct SOp {
    float v[DH / 2];
  };
  template <int DH>
  __device__ static __forceinline__ SOp<DH> pack_head(const f32x16& x, int j) {
    SOp<DH> o;
#pragma unroll
    for (int t = 0; t < DH / 2; ++t) o.v[t] = x[(DH / 2) * j + t];
    return o;
  }
  template <int DH>
  __device__ static __forceinline__ f32x16 scores_packed(const SOp<DH>& a, const SOp<DH>& b, f32x16 c) {
#pragma unroll
    for (int t = 0; t < DH / 2; ++t) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[t], b.v[t], c, 0, 0, 0);
    return c;
  }
  template <int DH>
  __device__ static __forceinline__ f32x16 scores(const f32x16& kv, const f32x16& qv, int j, f32x16 c) {
    constexpr int PER = DH / 2;
#pragma unroll
    for (int t = 0; t < PER; ++t) c = __builtin_amdgcn_mfma_f32_32x32x2f32(kv[PER * j + t], qv[PER * j + t], c, 0, 0, 0);
    return c;
  }
};

// Packed weight fragment (out-block ob, in-block ib, k-step s) of a matrix
// W[in][out] (x @ W convention): lane l holds W[32 ib + tile_idx(s*KPL+t, l/32)][32 ob + l%32]
// for t < KPL; fragment f occupies elements [f*64*KPL, (f+1)*64*KPL).
template <class P>
__device__ __forceinline__ typename P::op_t ld_frag(const typename P::elem_t* base, int frag, int lane) {
  if constexpr (P::KPL == 8) {
    return *reinterpret_cast<const bf16x8*>(base + ((size_t)frag * 64 + lane) * 8);
  } else {
    return base[(size_t)frag * 64 + lane];
  }
}

// Per-layer packed-weight offsets (elements), for width D and MLP width M.
template <int D, int M>
struct LayerPack {
  static constexpr int NB = D / 32, MB = M / 32;
  static constexpr int WQ = 0, WK = D * D, WV = 2 * D * D, WO = 3 * D * D;
  static constexpr int W1 = 4 * D * D;        // [MB ob][NB ib][STEPS] fragments
  static constexpr int W2 = 4 * D * D + D * M;  // [NB ob][MB ib][STEPS]
  static constexpr int TOTAL = 4 * D * D + 2 * D * M;
};

// Row validity and configuration slot of lane row lr in block g (see the forward).
struct RowMap {
  int n, cpb;
  bool span;
  __device__ void at(int64_t g, int lr, int64_t E, int64_t& entry, int& pass, int& row_in_cfg, bool& valid) const {
    if (span) {
      const int64_t tile = g >> 1;
      const int rb = (int)(g & 1);
      entry = tile >> 1;
      pass = (int)(tile & 1);
      row_in_cfg = rb * 32 + lr;
      valid = row_in_cfg < n && entry < E;
    } else {
      pass = (int)(g & 1);
      const int slot = lr / n;
      entry = (g >> 1) * cpb + slot;
      row_in_cfg = lr % n;
      valid = slot < cpb && entry < E;
    }
  }
};

// Sum and maximum of a value over the two halves of the wave (lanes l and l ^ 32) on
// the vector ALU (v_permlane32_swap: after swapping the upper half of one copy
// with the lower half of another, the two registers hold the lower and upper
// halves' values in every lane), instead of a round trip through the LDS
// crossbar.  Both operations are commutative, so every lane gets the same bits as
// x + shfl_xor(x, 32).  All 64 lanes must be active.
__device__ __forceinline__ float xor32_sum(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xor32_max(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

// Bounded global access through a buffer resource over [p, p + bytes): loads outside it
// return 0 and stores outside it are dropped by the hardware.  A wave can then keep one
// unconditional sequence of memory operations (bytes = 0 disables them): the loads and
// stores of a wave retire in order on one counter, and an access under a branch makes the
// compiler wait for every outstanding one at the next use of a load issued before it.
// p must be wave-uniform.
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ bf16x8 rld8(__amdgpu_buffer_rsrc_t r, int voff, int soff = 0) {
  return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ float2 rld2(__amdgpu_buffer_rsrc_t r, int voff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
}
__device__ __forceinline__ float4 rld4(__amdgpu_buffer_rsrc_t r, int voff, int soff = 0) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void rst2(__amdgpu_buffer_rsrc_t r, int voff, float2 v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(int __attribute__((ext_vector_type(2))), v), r, voff, 0, 0);
}
__device__ __forceinline__ void rst4(__amdgpu_buffer_rsrc_t r, int voff, float4 v, int soff = 0) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, v), r, voff, soff, 0);
}

// Workgroup barrier that orders LDS accesses only: global loads (a prefetch of the next
// tile) and stores stay in flight across it, where __syncthreads would wait for them.
__device__ __forceinline__ void barrier_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Exact ReLU of the feed-forward sub-layer as a signed integer maximum of the bits with 0:
// one instruction (a float maximum first quiets its inputs, a second instruction).  A
// negative value or -0 gives +0; it differs from x > 0 ? x : 0 only for a NaN input, which
// it passes on instead of replacing by 0.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }
__device__ __forceinline__ float PF32::relu_op(const f32x16& v, int s) { return relu(v[s]); }

}  // namespace tdo
