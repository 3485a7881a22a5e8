// Backward pass of the transformer density operator: vector-Jacobian products
// of log rho with respect to every parameter, for per-pass seeds (dF0, dF1) on
// the head outputs z = F0 + i F1.
//
// Per layer two kernels run in reverse order, each recomputing the layer's
// internals from the activations saved by the forward pass:
//   MLP:       u = b1 + x W1, dh = g W2^T, du = dh [u > 0], dx = g + du W1^T,
//              dW1 += x^T du, dW2 += relu(u)^T g, db1 += sum du, db2 += sum g;
//   attention: q, k, v, P = softmax(q k^T / sqrt(dh)) per head, O = P v;
//              dO = dx W_O^T, dP = dO v^T, dS = P (dP - rowsum(P dP)) / sqrt(dh),
//              dq = dS k, dk = dS^T q, dv = P^T dO, dx += dq Wq^T + dk Wk^T + dv Wv^T,
//              dW_O += O^T dx, dWq += x^T dq, dWk += x^T dk, dWv += x^T dv.
// Contractions over features chain in registers exactly as in the forward;
// contractions over rows (attention over keys/queries and all weight
// gradients) take operands whose lanes enumerate features, obtained either by
// computing the product in the (row x feature) orientation or by a transpose
// of a 32x32 tile through a wave-private LDS scratch.  Weight gradients of one
// block are added into workgroup-shared FP32 accumulators in LDS; at the end
// each workgroup writes its accumulators to a private partial buffer, and the
// partials are summed in FP64 in a fixed order.
#include "common.h"
#include "net.h"
#include "netapi.h"

namespace tdo {

constexpr int TS = 36;  // row stride (floats) of the transpose scratch

// Natural row index of value i of lane half h in an operand built by transpose_tile.
template <class P>
__device__ __forceinline__ int nat_idx(int i, int h) {
  return (i / P::KPL) * (2 * P::KPL) + h * P::KPL + (i % P::KPL);
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Input: a 32x32 tile in MFMA result layout (element (m, n) = value r of lane
// n + 32h with m = tile_idx(r, h)).  Output: the same tile with lane -> m and
// value i -> n = nat_idx(i, h), i.e. an operand for a contraction over n.
template <class P>
__device__ __forceinline__ f32x16 transpose_tile(const f32x16& v, float* sc, int lane) {
  const int h = lane >> 5, n = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) sc[tile_idx(r, h) * TS + n] = v[r];
  wave_lds_sync();
  f32x16 o;
  const float* row = sc + n * TS;
  if constexpr (P::KPL == 8) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = *reinterpret_cast<const float4*>(row + 16 * (q >> 1) + 8 * h + 4 * (q & 1));
      o[4 * q] = t.x; o[4 * q + 1] = t.y; o[4 * q + 2] = t.z; o[4 * q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) o[i] = row[nat_idx<P>(i, h)];
  }
  wave_lds_sync();
  return o;
}

template <class P>
__device__ __forceinline__ typename P::op_t masked_op(const f32x16& v, int s, bool keep) {
  const typename P::op_t o = P::op(v, s);
  return keep ? o : typename P::op_t{};
}

// Add a 32x32 result tile into an LDS matrix: value r of lane l goes to
// row m0 + tile_idx(r, h), column c0 + l%32, row stride ld.
__device__ __forceinline__ void lds_add_tile(float* base, int ld, int m0, int c0, const f32x16& v, int lane) {
  const int h = lane >> 5, n = lane & 31;
#pragma unroll
  for (int r = 0; r < 16; ++r) atomicAdd(base + (m0 + tile_idx(r, h)) * ld + c0 + n, v[r]);
}

template <class T>
__device__ __forceinline__ void load_tile(const T* src, f32x16& v) {
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = (float)src[r];
}
__device__ __forceinline__ void load_tile(const float* src, f32x16& v) {
  const float4* p = reinterpret_cast<const float4*>(src);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 t = p[q];
    v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
  }
}
__device__ __forceinline__ void store_tile(float* dst, const f32x16& v) {
  float4* p = reinterpret_cast<float4*>(dst);
#pragma unroll
  for (int q = 0; q < 4; ++q) p[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// ------------------------------------------------------------------ MLP backward
template <class P, int D>
__global__ void __launch_bounds__(256) k_bwd_mlp(BwdArgs a) {
  constexpr int NB = D / 32, ST = P::STEPS;
  using elem_t = typename P::elem_t;
  using save_t = typename P::save_t;
  using op_t = typename P::op_t;
  extern __shared__ __align__(16) float sm[];
  const int M = a.M, MB = M / 32;
  float* dW1 = sm;                // [D][M]
  float* dW2 = dW1 + D * M;       // [M][D]
  float* db1 = dW2 + M * D;       // [M]
  float* db2 = db1 + M;           // [D]
  float* scr = db2 + D;           // [4 waves][32 * TS]
  const int accn = 2 * D * M + M + D;
  for (int i = threadIdx.x; i < accn; i += blockDim.x) sm[i] = 0.f;
  __syncthreads();

  const elem_t* Wf = reinterpret_cast<const elem_t*>(a.wf);
  const elem_t* Wb = reinterpret_cast<const elem_t*>(a.wb);
  const elem_t* W1f = Wf + 4 * D * D;            // [MB][NB][ST]
  const elem_t* W2T = Wb + 4 * D * D;            // [MB][NB][ST]
  const elem_t* W1T = Wb + 4 * D * D + D * M;    // [NB][MB][ST]
  const int lane = threadIdx.x & 63, h = lane >> 5, lr = lane & 31, wave = threadIdx.x >> 6;
  float* sc = scr + wave * 32 * TS;
  const int64_t E = a.n_entries_dev ? *a.n_entries_dev : a.n_entries;
  const RowMap rm{a.n, a.cpb, a.span != 0};
  const int64_t nblk = a.span ? 4 * E : 2 * ((E + a.cpb - 1) / a.cpb);

  for (int64_t g = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; g < nblk; g += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    f32x16 xm[NB], gv[NB];
    const save_t* xs = reinterpret_cast<const save_t*>(a.save_mid);
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) load_tile(xs + ((g * NB + ib) * 64 + lane) * 16, xm[ib]);
    if (a.seeds) {
      int64_t e; int pass, ric; bool valid;
      rm.at(g, lr, E, e, pass, ric, valid);
      float s0 = 0.f, s1 = 0.f;
      if (valid) { s0 = a.seeds[(e * 2 + pass) * 2] / (float)a.n; s1 = a.seeds[(e * 2 + pass) * 2 + 1] / (float)a.n; }
#pragma unroll
      for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int f = 32 * ob + tile_idx(r, h);
          gv[ob][r] = f < a.d_real ? s0 * a.head_w[2 * f] + s1 * a.head_w[2 * f + 1] : 0.f;
        }
    } else {
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) load_tile(a.g_in + ((g * NB + ob) * 64 + lane) * 16, gv[ob]);
    }
    op_t xo[NB][ST], go[NB][ST];
#pragma unroll
    for (int ib = 0; ib < NB; ++ib)
#pragma unroll
      for (int s = 0; s < ST; ++s) { xo[ib][s] = P::op(xm[ib], s); go[ib][s] = P::op(gv[ib], s); }
    f32x16 xT[NB], gT[NB];
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) { xT[ib] = transpose_tile<P>(xm[ib], sc, lane); gT[ib] = transpose_tile<P>(gv[ib], sc, lane); }
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {  // db2 += sum over rows of g
      float t = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) t += gT[ob][i];
      t += __shfl_xor(t, 32, 64);
      if (h == 0) atomicAdd(db2 + 32 * ob + lr, t);
    }
    f32x16 dxm[NB];
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) dxm[ob] = gv[ob];
#pragma unroll 1
    for (int c = 0; c < MB; ++c) {
      f32x16 u, dh = f32x16{};  // u accumulates onto b1, in the forward's order
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r] = a.b1[32 * c + tile_idx(r, h)];
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          u = P::mma(ld_frag<P>(W1f, (c * NB + ib) * ST + s, lane), xo[ib][s], u);
          dh = P::mma(ld_frag<P>(W2T, (c * NB + ib) * ST + s, lane), go[ib][s], dh);
        }
      f32x16 hh, du;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float uu = u[r];
        hh[r] = relu(uu);
        du[r] = uu > 0.f ? dh[r] : 0.f;
      }
#pragma unroll
      for (int ob = 0; ob < NB; ++ob)
#pragma unroll
        for (int s = 0; s < ST; ++s) dxm[ob] = P::mma(ld_frag<P>(W1T, (ob * MB + c) * ST + s, lane), P::op(du, s), dxm[ob]);
      const f32x16 hT = transpose_tile<P>(hh, sc, lane);
      const f32x16 duT = transpose_tile<P>(du, sc, lane);
      {
        float t = 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) t += duT[i];
        t += __shfl_xor(t, 32, 64);
        if (h == 0) atomicAdd(db1 + 32 * c + lr, t);
      }
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {  // dW1[D-in][hidden] += x^T du
        f32x16 acc = f32x16{};
#pragma unroll
        for (int s = 0; s < ST; ++s) acc = P::mma(P::op(xT[ib], s), P::op(duT, s), acc);
        lds_add_tile(dW1, M, 32 * ib, 32 * c, acc, lane);
      }
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) {  // dW2[hidden][D-out] += relu(u)^T g
        f32x16 acc = f32x16{};
#pragma unroll
        for (int s = 0; s < ST; ++s) acc = P::mma(P::op(hT, s), P::op(gT[ob], s), acc);
        lds_add_tile(dW2, D, 32 * c, 32 * ob, acc, lane);
      }
    }
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) store_tile(a.g_out + ((g * NB + ob) * 64 + lane) * 16, dxm[ob]);
  }
  __syncthreads();
  float* part = a.partial + (int64_t)blockIdx.x * accn;
  for (int i = threadIdx.x; i < accn; i += blockDim.x) part[i] = sm[i];
}

// ------------------------------------------------------------------ attention backward
template <class P, int D, int DH, bool SPAN>
__global__ void __launch_bounds__(256) k_bwd_attn(BwdArgs a) {
  constexpr int NB = D / 32, ST = P::STEPS, NBR = SPAN ? 2 : 1, HPB = 32 / DH;
  using elem_t = typename P::elem_t;
  using save_t = typename P::save_t;
  using op_t = typename P::op_t;
  extern __shared__ __align__(16) float sm[];
  float* dWq = sm;               // [D][D] each: (D-in, attention feature)
  float* dWk = dWq + D * D;
  float* dWv = dWk + D * D;
  float* dWo = dWv + D * D;      // (attention feature, D-out)
  float* scr = dWo + D * D;
  for (int i = threadIdx.x; i < 4 * D * D; i += blockDim.x) sm[i] = 0.f;
  __syncthreads();

  const elem_t* Wf = reinterpret_cast<const elem_t*>(a.wf);
  const elem_t* Wb = reinterpret_cast<const elem_t*>(a.wb);
  const elem_t *Wq = Wf, *Wk = Wf + D * D, *Wv = Wf + 2 * D * D;
  const elem_t *WqT = Wb, *WkT = Wb + D * D, *WvT = Wb + 2 * D * D, *WoT = Wb + 3 * D * D;
  const int lane = threadIdx.x & 63, h = lane >> 5, lr = lane & 31, wave = threadIdx.x >> 6;
  float* sc = scr + wave * 32 * TS;
  const int64_t E = a.n_entries_dev ? *a.n_entries_dev : a.n_entries;
  const int n = a.n, cpb = a.cpb;
  const int64_t ntiles = SPAN ? 2 * E : 2 * ((E + cpb - 1) / cpb);
  const float sc2 = a.score_scale, isd = a.inv_sqrt_dh;

  for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave; tile < ntiles;
       tile += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    const int64_t e0 = SPAN ? (tile >> 1) : (tile >> 1) * cpb;
    const int64_t gb0 = tile * NBR;
    int rslot[NBR];
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb) rslot[rb] = SPAN ? 0 : lr / n;
    (void)e0;

    f32x16 xT[NBR][NB], dmT[NBR][NB], dx[NBR][NB];
    op_t xo[NBR][NB][ST], dmo[NBR][NB][ST];
    const save_t* xs = reinterpret_cast<const save_t*>(a.save_x);
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        f32x16 t;
        load_tile(xs + (((gb0 + rb) * NB + ib) * 64 + lane) * 16, t);
#pragma unroll
        for (int s = 0; s < ST; ++s) xo[rb][ib][s] = P::op(t, s);
        xT[rb][ib] = transpose_tile<P>(t, sc, lane);
        load_tile(a.g_in + (((gb0 + rb) * NB + ib) * 64 + lane) * 16, t);
        dx[rb][ib] = t;
#pragma unroll
        for (int s = 0; s < ST; ++s) dmo[rb][ib][s] = P::op(t, s);
        dmT[rb][ib] = transpose_tile<P>(t, sc, lane);
      }

#pragma unroll 1
    for (int hb = 0; hb < NB; ++hb) {
      f32x16 q[NBR], k[NBR], vR[NBR], vD[NBR], kR[NBR], dO[NBR];
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb) {
        q[rb] = k[rb] = vR[rb] = vD[rb] = kR[rb] = dO[rb] = f32x16{};
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            const int f = (hb * NB + ib) * ST + s;
            const op_t wq = ld_frag<P>(Wq, f, lane), wk = ld_frag<P>(Wk, f, lane), wv = ld_frag<P>(Wv, f, lane);
            q[rb] = P::mma(wq, xo[rb][ib][s], q[rb]);
            k[rb] = P::mma(wk, xo[rb][ib][s], k[rb]);
            vD[rb] = P::mma(wv, xo[rb][ib][s], vD[rb]);
            vR[rb] = P::mma(xo[rb][ib][s], wv, vR[rb]);
            kR[rb] = P::mma(xo[rb][ib][s], wk, kR[rb]);
            dO[rb] = P::mma(ld_frag<P>(WoT, f, lane), dmo[rb][ib][s], dO[rb]);
          }
      }
      f32x16 qT[NBR], dOT[NBR];
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb) { qT[rb] = transpose_tile<P>(q[rb], sc, lane); dOT[rb] = transpose_tile<P>(dO[rb], sc, lane); }
      f32x16 o[NBR], dq[NBR], dk[NBR], dv[NBR];
      float invl[NBR][HPB];
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb) o[rb] = dq[rb] = dk[rb] = dv[rb] = f32x16{};
#pragma unroll
      for (int j = 0; j < HPB; ++j) {
        const bool mine = (lr / DH) == j;
#pragma unroll
        for (int qb = 0; qb < NBR; ++qb) {
          f32x16 p[NBR], dp[NBR];
          float m = -INFINITY;
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb) {
            if (!SPAN && kb != qb) continue;
            p[kb] = P::template scores<DH>(k[kb], q[qb], j, f32x16{});
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int key = kb * 32 + tile_idx(r, h);
              bool ok;
              if (SPAN) ok = key < n;
              else ok = a.masked ? ((key / n) == rslot[qb] && (key / n) < cpb) : true;
              const float s2 = ok ? p[kb][r] * sc2 : -INFINITY;
              p[kb][r] = s2;
              m = fmaxf(m, s2);
            }
          }
          m = fmaxf(m, __shfl_xor(m, 32, 64));
          float l = 0.f;
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb) {
            if (!SPAN && kb != qb) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const float e = (m == -INFINITY) ? 0.f : exp2f(p[kb][r] - m);
              p[kb][r] = e;
              l += e;
            }
          }
          l += __shfl_xor(l, 32, 64);
          const float il = l > 0.f ? 1.0f / l : 0.f;
          invl[qb][j] = il;
          // dP^T (keys x queries) = V_j dO_j^T; Delta = sum_k P dP
          float delta = 0.f;
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb) {
            if (!SPAN && kb != qb) continue;
            dp[kb] = P::template scores<DH>(vD[kb], dO[qb], j, f32x16{});
#pragma unroll
            for (int r = 0; r < 16; ++r) delta += p[kb][r] * dp[kb][r];
          }
          delta += __shfl_xor(delta, 32, 64);
          delta *= il;
#pragma unroll
          for (int kb = 0; kb < NBR; ++kb) {
            if (!SPAN && kb != qb) continue;
            // O recompute (unnormalised; scaled by 1/l below)
#pragma unroll
            for (int s = 0; s < ST; ++s) o[qb] = P::mma(masked_op<P>(vR[kb], s, mine), P::op(p[kb], s), o[qb]);
            f32x16 ds, pn;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              pn[r] = p[kb][r] * il;
              ds[r] = pn[r] * (dp[kb][r] - delta) * isd;
            }
            // dq^T (feature x queries) += K_j^T dS^T   (keys in result order on both sides)
#pragma unroll
            for (int s = 0; s < ST; ++s) dq[qb] = P::mma(masked_op<P>(kR[kb], s, mine), P::op(ds, s), dq[qb]);
            // dk^T (feature x keys) += Q_j^T dS, dv^T (feature x keys) += dO_j^T P   (queries in natural order)
            const f32x16 dsT = transpose_tile<P>(ds, sc, lane);
            const f32x16 pT = transpose_tile<P>(pn, sc, lane);
#pragma unroll
            for (int s = 0; s < ST; ++s) {
              dk[kb] = P::mma(masked_op<P>(qT[qb], s, mine), P::op(dsT, s), dk[kb]);
              dv[kb] = P::mma(masked_op<P>(dOT[qb], s, mine), P::op(pT, s), dv[kb]);
            }
          }
        }
      }
#pragma unroll
      for (int rb = 0; rb < NBR; ++rb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) o[rb][r] *= invl[rb][DH == 8 ? r / 4 : r / 8];
        const f32x16 oT = transpose_tile<P>(o[rb], sc, lane);
#pragma unroll
        for (int ob = 0; ob < NB; ++ob) {  // dW_O[attn][D-out] += O^T dx_mid
          f32x16 acc = f32x16{};
#pragma unroll
          for (int s = 0; s < ST; ++s) acc = P::mma(P::op(oT, s), P::op(dmT[rb][ob], s), acc);
          lds_add_tile(dWo, D, 32 * hb, 32 * ob, acc, lane);
        }
#pragma unroll
        for (int ob = 0; ob < NB; ++ob)
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            const int f = (ob * NB + hb) * ST + s;
            dx[rb][ob] = P::mma(ld_frag<P>(WqT, f, lane), P::op(dq[rb], s), dx[rb][ob]);
            dx[rb][ob] = P::mma(ld_frag<P>(WkT, f, lane), P::op(dk[rb], s), dx[rb][ob]);
            dx[rb][ob] = P::mma(ld_frag<P>(WvT, f, lane), P::op(dv[rb], s), dx[rb][ob]);
          }
        const f32x16 dqT = transpose_tile<P>(dq[rb], sc, lane);
        const f32x16 dkT = transpose_tile<P>(dk[rb], sc, lane);
        const f32x16 dvT = transpose_tile<P>(dv[rb], sc, lane);
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {  // dW{q,k,v}[D-in][attn] += x^T d{q,k,v}
          f32x16 aq = f32x16{}, ak = f32x16{}, av = f32x16{};
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            const op_t xa = P::op(xT[rb][ib], s);
            aq = P::mma(xa, P::op(dqT, s), aq);
            ak = P::mma(xa, P::op(dkT, s), ak);
            av = P::mma(xa, P::op(dvT, s), av);
          }
          lds_add_tile(dWq, D, 32 * ib, 32 * hb, aq, lane);
          lds_add_tile(dWk, D, 32 * ib, 32 * hb, ak, lane);
          lds_add_tile(dWv, D, 32 * ib, 32 * hb, av, lane);
        }
      }
    }
#pragma unroll
    for (int rb = 0; rb < NBR; ++rb)
#pragma unroll
      for (int ob = 0; ob < NB; ++ob) store_tile(a.g_out + (((gb0 + rb) * NB + ob) * 64 + lane) * 16, dx[rb][ob]);
  }
  __syncthreads();
  float* part = a.partial + (int64_t)blockIdx.x * 4 * D * D;
  for (int i = threadIdx.x; i < 4 * D * D; i += blockDim.x) part[i] = sm[i];
}

// ------------------------------------------------------------------ head and embedding
// dW_head[f][k] += sum over configuration-passes of (mean over its rows of x_L[f]) dF_k,
// db_head[k] += dF_k.  One wave per block of the saved x_L (lane -> row, values ->
// features): each lane adds x_L[row][f] dF_k / n for its row into FP64
// accumulators; once per launch the lanes and the waves of a workgroup are summed in a
// fixed order into the workgroup's slot, and k_reduce_head adds the slots to the gradient.
template <class P, int D>
__global__ void __launch_bounds__(256) k_bwd_head(const void* __restrict__ save_last, const float* __restrict__ seeds,
                                                  const int64_t* E_dev, int64_t E_host, int n, int cpb, int span,
                                                  int d_real, double* __restrict__ part) {
  using save_t = typename P::save_t;
  constexpr int NB = D / 32;
  const int64_t E = E_dev ? *E_dev : E_host;
  const RowMap rm{n, cpb, span != 0};
  const int64_t nblk = span ? 4 * E : 2 * ((E + cpb - 1) / cpb);
  const int lane = threadIdx.x & 63, h = lane >> 5, lr = lane & 31, wave = threadIdx.x >> 6;
  const save_t* xs = reinterpret_cast<const save_t*>(save_last);
  const float inv_n = 1.0f / (float)n;
  double a0[NB][16], a1[NB][16], c0 = 0.0, c1 = 0.0;
#pragma unroll
  for (int ob = 0; ob < NB; ++ob)
#pragma unroll
    for (int r = 0; r < 16; ++r) a0[ob][r] = a1[ob][r] = 0.0;
  // no early exit for padding rows (their seeds are taken as 0: the forward wrote finite values
  // for them, which then add exactly 0), so that two blocks' loads can be in flight at once
#pragma unroll 2
  for (int64_t g = (int64_t)blockIdx.x * 4 + wave; g < nblk; g += (int64_t)gridDim.x * 4) {
    int64_t e; int pass, ric; bool valid;
    rm.at(g, lr, E, e, pass, ric, valid);
    float s0 = 0.f, s1 = 0.f;
    if (valid) {
      s0 = seeds[(e * 2 + pass) * 2] * inv_n;
      s1 = seeds[(e * 2 + pass) * 2 + 1] * inv_n;
    }
    if (h == 0) { c0 += s0; c1 += s1; }
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
      f32x16 v;
      load_tile(xs + ((g * NB + ob) * 64 + lane) * 16, v);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        a0[ob][r] += (double)(v[r] * s0);
        a1[ob][r] += (double)(v[r] * s1);
      }
    }
  }
  // sum over the 32 rows (lanes of one half) and then over the 4 waves, in a fixed order, into
  // this workgroup's slot part[block][2 d_real + 2] ([feature][2] head weights, then the bias)
  __shared__ double red[4][2 * D + 2];
#pragma unroll
  for (int ob = 0; ob < NB; ++ob)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double u0 = a0[ob][r], u1 = a1[ob][r];
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) { u0 += __shfl_xor(u0, o, 64); u1 += __shfl_xor(u1, o, 64); }
      const int f = 32 * ob + tile_idx(r, h);
      if (lr == 0) {
        red[wave][2 * f] = u0;
        red[wave][2 * f + 1] = u1;
      }
    }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) { c0 += __shfl_xor(c0, o, 64); c1 += __shfl_xor(c1, o, 64); }
  if (lane == 0) {
    red[wave][2 * D] = c0;
    red[wave][2 * D + 1] = c1;
  }
  __syncthreads();
  const int len = 2 * d_real + 2;
  for (int i = threadIdx.x; i < len; i += 256) {
    const int k = i < 2 * d_real ? i : 2 * D + (i - 2 * d_real);
    part[(int64_t)blockIdx.x * len + i] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
  }
}

// Sum of the head kernel's workgroup slots, one workgroup per entry in a fixed order:
// gw[i] (i < 2 d_real) or gb[i - 2 d_real] += sum over the nparts slots.
__global__ void __launch_bounds__(256) k_reduce_head(const double* __restrict__ part, int nparts, int d_real,
                                                     double* __restrict__ gw, double* __restrict__ gb) {
  __shared__ double sh[256];
  const int len = 2 * d_real + 2, i = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int p = t; p < nparts; p += 256) s += part[(int64_t)p * len + i];
  sh[t] = s;
  __syncthreads();
#pragma unroll
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) {
    if (i < 2 * d_real) gw[i] += sh[0];
    else gb[i - 2 * d_real] += sh[0];
  }
}

// dT[code][f] += sum over rows with that window code of dx_0[row][f], as a contraction
// over the rows of each block: C[f][code] = sum_row dx_0[row][f] onehot[row][code].  It runs
// on the BF16 matrix cores without losing FP32 accuracy: every FP32 value of dx_0 is split
// exactly into three BF16 terms (hi + mid + lo = x, each term the next 8 significant bits),
// the terms are transposed on the matrix cores (lane -> feature, values -> rows), and each is
// multiplied by the 0/1 operand: every product is exact and the sums accumulate in FP32 as
// in an FP32 contraction.  Accumulated in registers by every wave over its blocks and
// written to the wave's partial slot [64][D] once per launch.
template <int D>
__global__ void __launch_bounds__(256) k_embed_onehot(const float* __restrict__ dx0, const uint64_t* __restrict__ ecfg,
                                                      const int64_t* E_dev, int64_t E_host, int n, int cpb, int span,
                                                      float* __restrict__ partial) {
  constexpr int NB = D / 32;
  __shared__ uint32_t codes_s[4][8];  // per wave: window code of each of the 32 rows (byte r), 255 for padding
  const int64_t E = E_dev ? *E_dev : E_host;
  const RowMap rm{n, cpb, span != 0};
  const int64_t nblk = span ? 4 * E : 2 * ((E + cpb - 1) / cpb);
  const int lane = threadIdx.x & 63, h = lane >> 5, lr = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint8_t* cb = reinterpret_cast<uint8_t*>(codes_s[wave]);
  bf16x8 eye[2];  // permutation operands of the transposes: eye[s][t] = [tile_idx(8 s + t, h) == lr]
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
    for (int t2 = 0; t2 < 8; ++t2) eye[s2][t2] = (__bf16)(tile_idx(8 * s2 + t2, h) == lr ? 1.0f : 0.0f);
  auto mfma16 = [](const bf16x8& a, const bf16x8& b, const f32x16& c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  };
  f32x16 acc[NB][2];
#pragma unroll
  for (int ft = 0; ft < NB; ++ft) acc[ft][0] = acc[ft][1] = f32x16{};
  for (int64_t g = (int64_t)blockIdx.x * 4 + wave; g < nblk; g += (int64_t)gridDim.x * 4) {
    // window code of this lane's row (255 if the row is padding), shared through LDS
    {
      int64_t e; int pass, ric; bool valid;
      rm.at(g, lr, E, e, pass, ric, valid);
      int code = 255;
      if (valid) {
        const uint64_t al = ecfg[2 * e], be = ecfg[2 * e + 1];
        const uint64_t c0 = pass ? be : al, c1 = pass ? al : be;
        code = 0;
        for (int k = 0; k < 3; ++k) {
          int s = ric + k;
          s = s >= n ? s - n : s;
          code += ((int)((c0 >> s) & 1ull) + 2 * (int)((c1 >> s) & 1ull)) << (2 * k);
        }
      }
      if (h == 0) cb[lr] = (uint8_t)code;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    // one-hot operands: lane (code 32 ct + lr, half h), value t of k-step s -> row tile_idx(8 s + t, h)
    bf16x8 oh[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const uint32_t w0 = codes_s[wave][4 * s + h], w1 = codes_s[wave][4 * s + 2 + h];  // rows 16s+4h.., 16s+8+4h..
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const uint32_t c = ((t < 4 ? w0 : w1) >> (8 * (t & 3))) & 255u;
          oh[ct][s][t] = (__bf16)(c == (uint32_t)(32 * ct + lr) ? 1.0f : 0.0f);
        }
    }
    __builtin_amdgcn_wave_barrier();  // codes read before the next block's codes are written
#pragma unroll
    for (int ft = 0; ft < NB; ++ft) {
      const float4* src = reinterpret_cast<const float4*>(dx0 + ((g * NB + ft) * 64 + lane) * 16);
      float x[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 v = src[q];
        x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
      }
      bf16x8 tm[3][2];  // hi, mid, lo: R layout (lane -> row, values -> features tile_idx(r, h))
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const __bf16 hi = (__bf16)x[r];
        const float r1 = x[r] - (float)hi;
        const __bf16 mid = (__bf16)r1;
        const __bf16 lo = (__bf16)(r1 - (float)mid);
        tm[0][r >> 3][r & 7] = hi;
        tm[1][r >> 3][r & 7] = mid;
        tm[2][r >> 3][r & 7] = lo;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // transposed term: lane -> feature 32 ft + lr, value r -> row tile_idx(r, h) (exact)
        const f32x16 tt = mfma16(tm[k][1], eye[1], mfma16(tm[k][0], eye[0], f32x16{}));
        bf16x8 ta[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int t = 0; t < 8; ++t) ta[s][t] = (__bf16)tt[8 * s + t];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int s = 0; s < 2; ++s) acc[ft][ct] = mfma16(ta[s], oh[ct][s], acc[ft][ct]);
      }
    }
  }
  float* part = partial + ((int64_t)blockIdx.x * 4 + wave) * 64 * D;
#pragma unroll
  for (int ft = 0; ft < NB; ++ft)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 16; ++r) part[(32 * ct + lr) * D + 32 * ft + tile_idx(r, h)] = acc[ft][ct][r];
}

// Chain rule from the table gradient dT[64][D] (FP64) into the convolution parameters, in FP64
// (recomputes the table's pre-activations).  One workgroup per window code: the code's
// contribution to every parameter gradient goes to its slot part[code][4d + d + 2d^2 + d] (the
// gradient's layout); k_embed_params_sum adds the slots in code order.
__global__ void __launch_bounds__(64) k_embed_params(const float* __restrict__ params, const double* __restrict__ dT,
                                                     int d, int D, double* __restrict__ part) {
  // grad layout: conv1_w [2][2][d], conv1_b [d], conv2_w [2][d][d], conv2_b [d]
  __shared__ double ea[64], eb[64], gpre[64];
  const float* w1 = params;
  const float* b1 = params + 4 * d;
  const float* w2 = b1 + d;
  const float* b2 = w2 + 2 * d * d;
  const int64_t len = 6LL * d + 2LL * d * d;
  double* p = part + (int64_t)blockIdx.x * len;
  double* p_w1 = p;
  double* p_b1 = p + 4 * d;
  double* p_w2 = p_b1 + d;
  double* p_b2 = p_w2 + 2 * d * d;
  auto spin = [](int t, int ch) { return 1.0 - 2.0 * (double)((t >> ch) & 1); };
  auto phi = [](double u) { return 0.5 * u * (1.0 + erf(u * 0.7071067811865476)); };
  auto dphi = [](double u) { return 0.5 * (1.0 + erf(u * 0.7071067811865476)) + u * 0.3989422804014327 * exp(-0.5 * u * u); };
  const int t = threadIdx.x, code = blockIdx.x;
  const int t0 = code & 3, t1 = (code >> 2) & 3, t2 = (code >> 4) & 3;
  double pa = 0, pb = 0;
  if (t < d) {
    pa = b1[t] + spin(t0, 0) * w1[t] + spin(t0, 1) * w1[d + t] + spin(t1, 0) * w1[2 * d + t] + spin(t1, 1) * w1[3 * d + t];
    pb = b1[t] + spin(t1, 0) * w1[t] + spin(t1, 1) * w1[d + t] + spin(t2, 0) * w1[2 * d + t] + spin(t2, 1) * w1[3 * d + t];
    ea[t] = phi(pa);
    eb[t] = phi(pb);
  }
  __syncthreads();
  if (t < d) {  // output feature o = t: pre-activation and its gradient
    double acc = b2[t];
    for (int c = 0; c < d; ++c) acc += ea[c] * w2[c * d + t] + eb[c] * w2[d * d + c * d + t];
    gpre[t] = dT[code * D + t] * dphi(acc);
  }
  __syncthreads();
  if (t < d) {
    p_b2[t] = gpre[t];
    for (int c = 0; c < d; ++c) {  // thread t = output channel o (coalesced rows)
      p_w2[c * d + t] = ea[c] * gpre[t];
      p_w2[d * d + c * d + t] = eb[c] * gpre[t];
    }
    double da = 0, db = 0;  // thread t = input channel c
    for (int o = 0; o < d; ++o) { da += w2[t * d + o] * gpre[o]; db += w2[d * d + t * d + o] * gpre[o]; }
    const double ga = da * dphi(pa), gb = db * dphi(pb);
    p_b1[t] = ga + gb;
    p_w1[t] = spin(t0, 0) * ga + spin(t1, 0) * gb;
    p_w1[d + t] = spin(t0, 1) * ga + spin(t1, 1) * gb;
    p_w1[2 * d + t] = spin(t1, 0) * ga + spin(t2, 0) * gb;
    p_w1[3 * d + t] = spin(t1, 1) * ga + spin(t2, 1) * gb;
  }
}

// grad[i] += sum over the 64 codes, in code order, of part[code][i].
__global__ void k_embed_params_sum(const double* __restrict__ part, int64_t len, double* __restrict__ grad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < 64; ++c) s += part[c * len + i];
    grad[i] += s;
  }
}

// Sum nparts FP32 partials of length len in index order into FP64 out[i] (+=).
// A workgroup of 256 threads sums EPB consecutive elements over all nparts partials:
// G = 256 / EPB groups of threads each take every G-th partial, and the group sums are
// added in a fixed order (deterministic), so that enough loads are in flight per element.
template <int EPB>
__global__ void __launch_bounds__(256) k_reduce_partials(const float* __restrict__ part, int nparts, int64_t len,
                                                         double* __restrict__ out) {
  constexpr int G = 256 / EPB;
  __shared__ double sh[G][EPB];
  const int j = threadIdx.x % EPB, g = threadIdx.x / EPB;
  const int64_t i = (int64_t)blockIdx.x * EPB + j;
  double s = 0.0;
  if (i < len) {
#pragma unroll 8
    for (int p = g; p < nparts; p += G) s += (double)part[(int64_t)p * len + i];
  }
  sh[g][j] = s;
  __syncthreads();
  if (g == 0 && i < len) {
    double t = sh[0][j];
#pragma unroll
    for (int q = 1; q < G; ++q) t += sh[q][j];
    out[i] += t;
  }
}

// Scatter a padded FP64 layer gradient into the flat parameter gradient (+=, scaled).
//  layer accumulators: mlp = [dW1 D*M][dW2 M*D][db1 M][db2 D], attn = [dWq][dWk][dWv][dWo] (D*D each)
__global__ void k_scatter_layer(const double* __restrict__ mlp, const double* __restrict__ attn, int d, int D, int M,
                                double scale, double* __restrict__ g) {
  const int64_t tot = 4LL * d * d + 2LL * d * M + M + d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
    double v;
    if (i < 4LL * d * d) {
      const int mt = (int)(i / (d * d)), rem = (int)(i % (d * d)), r = rem / d, c = rem % d;
      v = attn[(int64_t)mt * D * D + r * D + c];
    } else if (i < 4LL * d * d + (int64_t)d * M) {
      const int64_t k = i - 4LL * d * d;
      const int r = (int)(k / M), c = (int)(k % M);
      v = mlp[(int64_t)r * M + c];
    } else if (i < 4LL * d * d + (int64_t)d * M + M) {
      v = mlp[2LL * D * M + (i - 4LL * d * d - (int64_t)d * M)];
    } else if (i < 4LL * d * d + 2LL * d * M + M) {
      const int64_t k = i - 4LL * d * d - (int64_t)d * M - M;
      const int r = (int)(k / d), c = (int)(k % d);
      v = mlp[(int64_t)D * M + (int64_t)r * D + c];
    } else {
      v = mlp[2LL * D * M + M + (i - 4LL * d * d - 2LL * d * M - M)];
    }
    g[i] += scale * v;
  }
}

// ------------------------------------------------------------------ launchers
template <class P, int D>
static int32_t mlp_t(const BwdArgs& a, int blocks, hipStream_t st) {
  const size_t lds = (size_t)(2 * D * a.M + a.M + D) * 4 + 4 * 32 * TS * 4;
  auto k = k_bwd_mlp<P, D>;
  TDO_TRY(allow_full_lds((const void*)k));
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, st, a);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

template <class P, int D, int DH, bool SPAN>
static int32_t attn_t(const BwdArgs& a, int blocks, hipStream_t st) {
  const size_t lds = (size_t)4 * D * D * 4 + 4 * 32 * TS * 4;
  auto k = k_bwd_attn<P, D, DH, SPAN>;
  TDO_TRY(allow_full_lds((const void*)k));
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), lds, st, a);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

size_t bwd_mlp_lds(int D, int M) { return (size_t)(2 * D * M + M + D) * 4 + 4 * 32 * TS * 4; }

int32_t launch_bwd_mlp(const BwdArgs& a, bool bf16, int D, int blocks, hipStream_t st) {
  if (D == 32) return bf16 ? mlp_t<PBF16, 32>(a, blocks, st) : mlp_t<PF32, 32>(a, blocks, st);
  if (D == 64) return bf16 ? mlp_t<PBF16, 64>(a, blocks, st) : mlp_t<PF32, 64>(a, blocks, st);
  return set_error(TDO_EUNSUPPORTED, "no MLP backward kernel for width %d", D);
}

template <class P>
static int32_t attn_p(const BwdArgs& a, int D, int DH, int blocks, hipStream_t st) {
  const bool sp = a.span != 0;
  if (D == 32 && DH == 8) return sp ? attn_t<P, 32, 8, true>(a, blocks, st) : attn_t<P, 32, 8, false>(a, blocks, st);
  if (D == 64 && DH == 8) return sp ? attn_t<P, 64, 8, true>(a, blocks, st) : attn_t<P, 64, 8, false>(a, blocks, st);
  if (D == 64 && DH == 16) return sp ? attn_t<P, 64, 16, true>(a, blocks, st) : attn_t<P, 64, 16, false>(a, blocks, st);
  return set_error(TDO_EUNSUPPORTED, "no attention backward kernel for width %d, head width %d", D, DH);
}

int32_t launch_bwd_attn(const BwdArgs& a, bool bf16, int D, int DH, int blocks, hipStream_t st) {
  return bf16 ? attn_p<PBF16>(a, D, DH, blocks, st) : attn_p<PF32>(a, D, DH, blocks, st);
}

int32_t launch_bwd_head(bool bf16, int D, const void* save_last, const float* seeds, const int64_t* E_dev,
                        int64_t E_host, int n, int cpb, int span, int d_real, double* gw, double* gb, double* part,
                        hipStream_t st) {
  constexpr int G = HEAD_BLOCKS;
  if (D == 32) {
    if (bf16) hipLaunchKernelGGL((k_bwd_head<PBF16, 32>), dim3(G), dim3(256), 0, st, save_last, seeds, E_dev, E_host, n, cpb, span, d_real, part);
    else hipLaunchKernelGGL((k_bwd_head<PF32, 32>), dim3(G), dim3(256), 0, st, save_last, seeds, E_dev, E_host, n, cpb, span, d_real, part);
  } else {
    if (bf16) hipLaunchKernelGGL((k_bwd_head<PBF16, 64>), dim3(G), dim3(256), 0, st, save_last, seeds, E_dev, E_host, n, cpb, span, d_real, part);
    else hipLaunchKernelGGL((k_bwd_head<PF32, 64>), dim3(G), dim3(256), 0, st, save_last, seeds, E_dev, E_host, n, cpb, span, d_real, part);
  }
  TDO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_head, dim3(2 * d_real + 2), dim3(256), 0, st, part, G, d_real, gw, gb);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_embed_scatter(int D, const float* dx0, const uint64_t* ecfg, const int64_t* E_dev, int64_t E_host,
                             int n, int cpb, int span, float* partial, int blocks, hipStream_t st) {
  // `blocks` workgroups of 4 waves; each wave writes one [64][D] partial (4 * blocks partials)
  if (D == 32) hipLaunchKernelGGL(k_embed_onehot<32>, dim3(blocks), dim3(256), 0, st, dx0, ecfg, E_dev, E_host, n, cpb, span, partial);
  else hipLaunchKernelGGL(k_embed_onehot<64>, dim3(blocks), dim3(256), 0, st, dx0, ecfg, E_dev, E_host, n, cpb, span, partial);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_embed_params(const float* params, const double* dT, int d, int D, double* grad, double* part,
                            hipStream_t st) {
  TDO_CHECK(d <= 64, TDO_EUNSUPPORTED, "embedding chain rule: width %d > 64", d);
  const int64_t len = 6LL * d + 2LL * d * d;
  hipLaunchKernelGGL(k_embed_params, dim3(64), dim3(64), 0, st, params, dT, d, D, part);
  TDO_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_embed_params_sum, dim3((unsigned)ceil_div(len, 256)), dim3(256), 0, st, part, len, grad);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_reduce_partials(const float* part, int nparts, int64_t len, double* out, hipStream_t st) {
  if (len <= 0) return TDO_OK;
  if (ceil_div(len, 64) >= 256) {  // enough workgroups with 4 groups of partials
    hipLaunchKernelGGL(k_reduce_partials<64>, dim3((unsigned)ceil_div(len, 64)), dim3(256), 0, st, part, nparts, len, out);
  } else {
    hipLaunchKernelGGL(k_reduce_partials<16>, dim3((unsigned)ceil_div(len, 16)), dim3(256), 0, st, part, nparts, len, out);
  }
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_scatter_layer(const double* mlp, const double* attn, int d, int D, int M, double scale, double* g,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_layer, dim3(256), dim3(256), 0, st, mlp, attn, d, D, M, scale, g);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // namespace tdo
