// Backward of the residual multi-head attention sub-layer y = x + concat_h(O_h) W_O,
// O_h = softmax(Q_h K_h^T / sqrt(dh)) V_h, Q = x Wq, K = x Wk, V = x Wv
// (Eq. attn-head-appendix), for width 64 with BF16 MFMA operands and FP32
// accumulation, chains of n <= 32 sites (configurations never span blocks):
//   dO = g W_O^T;  per head: P = exp2(S - lse) from the log2 row normalisers lse the forward
//   saved (the scores S here are the same bits as there), dP' = (dO / sqrt(dh)) V^T,
//   dS = P (dP' - rowsum(P dP')) (= P (dP - rowsum(P dP)) / sqrt(dh)),
//   dQ = dS K, dK = dS^T Q, dV = P^T dO;  dx = g + dQ Wq^T + dK Wk^T + dV Wv^T;
//   dW_O += O^T g, dWq += x^T dQ, dWk += x^T dK, dWv += x^T dV.
//
// Work decomposition.  A workgroup of 4 waves walks tiles of 2 blocks of 32 rows; wave w
// handles head block w / 2 (attention features [32 (w/2), 32 (w/2) + 32)) of block w % 2 of
// the tile, then owns one whole weight gradient (w = 0..3: Wq, Wk, Wv, W_O), accumulated in
// registers for the whole launch.  Two such workgroups run on each CU (80 KB of LDS each), so
// the two waves of a SIMD belong to different workgroups: their barriers are independent and
// they drift into different phases of their tiles (one in the matrix-core-heavy projections
// or gradient products while the other runs its softmax), which a single 8-wave workgroup
// over 4 blocks, whose waves all meet at every barrier, did not allow.  After the workgroup
// barrier that follows the staging, the wave of head block hb forms dx for output features
// [32 hb, 32 hb + 32), reading the other head block's dQ, dK, dV from the staging.
//
// Block phase (one wave per head block).  Every contraction over keys or queries needs its
// operands with lanes enumerating features and values enumerating rows, the
// transpose of what the projections give, and the contractions over queries need the
// probability and dS tiles key-major, the transpose of how they are computed.  All of these
// go through LDS: the tile is written as it is and read back with gfx950's transposing LDS
// read (ds_read_b64_tr_b16), which costs no matrix-core work.  Each head's products go
// into fresh accumulators of which only that head's features are kept, so no operand is
// masked per head.
//
// Gradient phase (all waves).  x, g, O, dQ, dK, dV of each block are staged
// in LDS row-major (one 16-byte write per operand and lane, see stage_r), and read
// back as row-contraction operands with the transposing read.  After a workgroup
// barrier, wave w adds the tile's 2 x 32 rows into its gradient.  Each workgroup
// writes its four gradients once per launch to its partial slot [4 D^2] (Wq, Wk, Wv as
// (in, attention feature), W_O as (attention feature, out)); the slots are
// summed in FP64 afterwards.
//
// The kernel for 32 < n <= 64 further down works the same way over two row blocks.
#include "common.h"
#include "net.h"
#include "netapi.h"

namespace tdo {

namespace {

constexpr int MAT = 64 * 32;  // one staged matrix: 32 rows x 64 features (BF16)
constexpr int ATTN_BPT = 2;   // blocks of 32 rows a tile of the n <= 32 kernel (its workgroup: 2 BPT waves)
enum { SX = 0, SG = 1, SQ = 2, SK = 3, SV = 4, SO = 5, NSTAGE = 6 };

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ f32x16 mfma16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
// Row-major staged matrix of 32 rows x 64 features (BF16) for gfx950's transposing LDS read.
// A row is 128 bytes, 8 units of 16 bytes; unit u = 4 fb + 2 s + hh holds the two 4-feature
// chunks 32 fb + 16 s + 4 hh + (0..3) and 32 fb + 16 s + 8 + 4 hh + (0..3): exactly the BF16
// operand s of lane half hh of the row-major tile of feature block fb, so a lane stages an
// operand with one 16-byte write.  Unit u of row r sits at position u ^ f(r), f(r) = (bit 1 of
// r, bit 2 of r, bit 0 of r) as bits (2, 1, 0).  Measured on gfx950 (bank-conflict counter of
// an LDS probe): a 16-byte write serves 8 lanes per cycle over 128 bytes, a transposing read 32
// lanes per cycle over 64 banks of 4 bytes; f gives the 8 rows of a write phase 8 distinct
// units and the 4 rows of a read phase (rows 4k .. 4k+3, both feature halves) 64 distinct
// banks.
__device__ __forceinline__ int rsw(int u, int row) {
  return u ^ ((((row >> 1) & 1) << 2) | (((row >> 2) & 1) << 1) | (row & 1));
}
// The lane's part of its row's unit offsets: unit 4 fb + 2 s + h of row lr starts at element
// rh ^ (32 fb + 16 s), rh = 64 lr | ((8 h) ^ 8 f(lr)) (the XOR acts on bits 3..5 only).  One
// register for every staged write and row read of the lane, instead of one per unit.
__device__ __forceinline__ int stage_rh(int lr, int h) { return lr * 64 | (rsw(h, lr) * 8); }
__device__ __forceinline__ void stage_r(__bf16* m, int fb, const bf16x8& o0, const bf16x8& o1, int rh) {
  *reinterpret_cast<bf16x8*>(m + (rh ^ (32 * fb))) = o0;
  *reinterpret_cast<bf16x8*>(m + (rh ^ (32 * fb + 16))) = o1;
}
// The same writes with the offsets formed from the row and the lane half (the compiler keeps
// them as it sees fit): the 32 < n <= 64 kernel measured faster with this form.
__device__ __forceinline__ void stage_r(__bf16* m, int fb, const bf16x8& o0, const bf16x8& o1, int lr, int h) {
  *reinterpret_cast<bf16x8*>(m + lr * 64 + rsw(4 * fb + h, lr) * 8) = o0;
  *reinterpret_cast<bf16x8*>(m + lr * 64 + rsw(4 * fb + 2 + h, lr) * 8) = o1;
}
// ds_read_b64_tr_b16: within each group of 16 lanes, lane 4t + u supplies the address of 4
// consecutive BF16 values and lane 4u + c receives, as its value t, value c of lane 4t + u.
__device__ __forceinline__ s16x4 tr16(const __bf16* p) {
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4*)(p));
}
// Element offset that lane (16 g + 4 t + u) of a transposing read addresses in a staged matrix:
// row `row`, the 4-feature chunk 16 (g & 1) + 4 u of feature block fb.
__device__ __forceinline__ int tr_off(int row, int fb, int lane) {
  const int g = lane >> 4, u = lane & 3;
  return row * 64 + rsw(4 * fb + 2 * (g & 1) + (u & 1), row) * 8 + 4 * (u >> 1);
}
// Feature-major operand read from a staged matrix: lane l gets feature 32 fb + l % 32 at 8 rows,
// value 4 rd + t from row 8 rd + (row of off).  off = tr_off(row of this lane's t, fb, l) plus
// the offset of whole 16-row parts; 8 rows further keep the unit positions (f reads rows
// modulo 8), so the second read is 512 elements on.
__device__ __forceinline__ bf16x8 tr_op(const __bf16* m, int off) {
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  const s16x4 a = tr16(m + off), b = tr16(m + off + 8 * 64);
  return __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

// -l (a softmax normaliser negated) as three BF16 terms with hi + mid + lo = -l exactly
// (each term the next 8 significant bits; -inf stays in hi), packed as two operand registers.
__device__ __forceinline__ u32x2 neg_terms(float l) {
  const float x = -l;
  const float hi = (float)(__bf16)x;
  const float r1 = __builtin_isinf(x) ? 0.f : x - hi;
  const float mid = (float)(__bf16)r1;
  const float lo = (float)(__bf16)(r1 - mid);
  return (u32x2){pk2(hi, mid), pk2(lo, 0.f)};
}

}  // namespace

// Two workgroups per CU (LDS 80 KB each, two waves per SIMD, one of each workgroup).
template <int DH, bool MASKED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) k_bwd_attn_bf16(BwdArgs a) {
  constexpr int D = 64, NB = 2, ST = 2, HPB = 32 / DH, NT = 256, BPT = ATTN_BPT;
  extern __shared__ __align__(16) char smem[];
  __bf16* Wl = reinterpret_cast<__bf16*>(smem);      // Wq, Wk, Wv, W_O^T fragments [4][D*D]
  __bf16* stg = Wl + 4 * D * D;                       // [BPT blocks][NSTAGE][MAT]

  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, lr = lane & 31;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform (scalar branches below)
  const int bw = w & 1, hb = w >> 1;  // block of the tile, head block
  {
    const int4* sf = reinterpret_cast<const int4*>(a.wf);
    const int4* sb = reinterpret_cast<const int4*>(a.wb);
    int4* dl = reinterpret_cast<int4*>(Wl);
    for (int i = t; i < 3 * D * D / 8; i += NT) dl[i] = sf[i];
    for (int i = t; i < D * D / 8; i += NT) dl[3 * D * D / 8 + i] = sb[3 * D * D / 8 + i];
  }
  const __bf16 *Wq = Wl, *Wk = Wl + D * D, *Wv = Wl + 2 * D * D, *WoT = Wl + 3 * D * D;
  // Wq^T, Wk^T, Wv^T fragments [3][D*D] BF16 in global memory (L2-resident), read through a
  // buffer resource: one lane offset shared by all fragments and a uniform offset per
  // fragment, instead of one 64-bit address per fragment kept live across the tile loop
  const __amdgpu_buffer_rsrc_t WT = rsrc(a.wb, 3 * D * D * 2);
  __syncthreads();

  const int64_t E = a.n_entries_dev ? *a.n_entries_dev : a.n_entries;
  const int n = a.n, cpb = a.cpb;
  const int64_t nblk = 2 * ((E + cpb - 1) / cpb);
  const int64_t ntile = (nblk + BPT - 1) / BPT;
  const float sc = a.score_scale, isd = a.inv_sqrt_dh;
  // valid (query, key) pairs of this lane's row lr against rows tile_idx(r, h): same configuration
  // slot, slot < cpb (symmetric, so the same bits serve query-major and key-major tiles)
  uint32_t okbits = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int other = tile_idx(r, h) / n;
    okbits |= (other == lr / n && other < cpb) ? (1u << r) : 0u;
  }

  // this lane's transposing-read offsets per feature block: rows tile_idx(8 s + 4 rd + t, l / 32),
  // t = (l & 15) >> 2 (the key order of the score tiles, and the row order of the gradient
  // products' K steps), 16 s rows on for operand s
  const int tb[2] = {tr_off(4 * h + ((lane & 15) >> 2), 0, lane), tr_off(4 * h + ((lane & 15) >> 2), 1, lane)};
  const int thb = hb ? tb[1] : tb[0];
  int rh = stage_rh(lr, h);

  f32x16 dW[NB][NB];  // weight gradient w (Wq, Wk, Wv, W_O), all 64 x 64
#pragma unroll
  for (int k = 0; k < NB; ++k)
#pragma unroll
    for (int j = 0; j < NB; ++j) dW[k][j] = f32x16{};

  // x (layer input, saved in BF16) and g (gradient of the sub-layer output) of block gb, lane ->
  // row, values -> features 32 ib + tile_idx(r, h); loaded one tile ahead, so that the
  // latency of the loads is covered by the previous tile's gradient phase
  bf16x8 xn[NB][ST];
  float4 gn[NB][4];
  float ln[HPB];  // the forward's log2 softmax normalisers of this lane's query row, heads of head block hb
  auto fetch = [&](int64_t tl) {
    // the block's saved normalisers, x and g through buffer resources at the block (scalar
    // bases and one lane offset each, no 64-bit addresses per lane); past the last block the
    // resources are empty and the loads return zeros
    const int64_t g = (int64_t)BPT * tl + bw;
    const bool ok = tl < ntile && g < nblk;
    const int64_t gg = ok ? g : 0;
    const auto lres = rsrc(a.lse + gg * 32 * (NB * HPB), ok ? 32 * NB * HPB * 4 : 0);
    const auto xres = rsrc(reinterpret_cast<const __bf16*>(a.save_x) + gg * NB * 64 * 16, ok ? NB * 64 * 16 * 2 : 0);
    const auto gres = rsrc(a.g_in + gg * NB * 64 * 16, ok ? NB * 64 * 16 * 4 : 0);
    // the lane offsets (lane * 32 for x, lane * 64 for g) formed here from the lane id, not kept
    // in registers across the tile loop
    int l32;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0\n\tv_lshlrev_b32 %0, 5, %0" : "=v"(l32));
    if constexpr (HPB == 4) {
      // row lr's normalisers at lr * 32 bytes: the x offset with the lane half masked off
      const float4 v = rld4(lres, l32 & 0x3ff, hb * HPB * 4);
      ln[0] = v.x; ln[1] = v.y; ln[2] = v.z; ln[3] = v.w;
    } else {
      static_assert(NB * HPB * 4 == 16, "row lr's two normalisers of each head block at lr * 16 bytes");
      const float2 v = rld2(lres, ((l32 & 0x3ff) >> 1) + hb * HPB * 4);
      ln[0] = v.x; ln[1] = v.y;
    }
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      xn[ib][0] = rld8(xres, l32, ib * 64 * 16 * 2);
      xn[ib][1] = rld8(xres, l32, ib * 64 * 16 * 2 + 16);
#pragma unroll
      for (int q = 0; q < 4; ++q) gn[ib][q] = rld4(gres, 2 * l32, ib * 64 * 64 + 16 * q);
    }
  };
  fetch(blockIdx.x);

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    // rh opaque to the loop: the unit offsets rh ^ c are formed where used, not kept in registers
    asm volatile("" : "+v"(rh));
    // ================= block phase: head block hb of block gb
    const int64_t gb = (int64_t)BPT * tile + bw;
    const bool valid = gb < nblk;
    __bf16* S = stg + bw * NSTAGE * MAT;
    // the block's x and g as BF16 operands (values tile_idx(8 s + t, h))
    bf16x8 xo[NB][ST], go[NB][ST];
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      f32x16 gr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        gr[4 * q] = gn[ib][q].x; gr[4 * q + 1] = gn[ib][q].y; gr[4 * q + 2] = gn[ib][q].z; gr[4 * q + 3] = gn[ib][q].w;
      }
      xo[ib][0] = xn[ib][0];
      xo[ib][1] = xn[ib][1];
      go[ib][0] = cvt8(gr, 0);
      go[ib][1] = cvt8(gr, 1);
    }
    // the wave of head block 0 stages x, the other g
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      if (hb == 0) stage_r(S + SX * MAT, ib, xo[ib][0], xo[ib][1], rh);
      else stage_r(S + SG * MAT, ib, go[ib][0], go[ib][1], rh);
    }

    // projections of the 32 attention features of head block hb, row-major (*R: lane -> row,
    // values -> features), packed to BF16 operands right away to keep the register peak low:
    // per-head score operands (q scaled by log2(e)/sqrt(dh), dO by 1/sqrt(dh)).  The
    // feature-major tiles (*F: lane -> feature, values -> rows in the key order of the score
    // tiles) are read back transposed from LDS; dK and dV, formed from the scaled q and dO,
    // are rescaled in the head loop.
    using sop = PBF16::SOp<DH>;
    sop QRp[HPB], KRp[HPB], VRp[HPB], ORp[HPB];
    bf16x8 QFb[ST], KFb[ST], VFb[ST], OFb[ST];
    // row-major operand s (values 8s .. 8s+7) of a projection from its per-head packs
    auto rop = [&](const sop (&P)[HPB], int s) -> bf16x8 {
      if constexpr (DH == 8) {
        const u32x2 lo = __builtin_bit_cast(u32x2, P[2 * s].v), hi = __builtin_bit_cast(u32x2, P[2 * s + 1].v);
        return __builtin_bit_cast(bf16x8, (u32x4){lo[0], lo[1], hi[0], hi[1]});
      } else {
        return P[s].v;
      }
    };
    {
      f32x16 QR = {}, KR = {};
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          const int f = ((hb * NB + ib) * ST + s) * 64 + lane;
          const bf16x8 wq = ld8(Wq + f * 8), wk = ld8(Wk + f * 8);
          QR = mfma16(wq, xo[ib][s], QR);
          KR = mfma16(wk, xo[ib][s], KR);
        }
#pragma unroll
      for (int r = 0; r < 16; ++r) QR[r] *= sc;
#pragma unroll
      for (int j = 0; j < HPB; ++j) {
        QRp[j] = PBF16::pack_head<DH>(QR, j);
        KRp[j] = PBF16::pack_head<DH>(KR, j);
      }
      // feature-major tiles through LDS: this wave's feature half of the dQ and dK staging
      // slots is free until it stages dQ and dK there after the head loop
      stage_r(S + SQ * MAT, hb, rop(QRp, 0), rop(QRp, 1), rh);
      stage_r(S + SK * MAT, hb, rop(KRp, 0), rop(KRp, 1), rh);
#pragma unroll
      for (int s = 0; s < ST; ++s) { QFb[s] = tr_op(S + SQ * MAT, thb + 1024 * s); KFb[s] = tr_op(S + SK * MAT, thb + 1024 * s); }
    }
    {
      f32x16 VR = {}, OR = {};  // V and dO = g W_O^T
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          const int f = ((hb * NB + ib) * ST + s) * 64 + lane;
          const bf16x8 wv = ld8(Wv + f * 8), wo = ld8(WoT + f * 8);
          VR = mfma16(wv, xo[ib][s], VR);
          OR = mfma16(wo, go[ib][s], OR);
        }
      // dO as the score operand of dP carries the factor 1/sqrt(dh) of dS
#pragma unroll
      for (int r = 0; r < 16; ++r) OR[r] *= isd;
#pragma unroll
      for (int j = 0; j < HPB; ++j) {
        VRp[j] = PBF16::pack_head<DH>(VR, j);
        ORp[j] = PBF16::pack_head<DH>(OR, j);
      }
      stage_r(S + SV * MAT, hb, rop(VRp, 0), rop(VRp, 1), rh);
      stage_r(S + SO * MAT, hb, rop(ORp, 0), rop(ORp, 1), rh);
#pragma unroll
      for (int s = 0; s < ST; ++s) { VFb[s] = tr_op(S + SV * MAT, thb + 1024 * s); OFb[s] = tr_op(S + SO * MAT, thb + 1024 * s); }
    }
    float lse[HPB];
#pragma unroll
    for (int j = 0; j < HPB; ++j) lse[j] = ln[j];
    // dQ, dK, dV and the attention output O, all row-major (lane -> row, values -> features).
    // Each head's products go into fresh accumulators with unmasked feature-major operands:
    // of such a product only values [VPH j, VPH (j + 1)) of each lane (the features of head j,
    // see tile_idx) are head j's result, and they are kept; the other values, formed from head
    // j's P or dS against other heads' features, are dropped.  No operand is masked per head.
    // The kept values are scaled where needed (dK and dV were formed from q scaled by sc and dO
    // scaled by 1/sqrt(dh)) and packed to BF16 operand words right away: value pair (2w, 2w + 1)
    // is word w % 4 of operand w / 4.
    constexpr int VPH = DH / 2;
    const float isc = 1.0f / sc, sdh = 1.0f / isd;
    u32x4 ow[ST], qw[ST], kw[ST], vw[ST];
#pragma unroll
    for (int j = 0; j < HPB; ++j) {
      // query-major tiles: lane -> query lr, values -> keys tile_idx(r, h)
      f32x16 sq;
      if constexpr (DH == 8) {
        // S - lse on the matrix cores (one 16-deep product, the cost of the 8-deep one): the head's
        // features at k = 8h + 0..3 of both operands, and in the first half's lanes the query's
        // -lse as three exact BF16 terms against ones at k = 4..6
        const u32x2 kb = __builtin_bit_cast(u32x2, KRp[j].v), qb = __builtin_bit_cast(u32x2, QRp[j].v);
        const u32x2 t = neg_terms(lse[j]);
        const uint32_t one2 = pk2(1.f, 1.f), one1 = pk2(1.f, 0.f);
        const bf16x8 ko = __builtin_bit_cast(bf16x8, (u32x4){kb[0], kb[1], h == 0 ? one2 : 0u, h == 0 ? one1 : 0u});
        const bf16x8 qo = __builtin_bit_cast(bf16x8, (u32x4){qb[0], qb[1], h == 0 ? t[0] : 0u, h == 0 ? t[1] : 0u});
        sq = mfma16(ko, qo, f32x16{});
      } else {
        sq = PBF16::scores_packed<DH>(KRp[j], QRp[j], f32x16{});
      }
      f32x16 dpq = PBF16::scores_packed<DH>(VRp[j], ORp[j], f32x16{});
      if constexpr (MASKED) {  // a compile-time choice keeps the head loop one scheduling region
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (!((okbits >> r) & 1u)) sq[r] = -INFINITY;
      }
      // P from the forward's normaliser of the row (its scores are the same bits); +inf for a
      // query with no key gives P = 0
      float dl = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        sq[r] = __builtin_amdgcn_exp2f(DH == 8 ? sq[r] : sq[r] - lse[j]);  // P
        dl += sq[r] * dpq[r];
      }
      dl = xor32_sum(dl);
#pragma unroll
      for (int r = 0; r < 16; ++r) dpq[r] = sq[r] * (dpq[r] - dl);  // dS (dP carries 1/sqrt(dh))
      bf16x8 Pq[ST], Sq[ST];
#pragma unroll
      for (int s = 0; s < ST; ++s) { Pq[s] = cvt8(sq, s); Sq[s] = cvt8(dpq, s); }
      // key-major P and dS (lane -> key, values -> queries) through LDS: written query-major into
      // this wave's half of the dQ and dK staging slots (free until the staging after the head loop;
      // the previous head's reads of them are ordered before these writes), read back transposed
      // after the query-major products below are issued
      stage_r(S + SQ * MAT, hb, Pq[0], Pq[1], rh);
      stage_r(S + SK * MAT, hb, Sq[0], Sq[1], rh);
      // two products at a time (four fresh accumulators at once would not fit in the registers)
      {
        f32x16 to = {}, tq = {};
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          to = mfma16(VFb[s], Pq[s], to);  // O[q][f]  = sum_k P[q][k] V[k][f]
          tq = mfma16(KFb[s], Sq[s], tq);  // dQ[q][f] = sum_k dS[q][k] K[k][f]
        }
#pragma unroll
        for (int w = VPH * j / 2; w < VPH * (j + 1) / 2; ++w) {
          ow[w / 4][w % 4] = pk2(to[2 * w], to[2 * w + 1]);
          qw[w / 4][w % 4] = pk2(tq[2 * w], tq[2 * w + 1]);
        }
      }
      {
        bf16x8 Pk[ST], Sk[ST];
#pragma unroll
        for (int s = 0; s < ST; ++s) { Pk[s] = tr_op(S + SQ * MAT, thb + 1024 * s); Sk[s] = tr_op(S + SK * MAT, thb + 1024 * s); }
        f32x16 tk = {}, tv = {};
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          tk = mfma16(QFb[s], Sk[s], tk);  // dK[k][f] = sum_q dS[q][k] Q[q][f]
          tv = mfma16(OFb[s], Pk[s], tv);  // dV[k][f] = sum_q P[q][k] dO[q][f]
        }
#pragma unroll
        for (int w = VPH * j / 2; w < VPH * (j + 1) / 2; ++w) {
          kw[w / 4][w % 4] = pk2(tk[2 * w] * isc, tk[2 * w + 1] * isc);
          vw[w / 4][w % 4] = pk2(tv[2 * w] * sdh, tv[2 * w + 1] * sdh);
        }
      }
      // heads are independent now: keep the scheduler from interleaving them, which would
      // hold several heads' score tiles and accumulators in registers at once
    }
    // stage dQ, dK, dV and O (R layout -> [feature][row])
    bf16x8 dq[ST], dk[ST], dv[ST];
#pragma unroll
    for (int s = 0; s < ST; ++s) {
      dq[s] = __builtin_bit_cast(bf16x8, qw[s]);
      dk[s] = __builtin_bit_cast(bf16x8, kw[s]);
      dv[s] = __builtin_bit_cast(bf16x8, vw[s]);
    }
    stage_r(S + SQ * MAT, hb, dq[0], dq[1], rh);
    stage_r(S + SK * MAT, hb, dk[0], dk[1], rh);
    stage_r(S + SV * MAT, hb, dv[0], dv[1], rh);
    stage_r(S + SO * MAT, hb, __builtin_bit_cast(bf16x8, ow[0]), __builtin_bit_cast(bf16x8, ow[1]), rh);
    // dx = g + dQ Wq^T + dK Wk^T + dV Wv^T, output feature block hb from this wave: after the
    // barrier it reads the other head block's dQ, dK, dV from the staging (the 16-byte operands
    // that wave staged) and sums (g + terms of attention block 0) + terms of attention block 1.
    // g is loaded before the barrier, where the wave may wait for the other waves.
    auto dx_terms = [&](int ib, const bf16x8 (&q)[ST], const bf16x8 (&k)[ST], const bf16x8 (&v)[ST]) {
      f32x16 acc = {};
      const int voff = lane * 16;  // fragment ((hb NB + ib) ST + s) of each matrix, ib in the scalar offset
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        const int so = ((hb * NB + ib) * ST + s) * 64 * 16;
        acc = mfma16(rld8(WT, voff, so), q[s], acc);
        acc = mfma16(rld8(WT, voff, so + D * D * 2), k[s], acc);
        acc = mfma16(rld8(WT, voff, so + 2 * D * D * 2), v[s], acc);
      }
      return acc;
    };
    // the block's g and dx through buffer resources at the block (a wave-uniform base and one
    // lane offset, instead of 64-bit addresses per lane kept live across the tile loop); empty
    // past the last block
    constexpr uint32_t BLK_BYTES = NB * 64 * 16 * sizeof(float);
    const auto gres = rsrc(a.g_in + (valid ? gb : 0) * NB * 64 * 16, valid ? BLK_BYTES : 0);
    const auto dres = rsrc(a.g_out + (valid ? gb : 0) * NB * 64 * 16, valid ? BLK_BYTES : 0);
    float4 sv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) sv[q] = rld4(gres, lane * 64, hb * 64 * 64 + 16 * q);
    barrier_lds();  // staging of both head blocks in LDS
    if (valid) {
      bf16x8 oq[ST], ok[ST], ov[ST];  // the other head block's operands, as it staged them
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        const int e = rh ^ (32 * (hb ^ 1) + 16 * s);
        oq[s] = ld8(S + SQ * MAT + e);
        ok[s] = ld8(S + SK * MAT + e);
        ov[s] = ld8(S + SV * MAT + e);
      }
      f32x16 a0, a1;
      if (hb == 0) {
        a0 = dx_terms(0, dq, dk, dv);
        a1 = dx_terms(1, oq, ok, ov);
      } else {
        a0 = dx_terms(0, oq, ok, ov);
        a1 = dx_terms(1, dq, dk, dv);
      }
      // all four results formed before the first store: the stores' data registers are then not
      // rewritten by the vector ALU right behind the store that reads them
      float4 o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 g = sv[q];
        o[q] = make_float4((g.x + a0[4 * q]) + a1[4 * q], (g.y + a0[4 * q + 1]) + a1[4 * q + 1],
                           (g.z + a0[4 * q + 2]) + a1[4 * q + 2], (g.w + a0[4 * q + 3]) + a1[4 * q + 3]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) rst4(dres, lane * 64, o[q], hb * 64 * 64 + 16 * q);
    }
    // issued after the dx step, whose loads would otherwise wait behind these in the in-order load counter
    fetch(tile + gridDim.x);

    // ================= gradient phase: wave w adds the tile's rows into its weight gradient rows
    {
      const int am = (w < 3) ? SX : SO;      // A operand: x (for Wq, Wk, Wv) or O (for W_O)
      const int bm = (w < 3) ? SQ + w : SG;  // B operand: dQ, dK, dV or g
#pragma unroll
      for (int b = 0; b < BPT; ++b) {
        const __bf16* A = stg + (b * NSTAGE + am) * MAT;
        const __bf16* B = stg + (b * NSTAGE + bm) * MAT;
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          bf16x8 av[NB], bv[NB];
#pragma unroll
          for (int k = 0; k < NB; ++k) av[k] = tr_op(A, tb[k] + 1024 * s);
#pragma unroll
          for (int j = 0; j < NB; ++j) bv[j] = tr_op(B, tb[j] + 1024 * s);
#pragma unroll
          for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int j = 0; j < NB; ++j) dW[k][j] = mfma16(av[k], bv[j], dW[k][j]);
        }
      }
    }
    barrier_lds();  // staging read before the next tile overwrites it
  }

  float* part = a.partial + (int64_t)blockIdx.x * 4 * D * D + (int64_t)w * D * D;
#pragma unroll
  for (int k = 0; k < NB; ++k)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) part[(32 * k + tile_idx(r, h)) * D + 32 * j + lr] = dW[k][j][r];
}

// Chains of 32 < n <= 64 sites: one configuration-pass spans two blocks (rows 0-31, 32-63;
// rows >= n are padding, and keys >= n are masked).  A workgroup of 4 waves (one per SIMD,
// all its registers) walks tiles of 4 blocks = 2 configuration-passes; wave w handles head
// block w % 2 of configuration-pass w / 2 over both of its blocks: score, P and dS tiles are
// 2 x 2 (query block x key block), P comes from the forward's normalisers, dK and dV of a
// key block sum over both query blocks.  Staging, the transposes through the transposing
// LDS read, dx by output feature block and the per-wave weight gradients (wave w owns all
// of Wq, Wk, Wv, W_O for w = 0..3) are those of the kernel above; the products
// keep feature-major operands masked per head (fresh accumulators per head would not fit
// next to the 2 x 2 tiles).  Padding rows add nothing: their keys have P = 0 and their
// incoming gradient is 0 (it is formed from the seeds of valid rows only).
// PAD16 (n <= 48): rows 48..63 of a pass are padding, so every product whose contraction runs
// over them adds exact zeros (keys: P = 0; queries: dS = 0 and dO = 0; rows of the weight
// gradients: dQ, dK, dV, g = 0) and is skipped; the staged tiles are still written whole.
template <int DH, bool MASKED, bool PAD16>
__global__ void __launch_bounds__(256) k_bwd_attn_span_bf16(BwdArgs a) {
  constexpr int D = 64, NB = 2, ST = 2, HPB = 32 / DH;
  extern __shared__ __align__(16) char smem[];
  __bf16* Wl = reinterpret_cast<__bf16*>(smem);
  __bf16* stg = Wl + 4 * D * D;

  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, lr = lane & 31;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int cp = w >> 1, hb = w & 1;  // configuration-pass of the tile, head block
  {
    const int4* sf = reinterpret_cast<const int4*>(a.wf);
    const int4* sb = reinterpret_cast<const int4*>(a.wb);
    int4* dl = reinterpret_cast<int4*>(Wl);
    for (int i = t; i < 3 * D * D / 8; i += 256) dl[i] = sf[i];
    for (int i = t; i < D * D / 8; i += 256) dl[3 * D * D / 8 + i] = sb[3 * D * D / 8 + i];
  }
  const __bf16 *Wq = Wl, *Wk = Wl + D * D, *Wv = Wl + 2 * D * D, *WoT = Wl + 3 * D * D;
  const __amdgpu_buffer_rsrc_t WT = rsrc(a.wb, 3 * D * D * 2);
  __syncthreads();

  const int64_t E = a.n_entries_dev ? *a.n_entries_dev : a.n_entries;
  const int n = a.n;
  const int64_t ntile = E;  // 4 blocks (2 configuration-passes) per entry
  const float sc = a.score_scale, isd = a.inv_sqrt_dh;
  // transposing-read offsets, as in the kernel above
  const int tb[2] = {tr_off(4 * h + ((lane & 15) >> 2), 0, lane), tr_off(4 * h + ((lane & 15) >> 2), 1, lane)};
  const int thb = hb ? tb[1] : tb[0];
  // valid keys of the second key block: rows 32 + tile_idx(r, h) < n (the first block is all valid)
  uint32_t ok1 = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) ok1 |= (32 + tile_idx(r, h) < n) ? (1u << r) : 0u;

  f32x16 dW[NB][NB];  // weight gradient w (Wq, Wk, Wv, W_O)
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) dW[i][j] = f32x16{};

  // x, g and the forward's normalisers of the two blocks, one tile ahead
  bf16x8 xn[2][NB][ST];
  float4 gn[2][NB][4];
  float ln[2][HPB];
  auto fetch = [&](int64_t tl) {
    const bool ok = tl < ntile;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int64_t g = ok ? 4 * tl + 2 * cp + rb : 0;
      const float* ls = a.lse + (g * 32 + lr) * (NB * HPB) + hb * HPB;
#pragma unroll
      for (int j = 0; j < HPB; ++j) ln[rb][j] = ls[j];
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        const __bf16* xs = reinterpret_cast<const __bf16*>(a.save_x) + ((g * NB + ib) * 64 + lane) * 16;
        xn[rb][ib][0] = ld8(xs);
        xn[rb][ib][1] = ld8(xs + 8);
        const float4* gs = reinterpret_cast<const float4*>(a.g_in + ((g * NB + ib) * 64 + lane) * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) gn[rb][ib][q] = gs[q];
      }
    }
  };
  fetch(blockIdx.x);

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    // ================= block phase: head block hb of configuration-pass cp (blocks 2 cp, 2 cp + 1)
    bf16x8 xo[2][NB][ST], go[2][NB][ST];
    float lse[2][HPB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
      for (int j = 0; j < HPB; ++j) lse[rb][j] = ln[rb][j];
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        f32x16 gr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          gr[4 * q] = gn[rb][ib][q].x; gr[4 * q + 1] = gn[rb][ib][q].y;
          gr[4 * q + 2] = gn[rb][ib][q].z; gr[4 * q + 3] = gn[rb][ib][q].w;
        }
        xo[rb][ib][0] = xn[rb][ib][0];
        xo[rb][ib][1] = xn[rb][ib][1];
        go[rb][ib][0] = cvt8(gr, 0);
        go[rb][ib][1] = cvt8(gr, 1);
      }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      __bf16* S = stg + (2 * cp + rb) * NSTAGE * MAT;
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        if (hb == 0) stage_r(S + SX * MAT, ib, xo[rb][ib][0], xo[rb][ib][1], lr, h);
        else stage_r(S + SG * MAT, ib, go[rb][ib][0], go[rb][ib][1], lr, h);
      }
    }
    // projections of head block hb for both blocks (see the kernel above: the feature-major
    // tiles are read back transposed from this wave's half of the dQ..O staging slots; dK, dV
    // rescaled below)
    using sop = PBF16::SOp<DH>;
    sop QRp[2][HPB], KRp[2][HPB], VRp[2][HPB], ORp[2][HPB];
    bf16x8 QFb[2][ST], KFb[2][ST], VFb[2][ST], OFb[2][ST];
    auto rop = [&](const sop (&P)[HPB], int s) -> bf16x8 {
      if constexpr (DH == 8) {
        const u32x2 lo = __builtin_bit_cast(u32x2, P[2 * s].v), hi = __builtin_bit_cast(u32x2, P[2 * s + 1].v);
        return __builtin_bit_cast(bf16x8, (u32x4){lo[0], lo[1], hi[0], hi[1]});
      } else {
        return P[s].v;
      }
    };
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      {
        f32x16 QR = {}, KR = {};
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            const int f = ((hb * NB + ib) * ST + s) * 64 + lane;
            const bf16x8 wq = ld8(Wq + f * 8), wk = ld8(Wk + f * 8);
            QR = mfma16(wq, xo[rb][ib][s], QR);
            KR = mfma16(wk, xo[rb][ib][s], KR);
          }
#pragma unroll
        for (int r = 0; r < 16; ++r) QR[r] *= sc;
#pragma unroll
        for (int j = 0; j < HPB; ++j) {
          QRp[rb][j] = PBF16::pack_head<DH>(QR, j);
          KRp[rb][j] = PBF16::pack_head<DH>(KR, j);
        }
        __bf16* S = stg + (2 * cp + rb) * NSTAGE * MAT;
        stage_r(S + SQ * MAT, hb, rop(QRp[rb], 0), rop(QRp[rb], 1), lr, h);
        stage_r(S + SK * MAT, hb, rop(KRp[rb], 0), rop(KRp[rb], 1), lr, h);
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          QFb[rb][s] = tr_op(S + SQ * MAT, thb + 1024 * s);
          KFb[rb][s] = tr_op(S + SK * MAT, thb + 1024 * s);
        }
      }
      {
        f32x16 VR = {}, OR = {};
#pragma unroll
        for (int ib = 0; ib < NB; ++ib)
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            const int f = ((hb * NB + ib) * ST + s) * 64 + lane;
            const bf16x8 wv = ld8(Wv + f * 8), wo = ld8(WoT + f * 8);
            VR = mfma16(wv, xo[rb][ib][s], VR);
            OR = mfma16(wo, go[rb][ib][s], OR);
          }
        // dO as the score operand of dP carries the factor 1/sqrt(dh) of dS
#pragma unroll
        for (int r = 0; r < 16; ++r) OR[r] *= isd;
#pragma unroll
        for (int j = 0; j < HPB; ++j) {
          VRp[rb][j] = PBF16::pack_head<DH>(VR, j);
          ORp[rb][j] = PBF16::pack_head<DH>(OR, j);
        }
        __bf16* S = stg + (2 * cp + rb) * NSTAGE * MAT;
        stage_r(S + SV * MAT, hb, rop(VRp[rb], 0), rop(VRp[rb], 1), lr, h);
        stage_r(S + SO * MAT, hb, rop(ORp[rb], 0), rop(ORp[rb], 1), lr, h);
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          VFb[rb][s] = tr_op(S + SV * MAT, thb + 1024 * s);
          OFb[rb][s] = tr_op(S + SO * MAT, thb + 1024 * s);
        }
      }
    }
    // dQ, dK, dV and O row-major (lane -> row, values -> features), accumulated over heads with
    // the feature-major operands masked to the head; the key-major P and dS of a (query block,
    // key block) pair through this wave's half of the dQ and dK staging slots of block 2 cp
    // (free until the staging after the head loop)
    __bf16* const PS = stg + (2 * cp) * NSTAGE * MAT + SQ * MAT;
    __bf16* const DS = stg + (2 * cp) * NSTAGE * MAT + SK * MAT;
    f32x16 dQR[2], dKR[2], dVR[2], AOR[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) dQR[rb] = dKR[rb] = dVR[rb] = AOR[rb] = f32x16{};
#pragma unroll
    for (int j = 0; j < HPB; ++j) {
      const bool mine = (lr / DH) == j;
      const bf16x8 z = {};
#pragma unroll
      for (int qb = 0; qb < 2; ++qb) {
        // query-major tiles of query block qb against key block kb
        f32x16 sq[2], dpq[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          sq[kb] = PBF16::scores_packed<DH>(KRp[kb][j], QRp[qb][j], f32x16{});
          dpq[kb] = PBF16::scores_packed<DH>(VRp[kb][j], ORp[qb][j], f32x16{});
        }
        if constexpr (MASKED) {
#pragma unroll
          for (int r = 0; r < 16; ++r)
            if (!((ok1 >> r) & 1u)) sq[1][r] = -INFINITY;
        }
        float dl = 0.f;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            if (PAD16 && kb == 1 && r >= 8) {  // keys 48..63: P = 0, no exponential
              sq[1][r] = 0.f;
              continue;
            }
            sq[kb][r] = __builtin_amdgcn_exp2f(sq[kb][r] - lse[qb][j]);  // P
            dl += sq[kb][r] * dpq[kb][r];
          }
        dl = xor32_sum(dl);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
          for (int r = 0; r < 16; ++r)  // dS (dP carries 1/sqrt(dh)); 0 at keys 48..63
            dpq[kb][r] = (PAD16 && kb == 1 && r >= 8) ? 0.f : sq[kb][r] * (dpq[kb][r] - dl);
          bf16x8 Pq[ST], Sq[ST];
#pragma unroll
          for (int s = 0; s < ST; ++s) { Pq[s] = cvt8(sq[kb], s); Sq[s] = cvt8(dpq[kb], s); }
          stage_r(PS, hb, Pq[0], Pq[1], lr, h);
          stage_r(DS, hb, Sq[0], Sq[1], lr, h);
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            if (PAD16 && kb == 1 && s == 1) continue;  // keys 48..63
            AOR[qb] = mfma16(mine ? VFb[kb][s] : z, Pq[s], AOR[qb]);  // O[q][f]  += P[q][k] V[k][f]
            dQR[qb] = mfma16(mine ? KFb[kb][s] : z, Sq[s], dQR[qb]);  // dQ[q][f] += dS[q][k] K[k][f]
          }
#pragma unroll
          for (int s = 0; s < ST; ++s) {
            if (PAD16 && qb == 1 && s == 1) continue;  // queries 48..63
            const bf16x8 Pk = tr_op(PS, thb + 1024 * s), Sk = tr_op(DS, thb + 1024 * s);
            dKR[kb] = mfma16(mine ? QFb[qb][s] : z, Sk, dKR[kb]);     // dK[k][f] += dS[q][k] Q[q][f]
            dVR[kb] = mfma16(mine ? OFb[qb][s] : z, Pk, dVR[kb]);     // dV[k][f] += P[q][k] dO[q][f]
          }
        }
      }
    }
    bf16x8 dq[2][ST], dk[2][ST], dv[2][ST];
    const float isc = 1.0f / sc, sdh = 1.0f / isd;  // dK, dV were formed from the scaled q and dO
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      __bf16* S = stg + (2 * cp + rb) * NSTAGE * MAT;
#pragma unroll
      for (int r = 0; r < 16; ++r) { dKR[rb][r] *= isc; dVR[rb][r] *= sdh; }
#pragma unroll
      for (int s = 0; s < ST; ++s) { dq[rb][s] = cvt8(dQR[rb], s); dk[rb][s] = cvt8(dKR[rb], s); dv[rb][s] = cvt8(dVR[rb], s); }
      stage_r(S + SQ * MAT, hb, dq[rb][0], dq[rb][1], lr, h);
      stage_r(S + SK * MAT, hb, dk[rb][0], dk[rb][1], lr, h);
      stage_r(S + SV * MAT, hb, dv[rb][0], dv[rb][1], lr, h);
      stage_r(S + SO * MAT, hb, cvt8(AOR[rb], 0), cvt8(AOR[rb], 1), lr, h);
    }
    // dx (as in the kernel above): output feature block hb from this wave, for both of its row
    // blocks; the other head block's dQ, dK, dV are read back from the staging after the barrier
    auto dx_terms = [&](int ib, const bf16x8 (&q)[ST], const bf16x8 (&k)[ST], const bf16x8 (&v)[ST]) {
      f32x16 acc = {};
      const int voff = (ib * ST * 64 + lane) * 16;
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        const int so = (hb * NB * ST + s) * 64 * 16;
        acc = mfma16(rld8(WT, voff, so), q[s], acc);
        acc = mfma16(rld8(WT, voff, so + D * D * 2), k[s], acc);
        acc = mfma16(rld8(WT, voff, so + 2 * D * D * 2), v[s], acc);
      }
      return acc;
    };
    float4 sv[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int64_t gb = 4 * tile + 2 * cp + rb;
#pragma unroll
      for (int q = 0; q < 4; ++q) sv[rb][q] = reinterpret_cast<const float4*>(a.g_in + ((gb * NB + hb) * 64 + lane) * 16)[q];
    }
    barrier_lds();  // staging of both head blocks in LDS
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int64_t gb = 4 * tile + 2 * cp + rb;
      const __bf16* S = stg + (2 * cp + rb) * NSTAGE * MAT;
      bf16x8 oq[ST], ok[ST], ov[ST];  // the other head block's operands, as it staged them
#pragma unroll
      for (int s = 0; s < ST; ++s) {
        const int e = lr * 64 + rsw(4 * (hb ^ 1) + 2 * s + h, lr) * 8;
        oq[s] = ld8(S + SQ * MAT + e);
        ok[s] = ld8(S + SK * MAT + e);
        ov[s] = ld8(S + SV * MAT + e);
      }
      f32x16 a0, a1;
      if (hb == 0) {
        a0 = dx_terms(0, dq[rb], dk[rb], dv[rb]);
        a1 = dx_terms(1, oq, ok, ov);
      } else {
        a0 = dx_terms(0, oq, ok, ov);
        a1 = dx_terms(1, dq[rb], dk[rb], dv[rb]);
      }
      // all four results formed before the first store (see the kernel above)
      float4 o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 g = sv[rb][q];
        o[q] = make_float4((g.x + a0[4 * q]) + a1[4 * q], (g.y + a0[4 * q + 1]) + a1[4 * q + 1],
                           (g.z + a0[4 * q + 2]) + a1[4 * q + 2], (g.w + a0[4 * q + 3]) + a1[4 * q + 3]);
      }
      float4* dst = reinterpret_cast<float4*>(a.g_out + ((gb * NB + hb) * 64 + lane) * 16);
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[q] = o[q];
    }
    fetch(tile + gridDim.x);

    // ================= gradient phase: wave w adds the tile's rows into weight gradient w
    {
      const int am = (w < 3) ? SX : SO;
      const int bm = (w < 3) ? SQ + w : SG;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const __bf16* A = stg + (b * NSTAGE + am) * MAT;
        const __bf16* B = stg + (b * NSTAGE + bm) * MAT;
#pragma unroll
        for (int s = 0; s < ST; ++s) {
          if (PAD16 && (b & 1) && s == 1) continue;  // rows 48..63 of the pass
          bf16x8 av[NB], bv[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            av[i] = tr_op(A, tb[i] + 1024 * s);
            bv[i] = tr_op(B, tb[i] + 1024 * s);
          }
#pragma unroll
          for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < NB; ++j) dW[i][j] = mfma16(av[i], bv[j], dW[i][j]);
        }
      }
    }
    barrier_lds();  // staging read before the next tile overwrites it
  }

  float* part = a.partial + (int64_t)blockIdx.x * 4 * D * D + (int64_t)w * D * D;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) part[(32 * i + tile_idx(r, h)) * D + 32 * j + lr] = dW[i][j][r];
}

size_t bwd_attn_bf16_lds(int bpt) {
  return (size_t)(4 * 64 * 64 + bpt * NSTAGE * MAT) * sizeof(__bf16);
}

bool bwd_attn_bf16_supported(int d, int D, int DH, bool span) { return d == 64 && D == 64 && (DH == 8 || DH == 16); }

int bwd_attn_bf16_parts(int blocks, bool span) { return span ? blocks : 2 * blocks; }

int32_t launch_bwd_attn_bf16(const BwdArgs& a, int DH, int blocks, hipStream_t st) {
  const size_t lds = bwd_attn_bf16_lds(4);
  // written for distinct input and output gradient buffers
  TDO_CHECK(a.g_in != a.g_out, TDO_EINVAL, "BF16 attention backward cannot run in place");
  TDO_CHECK(a.lse != nullptr, TDO_EINVAL, "BF16 attention backward needs the forward's softmax normalisers");
  auto go = [&](auto kern) -> int32_t {
    TDO_TRY(allow_full_lds((const void*)kern));
    hipLaunchKernelGGL(kern, dim3(2 * blocks), dim3(256), bwd_attn_bf16_lds(ATTN_BPT), st, a);
    TDO_HIP(hipGetLastError());
    return TDO_OK;
  };
  if (a.span) {
    auto go4 = [&](auto kern) -> int32_t {
      TDO_TRY(allow_full_lds((const void*)kern));
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, st, a);
      TDO_HIP(hipGetLastError());
      return TDO_OK;
    };
    const bool m = a.n < 64, p16 = a.n <= 48;
    if (DH == 8)
      return p16 ? go4(k_bwd_attn_span_bf16<8, true, true>)
                 : (m ? go4(k_bwd_attn_span_bf16<8, true, false>) : go4(k_bwd_attn_span_bf16<8, false, false>));
    if (DH == 16)
      return p16 ? go4(k_bwd_attn_span_bf16<16, true, true>)
                 : (m ? go4(k_bwd_attn_span_bf16<16, true, false>) : go4(k_bwd_attn_span_bf16<16, false, false>));
    return set_error(TDO_EUNSUPPORTED, "BF16 attention backward: head width %d", DH);
  }
  if (DH == 8) return a.masked ? go(k_bwd_attn_bf16<8, true>) : go(k_bwd_attn_bf16<8, false>);
  if (DH == 16) return a.masked ? go(k_bwd_attn_bf16<16, true>) : go(k_bwd_attn_bf16<16, false>);
  return set_error(TDO_EUNSUPPORTED, "BF16 attention backward: head width %d", DH);
}

}  // namespace tdo
