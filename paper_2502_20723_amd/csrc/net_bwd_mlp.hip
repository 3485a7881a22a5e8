// Backward of the residual feed-forward sub-layer y = x + relu(x W1 + b1) W2 + b2
// for width 64 with BF16 MFMA operands (FP32 accumulation):
//   u = b1 + x W1 (recomputed, with the forward's rounding order), dh = g W2^T, du = dh [u > 0], dx = g + du W1^T,
//   dW1 += x^T du, dW2 += relu(u)^T g, db1 += sum du, db2 += sum g.
//
// Work decomposition.  A workgroup (4 waves) walks 64-row tiles (two 32-row
// blocks of the activation layout) and keeps the weight gradients of the
// whole launch in registers: wave w owns the hidden units
// [w M/4, (w+1) M/4), i.e. its columns of dW1 and rows of dW2, so no
// gradient is ever added through memory until the launch ends.  Per tile:
//   1. the tile's x and g are staged in LDS twice: row-major (operands of
//      the contractions over features) and transposed (operands of the
//      contractions over rows), the transpose formed exactly on the matrix
//      cores.  Inside every 16-element group the index order is that of the
//      MFMA result layout (the two middle quads swapped, perm16), so that every
//      tile is written and read with 16-byte accesses; the weight operands
//      and W1's LDS copy take the same order along the contracted index;
//   2. each wave recomputes u and dh for its hidden units in the
//      (row x hidden) orientation, whose registers are directly the row-
//      contraction operands of dW1 and dW2, and writes du (transposed on the
//      matrix cores) to LDS;
//   3. each wave forms one 32x32 tile of dx = g + du W1^T from the du of all
//      hidden units.
// The workgroup's gradients are written once per launch to its slot of the
// partial buffer [2DM + M + D] (same layout as the generic kernel), and the
// slots are summed in FP64 afterwards.
#include "common.h"
#include "net.h"
#include "netapi.h"

namespace tdo {

namespace {

constexpr int RT = 64;  // rows per tile
constexpr int XS = 72;  // bf16 row stride of the 64-wide LDS tiles (144 bytes: conflict-free 16-byte reads)

// Position of tile row `row` in the transposed LDS tiles: inside each group
// of 16 rows the two middle quads are swapped, so that positions
// 16s + 8h + t (t < 8) hold rows tile_idx(8s + t, h) of the MFMA result layout.
__device__ __forceinline__ int perm16(int row) {
  const int q = row & 15;
  return (row & ~15) | ((q & 4) << 1) | ((q & 8) >> 1) | (q & 3);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ f32x16 mfma16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}


// Exact transpose of a 32x32 tile on the matrix cores, given as the two BF16
// operands of its R layout (lane -> m, values -> tile_idx(8 s + t, h)): the
// product with the 0/1 matrix eye[k][n] = [tile_idx(k) == n] returns lane ->
// former value index, values -> former lane index (result layout).
__device__ __forceinline__ f32x16 transpose_mfma(const bf16x8& x0, const bf16x8& x1, const bf16x8 (&eye)[2]) {
  return mfma16(x1, eye[1], mfma16(x0, eye[0], f32x16{}));
}

// Tiles of the 8-wave kernel: 64 BF16 columns per row (128 bytes, no padding) in perm16 order,
// 8 units of 16 bytes; unit u of row r sits at position u ^ f(r), f(r) = (bit 1 of r, bit 2 of
// r, bit 0 xor bit 3 of r) as bits (2, 1, 0).  Measured on gfx950 (bank-conflict counter of an
// LDS probe): 16-byte writes serve 8 lanes per cycle over 128 bytes, 16-byte reads 16 lanes
// and transposing reads 32 lanes per cycle over 64 banks of 4 bytes; with f, the 8 rows of a
// write phase, the 16 rows of a read phase and the 4 rows x 2 column halves of a transposing
// read phase all fall on distinct banks.
constexpr int XR = 64;  // row stride (bf16)
__device__ __forceinline__ int usw(int u, int row) {
  return u ^ ((((row >> 1) & 1) << 2) | (((row >> 2) & 1) << 1) | ((row ^ (row >> 3)) & 1));
}
// gfx950's transposing LDS read (ds_read_b64_tr_b16): within each group of 16 lanes, lane
// 4t + u supplies the address of 4 consecutive BF16 values and lane 4u + c receives, as its
// value t, value c of lane 4t + u.  Two such reads give lane l column 32 cb + l % 32 at 8 rows
// (values 4 rd + t from row 8 rd + 4 (l / 32) + t of the 16-row part at p): the row-
// contraction operand of the tile, with no transpose on the matrix cores.  off[rd] is the
// lane's offset for rows 8 rd + ... (mlp_toff); f depends on row bit 3, so the two reads have
// offsets of their own.
__device__ __forceinline__ int mlp_toff(int rd, int cb, int lane) {
  const int g = lane >> 4, u = lane & 3, row = 8 * rd + 4 * (lane >> 5) + ((lane & 15) >> 2);
  return row * XR + usw(4 * cb + 2 * (g & 1) + (u & 1), row) * 8 + 4 * (u >> 1);
}
__device__ __forceinline__ bf16x8 tr_op(const __bf16* p, const int (&off)[2]) {
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
  const s16x4 a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + off[0]));
  const s16x4 b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p + off[1]));
  return __builtin_bit_cast(bf16x8, (s16x8)__builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

}  // namespace

// SEEDS: the last layer, whose incoming gradient is formed from the per-configuration seeds
// (g_in NULL); otherwise g is read from g_in.
template <int M, bool SEEDS>
__global__ void __launch_bounds__(256) k_bwd_mlp_bf16(BwdArgs a) {
  constexpr int D = 64, NB = 2, HW = M / 4, HT = HW / 32, KS = M / 16, DUS = M + 8;
  static_assert(HT >= 1 && HT <= 2 && HW % 32 == 0, "hidden width 128 or 256");
  extern __shared__ __align__(16) char smem[];
  __bf16* XA = reinterpret_cast<__bf16*>(smem);  // [RT][XS]   x, row-major
  __bf16* XT = XA + RT * XS;                      // [D][XS]    x^T, permuted rows
  __bf16* GA = XT + D * XS;                       // [RT][XS]   g, row-major
  __bf16* GT = GA + RT * XS;                      // [D][XS]    g^T, permuted rows
  __bf16* DU = GT + D * XS;                       // [RT][DUS]  du, row-major, hidden units in perm16 order
  __bf16* W1s = DU + RT * DUS;                    // [D][DUS]   W1 (operand of dx = du W1^T), same order
  float* db2s = reinterpret_cast<float*>(W1s + D * DUS);  // [2 blocks of the tile][D]
  float4* GF = reinterpret_cast<float4*>(db2s + 2 * D);   // [4 waves][4][64]: g in FP32 for the residual of dx
  float2* hws = reinterpret_cast<float2*>(GF + 4 * 4 * 64);  // SEEDS: head weight pairs [D], zero past d

  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, lr = lane & 31;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int64_t E = a.n_entries_dev ? *a.n_entries_dev : a.n_entries;
  const RowMap rm{a.n, a.cpb, a.span != 0};
  const int64_t nblk = a.span ? 4 * E : 2 * ((E + a.cpb - 1) / a.cpb);
  const int64_t ntile = (nblk + 1) / 2;

  // ---- weights of this wave, as BF16 MFMA operands (read once per launch)
  const int hid0 = HW * w;  // first hidden unit owned by this wave
  bf16x8 w1b[HT][4], w2b[HT][4];
#pragma unroll
  for (int nt = 0; nt < HT; ++nt)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int hid = hid0 + 32 * nt + lr, f = perm16(16 * s + 8 * h + k);  // order of XA, GA
        w1b[nt][s][k] = (__bf16)a.w1[f * M + hid];  // B[k = in][n = hidden] = W1[in][hidden]
        w2b[nt][s][k] = (__bf16)a.w2[hid * D + f];  // B[k = out][n = hidden] = W2[hidden][out]
      }
  const int rb3 = w >> 1, it3 = w & 1;  // tile of dx formed by this wave
  for (int i = t; i < D * M; i += 256) W1s[(i / M) * DUS + perm16(i % M)] = (__bf16)a.w1[i];
  // permutation operands of transpose_mfma: eye[s][t] = [tile_idx(8 s + t, h) == lr]
  bf16x8 eye[2];
#pragma unroll
  for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
    for (int t2 = 0; t2 < 8; ++t2) eye[s2][t2] = (__bf16)(tile_idx(8 * s2 + t2, h) == lr ? 1.0f : 0.0f);
  if constexpr (SEEDS)
    for (int i = t; i < D; i += 256) hws[i] = i < a.d_real ? make_float2(a.head_w[2 * i], a.head_w[2 * i + 1]) : make_float2(0.f, 0.f);
  __syncthreads();  // W1s (and the head weights) initialised before any use
  float bias[HT];
#pragma unroll
  for (int nt = 0; nt < HT; ++nt) bias[nt] = a.b1[hid0 + 32 * nt + lr];

  f32x16 dW1[NB][HT], dW2[HT][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int nt = 0; nt < HT; ++nt) { dW1[i][nt] = f32x16{}; dW2[nt][i] = f32x16{}; }
  float db1[HT], db2[16];
#pragma unroll
  for (int nt = 0; nt < HT; ++nt) db1[nt] = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) db2[r] = 0.f;

  // staging role of this thread: block sb of the tile, feature block sob, lane sl
  const int sb = w >> 1, sob = w & 1, sl = lane, srow = 32 * sb + (sl & 31), sh = sl >> 5;

  // x and (when it comes from memory) g of this thread's staging role, loaded one tile
  // ahead so that the previous tile's phases cover the latency of the loads
  bf16x8 xn[2];
  float4 gn[4];
  float2 sn;  // SEEDS: (dF0, dF1) of this lane's row
  auto fetch = [&](int64_t tl) {  // zeros past the last block
    const int64_t g = 2 * tl + sb;
    const bool ok = tl < ntile && g < nblk;
    const auto rx = rsrc(reinterpret_cast<const __bf16*>(a.save_mid) + (g * NB + sob) * 64 * 16, ok ? 64 * 16 * 2 : 0);
    xn[0] = rld8(rx, sl * 32);
    xn[1] = rld8(rx, sl * 32 + 16);
    if constexpr (!SEEDS) {
      const auto rg = rsrc(a.g_in + (g * NB + sob) * 64 * 16, ok ? 64 * 16 * 4 : 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) gn[q] = rld4(rg, sl * 64 + 16 * q);
    } else {
      int64_t e;
      int pass, ric;
      bool rv;
      rm.at(ok ? g : 0, sl & 31, E, e, pass, ric, rv);
      const auto rs = rsrc(a.seeds, ok ? (uint32_t)(E * 4 * sizeof(float)) : 0u);
      sn = rld2(rs, rv ? (int)((e * 2 + pass) * 2 * sizeof(float)) : 0x7ffffff0);  // out of range: zeros
    }
  };
  fetch(blockIdx.x);
  {
    // the same number of stores after the prefetch on the path into the loop as at the end of
    // every tile (dropped: the resource is empty), so that the wait for the prefetch at the top
    // of the loop need not cover the stores
    const auto rz = rsrc(a.g_out, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) rst4(rz, 16 * i, make_float4(0.f, 0.f, 0.f, 0.f));
  }

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    // ---- 1. stage x and g of the tile (wave = role (block sb, feature block sob))
    {
      const int64_t gb = 2 * tile + sb;
      bf16x8 xo[2], go[2];
      if (gb < nblk) {
        xo[0] = xn[0];
        xo[1] = xn[1];
        float g[16];
        if constexpr (SEEDS) {
          // g = (dF0 head_w[:, 0] + dF1 head_w[:, 1]) / n from the pooled head (per row's configuration-pass)
          const float s0 = sn.x / (float)a.n, s1 = sn.y / (float)a.n;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float2 hw = hws[32 * sob + tile_idx(r, sh)];
            g[r] = s0 * hw.x + s1 * hw.y;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            g[4 * q] = gn[q].x; g[4 * q + 1] = gn[q].y; g[4 * q + 2] = gn[q].z; g[4 * q + 3] = gn[q].w;
          }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) db2[r] += g[r];
#pragma unroll
        for (int s = 0; s < 2; ++s) go[s] = cvt8(g, s);
        // the same wave and lane form the dx tile (block sb, features sob) in phase 3
#pragma unroll
        for (int q = 0; q < 4; ++q) GF[(w * 4 + q) * 64 + lane] = make_float4(g[4 * q], g[4 * q + 1], g[4 * q + 2], g[4 * q + 3]);
      } else {
        xo[0] = xo[1] = go[0] = go[1] = bf16x8{};
      }
      // row-major: value t of operand s is feature 32 sob + tile_idx(8 s + t, sh), position 32 sob + 16 s + 8 sh + t
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        *reinterpret_cast<bf16x8*>(XA + srow * XS + 32 * sob + 16 * s + 8 * sh) = xo[s];
        *reinterpret_cast<bf16x8*>(GA + srow * XS + 32 * sob + 16 * s + 8 * sh) = go[s];
      }
      // transposed: lane -> feature 32 sob + lr, values -> rows of block sb in perm16 order
      const f32x16 xt = transpose_mfma(xo[0], xo[1], eye), gt = transpose_mfma(go[0], go[1], eye);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        *reinterpret_cast<bf16x8*>(XT + (32 * sob + lr) * XS + 32 * sb + 16 * s + 8 * h) = cvt8(xt, s);
        *reinterpret_cast<bf16x8*>(GT + (32 * sob + lr) * XS + 32 * sb + 16 * s + 8 * h) = cvt8(gt, s);
      }
    }
    barrier_lds();
    fetch(tile + gridDim.x);

    // ---- 2. hidden units of this wave: u, dh, du; dW1, dW2, db1; du to LDS
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      f32x16 u[HT], dh[HT];
#pragma unroll
      for (int nt = 0; nt < HT; ++nt) {  // u accumulates onto b1, in the forward's order
        dh[nt] = f32x16{};
#pragma unroll
        for (int r = 0; r < 16; ++r) u[nt][r] = bias[nt];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bf16x8 xa = ld8(XA + (32 * rb + lr) * XS + 16 * s + 8 * h);
        const bf16x8 ga = ld8(GA + (32 * rb + lr) * XS + 16 * s + 8 * h);
#pragma unroll
        for (int nt = 0; nt < HT; ++nt) {
          u[nt] = mfma16(xa, w1b[nt][s], u[nt]);    // (row x hidden): lane -> hidden, values -> rows
          dh[nt] = mfma16(ga, w2b[nt][s], dh[nt]);
        }
      }
#pragma unroll
      for (int nt = 0; nt < HT; ++nt)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float uu = u[nt][r];
          const float d = uu > 0.f ? dh[nt][r] : 0.f;
          u[nt][r] = uu > 0.f ? uu : 0.f;  // relu(u)
          dh[nt][r] = d;                   // du
          db1[nt] += d;
        }
      bf16x8 duo[HT][2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int pos = 32 * rb + 16 * s + 8 * h;
        bf16x8 xt[NB], gt[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          xt[i] = ld8(XT + (32 * i + lr) * XS + pos);
          gt[i] = ld8(GT + (32 * i + lr) * XS + pos);
        }
#pragma unroll
        for (int nt = 0; nt < HT; ++nt) {
          duo[nt][s] = cvt8(dh[nt], s);
          const bf16x8 ho = cvt8(u[nt], s);
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            dW1[i][nt] = mfma16(xt[i], duo[nt][s], dW1[i][nt]);  // (in x hidden)
            dW2[nt][i] = mfma16(ho, gt[i], dW2[nt][i]);          // (hidden x out)
          }
        }
      }
      // du transposed (lane -> row, values -> hidden units in perm16 order), 16-byte writes
#pragma unroll
      for (int nt = 0; nt < HT; ++nt) {
        const f32x16 dut = transpose_mfma(duo[nt][0], duo[nt][1], eye);
#pragma unroll
        for (int s = 0; s < 2; ++s)
          *reinterpret_cast<bf16x8*>(DU + (32 * rb + lr) * DUS + hid0 + 32 * nt + 16 * s + 8 * h) = cvt8(dut, s);
      }
    }
    barrier_lds();

    // ---- 3. dx tile (rows of block rb3, features of block it3) = g + du W1^T
    {
      const int64_t gb = 2 * tile + rb3;
      f32x16 acc = f32x16{};
#pragma unroll
      for (int s = 0; s < KS; ++s)  // A[m = in][k = hidden] = W1, B[k = hidden][n = row] = du
        acc = mfma16(ld8(W1s + (32 * it3 + lr) * DUS + 16 * s + 8 * h), ld8(DU + (32 * rb3 + lr) * DUS + 16 * s + 8 * h), acc);
      // stores issued by every wave (dropped past the last block): see the loop entry
      const auto ro = rsrc(a.g_out + (gb * NB + it3) * 64 * 16, gb < nblk ? 64 * 16 * 4 : 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 g = GF[(w * 4 + q) * 64 + lane];  // staged by this lane in phase 1
        rst4(ro, lane * 64 + 16 * q,
             make_float4(acc[4 * q] + g.x, acc[4 * q + 1] + g.y, acc[4 * q + 2] + g.z, acc[4 * q + 3] + g.w));
      }
    }
    barrier_lds();
  }

  // ---- write this workgroup's gradients: dW1 [D][M], dW2 [M][D], db1 [M], db2 [D]
  float* part = a.partial + (int64_t)blockIdx.x * (2 * D * M + M + D);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int nt = 0; nt < HT; ++nt)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        part[(32 * i + tile_idx(r, h)) * M + hid0 + 32 * nt + lr] = dW1[i][nt][r];
        part[D * M + (hid0 + 32 * nt + tile_idx(r, h)) * D + 32 * i + lr] = dW2[nt][i][r];
      }
#pragma unroll
  for (int nt = 0; nt < HT; ++nt) {
    const float v = db1[nt] + __shfl_xor(db1[nt], 32, 64);
    if (h == 0) part[2 * D * M + hid0 + 32 * nt + lr] = v;
  }
  // db2: the 32 rows of each lane half summed by a fixed butterfly, then the two
  // blocks of the tile in a fixed order (deterministic, unlike atomics)
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float v = db2[r];
#pragma unroll
    for (int m = 1; m < 32; m <<= 1) v += __shfl_xor(v, m, 64);
    if ((sl & 31) == 0) db2s[sb * D + 32 * sob + tile_idx(r, sh)] = v;
  }
  __syncthreads();
  if (t < D) part[2 * D * M + M + t] = db2s[t] + db2s[D + t];
}

// Variant for m = 256 with 8 waves, two per SIMD (one wave's latencies overlap the
// other's work).  Wave w owns hidden units [32 w, 32 w + 32): its weight operands and
// gradients fit in half of a SIMD's registers.  Roles per tile (q = w mod 4: block q/2,
// feature block q mod 2): waves 0-3 stage x, waves 4-7 stage g and keep it in FP32 for the
// residual of dx.  The four 32x32 tiles of dx are split over the hidden units in halves:
// wave q sums hidden [128, 256) and leaves its part in LDS; after a barrier wave q + 4,
// which staged g of the same tile, adds hidden [0, 128), that part and the residual, and
// writes dx.  Every cross-wave use of LDS is ordered by one of the three barriers of a tile.
// Unlike the 4-wave kernel, no tile is transposed on the matrix cores: the contractions over
// rows read x and g, and dx reads du, with gfx950's transposing LDS read (tr_op), from
// x and g staged row-major and du staged as (hidden x row), the orientation it is formed in.
template <bool SEEDS>
__global__ void __launch_bounds__(512) k_bwd_mlp8_bf16(BwdArgs a) {
  constexpr int M = 256, D = 64, NB = 2, DUS = M + 8;
  extern __shared__ __align__(16) char smem[];
  __bf16* XA = reinterpret_cast<__bf16*>(smem);  // [RT][XR]   x, row-major (features in perm16 order, usw units)
  __bf16* GA = XA + RT * XR;                      // [RT][XR]   g, row-major
  __bf16* DT = GA + RT * XR;                      // [M][XR]    du, (hidden x row), rows in perm16 order
  __bf16* W1s = DT + M * XR;                      // [D][DUS]   W1 (operand of dx = du W1^T), hidden in perm16 order
  float* db2s = reinterpret_cast<float*>(W1s + D * DUS);     // [2 blocks of the tile][D]
  float4* GF = reinterpret_cast<float4*>(db2s + 2 * D);      // [4 roles][4][64]: g in FP32
  float4* XD = GF + 4 * 4 * 64;                              // [4 tiles][4][64]: dx over hidden [128, 256)
  float2* hws = reinterpret_cast<float2*>(XD + 4 * 4 * 64);  // SEEDS: head weight pairs [D], zero past d

  const int t = threadIdx.x, lane = t & 63, h = lane >> 5, lr = lane & 31;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
  const int q = w & 3, sb = q >> 1, sob = q & 1, srow = 32 * sb + lr;
  const bool gw = w >= 4;  // stages g and finishes dx
  const int64_t E = a.n_entries_dev ? *a.n_entries_dev : a.n_entries;
  const RowMap rm{a.n, a.cpb, a.span != 0};
  const int64_t nblk = a.span ? 4 * E : 2 * ((E + a.cpb - 1) / a.cpb);
  const int64_t ntile = (nblk + 1) / 2;

  // ---- weights of this wave, as BF16 MFMA operands (read once per launch)
  const int hid = 32 * w + lr;  // hidden unit of this lane in (row x hidden) results
  bf16x8 w1b[4], w2b[4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int f = perm16(16 * s + 8 * h + k);  // order of XA, GA
      w1b[s][k] = (__bf16)a.w1[f * M + hid];     // B[k = in][n = hidden] = W1[in][hidden]
      w2b[s][k] = (__bf16)a.w2[hid * D + f];     // B[k = out][n = hidden] = W2[hidden][out]
    }
  for (int i = t; i < D * M; i += 512) W1s[(i / M) * DUS + perm16(i % M)] = (__bf16)a.w1[i];
  if constexpr (SEEDS)
    for (int i = t; i < D; i += 512) hws[i] = i < a.d_real ? make_float2(a.head_w[2 * i], a.head_w[2 * i + 1]) : make_float2(0.f, 0.f);
  // this lane's transposing-read offsets (see tr_op): rows 8 rd + 4 h + t of a 16-row part, i.e.
  // rows 32 rb + tile_idx(8 s + 4 rd + t, h) of the tile with the part at row 32 rb + 16 s
  const int toff[2][2] = {{mlp_toff(0, 0, lane), mlp_toff(1, 0, lane)}, {mlp_toff(0, 1, lane), mlp_toff(1, 1, lane)}};
  // unit positions of this lane's row (rows 32 k + lr all share usw): 16-byte unit u = c / 8 + h
  // with c a multiple of 16 sits at element (c ^ G8) of the row
  int G8 = usw(h, lr) * 8;
  __syncthreads();  // W1s and the head weights initialised before any use
  const float bias = a.b1[hid];

  f32x16 dW1[NB], dW2[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) dW1[i] = dW2[i] = f32x16{};
  float db1 = 0.f, db2[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) db2[r] = 0.f;

  // x (waves 0-3) or g (waves 4-7) of this wave's role, loaded one tile ahead (zeros past the end)
  bf16x8 xn[2];
  float4 gn[4];
  float2 sn;
  auto fetch = [&](int64_t tl) {
    const int64_t g = 2 * tl + sb;
    const bool ok = tl < ntile && g < nblk;
    // 32 x the lane id, formed here from the hardware's lane count (three instructions) rather
    // than held in a register across the tile loop
    int lo;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0\n\tv_lshlrev_b32 %0, 5, %0" : "=v"(lo));
    if (!gw) {
      const auto rx = rsrc(reinterpret_cast<const __bf16*>(a.save_mid) + (g * NB + sob) * 64 * 16, ok ? 64 * 16 * 2 : 0);
      xn[0] = rld8(rx, lo);
      xn[1] = rld8(rx, lo, 16);
    } else if constexpr (!SEEDS) {
      const auto rg = rsrc(a.g_in + (g * NB + sob) * 64 * 16, ok ? 64 * 16 * 4 : 0);
#pragma unroll
      for (int k = 0; k < 4; ++k) gn[k] = rld4(rg, 2 * lo, 16 * k);
    } else {
      int64_t e;
      int pass, ric;
      bool rv;
      rm.at(ok ? g : 0, lr, E, e, pass, ric, rv);
      const auto rs = rsrc(a.seeds, ok ? (uint32_t)(E * 4 * sizeof(float)) : 0u);
      sn = rld2(rs, rv ? (int)((e * 2 + pass) * 2 * sizeof(float)) : 0x7ffffff0);  // out of range: zeros
    }
  };
  fetch(blockIdx.x);
  {
    // the same stores after the prefetch on the path into the loop as at the end of every tile
    // (dropped: empty resource), so that the wait for the prefetch need not cover the stores
    const auto rz = rsrc(a.g_out, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) rst4(rz, 16 * k, make_float4(0.f, 0.f, 0.f, 0.f));
  }

  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    // G8 made opaque here: the XOR offsets below are formed in the loop, one instruction each,
    // instead of being held in registers across it
    asm volatile("" : "+v"(G8));
    const int64_t gb = 2 * tile + sb;  // block of this wave's role
    // ---- 1. stage x (waves 0-3) or g (waves 4-7): row-major and transposed, 16-byte writes;
    // value t of operand s is feature 32 sob + tile_idx(8 s + t, h), position 32 sob + 16 s + 8 h + t
    if (!gw) {
#pragma unroll
      for (int s = 0; s < 2; ++s) *reinterpret_cast<bf16x8*>(XA + srow * XR + ((32 * sob + 16 * s) ^ G8)) = xn[s];
    } else {
      float g[16];
      if constexpr (SEEDS) {
        // g = (dF0 head_w[:, 0] + dF1 head_w[:, 1]) / n from the pooled head
        const float s0 = sn.x / (float)a.n, s1 = sn.y / (float)a.n;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float2 hw = hws[32 * sob + tile_idx(r, h)];
          g[r] = s0 * hw.x + s1 * hw.y;
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          g[4 * k] = gn[k].x; g[4 * k + 1] = gn[k].y; g[4 * k + 2] = gn[k].z; g[4 * k + 3] = gn[k].w;
        }
      }
      bf16x8 go[2];
#pragma unroll
      for (int r = 0; r < 16; ++r) db2[r] += g[r];
#pragma unroll
      for (int s = 0; s < 2; ++s) go[s] = cvt8(g, s);
#pragma unroll
      for (int k = 0; k < 4; ++k) GF[(q * 4 + k) * 64 + lane] = make_float4(g[4 * k], g[4 * k + 1], g[4 * k + 2], g[4 * k + 3]);
#pragma unroll
      for (int s = 0; s < 2; ++s) *reinterpret_cast<bf16x8*>(GA + srow * XR + ((32 * sob + 16 * s) ^ G8)) = go[s];
    }
    barrier_lds();
    fetch(tile + gridDim.x);

    // ---- 2. hidden units of this wave: u, dh, du; dW1, dW2, db1; du to LDS
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      f32x16 u, dh = {};  // u accumulates onto b1, in the forward's order
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r] = bias;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bf16x8 xa = ld8(XA + (32 * rb + lr) * XR + ((16 * s) ^ G8));
        const bf16x8 ga = ld8(GA + (32 * rb + lr) * XR + ((16 * s) ^ G8));
        u = mfma16(xa, w1b[s], u);  // (row x hidden): lane -> hidden, values -> rows
        dh = mfma16(ga, w2b[s], dh);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float uu = u[r];
        const float d = uu > 0.f ? dh[r] : 0.f;
        u[r] = uu > 0.f ? uu : 0.f;  // relu(u)
        dh[r] = d;                   // du
        db1 += d;
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 duo = cvt8(dh, s), ho = cvt8(u, s);
        // du as (hidden x row): one 16-byte write per lane, the layout x and g are staged in
        *reinterpret_cast<bf16x8*>(DT + hid * XR + ((32 * rb + 16 * s) ^ G8)) = duo;
        const int ro = (32 * rb + 16 * s) * XR;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          dW1[i] = mfma16(tr_op(XA + ro, toff[i]), duo, dW1[i]);  // (in x hidden)
          dW2[i] = mfma16(ho, tr_op(GA + ro, toff[i]), dW2[i]);   // (hidden x out)
        }
      }
    }
    barrier_lds();

    // ---- 3. dx tile (rows of block sb, features of block sob) = g + du W1^T, hidden in halves
    f32x16 acc = {};
    const int k0 = gw ? 0 : (M / 16) / 2;
#pragma unroll
    for (int s = 0; s < (M / 16) / 2; ++s)  // A[m = in][k = hidden] = W1, B[k = hidden][n = row] = du
      acc = mfma16(ld8(W1s + (32 * sob + lr) * DUS + 16 * (k0 + s) + 8 * h),
                   tr_op(DT + 16 * (k0 + s) * XR, toff[sb]), acc);
    if (!gw) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        XD[(q * 4 + k) * 64 + lane] = make_float4(acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]);
    }
    barrier_lds();
    {
      // stores issued by every wave (dropped unless this wave finishes a valid tile)
      const auto ro = rsrc(a.g_out + (gb * NB + sob) * 64 * 16, (gw && gb < nblk) ? 64 * 16 * 4 : 0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float4 o = XD[(q * 4 + k) * 64 + lane], g = GF[(q * 4 + k) * 64 + lane];
        rst4(ro, lane * 64 + 16 * k,
             make_float4(acc[4 * k] + o.x + g.x, acc[4 * k + 1] + o.y + g.y, acc[4 * k + 2] + o.z + g.z,
                         acc[4 * k + 3] + o.w + g.w));
      }
    }
  }

  // ---- write this workgroup's gradients: dW1 [D][M], dW2 [M][D], db1 [M], db2 [D]
  float* part = a.partial + (int64_t)blockIdx.x * (2 * D * M + M + D);
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      part[(32 * i + tile_idx(r, h)) * M + 32 * w + lr] = dW1[i][r];
      part[D * M + (32 * w + tile_idx(r, h)) * D + 32 * i + lr] = dW2[i][r];
    }
  {
    const float v = db1 + __shfl_xor(db1, 32, 64);
    if (h == 0) part[2 * D * M + hid] = v;
  }
  // db2 (waves 4-7): the 32 rows of each lane half by a fixed butterfly, then the two blocks
  // of the tile in a fixed order
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float v = db2[r];
#pragma unroll
    for (int m = 1; m < 32; m <<= 1) v += __shfl_xor(v, m, 64);
    if (gw && lr == 0) db2s[sb * D + 32 * sob + tile_idx(r, h)] = v;
  }
  __syncthreads();
  if (t < D) part[2 * D * M + M + t] = db2s[t] + db2s[D + t];
}

size_t bwd_mlp8_bf16_lds() {
  return (size_t)(2 * RT * XR + 256 * XR + 64 * (256 + 8)) * sizeof(__bf16) + 2 * 64 * sizeof(float) +
         2 * 4 * 4 * 64 * sizeof(float4) + 64 * sizeof(float2);
}

size_t bwd_mlp_bf16_lds(int M) {
  return (size_t)(2 * RT * XS + 2 * 64 * XS + (RT + 64) * (M + 8)) * sizeof(__bf16) + 2 * 64 * sizeof(float) +
         4 * 4 * 64 * sizeof(float4) + 64 * sizeof(float2);
}

bool bwd_mlp_bf16_supported(int d, int D, int M) { return d == 64 && D == 64 && (M == 128 || M == 256); }

int32_t launch_bwd_mlp_bf16(const BwdArgs& a, int blocks, hipStream_t st) {
  const bool seeds = a.g_in == nullptr;
  if (a.M == 256 && a.mlp_waves != 4) {
    auto go8 = [&](auto kern) -> int32_t {
      TDO_TRY(allow_full_lds((const void*)kern));
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(512), bwd_mlp8_bf16_lds(), st, a);
      TDO_HIP(hipGetLastError());
      return TDO_OK;
    };
    return seeds ? go8(k_bwd_mlp8_bf16<true>) : go8(k_bwd_mlp8_bf16<false>);
  }
  const size_t lds = bwd_mlp_bf16_lds(a.M);
  auto go = [&](auto kern) -> int32_t {
    TDO_TRY(allow_full_lds((const void*)kern));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, st, a);
    TDO_HIP(hipGetLastError());
    return TDO_OK;
  };
  switch (a.M) {
    case 128: return seeds ? go(k_bwd_mlp_bf16<128, true>) : go(k_bwd_mlp_bf16<128, false>);
    case 256: return seeds ? go(k_bwd_mlp_bf16<256, true>) : go(k_bwd_mlp_bf16<256, false>);
    default: return set_error(TDO_EUNSUPPORTED, "BF16 feed-forward backward: mlp width %d", a.M);
  }
}

}  // namespace tdo
