// Forward-mode derivative of log rho along a parameter direction (App. C, metric tensor of
// stochastic reconfiguration: S p = Re sum_b w_b conj(dO_b) (dO_b . p) needs O_b . p, the
// Jacobian-vector product), in FP32, and the matrix-free SR solve built on it.
//
// The network (main text "Transformer density operator ansatz"; App. B) is evaluated
// together with its tangent t(.) = d(.)/d eps at theta + eps p, stage by stage over a chunk
// of configurations, with activations in global memory (row r = (e * 2 + pass) * n + i):
//   embedding:  T and t(T) for the 64 window codes (two circular convolutions, GELU each);
//   per layer:  Q = X Wq, t(Q) = t(X) Wq + X t(Wq) (and K, V);
//               per head  S = Q K^T / sqrt(dh), t(S) = (t(Q) K^T + Q t(K)^T) / sqrt(dh),
//               P = softmax(S), t(P) = P (t(S) - rowsum(P t(S))), O = P V, t(O) = t(P) V + P t(V);
//               Y = X + O Wo, t(Y) = t(X) + t(O) Wo + O t(Wo);
//               H = max(0, Y W1 + b1), t(H) = [H > 0] (t(Y) W1 + Y t(W1) + t(b1));
//               X' = Y + H W2 + b2, t(X') = t(Y) + t(H) W2 + H t(W2) + t(b2);
//   head:       f = mean_i X_i Wh + bh, t(f) = mean_i (t(X_i) Wh + X_i t(Wh)) + t(bh), z = f0 + i f1;
//   log rho = log(e^{z1} + conj e^{z2}):  t(log rho) = (e^{z1} t(z1) + conj(e^{z2} t(z2))) / (e^{z1} + conj e^{z2}).
// The products are one tiled FP32 GEMM kernel (64 x 64 output tiles, LDS-staged operands);
// everything else is elementwise or per configuration-pass.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "netapi.h"
#include "train.h"

namespace tdo {

namespace {

__device__ __forceinline__ float gelu_f(float u) { return 0.5f * u * (1.0f + erff(u * 0.70710678118654752f)); }
// d/du [u Phi(u)] = Phi(u) + u phi(u)
__device__ __forceinline__ float gelu_d(float u) {
  return 0.5f * (1.0f + erff(u * 0.70710678118654752f)) + u * 0.39894228040143268f * expf(-0.5f * u * u);
}

}  // namespace

// Embedding table of the 64 window codes and its tangent (as k_embed_table): rows of d values.
__global__ void k_embed_table_jvp(const float* __restrict__ params, const float* __restrict__ tan, int d,
                                  float* __restrict__ T, float* __restrict__ Td) {
  __shared__ float e0[64], e1[64], e0d[64], e1d[64];
  const int code = blockIdx.x;
  const int t0 = code & 3, t1 = (code >> 2) & 3, t2 = (code >> 4) & 3;
  const float *w1 = params, *b1 = params + 4 * d, *w2 = b1 + d, *b2 = w2 + 2 * d * d;
  const float *w1d = tan, *b1d = tan + 4 * d, *w2d = b1d + d, *b2d = w2d + 2 * d * d;
  auto spin = [](int t, int ch) { return 1.0f - 2.0f * (float)((t >> ch) & 1); };
  for (int c = threadIdx.x; c < d; c += blockDim.x) {
    const float sa0 = spin(t0, 0), sa1 = spin(t0, 1), sb0 = spin(t1, 0), sb1 = spin(t1, 1), sc0 = spin(t2, 0),
                sc1 = spin(t2, 1);
    const float a = b1[c] + sa0 * w1[c] + sa1 * w1[d + c] + sb0 * w1[2 * d + c] + sb1 * w1[3 * d + c];
    const float ad = b1d[c] + sa0 * w1d[c] + sa1 * w1d[d + c] + sb0 * w1d[2 * d + c] + sb1 * w1d[3 * d + c];
    const float b = b1[c] + sb0 * w1[c] + sb1 * w1[d + c] + sc0 * w1[2 * d + c] + sc1 * w1[3 * d + c];
    const float bd = b1d[c] + sb0 * w1d[c] + sb1 * w1d[d + c] + sc0 * w1d[2 * d + c] + sc1 * w1d[3 * d + c];
    e0[c] = gelu_f(a);
    e0d[c] = gelu_d(a) * ad;
    e1[c] = gelu_f(b);
    e1d[c] = gelu_d(b) * bd;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < d; o += blockDim.x) {
    float acc = b2[o], accd = b2d[o];
    for (int c = 0; c < d; ++c) {
      acc += e0[c] * w2[c * d + o] + e1[c] * w2[d * d + c * d + o];
      accd += e0d[c] * w2[c * d + o] + e0[c] * w2d[c * d + o] + e1d[c] * w2[d * d + c * d + o] +
              e1[c] * w2d[d * d + c * d + o];
    }
    T[code * d + o] = gelu_f(acc);
    Td[code * d + o] = gelu_d(acc) * accd;
  }
}

// Rows of the embedding: X[r] = T[code], t(X)[r] = t(T)[code], r = (e * 2 + pass) * n + i.
__global__ void k_jvp_embed(const uint64_t* __restrict__ cfg, int64_t E, int n, int d, const float* __restrict__ T,
                            const float* __restrict__ Td, float* __restrict__ X, float* __restrict__ Xd) {
  const int64_t total = E * 2 * n * d;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(idx % d);
    const int64_t r = idx / d;
    const int i = (int)(r % n);
    const int64_t ep = r / n;
    const int pass = (int)(ep & 1);
    const int64_t e = ep >> 1;
    const uint64_t a = cfg[2 * e], b = cfg[2 * e + 1];
    const uint64_t c0 = pass ? b : a, c1 = pass ? a : b;
    int code = 0;
    for (int k = 0; k < 3; ++k) {
      int s = i + k;
      s = s >= n ? s - n : s;
      code += ((int)((c0 >> s) & 1ull) + 2 * (int)((c1 >> s) & 1ull)) << (2 * k);
    }
    X[idx] = T[code * d + o];
    Xd[idx] = Td[code * d + o];
  }
}

// C[r][j] = sum_k A1[r][k] B1[k][j] (+ sum_k A2[r][k] B2[k][j]) (+ bias[j]) (+ Res[r][j]),
// A row stride lda (the first K columns), B row-major with row stride ldb, C and Res with
// row stride ldc.  epi 1: C = max(0, C); epi 2: C = 0 where Mask[r][j] <= 0 (Mask stride ldc).
// 64 x 64 output tile per workgroup of 256 threads, each 4 x 4; K in steps of 16 through LDS.
constexpr int GT = 64, GK = 16;
__global__ void __launch_bounds__(256) k_jvp_gemm(const float* __restrict__ A1, const float* __restrict__ B1,
                                                  const float* __restrict__ A2, const float* __restrict__ B2,
                                                  int64_t R, int K, int N, int lda, int ldb,
                                                  const float* __restrict__ bias, const float* __restrict__ Res,
                                                  const float* __restrict__ Mask, int epi, float* __restrict__ C,
                                                  int ldc) {
  __shared__ float As[GK][GT + 4], Bs[GK][GT + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t ntn = (N + GT - 1) / GT;
  const int64_t ntiles = ((R + GT - 1) / GT) * ntn;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = (tile / ntn) * GT;
    const int j0 = (int)(tile % ntn) * GT;
    float acc[4][4] = {};
    for (int pass = 0; pass < 2; ++pass) {
      const float* A = pass ? A2 : A1;
      const float* Bm = pass ? B2 : B1;
      if (!A) continue;
      for (int k0 = 0; k0 < K; k0 += GK) {
        // stage A[r0 .. r0+63][k0 .. k0+15] (transposed) and B[k0 .. k0+15][j0 .. j0+63]
        for (int q = threadIdx.x; q < GT * GK; q += 256) {
          const int rr = q / GK, kk = q % GK;
          const int64_t r = r0 + rr;
          As[kk][rr] = (r < R && k0 + kk < K) ? A[r * lda + k0 + kk] : 0.f;
          const int kb = q / GT, jj = q % GT;
          Bs[kb][jj] = (k0 + kb < K && j0 + jj < N) ? Bm[(int64_t)(k0 + kb) * ldb + j0 + jj] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
          float a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = As[kk][ty * 4 + u];
            b[u] = Bs[kk][tx * 4 + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t r = r0 + ty * 4 + u;
      if (r >= R) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + tx * 4 + v;
        if (j >= N) continue;
        float c = acc[u][v];
        if (bias) c += bias[j];
        if (Res) c += Res[r * ldc + j];
        if (epi == 1) c = fmaxf(c, 0.f);
        if (epi == 2 && !(Mask[r * ldc + j] > 0.f)) c = 0.f;
        C[r * ldc + j] = c;
      }
    }
  }
}

// Attention of one configuration-pass per workgroup, all heads in turn, with tangents:
// O = softmax(Q K^T / sqrt(dh)) V and t(O) from Q, K, V, t(Q), t(K), t(V) (rows of d).
__global__ void __launch_bounds__(256) k_jvp_attn(int64_t EP, int n, int d, int heads, float scale,
                                                  const float* __restrict__ Q, const float* __restrict__ Kx,
                                                  const float* __restrict__ V, const float* __restrict__ Qd,
                                                  const float* __restrict__ Kd, const float* __restrict__ Vd,
                                                  float* __restrict__ O, float* __restrict__ Od) {
  extern __shared__ float sm[];
  const int dh = d / heads;
  float* S = sm;               // [n][n] scores, then P
  float* Sd = S + n * n;       // tangents, then t(P)
  for (int64_t ep = blockIdx.x; ep < EP; ep += gridDim.x) {
    const int64_t base = ep * n * d;
    for (int h = 0; h < heads; ++h) {
      for (int q = threadIdx.x; q < n * n; q += blockDim.x) {
        const int i = q / n, k = q % n;
        float s = 0.f, sd = 0.f;
        for (int j = 0; j < dh; ++j) {
          const int64_t qi = base + (int64_t)i * d + h * dh + j, kk = base + (int64_t)k * d + h * dh + j;
          s += Q[qi] * Kx[kk];
          sd += Qd[qi] * Kx[kk] + Q[qi] * Kd[kk];
        }
        S[q] = s * scale;
        Sd[q] = sd * scale;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        float m = -INFINITY;
        for (int k = 0; k < n; ++k) m = fmaxf(m, S[i * n + k]);
        float l = 0.f;
        for (int k = 0; k < n; ++k) {
          const float p = expf(S[i * n + k] - m);
          S[i * n + k] = p;
          l += p;
        }
        const float inv = 1.0f / l;
        float dot = 0.f;
        for (int k = 0; k < n; ++k) {
          S[i * n + k] *= inv;
          dot += S[i * n + k] * Sd[i * n + k];
        }
        for (int k = 0; k < n; ++k) Sd[i * n + k] = S[i * n + k] * (Sd[i * n + k] - dot);
      }
      __syncthreads();
      for (int q = threadIdx.x; q < n * dh; q += blockDim.x) {
        const int i = q / dh, j = q % dh;
        float o = 0.f, od = 0.f;
        for (int k = 0; k < n; ++k) {
          const int64_t vk = base + (int64_t)k * d + h * dh + j;
          o += S[i * n + k] * V[vk];
          od += Sd[i * n + k] * V[vk] + S[i * n + k] * Vd[vk];
        }
        O[base + (int64_t)i * d + h * dh + j] = o;
        Od[base + (int64_t)i * d + h * dh + j] = od;
      }
      __syncthreads();
    }
  }
}

// Mean pooling and head per configuration-pass (one wave each): z = (f0, f1), t(z).
__global__ void k_jvp_head(int64_t EP, int n, int d, const float* __restrict__ X, const float* __restrict__ Xd,
                           const float* __restrict__ hw, const float* __restrict__ hb, const float* __restrict__ hwd,
                           const float* __restrict__ hbd, float* __restrict__ z, float* __restrict__ zd) {
  const int lane = threadIdx.x & 63;
  for (int64_t ep = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); ep < EP;
       ep += (int64_t)gridDim.x * (blockDim.x >> 6)) {
    float f0 = 0.f, f1 = 0.f, g0 = 0.f, g1 = 0.f;
    for (int q = lane; q < n * d; q += 64) {
      const int o = q % d;
      const float x = X[ep * n * d + q], xd = Xd[ep * n * d + q];
      f0 += x * hw[2 * o];
      f1 += x * hw[2 * o + 1];
      g0 += xd * hw[2 * o] + x * hwd[2 * o];
      g1 += xd * hw[2 * o + 1] + x * hwd[2 * o + 1];
    }
    f0 = wave_sum(f0);
    f1 = wave_sum(f1);
    g0 = wave_sum(g0);
    g1 = wave_sum(g1);
    if (lane == 0) {
      const float inv = 1.0f / (float)n;
      z[2 * ep] = f0 * inv + hb[0];
      z[2 * ep + 1] = f1 * inv + hb[1];
      zd[2 * ep] = g0 * inv + hbd[0];
      zd[2 * ep + 1] = g1 * inv + hbd[1];
    }
  }
}

// t(log rho) per configuration from z, t(z) of its two passes.
__global__ void k_jvp_combine(int64_t E, const float* __restrict__ z, const float* __restrict__ zd,
                              float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const float a0 = z[4 * e], a1 = z[4 * e + 1], b0 = z[4 * e + 2], b1 = z[4 * e + 3];
    const float mx = fmaxf(a0, b0);
    float s, c;
    const float ea = expf(a0 - mx), eb = expf(b0 - mx);
    sincosf(a1, &s, &c);
    const float w1r = ea * c, w1i = ea * s;   // e^{z1}
    sincosf(-b1, &s, &c);
    const float w2r = eb * c, w2i = eb * s;   // e^{conj z2}
    const float t1r = zd[4 * e], t1i = zd[4 * e + 1], t2r = zd[4 * e + 2], t2i = -zd[4 * e + 3];  // t(z1), conj t(z2)
    const float nr = w1r * t1r - w1i * t1i + w2r * t2r - w2i * t2i;
    const float ni = w1r * t1i + w1i * t1r + w2r * t2i + w2i * t2r;
    const float Sr = w1r + w2r, Si = w1i + w2i, nn = Sr * Sr + Si * Si;
    out[2 * e] = nn > 0.f ? (nr * Sr + ni * Si) / nn : 0.f;
    out[2 * e + 1] = nn > 0.f ? (ni * Sr - nr * Si) / nn : 0.f;
  }
}

__global__ void k_to_f32(const double* __restrict__ a, int64_t n, float* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

}  // namespace tdo

namespace tdo {

namespace {

size_t jvp_bytes_per_config(const NetPlan& np) {
  const size_t rows = 2 * (size_t)np.n;
  return rows * (12 * (size_t)np.pp.d + 2 * (size_t)np.pp.mlp) * 4 + 64;
}

int32_t gemm(const NetPlan& np, const float* A1, const float* B1, const float* A2, const float* B2, int64_t R, int K,
             int N, int lda, int ldb, const float* bias, const float* res, const float* mask, int epi, float* C, int ldc,
             hipStream_t st);

}  // namespace

// Lay out the forward-mode buffers from ar.used on, for at most B configurations and
// within max_bytes for the per-chunk part.
int32_t plan_jvp(const NetPlan& np, int64_t B, size_t max_bytes, Arena& ar, JvpWs* j) {
  const PackPlan& pp = np.pp;
  const size_t per = jvp_bytes_per_config(np);
  const size_t fixed = ((size_t)pp.nparams + 128 * (size_t)pp.d) * 4 + 20 * 256;
  TDO_CHECK(max_bytes >= fixed + per, TDO_ENOMEM,
            "workspace cannot hold the forward-mode buffers of one configuration (%zu bytes)", fixed + per);
  j->ec = std::max<int64_t>(1, std::min<int64_t>(B, (int64_t)((max_bytes - fixed) / per)));
  const size_t R = (size_t)j->ec * 2 * np.n, d = pp.d, m = pp.mlp;
  j->tanf = ar.take<float>(pp.nparams);
  j->T = ar.take<float>(64 * d);
  j->Td = ar.take<float>(64 * d);
  size_t* act[] = {&j->X, &j->Xd, &j->Y, &j->Yd, &j->Q, &j->K, &j->V, &j->Qd, &j->Kd, &j->Vd, &j->O, &j->Od};
  for (size_t* o : act) *o = ar.take<float>(R * d);
  j->H = ar.take<float>(R * m);
  j->Hd = ar.take<float>(R * m);
  j->z = ar.take<float>(4 * (size_t)j->ec);
  j->zd = ar.take<float>(4 * (size_t)j->ec);
  return TDO_OK;
}

namespace {

int32_t gemm(const NetPlan& np, const float* A1, const float* B1, const float* A2, const float* B2, int64_t R, int K,
             int N, int lda, int ldb, const float* bias, const float* res, const float* mask, int epi, float* C, int ldc,
             hipStream_t st) {
  const int64_t tiles = ((R + GT - 1) / GT) * ((N + GT - 1) / GT);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)np.num_cus * 8));
  hipLaunchKernelGGL(k_jvp_gemm, dim3(grid), dim3(256), 0, st, A1, B1, A2, B2, R, K, N, lda, ldb, bias, res, mask, epi,
                     C, ldc);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // namespace

// Tangent table (the embedding, once per tangent), then per chunk the network and its
// tangent; out[e] = t(log rho(cfg[e])) as (re, im).
int32_t run_jvp(const NetPlan& np, void* ws, const JvpWs& j, const float* params, const uint64_t* cfg, int64_t B,
                float* out, hipStream_t st) {
  const PackPlan& pp = np.pp;
  const int d = pp.d, m = pp.mlp, n = np.n, H = pp.heads;
  const float* tan = at<float>(ws, j.tanf);
  float *T = at<float>(ws, j.T), *Td = at<float>(ws, j.Td);
  hipLaunchKernelGGL(k_embed_table_jvp, dim3(64), dim3(64), 0, st, params, tan, d, T, Td);
  TDO_HIP(hipGetLastError());
  float *X = at<float>(ws, j.X), *Xd = at<float>(ws, j.Xd), *Y = at<float>(ws, j.Y), *Yd = at<float>(ws, j.Yd);
  float *Q = at<float>(ws, j.Q), *K = at<float>(ws, j.K), *V = at<float>(ws, j.V);
  float *Qd = at<float>(ws, j.Qd), *Kd = at<float>(ws, j.Kd), *Vd = at<float>(ws, j.Vd);
  float *O = at<float>(ws, j.O), *Od = at<float>(ws, j.Od), *Hh = at<float>(ws, j.H), *Hd = at<float>(ws, j.Hd);
  float *z = at<float>(ws, j.z), *zd = at<float>(ws, j.zd);
  const float scale = (float)(1.0 / std::sqrt((double)(d / H)));
  const size_t attn_lds = 2 * (size_t)n * n * sizeof(float);
  for (int64_t e0 = 0; e0 < B; e0 += j.ec) {
    const int64_t E = std::min(j.ec, B - e0), EP = 2 * E, R = EP * n;
    hipLaunchKernelGGL(k_jvp_embed, dim3((unsigned)std::min<int64_t>(ceil_div(R * d, 256), 65536)), dim3(256), 0, st,
                       cfg + 2 * e0, E, n, d, T, Td, X, Xd);
    TDO_HIP(hipGetLastError());
    for (int l = 0; l < pp.layers; ++l) {
      const int64_t o = pp.off_layer0 + (int64_t)l * pp.layer_stride;
      const float *wq = params + o, *wk = wq + d * d, *wv = wk + d * d, *wo = wv + d * d, *w1 = wo + d * d;
      const float *b1 = w1 + d * m, *w2 = b1 + m, *b2 = w2 + m * d;
      const float *tq = tan + o, *tk = tq + d * d, *tv = tk + d * d, *to = tv + d * d, *t1 = to + d * d;
      const float *tb1 = t1 + d * m, *t2 = tb1 + m, *tb2 = t2 + m * d;
      const float* W[3] = {wq, wk, wv};
      const float* Wt[3] = {tq, tk, tv};
      float* P[3] = {Q, K, V};
      float* Pd[3] = {Qd, Kd, Vd};
      for (int i = 0; i < 3; ++i) {
        TDO_TRY(gemm(np, X, W[i], nullptr, nullptr, R, d, d, d, d, nullptr, nullptr, nullptr, 0, P[i], d, st));
        TDO_TRY(gemm(np, Xd, W[i], X, Wt[i], R, d, d, d, d, nullptr, nullptr, nullptr, 0, Pd[i], d, st));
      }
      hipLaunchKernelGGL(k_jvp_attn, dim3((unsigned)std::min<int64_t>(EP, (int64_t)np.num_cus * 8)), dim3(256),
                         attn_lds, st, EP, n, d, H, scale, Q, K, V, Qd, Kd, Vd, O, Od);
      TDO_HIP(hipGetLastError());
      TDO_TRY(gemm(np, O, wo, nullptr, nullptr, R, d, d, d, d, nullptr, X, nullptr, 0, Y, d, st));
      TDO_TRY(gemm(np, Od, wo, O, to, R, d, d, d, d, nullptr, Xd, nullptr, 0, Yd, d, st));
      TDO_TRY(gemm(np, Y, w1, nullptr, nullptr, R, d, m, d, m, b1, nullptr, nullptr, 1, Hh, m, st));
      TDO_TRY(gemm(np, Yd, w1, Y, t1, R, d, m, d, m, tb1, nullptr, Hh, 2, Hd, m, st));
      TDO_TRY(gemm(np, Hh, w2, nullptr, nullptr, R, m, d, m, d, b2, Y, nullptr, 0, X, d, st));
      TDO_TRY(gemm(np, Hd, w2, Hh, t2, R, m, d, m, d, tb2, Yd, nullptr, 0, Xd, d, st));
    }
    hipLaunchKernelGGL(k_jvp_head, dim3((unsigned)std::min<int64_t>(ceil_div(EP, 4), 16384)), dim3(256), 0, st, EP, n,
                       d, X, Xd, params + pp.off_head_w, params + pp.off_head_b, tan + pp.off_head_w,
                       tan + pp.off_head_b, z, zd);
    hipLaunchKernelGGL(k_jvp_combine, dim3((unsigned)std::min<int64_t>(ceil_div(E, 256), 4096)), dim3(256), 0, st, E,
                       z, zd, out + 2 * e0);
    TDO_HIP(hipGetLastError());
  }
  return TDO_OK;
}

int32_t jvp_check(const Context& c, const tdo_arch_t* arch, int32_t n, int64_t B, NetPlan* np) {
  TDO_TRY(net_plan(&c, arch, n, false, np));
  TDO_CHECK(B >= 0, TDO_EINVAL, "B=%lld < 0", (long long)B);
  return TDO_OK;
}

int32_t jvp_tangent_f32(const double* p, int64_t P, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(P, 256), 4096))),
                     dim3(256), 0, st, p, P, out);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // namespace tdo

using namespace tdo;

extern "C" int32_t tdo_log_rho_jvp(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n,
                                   const uint64_t* cfg, int64_t B, const double* tangent, float* jvp,
                                   hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  NetPlan np;
  TDO_TRY(jvp_check(ctx->c, arch, n, B, &np));
  if (B == 0) return TDO_OK;
  TDO_CHECK(params && cfg && tangent && jvp, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  Arena ar;
  JvpWs j;
  TDO_CHECK(c.budget > 4096, TDO_ENOMEM, "workspace budget %zu too small", c.budget);
  TDO_TRY(plan_jvp(np, B, c.budget, ar, &j));
  TDO_TRY(ensure_workspace(&c, ar.used));
  TDO_TRY(jvp_tangent_f32(tangent, np.pp.nparams, at<float>(c.ws, j.tanf), stream));
  return run_jvp(np, c.ws, j, params, cfg, B, jvp, stream);
}
