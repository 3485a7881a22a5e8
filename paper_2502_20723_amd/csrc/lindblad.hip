// Rows of the vectorised Lindbladian, the local estimator L(x) and the FP64
// sample reductions.
//
// Row x = (alpha, beta) of Lhat = -i(H (x) 1 - 1 (x) H^T)
//   + sum_j gamma [L_j (x) L_j^* - 1/2 L_j^dag L_j (x) 1 - 1/2 1 (x) L_j^T L_j^*]
// (Eq. VecLin; App. A) for H of the Ising section (chain or 2D lattice) or of
// the Heisenberg section and L_j = sigma^-_j.  Worked out per slot type:
//   diagonal   -i[E(alpha) - E(beta)] - (gamma/2) (#up(alpha) + #up(beta)),
//              E the diagonal of H (Ising (V/4) sum s s; XYZ Jz sum s s + Bz sum s)
//   alpha move H(alpha, alpha') with a minus i:  Ising flip of site i, -i g/2;
//              XYZ flip of bond (i, i+1), -i (Jx - Jy s_i s_{i+1})
//   beta move  +i H(beta', beta): Ising +i g/2; XYZ +i (Jx - Jy s_i s_{i+1}) (beta's spins)
//   fields     alpha single flip -i Bx - By s_i; beta single flip +i Bx - By s_i
//   dissipator flip site i of alpha and beta, gamma, iff alpha_i = beta_i = 1
// (bit 1 = spin down; sigma^- = |1><0|).  Presence is decided exactly: an
// entry is emitted iff its exact value is nonzero, so connected indices are
// bit-exact across implementations.
#include "common.h"
#include "lindblad.h"

namespace tdo {

int32_t make_model(const tdo_model_t* m, ModelDev* out) {
  TDO_CHECK(m != nullptr, TDO_EINVAL, "model is NULL");
  TDO_CHECK(m->kind == 0 || m->kind == 1, TDO_EINVAL, "model kind %d is not 0 (Ising) or 1 (XYZ)", m->kind);
  TDO_CHECK(m->n >= 3 && m->n <= 64, TDO_EINVAL, "chain length n=%d outside [3, 64]", m->n);
  TDO_CHECK(m->rows >= 0, TDO_EINVAL, "rows=%d < 0", m->rows);
  ModelDev d{};
  d.kind = m->kind;
  d.n = m->n;
  d.rows = m->rows > 1 ? m->rows : 1;
  if (d.rows > 1) {
    TDO_CHECK(m->kind == 0, TDO_EINVAL, "a lattice (rows=%d) is defined for the Ising model only", m->rows);
    TDO_CHECK(m->n % d.rows == 0, TDO_EINVAL, "n=%d is not a multiple of rows=%d", m->n, m->rows);
  }
  d.cols = d.n / d.rows;
  for (int r = 0; r < d.rows; ++r) {
    d.h_last |= 1ull << (r * d.cols + d.cols - 1);
    d.h_first |= 1ull << (r * d.cols);
  }
  d.h_keep = low_mask(d.n) & ~d.h_last;
  d.low_cols = low_mask(d.cols);
  d.gam = m->gamma;
  d.gam2 = 0.5 * m->gamma;
  d.gamma_ok = m->gamma != 0.0;
  if (m->kind == 0) {
    d.V4 = m->V / 4.0;
    d.g2 = m->g / 2.0;
    d.hmove_eq = d.hmove_ne = (m->g != 0.0);
    d.has_fields = 0;
  } else {
    d.Jz = m->Jz;
    d.jm = m->Jx - m->Jy;
    d.jp = m->Jx + m->Jy;
    d.hmove_eq = (m->Jx != m->Jy);   // bond with equal spins: Jx - Jy
    d.hmove_ne = (m->Jx != -m->Jy);  // bond with different spins: Jx + Jy
    d.Bx = m->Bx;
    d.By = m->By;
    d.Bz = m->Bz;
    d.has_fields = (m->Bx != 0.0 || m->By != 0.0) ? 1 : 0;
  }
  d.nslots = (d.has_fields ? 5 : 3) * d.n + 1;
  *out = d;
  return TDO_OK;
}

// Exact test of Jz*p + Bz*q == 0 for small integers p, q: compare the two
// products as unevaluated sums (rounded product + exact fma residual).
__device__ __forceinline__ bool lin2_is_zero(double a, int p, double b, int q) {
  double x1 = a * (double)p, e1 = fma(a, (double)p, -x1);
  double x2 = -b * (double)q, e2 = fma(-b, (double)q, -x2);
  return x1 == x2 && e1 == e2;
}

// The model's fields as values in (scalar) registers.  Read straight from the kernel argument,
// a per-lane choice between two fields (e.g. Jx - Jy or Jx + Jy by the bond's spins) is
// compiled into one load from a per-lane address in the argument segment, waited on inside
// the slot loop; readfirstlane makes each field a register value, so the choice is a select.
__device__ __forceinline__ int in_reg(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double in_reg(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, (hi << 32) | lo);
}
// Wait for every vector memory operation of the wave (s_waitcnt vmcnt(0); the expcnt and
// lgkmcnt fields of the gfx9 encoding at their maxima, i.e. no wait on them).  Placed right
// after a batch of loads, it keeps the compiler from waiting for all outstanding stores at the
// first use of those loads inside a loop (the counter is shared and in order).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ uint64_t in_reg(uint64_t v) {
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (hi << 32) | lo;
}

__device__ __forceinline__ ModelDev in_regs(const ModelDev& m) {
  ModelDev r;
  r.kind = in_reg(m.kind); r.n = in_reg(m.n); r.nslots = in_reg(m.nslots); r.has_fields = in_reg(m.has_fields);
  r.gamma_ok = in_reg(m.gamma_ok); r.hmove_eq = in_reg(m.hmove_eq); r.hmove_ne = in_reg(m.hmove_ne);
  r.gam = in_reg(m.gam); r.gam2 = in_reg(m.gam2); r.V4 = in_reg(m.V4); r.g2 = in_reg(m.g2); r.Jz = in_reg(m.Jz);
  r.jm = in_reg(m.jm); r.jp = in_reg(m.jp); r.Bx = in_reg(m.Bx); r.By = in_reg(m.By); r.Bz = in_reg(m.Bz);
  r.rows = in_reg(m.rows); r.cols = in_reg(m.cols);
  r.h_last = in_reg(m.h_last); r.h_keep = in_reg(m.h_keep); r.h_first = in_reg(m.h_first);
  r.low_cols = in_reg(m.low_cols);
  return r;
}

// sum over the bonds of s_i s_j = (number of bonds) - 2 (bonds whose spins differ).
// Chain: bonds (i, i+1 mod n).  M x C lattice: the right neighbour within the row
// and the neighbour one row down, each distinct pair once (a ring of length 2 has
// one bond, a ring of length 1 none).
__device__ __forceinline__ int bond_sum(const ModelDev& m, uint64_t a) {
  const int n = m.n;
  if (m.rows == 1) return n - 2 * __popcll(a ^ rot_down(a, n));
  const int M = m.rows, C = m.cols;
  int nb = 0, nd = 0;
  if (C >= 3) {  // bit i of r: the right neighbour's spin, wrapping within the row
    const uint64_t r = ((a >> 1) & m.h_keep) | ((a << (C - 1)) & m.h_last);
    nd += __popcll(a ^ r);
    nb += n;
  } else if (C == 2) {
    nd += __popcll((a ^ (a >> 1)) & m.h_first);
    nb += M;
  }
  if (M >= 3) {  // bit i of r: the spin one row down, wrapping
    const uint64_t r = ((a >> C) | (a << (n - C))) & low_mask(n);
    nd += __popcll(a ^ r);
    nb += n;
  } else {  // M == 2
    nd += __popcll((a ^ (a >> C)) & m.low_cols);
    nb += C;
  }
  return nb - 2 * nd;
}

__device__ bool slot_entry(const ModelDev& m, uint64_t a, uint64_t b, int s, uint64_t& ya,
                           uint64_t& yb, float& cre, float& cim) {
  const int n = m.n;
  const uint64_t mask = low_mask(n);
  a &= mask;  // bits at positions >= n are ignored
  b &= mask;
  ya = a;
  yb = b;
  if (s == 0) {
    int nup = 2 * n - __popcll(a) - __popcll(b);
    int bsa = bond_sum(m, a);
    int bsb = bond_sum(m, b);
    double re = -m.gam2 * (double)nup, im;
    bool im_zero;
    if (m.kind == 0) {
      im = -m.V4 * (double)(bsa - bsb);
      im_zero = (m.V4 == 0.0) || (bsa == bsb);
    } else {
      int sa = n - 2 * __popcll(a), sb = n - 2 * __popcll(b);
      im = -(m.Jz * (double)(bsa - bsb) + m.Bz * (double)(sa - sb));
      im_zero = lin2_is_zero(m.Jz, bsa - bsb, m.Bz, sa - sb);
    }
    cre = (float)re;
    cim = (float)im;
    return !((!m.gamma_ok || nup == 0) && im_zero);
  }
  s -= 1;
  if (s < 2 * n) {  // Hamiltonian moves on alpha (s < n) or beta
    const bool on_a = s < n;
    const int i = on_a ? s : s - n;
    const uint64_t x = on_a ? a : b;
    const double sign = on_a ? -1.0 : 1.0;  // -i H(x) 1  vs  +i 1 (x) H^T
    uint64_t flip;
    double c;
    bool ok;
    if (m.kind == 0) {
      flip = 1ull << i;
      c = m.g2;
      ok = m.hmove_eq;
    } else {
      const int j = (i + 1) % n;
      const bool eq = ((x >> i) & 1ull) == ((x >> j) & 1ull);
      flip = (1ull << i) | (1ull << j);
      // choices between two fields go through in_reg, so that they stay selects of values
      // (not one load from a per-lane address)
      c = eq ? in_reg(m.jm) : in_reg(m.jp);  // Jx - Jy s_i s_j
      ok = eq ? in_reg(m.hmove_eq) : in_reg(m.hmove_ne);
    }
    if (on_a) ya = (a ^ flip) & mask; else yb = (b ^ flip) & mask;
    cre = 0.0f;
    cim = (float)(sign * c);
    return ok;
  }
  s -= 2 * n;
  if (m.has_fields) {
    if (s < 2 * n) {
      const bool on_a = s < n;
      const int i = on_a ? s : s - n;
      const uint64_t x = on_a ? a : b;
      const double si = ((x >> i) & 1ull) ? -1.0 : 1.0;
      if (on_a) ya = a ^ (1ull << i); else yb = b ^ (1ull << i);
      cre = (float)(-m.By * si);
      cim = (float)(on_a ? -m.Bx : m.Bx);
      return true;  // has_fields means Bx != 0 or By != 0, so the value is nonzero
    }
    s -= 2 * n;
  }
  // dissipator gamma L_i (x) L_i^*: alpha_i = beta_i = 1 -> both 0
  const int i = s;
  const bool ok = m.gamma_ok && ((a >> i) & 1ull) && ((b >> i) & 1ull);
  ya = a ^ (1ull << i);
  yb = b ^ (1ull << i);
  cre = (float)m.gam;
  cim = 0.0f;
  return ok;
}

// One wave per row; lanes cover slots, valid entries compacted in slot order.  A wave takes
// its rows 64 at a time: lane i loads the configuration of the i-th of them (one coalesced
// load for 64 rows), each row reads its configuration from that lane, and the 64 counts are
// stored together, so the only per-row memory operations are the entries' stores.
__global__ void k_connected(ModelDev m_arg, const uint64_t* __restrict__ cfg, int64_t B, int kmax,
                            uint64_t* __restrict__ conn, float* __restrict__ mel,
                            int32_t* __restrict__ n_conn) {
  const ModelDev m = in_regs(m_arg);
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t r0 = wave0; r0 < B; r0 += 64 * nwaves) {
    const int64_t mine = r0 + lane * nwaves;
    ulonglong2 cl = make_ulonglong2(0, 0);
    if (mine < B) cl = reinterpret_cast<const ulonglong2*>(cfg)[mine];
    wait_vmem();
    const int nrows = (int)min<int64_t>(64, (B - r0 + nwaves - 1) / nwaves);
    int count = 0;
    for (int i = 0; i < nrows; ++i) {
      const int64_t row = r0 + i * nwaves;
      const uint64_t a = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(cl.x >> 32), i) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((uint32_t)cl.x, i);
      const uint64_t b = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(cl.y >> 32), i) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((uint32_t)cl.y, i);
      int base = 0;
      for (int s0 = 0; s0 < m.nslots; s0 += 64) {
        const int s = s0 + lane;
        uint64_t ya = 0, yb = 0;
        float cre = 0.f, cim = 0.f;
        const bool v = s < m.nslots && slot_entry(m, a, b, s, ya, yb, cre, cim);
        const uint64_t bal = __ballot(v);
        const int pos = base + __popcll(bal & ((1ull << lane) - 1ull));
        if (v && pos < kmax) {
          const int64_t o = row * kmax + pos;
          reinterpret_cast<ulonglong2*>(conn)[o] = make_ulonglong2(ya, yb);
          reinterpret_cast<float2*>(mel)[o] = make_float2(cre, cim);
        }
        base += __popcll(bal);
      }
      count = lane == i ? base : count;
    }
    if (mine < B) n_conn[mine] = count;
  }
}

// Internal evaluation list: per row, entry 0 is x itself (coefficient = the
// diagonal, possibly 0), followed by the valid off-diagonal entries in slot
// order.  Pass 1 counts, pass 2 (after a scan) fills.
__global__ void k_eval_count(ModelDev m_arg, const uint64_t* __restrict__ cfg, int64_t B,
                             int32_t* __restrict__ cnt) {
  const ModelDev m = in_regs(m_arg);
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t row = wave0; row < B; row += nwaves) {
    const uint64_t a = cfg[2 * row], b = cfg[2 * row + 1];
    int total = 1;
    for (int s0 = 1; s0 < m.nslots; s0 += 64) {
      const int s = s0 + lane;
      uint64_t ya, yb;
      float cre, cim;
      const bool v = s < m.nslots && slot_entry(m, a, b, s, ya, yb, cre, cim);
      total += __popcll(__ballot(v));
    }
    if (lane == 0) cnt[row] = total;
  }
}

__global__ void k_eval_fill(ModelDev m_arg, const uint64_t* __restrict__ cfg, int64_t B,
                            const int64_t* __restrict__ off, uint64_t* __restrict__ ecfg,
                            float* __restrict__ ecoef, int32_t* __restrict__ eowner) {
  const ModelDev m = in_regs(m_arg);
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t row = wave0; row < B; row += nwaves) {
    const uint64_t a = cfg[2 * row], b = cfg[2 * row + 1];
    const int64_t o = off[row];
    if (lane == 0) {
      uint64_t ya, yb;
      float cre, cim;
      slot_entry(m, a, b, 0, ya, yb, cre, cim);
      ecfg[2 * o] = a;
      ecfg[2 * o + 1] = b;
      ecoef[2 * o] = cre;
      ecoef[2 * o + 1] = cim;
      eowner[o] = (int32_t)row;
    }
    int base = 1;
    for (int s0 = 1; s0 < m.nslots; s0 += 64) {
      const int s = s0 + lane;
      uint64_t ya = 0, yb = 0;
      float cre = 0.f, cim = 0.f;
      const bool v = s < m.nslots && slot_entry(m, a, b, s, ya, yb, cre, cim);
      const uint64_t bal = __ballot(v);
      const int64_t e = o + base + __popcll(bal & ((1ull << lane) - 1ull));
      if (v) {
        ecfg[2 * e] = ya;
        ecfg[2 * e + 1] = yb;
        ecoef[2 * e] = cre;
        ecoef[2 * e + 1] = cim;
        eowner[e] = (int32_t)row;
      }
      base += __popcll(bal);
    }
  }
}

// Exclusive scan of int32 counts into int64 offsets, single workgroup of 1024.
__global__ void __launch_bounds__(1024) k_scan(const int32_t* __restrict__ cnt, int64_t B,
                                               int64_t* __restrict__ off, int64_t* __restrict__ total) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (B + 1023) / 1024;
  const int64_t lo = t * per, hi = (lo + per < B) ? lo + per : B;
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    int64_t v = (t >= d) ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = lo; i < hi; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) *total = part[1023];
}

__device__ __forceinline__ float2 cexpf_diff(float2 y, float2 x) {
  const float er = __expf(y.x - x.x);
  float sn, cs;
  __sincosf(y.y - x.y, &sn, &cs);
  return make_float2(er * cs, er * sn);
}

// L(x_b) = sum_k mel[b][k] exp(lr_conn[b][k] - lr_x[b]); one wave per row.  A wave takes its
// rows 64 at a time: lane i loads log rho(x) and the count of the i-th of them, each row reads
// them from that lane, and the 64 results are stored together, so inside the row loop there
// are only the entries' loads.  The next row's first 64 entries are loaded while the current
// row is reduced; entries are loaded up to kmax regardless of the count (in bounds) and those
// at or beyond the count are discarded by selection, so unwritten slots never enter the sum.
__global__ void k_lloc_fixed(int64_t B, const float2* __restrict__ lrx, const float2* __restrict__ mel,
                             const int32_t* __restrict__ ncon, int kmax,
                             const float2* __restrict__ lrc, float2* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t r0 = wave0; r0 < B; r0 += 64 * nwaves) {
    const int64_t mine = r0 + lane * nwaves;
    float2 xl = make_float2(0.f, 0.f);
    int kl = 0;
    if (mine < B) { xl = lrx[mine]; kl = min(ncon[mine], kmax); }
    const int nrows = (int)min<int64_t>(64, (B - r0 + nwaves - 1) / nwaves);
    float2 nc = make_float2(0.f, 0.f), nl = nc;
    if (lane < kmax) { nc = mel[r0 * kmax + lane]; nl = lrc[r0 * kmax + lane]; }
    wait_vmem();
    float2 res = make_float2(0.f, 0.f);
    for (int i = 0; i < nrows; ++i) {
      const int64_t row = r0 + i * nwaves;
      const float2 x = make_float2(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(xl.x), i)),
                                   __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xl.y), i)));
      const int k = __builtin_amdgcn_readlane(kl, i);
      const float2 c0 = nc, l0 = nl;
      const bool live = !(isinf(x.x) && x.x < 0.f);
      float re = 0.f, im = 0.f;
      if (live && lane < k) {
        const float2 e = cexpf_diff(l0, x);
        re = c0.x * e.x - c0.y * e.y;
        im = c0.x * e.y + c0.y * e.x;
      }
      if (live) {
        for (int j = lane + 64; j < k; j += 64) {
          const float2 c = mel[row * kmax + j];
          const float2 e = cexpf_diff(lrc[row * kmax + j], x);
          re += c.x * e.x - c.y * e.y;
          im += c.x * e.y + c.y * e.x;
        }
      }
      if (i + 1 < nrows && lane < kmax) {
        nc = mel[(row + nwaves) * kmax + lane];
        nl = lrc[(row + nwaves) * kmax + lane];
      }
      re = wave_sum(re);
      im = wave_sum(im);
      res = lane == i ? make_float2(re, im) : res;
    }
    if (mine < B) out[mine] = res;
  }
}

// Same on the compacted evaluation list; entry off[b] holds x itself.
__global__ void k_lloc_eval(int64_t B, const int64_t* __restrict__ off, const int32_t* __restrict__ cnt,
                            const float2* __restrict__ ecoef, const float2* __restrict__ elr,
                            float2* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t row = wave0; row < B; row += nwaves) {
    const int64_t o = off[row];
    const int k = cnt[row];
    const float2 x = elr[o];
    float re = 0.f, im = 0.f;
    if (!(isinf(x.x) && x.x < 0.f)) {
      for (int j = lane; j < k; j += 64) {
        const float2 c = ecoef[o + j];
        const float2 e = cexpf_diff(elr[o + j], x);
        re += c.x * e.x - c.y * e.y;
        im += c.x * e.y + c.y * e.x;
      }
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) out[row] = make_float2(re, im);
  }
}

// Deterministic FP64 reduction of sum w|L|^2 and sum w: fixed per-block
// partials, then one block adds them in index order.
constexpr int RED_BLOCKS = 512;

__global__ void __launch_bounds__(256) k_loss_partial(int64_t B, const float2* __restrict__ L,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ part) {
  __shared__ double s0[4], s1[4];
  double a = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < B; i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w ? w[i] : 1.0;
    const double re = L[i].x, im = L[i].y;
    a += wi * (re * re + im * im);
    c += wi;
  }
  a = wave_sum(a);
  c = wave_sum(c);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { s0[wv] = a; s1[wv] = c; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0[0] + s0[1] + s0[2] + s0[3];
    part[2 * blockIdx.x + 1] = s1[0] + s1[1] + s1[2] + s1[3];
  }
}

// acc[0] += sum of partials (w|L|^2), acc[1] += sum w; one wave, fixed order.
__global__ void k_loss_accum(const double* __restrict__ part, int nparts, double* __restrict__ acc) {
  const int lane = threadIdx.x;
  double a = 0.0, c = 0.0;
  for (int i = lane; i < nparts; i += 64) { a += part[2 * i]; c += part[2 * i + 1]; }
  a = wave_sum(a);
  c = wave_sum(c);
  if (lane == 0) { acc[0] += a; acc[1] += c; }
}

// ---------------------------------------------------------------- launchers
int32_t launch_connected(const ModelDev& m, const uint64_t* cfg, int64_t B, int kmax, uint64_t* conn,
                         float* mel, int32_t* n_conn, hipStream_t st) {
  if (B == 0) return TDO_OK;
  const int blocks = (int)std::min<int64_t>(ceil_div(B, 4), 8192);
  hipLaunchKernelGGL(k_connected, dim3(blocks), dim3(256), 0, st, m, cfg, B, kmax, conn, mel, n_conn);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_eval_list(const ModelDev& m, const uint64_t* cfg, int64_t B, int32_t* cnt, int64_t* off,
                         int64_t* total, uint64_t* ecfg, float* ecoef, int32_t* eowner, hipStream_t st) {
  const int blocks = (int)std::min<int64_t>(ceil_div(B, 4), 8192);
  hipLaunchKernelGGL(k_eval_count, dim3(blocks), dim3(256), 0, st, m, cfg, B, cnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, B, off, total);
  hipLaunchKernelGGL(k_eval_fill, dim3(blocks), dim3(256), 0, st, m, cfg, B, off, ecfg, ecoef, eowner);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_lloc_fixed(int64_t B, const float* lrx, const float* mel, const int32_t* ncon, int kmax,
                          const float* lrc, float* out, hipStream_t st) {
  if (B == 0) return TDO_OK;
  const int blocks = (int)std::min<int64_t>(ceil_div(B, 4), 8192);
  hipLaunchKernelGGL(k_lloc_fixed, dim3(blocks), dim3(256), 0, st, B, (const float2*)lrx,
                     (const float2*)mel, ncon, kmax, (const float2*)lrc, (float2*)out);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_lloc_eval(int64_t B, const int64_t* off, const int32_t* cnt, const float* ecoef,
                         const float* elr, float* out, hipStream_t st) {
  const int blocks = (int)std::min<int64_t>(ceil_div(B, 4), 8192);
  hipLaunchKernelGGL(k_lloc_eval, dim3(blocks), dim3(256), 0, st, B, off, cnt, (const float2*)ecoef,
                     (const float2*)elr, (float2*)out);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t launch_loss_accum(int64_t B, const float* L, const double* w, double* part, double* acc,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_loss_partial, dim3(RED_BLOCKS), dim3(256), 0, st, B, (const float2*)L, w, part);
  hipLaunchKernelGGL(k_loss_accum, dim3(1), dim3(64), 0, st, part, RED_BLOCKS, acc);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

}  // namespace tdo
