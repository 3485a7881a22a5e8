// C-ABI entry points of libtdo (declared and documented in include/tdo.h):
// argument validation, workspace planning and the launch sequences.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"
#include "lindblad.h"
#include "netapi.h"
#include "train.h"

namespace tdo {

static thread_local std::string g_err;

int32_t set_error(int32_t code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
void clear_error() { g_err.clear(); }

int32_t allow_full_lds(const void* kern) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, int>> done;
  int dev = 0;
  TDO_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  for (const auto& d : done)
    if (d.first == kern && d.second == dev) return TDO_OK;
  TDO_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  done.emplace_back(kern, dev);
  return TDO_OK;
}

// ---------------------------------------------------------------- profiler
hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void Profiler::recycle() {
  for (auto& r : recs) {
    pool.push_back(r.start);
    pool.push_back(r.stop);
  }
  recs.clear();
}

void Profiler::destroy() {
  recycle();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

ProfScope::ProfScope(Profiler* p_, const char* name_, hipStream_t st_) : p(p_), name(name_), st(st_) {
  if (p && p->enabled && !p->suspended) {
    start = p->get();
    if (start) (void)hipEventRecord(start, st);
  }
}

ProfScope::~ProfScope() {
  if (!start) return;
  hipEvent_t stop = p->get();
  if (!stop) {
    p->pool.push_back(start);
    return;
  }
  (void)hipEventRecord(stop, st);
  p->recs.push_back({name, start, stop});
}

// ---------------------------------------------------------------- ordering and parameter checks
int32_t WsOrder::begin(Context* c_, hipStream_t st_) {
  c = c_;
  st = st_;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  TDO_HIP(hipStreamIsCapturing(st, &cap));
  active = cap == hipStreamCaptureStatusNone;
  if (active && c->ws_recorded && c->ws_stream != st) TDO_HIP(hipStreamWaitEvent(st, c->ws_done, 0));
  return TDO_OK;
}

WsOrder::~WsOrder() {
  if (!active || !c->ws_done) return;
  if (hipEventRecord(c->ws_done, st) == hipSuccess) {
    c->ws_stream = st;
    c->ws_recorded = true;
  } else {
    (void)hipGetLastError();
  }
}

// One workgroup counts the values whose exponent field is all ones (inf or nan) and
// writes (or adds) the count: a fixed-size read of a parameter vector, a few microseconds.
__global__ void __launch_bounds__(1024) k_count_nonfinite(const float* __restrict__ p, int64_t n, int accumulate,
                                                          uint32_t* __restrict__ out) {
  __shared__ uint32_t part[16];
  uint32_t cnt = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    cnt += ((__float_as_uint(p[i]) & 0x7f800000u) == 0x7f800000u) ? 1u : 0u;
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, WAVE);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
    out[0] = accumulate ? out[0] + t : t;
  }
}

static bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cap != hipStreamCaptureStatusNone;
}

int32_t count_nonfinite(Context* c, const float* p, int64_t n, bool accumulate, hipStream_t st) {
  if (capturing(st)) return TDO_OK;
  if (!c->nf_dev) {
    TDO_HIP(hipMalloc(&c->nf_dev, 256));
    TDO_HIP(hipHostMalloc(&c->nf_host, 256, hipHostMallocDefault));
  }
  hipLaunchKernelGGL(k_count_nonfinite, dim3(1), dim3(1024), 0, st, p, n, accumulate ? 1 : 0, c->nf_dev);
  TDO_HIP(hipGetLastError());
  return TDO_OK;
}

int32_t check_nonfinite(Context* c, hipStream_t st, const char* what) {
  if (capturing(st) || !c->nf_dev) return TDO_OK;
  TDO_HIP(hipMemcpyAsync(c->nf_host, c->nf_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  TDO_HIP(hipStreamSynchronize(st));
  TDO_CHECK(c->nf_host[0] == 0, TDO_ENONFINITE, "%s: %u parameter values are inf or nan", what, c->nf_host[0]);
  return TDO_OK;
}

int32_t check_params_finite(Context* c, const float* p, int64_t n, hipStream_t st) {
  TDO_TRY(count_nonfinite(c, p, n, false, st));
  return check_nonfinite(c, st, "params");
}

int32_t ensure_workspace(Context* c, size_t bytes) {
  if (bytes <= c->ws_size) return TDO_OK;
  TDO_CHECK(bytes <= c->budget, TDO_ENOMEM, "workspace of %zu bytes exceeds the context budget of %zu bytes",
            bytes, c->budget);
  TDO_HIP(hipSetDevice(c->device));
  if (c->ws) {
    TDO_HIP(hipDeviceSynchronize());
    TDO_HIP(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_size = 0;
  }
  // grow geometrically so that a sequence of growing requests allocates rarely
  size_t want = std::min(c->budget, std::max(bytes, (size_t)(1.5 * (double)bytes)));
  hipError_t e = hipMalloc(&c->ws, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    e = hipMalloc(&c->ws, bytes);
    want = bytes;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->ws = nullptr;
    return set_error(TDO_ENOMEM, "hipMalloc of %zu workspace bytes failed: %s", bytes, hipGetErrorString(e));
  }
  c->ws_size = want;
  return TDO_OK;
}

int32_t net_plan(const Context* c, const tdo_arch_t* arch, int n, bool bf16, NetPlan* np) {
  TDO_TRY(make_pack_plan(arch, &np->pp));
  TDO_CHECK(n >= 3 && n <= 64, TDO_EINVAL, "chain length n=%d outside [3, 64]", n);
  np->bf16 = bf16;
  np->n = n;
  np->D = np->pp.D;
  np->DH = arch->d / arch->heads;
  np->span = n > 32;
  np->cpb = np->span ? 1 : 32 / n;
  np->masked = np->span ? (n < 64) : !(np->cpb == 1 && n == 32);
  np->score_scale = (float)(1.4426950408889634 / std::sqrt((double)np->DH));
  np->elem = bf16 ? 2 : 4;
  np->num_cus = c->num_cus;
  np->prof = const_cast<Profiler*>(&c->prof);
  np->fwd_wg_per_cu = 1;
  np->fwd_waves = bf16 ? 8 : 4;
  np->mlp_waves = (bf16 && np->pp.M == 256) ? 8 : 4;
  const uint64_t key = tune_key(*np);
  for (const TuneEntry& e : c->tune)
    if (e.key == key) {
      np->fwd_wg_per_cu = e.fwd_wg_per_cu;
      np->fwd_waves = e.fwd_waves;
      np->mlp_waves = e.mlp_waves;
    }
  return TDO_OK;
}

int64_t blocks_for(const NetPlan& np, int64_t E) { return np.span ? 4 * E : 2 * ((E + np.cpb - 1) / np.cpb); }

// Forward over E entries whose configurations are ecfg; z [E][2][2].
int32_t run_forward(const NetPlan& np, const NetWeights& w, const uint64_t* ecfg, int64_t E, const int64_t* E_dev,
                    float* xa, float* xb, const Saves* sv, float* z, hipStream_t st) {
  const PackPlan& pp = np.pp;
  const int L = pp.layers;
  for (int l = 0; l < L; ++l) {
    FwdArgs a{};
    a.wpack = static_cast<const char*>(w.wpack) + (size_t)l * pp.layer_elems * np.elem;
    a.b1 = w.b1 + (size_t)l * pp.M;
    a.b2 = w.b2 + (size_t)l * pp.D;
    a.table = w.table;
    a.ecfg = ecfg;
    a.n_entries_dev = E_dev;
    a.n_entries = E;
    a.x_in = (l % 2 == 0) ? xb : xa;  // layer l reads what layer l-1 wrote
    a.x_out = (l % 2 == 0) ? xa : xb;
    if (sv) {
      a.save_x = static_cast<char*>(sv->x) + (size_t)l * sv->layer_bytes;
      a.save_mid = static_cast<char*>(sv->mid) + (size_t)l * sv->layer_bytes;
      a.save_lse = sv->lse ? sv->lse + (size_t)l * sv->lse_layer : nullptr;
      a.save_last = sv->last;
    }
    a.head_w = w.head_w;
    a.head_b = w.head_b;
    a.z = z;
    a.n = np.n;
    a.cpb = np.cpb;
    a.d_real = pp.d;
    a.M = pp.M;
    a.score_scale = np.score_scale;
    a.first = l == 0;
    a.last = l == L - 1;
    a.masked = np.masked;
    a.blocks_per_cu = np.fwd_wg_per_cu;
    a.waves = np.fwd_waves;
    ProfScope ps(np.prof, "fwd_layer", st);
    TDO_TRY(launch_fwd_layer(a, np.bf16, np.D, np.DH, np.span, np.num_cus, st));
  }
  return TDO_OK;
}

int32_t pack_weights(const NetPlan& np, const float* params, NetWeights* w, hipStream_t st) {
  TDO_TRY(launch_pack_forward(np.pp, params, np.bf16, w->wpack, w->b1, w->b2, st));
  TDO_TRY(launch_embed_table(params, np.pp.d, np.D, w->table, st));
  w->head_w = params + np.pp.off_head_w;
  w->head_b = params + np.pp.off_head_b;
  return TDO_OK;
}

void carve_weights(const NetPlan& np, Arena& ar, size_t* offs) {
  const PackPlan& pp = np.pp;
  offs[0] = ar.take<char>((size_t)pp.layer_elems * pp.layers * np.elem);
  offs[1] = ar.take<float>((size_t)pp.layers * pp.M);
  offs[2] = ar.take<float>((size_t)pp.layers * pp.D);
  offs[3] = ar.take<float>(64 * (size_t)pp.D);
}

NetWeights weights_at(void* ws, const size_t* offs) {
  NetWeights w{};
  w.wpack = at<char>(ws, offs[0]);
  w.b1 = at<float>(ws, offs[1]);
  w.b2 = at<float>(ws, offs[2]);
  w.table = at<float>(ws, offs[3]);
  return w;
}

}  // namespace tdo

using namespace tdo;

extern "C" {

const char* tdo_last_error(void) { return g_err.c_str(); }

int32_t tdo_ctx_create(tdo_ctx_t** ctx, int32_t device, size_t workspace_bytes) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  int ndev = 0;
  TDO_HIP(hipGetDeviceCount(&ndev));
  TDO_CHECK(device >= 0 && device < ndev, TDO_EINVAL, "device %d not in [0, %d)", device, ndev);
  TDO_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  TDO_HIP(hipGetDeviceProperties(&prop, device));
  TDO_CHECK(std::strncmp(prop.gcnArchName, "gfx950", 6) == 0, TDO_EUNSUPPORTED,
            "device %d is %s; this library is built for gfx950 (MI355X) only", device, prop.gcnArchName);
  tdo_ctx_t* c = new (std::nothrow) tdo_ctx_t;
  TDO_CHECK(c != nullptr, TDO_ENOMEM, "out of host memory");
  c->c.device = device;
  c->c.num_cus = prop.multiProcessorCount;
  c->c.budget = workspace_bytes ? workspace_bytes : (size_t(8) << 30);
  tune_cache_load(&c->c);
  {
    const int32_t s = noalloc_setup(device);
    if (s != TDO_OK) {
      delete c;
      return s;
    }
  }
  if (hipEventCreateWithFlags(&c->c.ws_done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return set_error(TDO_EHIP, "hipEventCreateWithFlags failed");
  }
  *ctx = c;
  return TDO_OK;
}

int32_t tdo_ctx_destroy(tdo_ctx_t* ctx) {
  clear_error();
  if (!ctx) return TDO_OK;
  TDO_HIP(hipSetDevice(ctx->c.device));
  TDO_HIP(hipDeviceSynchronize());
  ctx->c.prof.destroy();
  if (ctx->c.graph.exec) TDO_HIP(hipGraphExecDestroy(ctx->c.graph.exec));
  if (ctx->c.ws) TDO_HIP(hipFree(ctx->c.ws));
  if (ctx->c.nf_dev) TDO_HIP(hipFree(ctx->c.nf_dev));
  if (ctx->c.nf_host) TDO_HIP(hipHostFree(ctx->c.nf_host));
  if (ctx->c.ws_done) TDO_HIP(hipEventDestroy(ctx->c.ws_done));
  delete ctx;
  return TDO_OK;
}

int32_t tdo_profile(tdo_ctx_t* ctx, int32_t enable) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_HIP(hipSetDevice(ctx->c.device));
  for (auto& r : ctx->c.prof.recs) TDO_HIP(hipEventSynchronize(r.stop));
  ctx->c.prof.recycle();
  ctx->c.prof.enabled = enable != 0;
  return TDO_OK;
}

int32_t tdo_profile_read(tdo_ctx_t* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  clear_error();
  TDO_CHECK(ctx && kernel && total_ms && launches, TDO_EINVAL, "NULL argument");
  TDO_HIP(hipSetDevice(ctx->c.device));
  double t = 0.0;
  int64_t k = 0;
  for (auto& r : ctx->c.prof.recs) {
    if (std::strcmp(r.name, kernel) != 0) continue;
    TDO_HIP(hipEventSynchronize(r.stop));
    float ms = 0.f;
    TDO_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    t += ms;
    ++k;
  }
  *total_ms = t;
  *launches = k;
  return TDO_OK;
}

int64_t tdo_num_params(const tdo_arch_t* arch) {
  clear_error();
  PackPlan pp;
  if (make_pack_plan(arch, &pp) != TDO_OK) return -1;
  return pp.nparams;
}

int32_t tdo_connected(tdo_ctx_t* ctx, const tdo_model_t* model, const uint64_t* cfg, int64_t B, int32_t kmax,
                      uint64_t* conn, float* mel, int32_t* n_conn, hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  ModelDev m;
  TDO_TRY(make_model(model, &m));
  TDO_CHECK(B >= 0, TDO_EINVAL, "B=%lld < 0", (long long)B);
  TDO_CHECK(kmax >= m.nslots, TDO_EINVAL, "kmax=%d smaller than the number of slots (%d) of a row", kmax,
            m.nslots);
  if (B == 0) return TDO_OK;
  TDO_CHECK(cfg && conn && mel && n_conn, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  return launch_connected(m, cfg, B, kmax, conn, mel, n_conn, stream);
}

int32_t tdo_local_lindbladian(tdo_ctx_t* ctx, int64_t B, const float* log_rho_x, const float* mel,
                              const int32_t* n_conn, int32_t kmax, const float* log_rho_conn, float* lloc,
                              hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(B >= 0 && kmax >= 1, TDO_EINVAL, "B=%lld, kmax=%d", (long long)B, kmax);
  if (B == 0) return TDO_OK;
  TDO_CHECK(log_rho_x && mel && n_conn && log_rho_conn && lloc, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  return launch_lloc_fixed(B, log_rho_x, mel, n_conn, kmax, log_rho_conn, lloc, stream);
}

int32_t tdo_log_rho(tdo_ctx_t* ctx, const tdo_arch_t* arch, const float* params, int32_t n, const uint64_t* cfg,
                    int64_t B, tdo_prec_t prec, float* log_rho, hipStream_t stream) {
  clear_error();
  TDO_CHECK(ctx != nullptr, TDO_EINVAL, "ctx is NULL");
  TDO_CHECK(prec == TDO_FP32 || prec == TDO_BF16, TDO_EINVAL, "unknown precision %d", (int)prec);
  NetPlan np;
  TDO_TRY(net_plan(&ctx->c, arch, n, prec == TDO_BF16, &np));
  TDO_CHECK(B >= 0, TDO_EINVAL, "B=%lld < 0", (long long)B);
  if (B == 0) return TDO_OK;
  TDO_CHECK(params && cfg && log_rho, TDO_EINVAL, "NULL buffer");
  TDO_HIP(hipSetDevice(ctx->c.device));
  Context& c = ctx->c;
  WsOrder order;
  TDO_TRY(order.begin(&c, stream));
  TDO_TRY(check_params_finite(&c, params, np.pp.nparams, stream));
  Arena ar;
  size_t woff[4];
  carve_weights(np, ar, woff);
  const size_t fixed = ar.used + 4096;
  const size_t per_block = 32 * (size_t)np.D * 4;
  TDO_CHECK(c.budget > fixed + 8 * per_block, TDO_ENOMEM, "workspace budget %zu too small", c.budget);
  // entries per chunk: two FP32 residual buffers + z
  const double per_entry = 2.0 * per_block * (np.span ? 4.0 : 2.0 / np.cpb) + 16.0;
  int64_t chunk = (int64_t)((double)(c.budget - fixed) / per_entry);
  chunk = std::min<int64_t>(chunk, B);
  chunk = std::max<int64_t>(np.cpb, chunk / np.cpb * np.cpb);
  const int64_t nblk = blocks_for(np, chunk);
  const size_t oxa = ar.take<float>((size_t)nblk * 32 * np.D);
  const size_t oxb = ar.take<float>((size_t)nblk * 32 * np.D);
  const size_t oz = ar.take<float>((size_t)chunk * 4);
  TDO_TRY(ensure_workspace(&c, ar.used));
  NetWeights w = weights_at(c.ws, woff);
  TDO_TRY(pack_weights(np, params, &w, stream));
  for (int64_t e0 = 0; e0 < B; e0 += chunk) {
    const int64_t E = std::min(chunk, B - e0);
    TDO_TRY(run_forward(np, w, cfg + 2 * e0, E, nullptr, at<float>(c.ws, oxa), at<float>(c.ws, oxb), nullptr,
                        at<float>(c.ws, oz), stream));
    TDO_TRY(launch_symmetrise(nullptr, E, at<float>(c.ws, oz), log_rho + 2 * e0, stream));
  }
  return TDO_OK;
}

}  // extern "C"
