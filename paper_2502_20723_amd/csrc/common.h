// Shared definitions of the tdo HIP library: error state, context, workspace,
// and small device helpers (wave reductions, packed configurations).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tdo.h"

namespace tdo {

// ---------------------------------------------------------------- errors
int32_t set_error(int32_t code, const char* fmt, ...);
void clear_error();

#define TDO_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::tdo::set_error(TDO_EHIP, "%s failed: %s (%s:%d)", #call,                \
                              hipGetErrorString(e_), __FILE__, __LINE__);              \
  } while (0)

#define TDO_CHECK(cond, code, ...)                     \
  do {                                                 \
    if (!(cond)) return ::tdo::set_error(code, __VA_ARGS__); \
  } while (0)

#define TDO_TRY(expr)              \
  do {                             \
    int32_t s_ = (expr);           \
    if (s_ != TDO_OK) return s_;   \
  } while (0)

// ---------------------------------------------------------------- profiling
// Optional per-kernel timing: when enabled, each launch of a named kernel
// group is bracketed by HIP events recorded on the launch stream.  Events come
// from a pool owned by the context and are read (and returned) on request.
struct Profiler {
  bool enabled = false;
  bool suspended = false;  // set while a launch sequence is recorded into a graph
  struct Rec {
    const char* name;
    hipEvent_t start, stop;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void recycle();
  void destroy();
};

struct ProfScope {
  Profiler* p;
  const char* name;
  hipStream_t st;
  hipEvent_t start = nullptr;
  ProfScope(Profiler* p_, const char* name_, hipStream_t st_);
  ~ProfScope();
};

// ---------------------------------------------------------------- graphs and tuning
// Recorded launch sequence of the batched loss/gradient: the arguments it was
// recorded for (including the workspace base), and the instantiated graph.
struct GraphCache {
  std::vector<uint8_t> seen_key, key;  // arguments of the last eager call / of the recording
  void* seen_ws = nullptr;
  void* ws = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Autotuned launch shapes: workgroups per CU of the forward layer kernel, per
// (chain length, precision, padded width, head width).
struct TuneEntry {
  uint64_t key;
  int fwd_wg_per_cu, fwd_waves, mlp_waves;
};


// Allow a kernel the whole 160 KB LDS of a CU, once per kernel and device per
// process (a host-side attribute, so later launches, also while a stream is
// being recorded into a graph, need no further runtime call).
int32_t allow_full_lds(const void* kern);

// ---------------------------------------------------------------- context
struct Context {
  int device = 0;
  int num_cus = 256;
  size_t budget = 0;
  void* ws = nullptr;
  size_t ws_size = 0;
  Profiler prof;
  GraphCache graph;
  std::vector<TuneEntry> tune;
  std::string tune_cache;  // path of the JSON cache of the tuned shapes, or empty
  // count of non-finite parameters (device) and its pinned host copy
  uint32_t* nf_dev = nullptr;
  uint32_t* nf_host = nullptr;
  // recorded at the end of the last call that used the workspace, on the stream it ran on
  hipEvent_t ws_done = nullptr;
  hipStream_t ws_stream = nullptr;
  bool ws_recorded = false;
};

// The autotuned shapes kept in a JSON file (the path in TDO_AUTOTUNE_CACHE): read when a
// context is created, rewritten when a call tunes a new shape.
void tune_cache_load(Context* c);
void tune_cache_save(const Context* c);

// Orders calls that share the context's workspace across streams: the call's stream
// first waits for the end of the previous call when that ran on another stream, and the
// end of this call is recorded when the guard goes out of scope.  Inactive while the
// stream is being captured into a graph (the library's own recording of the batched
// call orders its launches by the capturing stream alone).
struct WsOrder {
  Context* c = nullptr;
  hipStream_t st = nullptr;
  bool active = false;
  int32_t begin(Context* c_, hipStream_t st_);
  ~WsOrder();
};

// Non-finite parameters: count them on the stream (a read-only kernel, one workgroup per
// call; accumulate adds to the count of the previous call), then wait for the count.
// Both are skipped while the stream is being captured.
int32_t count_nonfinite(Context* c, const float* p, int64_t n, bool accumulate, hipStream_t st);
int32_t check_nonfinite(Context* c, hipStream_t st, const char* what);
// Both steps for one parameter vector.
int32_t check_params_finite(Context* c, const float* p, int64_t n, hipStream_t st);

// Device address of the no-allocation scratch array on a device, looked up once per device.
int32_t noalloc_setup(int device);

// Grow the context workspace to at least `bytes` (<= budget).
int32_t ensure_workspace(Context* c, size_t bytes);

// Bump allocator over a workspace region; all offsets aligned to 256 bytes.
struct Arena {
  size_t used = 0;
  template <class T>
  size_t take(size_t count) {
    size_t off = used;
    used = (used + count * sizeof(T) + 255) & ~size_t(255);
    return off;
  }
};

template <class T>
inline T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// ---------------------------------------------------------------- device helpers
constexpr int WAVE = 64;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__host__ __device__ inline uint64_t low_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// Cyclic shift by one site towards lower indices: bit i of the result is bit i+1 (mod n).
__host__ __device__ inline uint64_t rot_down(uint64_t x, int n) {
  return ((x >> 1) | (x << (n - 1))) & low_mask(n);
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace tdo

struct tdo_ctx {
  tdo::Context c;
};
