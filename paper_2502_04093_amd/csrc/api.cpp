// C ABI of the IPComp library: contexts, streams, states and the three calls
// of the paper's problem statement (compress; retrieve at a fidelity; refine to
// a higher fidelity), plus the host-only planner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>
#include <unistd.h>

#include "ipc_internal.h"
#include "kernels.h"

using namespace ipc;

// ------------------------------------------------------------------ objects

// Tuned column lengths (chunk rows per workgroup) of the fused level
// launches, per field shape, dtype and interpolation; 0 = the default rule
struct TuneKey {
  int64_t d[3];
  int dtype, interp;
  bool operator<(const TuneKey &o) const {
    return std::tie(d[0], d[1], d[2], dtype, interp) < std::tie(o.d[0], o.d[1], o.d[2], o.dtype, o.interp);
  }
};
struct TuneVal {
  int32_t zseg_c[32];  // compression, by level
  int32_t zseg_r[32];  // retrieval, by level
};
// the batch schedule chosen for a shape: graph replays or direct launches,
// and the persistent grid of a full queue slot (workgroups per CU)
struct BatchTune {
  int graphs_r = 0, graphs_c = 0;
  uint32_t per_cu_r = 0, per_cu_c = 0;
};

struct ipc_ctx {
  int device = 0;
  std::map<TuneKey, TuneVal> tuned;     // autotuner results
  int forced_zseg = 0;                  // while tuning: every level uses this
  void *dev_zero = nullptr;             // 256 zero bytes on the device
  int n_cu = 256;                       // compute units of the device
  hipStream_t stream = nullptr;
  // no stream was given: a blocking stream the context creates, which HIP
  // orders after the work queued on the null stream before each of its
  // operations (and the null stream's later work after them), so inputs
  // written there are complete before they are read
  hipStream_t owned = nullptr;
  hipEvent_t ev_copy = nullptr;  // a compression's summary copy (the host waits on it alone)
  std::string err;
  std::multimap<size_t, void *> cache;  // freed device blocks by size
  size_t cached_bytes = 0;
  // reusable workspace
  void *ws_xh = nullptr;
  size_t ws_xh_bytes = 0;
  void *ws_summary = nullptr;
  size_t ws_summary_bytes = 0;
  void *ws_out = nullptr;
  size_t ws_out_cap = 0;  // records
  void *ws_g[2] = {nullptr, nullptr};   // compact coarse grids (by level parity)
  size_t ws_g_bytes[2] = {0, 0};
  void *ws_args = nullptr;              // PassArgs of the current call
  size_t ws_args_bytes = 0;
  std::vector<PassArgs> args_host;      // what ws_args holds ...
  void *args_dev_at = nullptr;          // ... while it is this allocation
  void *ws_cnt = nullptr;               // outlier index scratch: per-chunk counts, block sums
  size_t ws_cnt_bytes = 0;
  void *ws_rows = nullptr;              // fused-level compression: per-workgroup rows
  size_t ws_rows_bytes = 0;
  void *host_summary = nullptr;         // pinned copy of the compression summary
  size_t host_summary_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // this device's copy of the no-allocation scratch (null if it could not be
  // resolved; ipc_retrieve_noalloc then fails with IPC_EHIP)
  void *scratch = nullptr;
  // per-pass timing
  bool profiling = false;
  std::vector<hipEvent_t> pev;   // 2 per pass
  std::vector<int> pev_pass;     // pass index of each timed pair
  std::vector<float> pass_ms;     // per pass (0 = not run)
  size_t prof_np = 0;
  int prof_only = -1;
  // batches as queue launches replayed from captured HIP graphs: 0 never
  // (direct launches), 1 always, 2 as the batch autotuner chose for the
  // batch's shape, else by field size
  int batch_graphs = 0;
  std::map<TuneKey, BatchTune> tuned_batch;
  // workgroups per CU of a full queue slot while a batch runs (0 = default)
  uint32_t per_cu_r = 0, per_cu_c = 0;
  std::map<std::vector<int>, hipGraphExec_t> graphs;  // by launch shape
  void *ws_q = nullptr;       // claim counters, then the queue table (fixed address)
  size_t ws_q_bytes = 0;
  void *host_q = nullptr;     // pinned staging of the queue table
  uint64_t graphs_captured = 0, graph_replays = 0;
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct ipc_stream {
  ipc_ctx *ctx = nullptr;
  StreamMeta meta;
  PlanTables tables;
  bool packed = false;         // payload placement
  bool host_payload = false;   // payload in pinned host memory the device reads
  DevBuf payload;              // u32 words
  DevBuf masks;                // u32 per chunk
  DevBuf chunk_off;            // u64 per chunk (packed placement only)
  DevBuf coded;                // entropy-coded payload (meta.coding == 1)
  DevBuf out_gchunk, out_local, out_bits, out_start;
  bool host_masks_valid = false;
  bool host_outliers_valid = true;  // meta.outliers holds the records (else only on the device)
  std::vector<PassArgs> args;
};

struct ipc_state {
  ipc_ctx *ctx = nullptr;
  const ipc_stream *stream = nullptr;
  std::vector<int> plan;
  DevBuf field;
  double bound = 0;
};

// ------------------------------------------------------------------ helpers

// Scratch of ipc_retrieve_noalloc: the compact coarse grids of a fused 3-D
// retrieval.  Every device the library runs on holds its own copy until the
// process ends.  In host code the array's name is not a device address: the
// device's copy is resolved once per device (device_scratch) and only that
// pointer is handed to kernels.
static __device__ __align__(256) unsigned char scratch[IPC_NOALLOC_SCRATCH_BYTES];

namespace {

struct Fail {
  ipc_status st;
};

// The address of `scratch` on `device`, which must be the current device;
// resolved on the first call per device and kept.  Null if it cannot be
// resolved.
void *device_scratch(int device) {
  static std::mutex mu;
  static std::map<int, void *> ptrs;
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptrs.find(device);
  if (it != ptrs.end()) return it->second;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;  // not kept: a later context tries again
  }
  ptrs[device] = p;
  return p;
}

// A named range on the ROCTx marker stream for the span of a library call
// (seen by rocprofv3 --marker-trace; nearly free when no tool listens)
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

// Host worker threads for parallel_for, started once per process and kept:
// starting threads per call had cost about as much as the planning they
// shared out.  One job at a time; a caller that finds the pool busy (another
// host thread's call) runs its job alone.
class WorkerPool {
 public:
  static WorkerPool &get() {
    static WorkerPool pool;
    return pool;
  }
  size_t helpers() const { return th_.size(); }
  // fn(i) for i in [0, n) on the helpers and the calling thread; false (and
  // nothing run) when the pool is busy
  bool run(size_t n, const std::function<void(size_t)> &fn) {
    // a forked child has none of the helpers
    if (getpid() != pid_) return false;
    std::unique_lock<std::mutex> busy(job_mu_, std::try_to_lock);
    if (!busy.owns_lock() || th_.empty()) return false;
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_.store(0);
      working_ = th_.size();
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return working_ == 0; });
    fn_ = nullptr;
    return true;
  }

 private:
  WorkerPool() : pid_(getpid()) {
    const size_t hw = std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
    try {
      for (size_t t = 1; t < hw; ++t) th_.emplace_back([this] { loop(); });
    } catch (...) {
    }
  }
  ~WorkerPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (std::thread &t : th_) t.join();
  }
  void work() {
    for (size_t i = next_.fetch_add(1); i < n_; i = next_.fetch_add(1)) (*fn_)(i);
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      work();
      std::lock_guard<std::mutex> lk(mu_);
      if (--working_ == 0) done_cv_.notify_one();
    }
  }
  pid_t pid_;
  std::vector<std::thread> th_;
  std::mutex job_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(size_t)> *fn_ = nullptr;
  size_t n_ = 0;
  std::atomic<size_t> next_{0};
  size_t working_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// fn(i) for i in [0, n) on up to 16 host threads (planning several requests:
// each plan reads only its stream's tables).  The first exception any call
// throws is rethrown once every call has returned.
template <typename Fn>
void parallel_for(size_t n, Fn fn) {
  std::exception_ptr err;
  std::mutex err_mu;
  const std::function<void(size_t)> job = [&](size_t i) {
    try {
      fn(i);
    } catch (...) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (!err) err = std::current_exception();
    }
  };
  if (n < 4 || !WorkerPool::get().run(n, job))
    for (size_t i = 0; i < n; ++i) job(i);
  if (err) std::rethrow_exception(err);
}

void set_err(ipc_ctx *ctx, const std::string &m) {
  if (ctx) ctx->err = m;
}

void hip_check(ipc_ctx *ctx, hipError_t e, const char *what) {
  if (e != hipSuccess) {
    set_err(ctx, std::string(what) + ": " + hipGetErrorString(e));
    throw Fail{e == hipErrorOutOfMemory ? IPC_ENOMEM : IPC_EHIP};
  }
}

// Start of a call that issues device work: the context's device becomes
// current.  (Ordering after the caller's null-stream work comes from the
// owned stream being a blocking stream: an explicit event on the null stream
// per call cost about 19 us of host time, as does querying the null stream.)
void enter_device(ipc_ctx *ctx) {
  hip_check(ctx, hipSetDevice(ctx->device), "hipSetDevice");
}

DevBuf dev_alloc(ipc_ctx *ctx, size_t bytes) {
  DevBuf b;
  b.bytes = bytes;
  if (bytes == 0) return b;
  auto it = ctx->cache.lower_bound(bytes);
  if (it != ctx->cache.end() && it->first <= bytes + bytes / 2 + 4096) {
    b.p = it->second;
    b.bytes = it->first;
    ctx->cached_bytes -= it->first;
    ctx->cache.erase(it);
    return b;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    // release the cache and retry once
    for (auto &kv : ctx->cache) (void)hipFree(kv.second);
    ctx->cache.clear();
    ctx->cached_bytes = 0;
    (void)hipGetLastError();
    e = hipMalloc(&b.p, bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_err(ctx, "device allocation of " + std::to_string(bytes) + " bytes failed");
    throw Fail{IPC_ENOMEM};
  }
  return b;
}

void dev_free(ipc_ctx *ctx, DevBuf &b) {
  if (b.p) {
    if (ctx) {
      ctx->cache.emplace(b.bytes, b.p);
      ctx->cached_bytes += b.bytes;
    } else {
      (void)hipFree(b.p);
    }
  }
  b.p = nullptr;
  b.bytes = 0;
}

void *ensure_ws(ipc_ctx *ctx, void *&p, size_t &have, size_t need) {
  if (have >= need && p) return p;
  if (p) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(p);
    p = nullptr;
    have = 0;
  }
  hipError_t e = hipMalloc(&p, need);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_err(ctx, "workspace allocation failed");
    throw Fail{IPC_ENOMEM};
  }
  have = need;
  return p;
}

void prof_begin(ipc_ctx *ctx, size_t n_passes) {
  ctx->pev_pass.clear();
  ctx->pass_ms.clear();
  ctx->prof_np = n_passes;
  if (!ctx->profiling) return;
  while (ctx->pev.size() < 2 * n_passes) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      set_err(ctx, "event creation failed");
      throw Fail{IPC_EHIP};
    }
    ctx->pev.push_back(e);
  }
}

void prof_mark(ipc_ctx *ctx, int pass, bool start) {
  if (!ctx->profiling) return;
  if (ctx->prof_only >= 0 && pass != ctx->prof_only) return;
  size_t k = ctx->pev_pass.size();
  if (start) {
    (void)hipEventRecord(ctx->pev[2 * k], ctx->stream);
  } else {
    (void)hipEventRecord(ctx->pev[2 * k + 1], ctx->stream);
    ctx->pev_pass.push_back(pass);
  }
}

// after the stream is synchronized
void prof_end(ipc_ctx *ctx) {
  if (!ctx->profiling) return;
  ctx->pass_ms.assign(ctx->prof_np, 0.0f);
  for (size_t k = 0; k < ctx->pev_pass.size(); ++k)
    (void)hipEventElapsedTime(&ctx->pass_ms[size_t(ctx->pev_pass[k])], ctx->pev[2 * k],
                              ctx->pev[2 * k + 1]);
}

PassArgs make_args(const Schedule &s, const PassGeom &p) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  for (int j = 0; j < 3; ++j) {
    a.dims3[j] = s.dims3[j];
    a.ldims[j] = p.ldims[j];
    a.tdims[j] = p.tdims[j];
    a.ct[j] = p.ct[j];
    a.tiles[j] = p.tiles[j];
    a.kinds[j] = p.kinds[j];
  }
  a.dim3 = p.dim3;
  a.h = p.h;
  a.n_chunks = p.n_chunks;
  a.chunk_base = p.chunk_base;
  a.slot_base = p.slot_base;
  a.wmax = uint32_t(p.wmax);
  a.pass_index = uint32_t(p.index);
  return a;
}

bool chunks_supported(const Schedule &s, std::string &err) {
  for (const PassGeom &p : s.passes)
    if (p.max_count > MAX_CHUNK_CODES) {
      err = "chunks larger than " + std::to_string(MAX_CHUNK_CODES) + " codes are not supported";
      return false;
    }
  return true;
}

template <typename F>
ipc_status guarded(ipc_ctx *ctx, F &&f) {
  try {
    f();
    return IPC_OK;
  } catch (const Fail &e) {
    return e.st;
  } catch (const std::bad_alloc &) {
    set_err(ctx, "host allocation failed");
    return IPC_ENOMEM;
  } catch (...) {
    set_err(ctx, "unexpected internal error");
    return IPC_EHIP;
  }
}

void free_stream_bufs(ipc_stream *s) {
  ipc_ctx *c = s->ctx;
  if (s->host_payload) {
    if (s->payload.p) (void)hipHostFree(s->payload.p);
    s->payload = DevBuf();
    s->host_payload = false;
  }
  dev_free(c, s->payload);
  dev_free(c, s->masks);
  dev_free(c, s->chunk_off);
  dev_free(c, s->coded);
  dev_free(c, s->out_gchunk);
  dev_free(c, s->out_local);
  dev_free(c, s->out_bits);
  dev_free(c, s->out_start);
}

void upload_outliers(ipc_ctx *ctx, ipc_stream *s) {
  size_t n = s->meta.outliers.size();
  s->meta.n_outliers = n;
  s->host_outliers_valid = true;
  if (n == 0) return;
  std::vector<uint64_t> gch(n), bits(n);
  std::vector<uint32_t> loc(n);
  for (size_t i = 0; i < n; ++i) {
    const OutlierRec &o = s->meta.outliers[i];
    gch[i] = uint64_t(s->meta.sched.passes[o.pass].chunk_base) + o.chunk;
    loc[i] = o.local;
    bits[i] = o.bits;
  }
  s->out_gchunk = dev_alloc(ctx, 8 * n);
  s->out_local = dev_alloc(ctx, 4 * n);
  s->out_bits = dev_alloc(ctx, 8 * n);
  hip_check(ctx, hipMemcpyAsync(s->out_gchunk.p, gch.data(), 8 * n, hipMemcpyHostToDevice, ctx->stream), "upload");
  hip_check(ctx, hipMemcpyAsync(s->out_local.p, loc.data(), 4 * n, hipMemcpyHostToDevice, ctx->stream), "upload");
  hip_check(ctx, hipMemcpyAsync(s->out_bits.p, bits.data(), 8 * n, hipMemcpyHostToDevice, ctx->stream), "upload");
  const uint64_t nc = uint64_t(s->meta.sched.n_chunks);
  s->out_start = dev_alloc(ctx, 4 * (nc + 1));
  hip_check(ctx, launch_out_start(static_cast<const uint64_t *>(s->out_gchunk.p), n, nc,
                                  static_cast<uint32_t *>(s->out_start.p), ctx->stream),
            "outlier index launch");
  hip_check(ctx, hipStreamSynchronize(ctx->stream), "upload");
}

// the device-sorted outlier records into meta.outliers (pass, chunk, local, bits)
// Descriptors of the stored blocks (payload order: chunks in order, planes
// 31 down to 0) built on the device into `blk` from three per-chunk tables
// made here: first block, raw word offset in the packed placement, codes.
// Coded offsets are filled separately (launch_ec_offsets).  `tabs` holds the
// uploaded tables until the caller synchronizes.
void device_blocks(ipc_ctx *ctx, const StreamMeta &m, DevBuf &blk, DevBuf &tabs) {
  const size_t nc = size_t(m.sched.n_chunks);
  std::vector<uint64_t> craw;
  packed_chunk_offsets(m, craw);  // nc + 1 entries
  std::vector<uint32_t> cblk(nc + 1), ccount(nc + 1, 0);
  uint32_t nb = 0;
  std::vector<uint32_t> cnt;
  for (const PassGeom &p : m.sched.passes) {
    chunk_counts(p, cnt);
    for (int64_t c = 0; c < p.n_chunks; ++c) {
      const size_t g = size_t(p.chunk_base + c);
      cblk[g] = nb;
      ccount[g] = cnt[size_t(c)];
      nb += uint32_t(__builtin_popcount(m.masks[g]));
    }
  }
  cblk[nc] = nb;
  const size_t b_raw = craw.size() * 8, b_blk = cblk.size() * 4, b_cnt = ccount.size() * 4;
  tabs = dev_alloc(ctx, b_raw + b_blk + b_cnt);
  char *t = static_cast<char *>(tabs.p);
  hip_check(ctx, hipMemcpyAsync(t, craw.data(), b_raw, hipMemcpyHostToDevice, ctx->stream), "upload");
  hip_check(ctx, hipMemcpyAsync(t + b_raw, cblk.data(), b_blk, hipMemcpyHostToDevice, ctx->stream), "upload");
  hip_check(ctx, hipMemcpyAsync(t + b_raw + b_blk, ccount.data(), b_cnt, hipMemcpyHostToDevice, ctx->stream),
            "upload");
  blk = dev_alloc(ctx, std::max<size_t>(sizeof(EcBlock), size_t(nb) * sizeof(EcBlock)));
  hip_check(ctx, launch_ec_blocks(reinterpret_cast<const uint32_t *>(t + b_raw),
                                  reinterpret_cast<const uint64_t *>(t),
                                  reinterpret_cast<const uint32_t *>(t + b_raw + b_blk), nc,
                                  static_cast<EcBlock *>(blk.p), ctx->stream),
            "block table launch");
}

void fetch_outliers(ipc_ctx *ctx, ipc_stream *s) {
  StreamMeta &m = s->meta;
  const size_t n = size_t(m.n_outliers);
  std::vector<uint64_t> gch(n), bits(n);
  std::vector<uint32_t> loc(n);
  if (n) {
    hip_check(ctx, hipMemcpyAsync(gch.data(), s->out_gchunk.p, 8 * n, hipMemcpyDeviceToHost, ctx->stream), "copy");
    hip_check(ctx, hipMemcpyAsync(loc.data(), s->out_local.p, 4 * n, hipMemcpyDeviceToHost, ctx->stream), "copy");
    hip_check(ctx, hipMemcpyAsync(bits.data(), s->out_bits.p, 8 * n, hipMemcpyDeviceToHost, ctx->stream), "copy");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "copy");
  }
  m.outliers.resize(n);
  const std::vector<PassGeom> &ps = m.sched.passes;
  size_t p = 0;
  for (size_t i = 0; i < n; ++i) {
    // records are sorted by global chunk, so the pass index only moves forward
    while (p + 1 < ps.size() && uint64_t(ps[p + 1].chunk_base) <= gch[i]) ++p;
    OutlierRec &o = m.outliers[i];
    o.pass = uint32_t(p);
    o.chunk = uint32_t(gch[i] - uint64_t(ps[p].chunk_base));
    o.local = loc[i];
    o.pad = 0;
    o.bits = bits[i];
  }
  s->host_outliers_valid = true;
}

void fill_info(const ipc_stream *s, const std::vector<int> &plan, double bound, uint32_t flags,
               uint64_t read, float tplan, float tdev, ipc_info *info) {
  if (!info) return;
  std::memset(info, 0, sizeof(*info));
  info->bound = bound;
  info->bytes_loaded = uint64_t(plan_loaded(s->tables, plan));
  info->bytes_total = s->meta.serialized_bytes;
  info->bytes_read = read;
  info->n_passes = uint32_t(plan.size());
  info->flags = flags;
  for (size_t i = 0; i < plan.size() && i < IPC_MAX_PASSES; ++i) info->plan[i] = uint8_t(plan[i]);
  info->t_plan_ms = tplan;
  info->t_device_ms = tdev;
}

// ---------------------------------------------------------------- fused 3-D levels

Level3Args level3_args(const Schedule &s, int l, int64_t fill = 1024);

// The fused level kernels cover 3-D fields with the default chunk shape and
// 2-D fields with chunks of 16 x 64 (the 3-D tile with a z extent of one
// plane, pass A absent), whose level-1 launch fits the grid limits (their tile
// arithmetic is 32-bit).
bool fused3(const Schedule &s) {
  const bool c3 = s.D == 3 && s.chunk_log2[0] == 1 && s.chunk_log2[1] == 4 && s.chunk_log2[2] == 6;
  const bool c2 = s.D == 2 && s.chunk_log2[0] == 4 && s.chunk_log2[1] == 6;
  if (!(s.K >= 1 && (c3 || c2))) return false;
  // 32-bit element offsets inside the kernels' two-plane slabs
  if (s.n_points >= (int64_t(1) << 31)) return false;
  for (int j = 0; j < 3; ++j)
    if (s.dims3[j] > (int64_t(1) << 24)) return false;
  const Level3Args A = level3_args(s, 1);
  return A.tiles_y <= 65535 && (A.tiles_z + A.zseg - 1) / A.zseg <= 65535;
}

// points of the coarse grid G_j (fine stride 2^j)
int64_t coarse_points(const Schedule &s, int j) {
  int64_t n = 1;
  for (int d = 0; d < 3; ++d) n *= ((s.dims3[d] - 1) >> j) + 1;
  return n;
}

// fine-field strides of one step of stride h along z, y, x
void level_strides(const Schedule &s, int64_t h, Level3Args &A) {
  A.sZ = h * s.dims3[1] * s.dims3[2];
  A.sY = h * s.dims3[2];
  A.sX = int32_t(h);
}

Level3Args anchor3_args(const Schedule &s) {
  Level3Args A;
  std::memset(&A, 0, sizeof(A));
  const PassGeom &p = s.passes[0];
  for (int j = 0; j < 3; ++j) {
    A.L[j] = int32_t(p.ldims[j]);
    A.G[j] = int32_t(p.ldims[j]);
  }
  level_strides(s, p.h, A);
  A.chunk_base[0] = p.chunk_base;
  A.slot_base[0] = p.slot_base;
  A.wmax[0] = uint32_t(p.wmax);
  A.pass_index[0] = 0;
  return A;
}

// `fill`: workgroups that make one full round of the device
Level3Args level3_args(const Schedule &s, int l, int64_t fill) {
  Level3Args A;
  std::memset(&A, 0, sizeof(A));
  const int64_t h = int64_t(1) << (l - 1);
  for (int j = 0; j < 3; ++j) {
    A.L[j] = int32_t((s.dims3[j] - 1) / h + 1);
    A.G[j] = int32_t((s.dims3[j] - 1) / (2 * h) + 1);
  }
  level_strides(s, h, A);
  A.tiles_z = (A.L[0] + 1) / 2;
  A.tiles_y = (A.L[1] + 15) / 16;
  A.tiles_x = (A.L[2] + 63) / 64;
  // chunk rows per workgroup: long columns amortize the coarse-plane halo and
  // the workgroup's set-up, so the longest (up to 16) that still fills the
  // device; small levels get single-step columns
  const int64_t nxy = int64_t(A.tiles_y) * A.tiles_x;
  A.zseg = 16;
  while (A.zseg > 1 && nxy * ((A.tiles_z + A.zseg - 1) / A.zseg) < fill) A.zseg >>= 1;
  // passes A, B, C are the level's passes along z, y, x; a 2-D field has no
  // pass along z: its slot A gets no targets (tdims 0), wmax 0 (which the
  // compression kernel reads as "no pass A": no chunk masks written) and pass
  // B's chunk table, so reads through it stay in bounds
  const int D = s.D;
  for (int p = 3 - D; p < 3; ++p) {
    const PassGeom &g = s.passes[size_t(1 + (s.K - l) * D + p - (3 - D))];
    for (int j = 0; j < 3; ++j) {
      A.tdims[p][j] = int32_t(g.tdims[j]);
      A.ct[p][j] = int32_t(g.ct[j]);
    }
    A.chunk_base[p] = g.chunk_base;
    A.slot_base[p] = g.slot_base;
    A.wmax[p] = uint32_t(g.wmax);
    A.pass_index[p] = uint32_t(g.index);
  }
  if (D == 2) {
    for (int j = 0; j < 3; ++j) {
      A.tdims[0][j] = 0;
      A.ct[0][j] = A.ct[1][j];
    }
    A.chunk_base[0] = A.chunk_base[1];
    A.slot_base[0] = A.slot_base[1];
    A.wmax[0] = 0;
    A.pass_index[0] = A.pass_index[1];
  }
  return A;
}

// stream index of the last pass of level l (the pass its fused launch is
// timed and reported under)
int level_last_pass(const Schedule &s, int l) { return 1 + (s.K - l) * s.D + s.D - 1; }

// resident workgroups per compute unit assumed when sizing the fused level
// launches (occupancy of the compression and retrieval kernels)
#ifndef IPC_WG_PER_CU_C
#define IPC_WG_PER_CU_C 4
#endif
#ifndef IPC_WG_PER_CU_R
#define IPC_WG_PER_CU_R 4
#endif

// workgroups of a fused level launch (its 1-D grid)
int64_t level3_wgs(const Level3Args &A) {
  return int64_t(A.tiles_x) * A.tiles_y * ((A.tiles_z + A.zseg - 1) / A.zseg);
}

// Arguments of the fused launch of level l of a stream, with the column
// length the autotuner chose for this shape (or the one being tried)
Level3Args level_args(const ipc_ctx *ctx, const StreamMeta &m, int l, bool compress) {
  Level3Args La = level3_args(m.sched, l, (compress ? IPC_WG_PER_CU_C : IPC_WG_PER_CU_R) * int64_t(ctx->n_cu));
  int z = ctx->forced_zseg;
  if (z == 0 && !ctx->tuned.empty() && l < 32) {
    TuneKey k{{m.sched.dims3[0], m.sched.dims3[1], m.sched.dims3[2]}, m.dtype, m.interp};
    auto it = ctx->tuned.find(k);
    if (it != ctx->tuned.end()) z = compress ? it->second.zseg_c[l] : it->second.zseg_r[l];
  }
  if (z > 0) La.zseg = z;
  return La;
}

// Bytes of the compact coarse grids G_j of a fused retrieval by level parity
// (G_j lives in buffer j & 1)
void coarse_need(const Schedule &s, size_t isz, size_t need[2]) {
  need[0] = need[1] = 0;
  for (int j = 1; j <= s.K; ++j)
    need[j & 1] = std::max(need[j & 1], size_t(coarse_points(s, j)) * isz);
}

// compact coarse-grid buffers: G_j lives in ws_g[j & 1]
void ensure_coarse(ipc_ctx *ctx, const Schedule &s, size_t isz) {
  size_t need[2];
  coarse_need(s, isz, need);
  for (int i = 0; i < 2; ++i)
    ensure_ws(ctx, ctx->ws_g[i], ctx->ws_g_bytes[i], std::max<size_t>(need[i], 8));
}

// what the retrieval kernels read of a stream
RetrieveIn retrieve_in(ipc_ctx *ctx, const ipc_stream *s) {
  RetrieveIn in;
  in.payload = static_cast<const uint32_t *>(s->payload.p);
  in.masks = static_cast<const uint32_t *>(s->masks.p);
  in.chunk_off = s->packed ? static_cast<const uint64_t *>(s->chunk_off.p) : nullptr;
  in.out_gchunk = static_cast<const uint64_t *>(s->out_gchunk.p);
  in.out_local = static_cast<const uint32_t *>(s->out_local.p);
  in.out_bits = static_cast<const uint64_t *>(s->out_bits.p);
  in.out_start = static_cast<const uint32_t *>(s->out_start.p);
  in.n_out = s->meta.n_outliers;
  in.zero = static_cast<const uint32_t *>(ctx->dev_zero);
  return in;
}

// run passes [s0, P) of a retrieval into `field`; the fused path keeps its
// coarse grids in `ws` (two buffers by level parity) when given, else in the
// context's workspace
void run_retrieve(ipc_ctx *ctx, const ipc_stream *s, const std::vector<int> &plan, int s0,
                  void *field, void *const *ws = nullptr) {
  const RetrieveIn in = retrieve_in(ctx, s);
  prof_begin(ctx, s->args.size());
  const Schedule &sc = s->meta.sched;
  if (fused3(sc)) {
    const size_t isz = s->meta.dtype == IPC_F32 ? 4 : 8;
    void *g[2];
    if (ws) {
      g[0] = ws[0];
      g[1] = ws[1];
    } else {
      ensure_coarse(ctx, sc, isz);
      g[0] = ctx->ws_g[0];
      g[1] = ctx->ws_g[1];
    }
    int l_start = sc.K;
    // a refinement that starts in the top level rebuilds the top coarse grid
    // from the anchors (always fully loaded, so the same values) instead of
    // gathering it from the resident field
    if (s0 <= 0 || sc.passes[size_t(s0)].level == sc.K) {
      Level3Args A = anchor3_args(sc);
      prof_mark(ctx, 0, true);
      hip_check(ctx, launch_anchor3_retrieve(s->meta.dtype, A, g[sc.K & 1], in, s->meta.eb,
                                             ctx->stream),
                "anchor kernel launch");
      prof_mark(ctx, 0, false);
    } else {
      // refinement: restart at the level of pass s0 from the resident field
      l_start = sc.passes[size_t(s0)].level;
      int64_t gd[3];
      for (int j = 0; j < 3; ++j) gd[j] = ((sc.dims3[j] - 1) >> l_start) + 1;
      hip_check(ctx, launch_gather_coarse(s->meta.dtype, field, sc.dims3, int64_t(1) << l_start,
                                          g[l_start & 1], gd, ctx->stream),
                "gather kernel launch");
    }
    for (int l = l_start; l >= 1; --l) {
      Level3Args La = level_args(ctx, s->meta, l, false);
      int disc[3];
      for (int p = 0; p < 3; ++p) disc[p] = plan[La.pass_index[p]];
      int pc = int(La.pass_index[2]);
      prof_mark(ctx, pc, true);
      hip_check(ctx, launch_level3_retrieve(s->meta.dtype, s->meta.interp, La, g[l & 1],
                                            l > 1 ? g[(l - 1) & 1] : field, disc, in,
                                            s->meta.eb, ctx->stream),
                "level kernel launch");
      prof_mark(ctx, pc, false);
    }
    return;
  }
  for (size_t i = size_t(s0); i < s->args.size(); ++i) {
    prof_mark(ctx, int(i), true);
    hip_check(ctx, launch_retrieve_pass(s->meta.dtype, s->meta.interp, s->args[i], field, plan[i],
                                        in, s->meta.eb, ctx->stream),
              "retrieve kernel launch");
    prof_mark(ctx, int(i), false);
  }
}

uint64_t verify_stream(ipc_ctx *ctx, const ipc_stream *s, const void *field_dev) {
  const size_t isz = s->meta.dtype == IPC_F32 ? 4 : 8;
  const uint64_t n = uint64_t(s->meta.sched.n_points);
  DevBuf rec = dev_alloc(ctx, std::max<size_t>(8, size_t(n) * isz));
  DevBuf cnt = dev_alloc(ctx, 8);
  uint64_t bad = 0;
  try {
    std::vector<int> full(s->args.size(), 0);
    run_retrieve(ctx, s, full, 0, rec.p);
    hip_check(ctx, hipMemsetAsync(cnt.p, 0, 8, ctx->stream), "memset");
    hip_check(ctx, launch_verify_bound(s->meta.dtype, field_dev, rec.p, n, s->meta.eb,
                                       static_cast<unsigned long long *>(cnt.p), ctx->stream),
              "verify launch");
    hip_check(ctx, hipMemcpyAsync(&bad, cnt.p, 8, hipMemcpyDeviceToHost, ctx->stream), "copy");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "verify");
  } catch (...) {
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, rec);
    dev_free(ctx, cnt);
    throw;
  }
  dev_free(ctx, rec);
  dev_free(ctx, cnt);
  return bad;
}

void errq_to_bound(ipc_stream *s);

// What ipc_options asks for once a stream's planes and tables exist: the
// bound form of the delta-y table, the entropy-coded lossless stage, the
// full-precision check
ipc_status finish_options(ipc_ctx *ctx, ipc_stream *s, const void *field_dev, const ipc_options *opts) {
  if (!opts) return IPC_OK;
  if (opts->errq_mode == IPC_ERRQ_BOUND) errq_to_bound(s);
  if (opts->debug_flags & IPC_DEBUG_VERIFY) {
    uint64_t bad = 0;
    ipc_status st = guarded(ctx, [&] {
      enter_device(ctx);
      bad = verify_stream(ctx, s, field_dev);
    });
    if (st != IPC_OK) return st;
    if (bad) {
      set_err(ctx, "verification: " + std::to_string(bad) + " points miss the error bound");
      return IPC_ECORRUPT;
    }
  }
  if (opts->lossless == IPC_LOSSLESS_CODED) return ipc_stream_entropy_code(ctx, s);
  return IPC_OK;
}

uint64_t plane_bytes_between(const ipc_stream *s, const std::vector<int> &lo,
                             const std::vector<int> &hi) {
  uint64_t tot = 0;
  for (size_t p = 0; p < lo.size(); ++p)
    for (int k = lo[p]; k < hi[p]; ++k) tot += uint64_t(s->tables.sizes[p * 32 + k]);
  return tot;
}

// Schedule, metadata, pass table and device buffers of a new stream
void setup_stream(ipc_ctx *ctx, ipc_stream *s, const uint64_t *dims, int ndim, int dtype, int interp,
                  double abs_eb, const ipc_options *opts) {
  int64_t d64[3];
  for (int j = 0; j < ndim; ++j) d64[j] = int64_t(dims[j]);
  int cl[3] = {0, 0, 0};
  if (opts)
    for (int j = 0; j < ndim; ++j) cl[j] = opts->chunk_log2[j];
  StreamMeta &m = s->meta;
  std::string e;
  if (!make_schedule(d64, ndim, cl, m.sched, e)) {
    set_err(ctx, e);
    throw Fail{IPC_EINVAL};
  }
  if (!chunks_supported(m.sched, e)) {
    set_err(ctx, e);
    throw Fail{IPC_EUNSUPPORTED};
  }
  int np = opts ? opts->nonprog_levels : 0;
  if (np < 0 || np > m.sched.K) {
    set_err(ctx, "nonprog_levels out of range");
    throw Fail{IPC_EINVAL};
  }
  if (opts && (opts->errq_mode > IPC_ERRQ_BOUND || opts->lossless > IPC_LOSSLESS_CODED ||
               (opts->debug_flags & ~(IPC_DEBUG_PER_PASS | IPC_DEBUG_VERIFY)) != 0)) {
    set_err(ctx, "unknown errq_mode, lossless mode or debug flag");
    throw Fail{IPC_EINVAL};
  }
  m.dtype = dtype;
  m.interp = interp;
  m.nonprog_levels = np;
  m.eb = abs_eb;
  m.qmax = dtype == IPC_F32 ? QMAX_F32 : QMAX_F64;
  const Schedule &sc = m.sched;
  for (const PassGeom &p : sc.passes) s->args.push_back(make_args(sc, p));
  s->payload = dev_alloc(ctx, size_t(sc.slot_words) * 4);
  s->masks = dev_alloc(ctx, size_t(sc.n_chunks) * 4);
}

// Metadata of a compressed stream from its summary block: n_out, maxabs bits,
// sizes [P][32] u64, errq [P][33] u32
void finish_stream(ipc_stream *s, const char *hostp, uint64_t nout) {
  StreamMeta &m = s->meta;
  const int P = int(m.sched.passes.size());
  uint64_t mb;
  std::memcpy(&mb, hostp + 8, 8);
  std::memcpy(&m.maxabs, &mb, 8);
  m.errq.resize(size_t(P) * 33);
  std::memcpy(m.errq.data(), hostp + 16 + size_t(P) * 32 * 8, m.errq.size() * 4);
  std::vector<uint64_t> sz(size_t(P) * 32);
  std::memcpy(sz.data(), hostp + 16, sz.size() * 8);
  m.outliers.clear();
  m.n_outliers = nout;
  s->host_outliers_valid = nout == 0;
  uint64_t words = 0;
  for (uint64_t v : sz) words += v / 4;
  m.payload_words = words;
  m.serialized_bytes = serialized_size(m);
  // planner tables from the device-computed plane sizes (no mask copy needed)
  s->tables = plan_tables_from_sizes(m, sz);
}

size_t summary_bytes(int P) { return 16 + size_t(P) * 32 * 8 + size_t(P) * 33 * 4; }

// Thm. 1's delta-y as a table fixed before compression: the largest change
// that discarding b negabinary digits can make to any code, which is Sec.
// 4.4.2's truncation uncertainty floor((2^(b+1) - 1) / 3), for every pass
void errq_to_bound(ipc_stream *s) {
  StreamMeta &m = s->meta;
  const size_t P = m.sched.passes.size();
  m.errq.assign(P * 33, 0u);
  for (size_t p = 0; p < P; ++p)
    for (int b = 0; b <= 32; ++b) m.errq[p * 33 + size_t(b)] = uint32_t(((uint64_t(1) << (b + 1)) - 1) / 3);
  s->tables.errq = m.errq;
}

// points of a full-precision reconstruction of `s` that miss the bound
uint64_t verify_stream(ipc_ctx *ctx, const ipc_stream *s, const void *field_dev);


// ---------------------------------------------------------------- batches

// Whether a field of these dims (and options) would take the fused level path
bool fused_dims(const uint64_t *dims, int ndim, const ipc_options *opts) {
  if (ndim != 2 && ndim != 3) return false;
  if (opts && (opts->debug_flags & IPC_DEBUG_PER_PASS)) return false;
  int64_t d64[3] = {0, 0, 0};
  int cl[3] = {0, 0, 0};
  for (int j = 0; j < ndim; ++j) {
    d64[j] = int64_t(dims[j]);
    if (opts) cl[j] = int(opts->chunk_log2[j]);
  }
  Schedule sc;
  std::string e;
  return make_schedule(d64, ndim, cl, sc, e) && fused3(sc);
}

// Compression of n fused 3-D fields with one launch per level over all of
// them (the levels of a field with fewer levels are skipped).  Each field
// keeps its own summary, outlier records, coarse grids and rows.  Fields
// whose outliers overflow their record capacity are flagged in `redo`.
template <typename T>
void compress_batch_fused(ipc_ctx *ctx, std::vector<ipc_stream *> &ss,
                          const void *const *fields, const double *ebs, std::vector<char> &redo) {
  const int n = int(ss.size());
  const int dtype = ss[0]->meta.dtype, interp = ss[0]->meta.interp;
  const size_t isz = sizeof(T);
  // per-field summary blocks and record ranges
  std::vector<size_t> sum_off(n + 1, 0), rec_off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const Schedule &sc = ss[i]->meta.sched;
    sum_off[i + 1] = sum_off[i] + ((summary_bytes(int(sc.passes.size())) + 255) & ~size_t(255));
    rec_off[i + 1] = rec_off[i] + std::max<size_t>(4096, size_t(sc.n_points / 1024));
  }
  char *summary = static_cast<char *>(ensure_ws(ctx, ctx->ws_summary, ctx->ws_summary_bytes, sum_off[n]));
  ensure_ws(ctx, ctx->ws_out, ctx->ws_out_cap, rec_off[n] * sizeof(OutlierRec));
  hip_check(ctx, hipMemsetAsync(summary, 0, sum_off[n], ctx->stream), "memset");
  // pass tables of all fields (the outlier index reads them)
  std::vector<PassArgs> args;
  std::vector<size_t> args_off(n);
  for (int i = 0; i < n; ++i) {
    args_off[i] = args.size();
    args.insert(args.end(), ss[i]->args.begin(), ss[i]->args.end());
  }
  DevBuf args_dev = dev_alloc(ctx, args.size() * sizeof(PassArgs));
  hip_check(ctx, hipMemcpyAsync(args_dev.p, args.data(), args.size() * sizeof(PassArgs),
                                hipMemcpyHostToDevice, ctx->stream), "upload");
  // coarse grids, two per field
  std::vector<DevBuf> g(2 * n);
  std::vector<CompressOut> o(n);
  int Kmax = 0;
  for (int i = 0; i < n; ++i) {
    const Schedule &sc = ss[i]->meta.sched;
    Kmax = std::max(Kmax, sc.K);
    size_t need[2] = {8, 8};
    for (int j = 1; j <= sc.K; ++j)
      need[j & 1] = std::max(need[j & 1], size_t(coarse_points(sc, j)) * isz);
    g[2 * i] = dev_alloc(ctx, need[0]);
    g[2 * i + 1] = dev_alloc(ctx, need[1]);
    char *sm = summary + sum_off[i];
    const int P = int(sc.passes.size());
    o[i].payload = static_cast<uint32_t *>(ss[i]->payload.p);
    o[i].masks = static_cast<uint32_t *>(ss[i]->masks.p);
    o[i].n_out = reinterpret_cast<unsigned long long *>(sm);
    o[i].maxabs_bits = reinterpret_cast<unsigned long long *>(sm + 8);
    o[i].sizes = reinterpret_cast<unsigned long long *>(sm + 16);
    o[i].errq = reinterpret_cast<uint32_t *>(sm + 16 + size_t(P) * 32 * 8);
    o[i].out_recs = static_cast<OutlierRec *>(ctx->ws_out) + rec_off[i];
    o[i].out_cap = rec_off[i + 1] - rec_off[i];
  }
  // the work lists of the level launches and every field's rows
  std::vector<BatchC<T>> ent;
  struct Launch { size_t off; int nf; uint32_t items; };
  std::vector<Launch> launches;
  std::vector<LevelRows> lr(n);
  for (LevelRows &r : lr) std::memset(&r, 0, sizeof(r));
  uint32_t rows = 0;
  for (int l = Kmax; l >= 1; --l) {
    Launch ln{ent.size(), 0, 0};
    for (int i = 0; i < n; ++i) {
      const Schedule &sc = ss[i]->meta.sched;
      if (l > sc.K) continue;
      Level3Args La = level_args(ctx, ss[i]->meta, l, true);
      La.row_base = rows;
      const uint32_t items = uint32_t(level3_wgs(La));
      LevelRows &r = lr[i];
      if (r.n >= MAX_LEVEL_LAUNCHES) {
        set_err(ctx, "too many levels for the fused kernels");
        throw Fail{IPC_EUNSUPPORTED};
      }
      r.row_base[r.n] = rows;
      r.n_rows[r.n] = items;
      for (int p = 0; p < 3; ++p) r.pass_index[r.n][p] = La.pass_index[p];
      ++r.n;
      rows += items;
      BatchC<T> e;
      std::memset(&e, 0, sizeof(e));
      e.L = La;
      e.x = static_cast<const T *>(fields[i]);
      e.gin = static_cast<const T *>(g[2 * i + (l & 1)].p);
      e.gout = l > 1 ? static_cast<T *>(g[2 * i + ((l - 1) & 1)].p) : nullptr;
      e.o = o[i];
      e.eb = ebs[i];
      e.two_eb = T(2.0 * ebs[i]);
      e.inv = T(1.0 / (2.0 * ebs[i]));
      e.qmax = T(sizeof(T) == 4 ? QMAX_F32 : QMAX_F64);
      e.item0 = ln.items;
      ent.push_back(e);
      ++ln.nf;
      ln.items += items;
    }
    launches.push_back(ln);
  }
  uint32_t *rows_p = static_cast<uint32_t *>(
      ensure_ws(ctx, ctx->ws_rows, ctx->ws_rows_bytes, size_t(rows) * WG_ROW * 4));
  for (BatchC<T> &e : ent) e.o.wg_rows = rows_p;
  for (int i = 0; i < n; ++i) o[i].wg_rows = rows_p;
  // one upload: the anchor jobs as a head table, the level work lists, and
  // the row-reduction jobs of every field's level launches
  std::vector<RowsJob> jobs;
  uint32_t most_rows = 0;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < lr[i].n; ++k) {
      RowsJob j;
      std::memset(&j, 0, sizeof(j));
      j.row_base = lr[i].row_base[k];
      j.n_rows = lr[i].n_rows[k];
      for (int p = 0; p < 3; ++p) j.pass_index[p] = lr[i].pass_index[k][p];
      j.errq = o[i].errq;
      j.maxabs_bits = o[i].maxabs_bits;
      j.sizes = o[i].sizes;
      most_rows = std::max(most_rows, j.n_rows);
      jobs.push_back(j);
    }
  const size_t heads_off = (sizeof(QueueTable) + 255) & ~size_t(255);
  const size_t ent_off = heads_off + ((size_t(n) * sizeof(HeadC<T>) + 255) & ~size_t(255));
  const size_t jobs_off = ent_off + ((ent.size() * sizeof(BatchC<T>) + 255) & ~size_t(255));
  std::vector<char> up(jobs_off + jobs.size() * sizeof(RowsJob), 0);
  QueueTable &tab = *reinterpret_cast<QueueTable *>(up.data());
  tab.n_heads = uint32_t(n);
  tab.heads_off = uint32_t(heads_off);
  tab.ent_off = uint32_t(ent_off);
  for (int i = 0; i < n; ++i) {
    HeadC<T> &h = reinterpret_cast<HeadC<T> *>(up.data() + heads_off)[i];
    const Schedule &sc = ss[i]->meta.sched;
    h.A = anchor3_args(sc);
    h.x = static_cast<const T *>(fields[i]);
    h.g = static_cast<T *>(g[2 * i + (sc.K & 1)].p);
    h.o = o[i];
    h.eb = ebs[i];
    h.two_eb = T(2.0 * ebs[i]);
    h.inv = T(1.0 / (2.0 * ebs[i]));
    h.qmax = T(sizeof(T) == 4 ? QMAX_F32 : QMAX_F64);
  }
  std::memcpy(up.data() + ent_off, ent.data(), ent.size() * sizeof(BatchC<T>));
  std::memcpy(up.data() + jobs_off, jobs.data(), jobs.size() * sizeof(RowsJob));
  DevBuf up_dev = dev_alloc(ctx, up.size());
  hip_check(ctx, hipMemcpyAsync(up_dev.p, up.data(), up.size(), hipMemcpyHostToDevice, ctx->stream), "upload");
  const QueueTable *tab_dev = static_cast<const QueueTable *>(up_dev.p);
  const BatchC<T> *ent_dev = reinterpret_cast<const BatchC<T> *>(static_cast<const char *>(up_dev.p) + ent_off);
  hip_check(ctx, launch_heads_compress(dtype, tab_dev, ctx->stream), "anchor kernel launch");
  for (const Launch &ln : launches)
    hip_check(ctx, launch_level3_compress_batch(dtype, interp, ent_dev + ln.off, ln.nf, ln.items, ctx->stream),
              "level kernel launch");
  hip_check(ctx, launch_rows_reduce_batch(
                     reinterpret_cast<const RowsJob *>(static_cast<const char *>(up_dev.p) + jobs_off),
                     uint32_t(jobs.size()), most_rows, rows_p, ctx->stream),
            "row reduction launch");
  if (ctx->host_summary_bytes < sum_off[n]) {
    if (ctx->host_summary) (void)hipHostFree(ctx->host_summary);
    ctx->host_summary = nullptr;
    ctx->host_summary_bytes = 0;
    hip_check(ctx, hipHostMalloc(&ctx->host_summary, sum_off[n], hipHostMallocDefault), "pinned alloc");
    ctx->host_summary_bytes = sum_off[n];
  }
  char *hostp = static_cast<char *>(ctx->host_summary);
  hip_check(ctx, hipMemcpyAsync(hostp, summary, sum_off[n], hipMemcpyDeviceToHost, ctx->stream), "copy");
  hip_check(ctx, hipStreamSynchronize(ctx->stream), "compress");
  for (int i = 0; i < n; ++i) {
    uint64_t nout;
    std::memcpy(&nout, hostp + sum_off[i], 8);
    if (nout > o[i].out_cap) {
      redo[i] = 1;
      continue;
    }
    finish_stream(ss[i], hostp + sum_off[i], nout);
    // the outlier index, sorted on the device, for the fields that have
    // outliers (a stream without any has no table); queued behind the
    // call's work and read only by later work on the same stream
    if (nout == 0) continue;
    ipc_stream *s = ss[i];
    const uint64_t nc = uint64_t(s->meta.sched.n_chunks);
    s->out_gchunk = dev_alloc(ctx, 8 * nout);
    s->out_local = dev_alloc(ctx, 4 * nout);
    s->out_bits = dev_alloc(ctx, 8 * nout);
    s->out_start = dev_alloc(ctx, 4 * (nc + 1));
    const size_t nb = (nc + 1 + 1023) / 1024;
    uint32_t *cnt = static_cast<uint32_t *>(
        ensure_ws(ctx, ctx->ws_cnt, ctx->ws_cnt_bytes, 4 * (nc + 1) + 4 * (nb + 1)));
    hip_check(ctx, launch_outlier_index_n(static_cast<const OutlierRec *>(o[i].out_recs), nout, o[i].n_out,
                                        static_cast<const PassArgs *>(args_dev.p) + args_off[i], nc,
                                        static_cast<uint32_t *>(s->out_start.p), cnt, cnt + (nc + 1),
                                        static_cast<uint64_t *>(s->out_gchunk.p),
                                        static_cast<uint32_t *>(s->out_local.p),
                                        static_cast<uint64_t *>(s->out_bits.p), ctx->stream),
              "outlier index launch");
  }
  dev_free(ctx, up_dev);
  dev_free(ctx, args_dev);
  for (DevBuf &b : g) dev_free(ctx, b);
}

// Retrieval of n fused 3-D streams (same dtype and interpolation) with one
// launch per level over all of them; plans given, fields allocated by the
// caller of this helper.
template <typename T>
void retrieve_batch_fused(ipc_ctx *ctx, const std::vector<const ipc_stream *> &ss,
                          const std::vector<std::vector<int>> &plans, const std::vector<void *> &out,
                          const std::vector<int> &l_start) {
  const int n = int(ss.size());
  const int dtype = ss[0]->meta.dtype, interp = ss[0]->meta.interp;
  const size_t isz = sizeof(T);
  std::vector<DevBuf> g(2 * n);
  std::vector<RetrieveIn> in(n);
  int Kmax = 0;
  for (int i = 0; i < n; ++i) {
    const ipc_stream *s = ss[i];
    const Schedule &sc = s->meta.sched;
    Kmax = std::max(Kmax, sc.K);
    size_t need[2] = {8, 8};
    for (int j = 1; j <= sc.K; ++j)
      need[j & 1] = std::max(need[j & 1], size_t(coarse_points(sc, j)) * isz);
    g[2 * i] = dev_alloc(ctx, need[0]);
    g[2 * i + 1] = dev_alloc(ctx, need[1]);
    RetrieveIn &r = in[i];
    r.payload = static_cast<const uint32_t *>(s->payload.p);
    r.masks = static_cast<const uint32_t *>(s->masks.p);
    r.chunk_off = s->packed ? static_cast<const uint64_t *>(s->chunk_off.p) : nullptr;
    r.out_gchunk = static_cast<const uint64_t *>(s->out_gchunk.p);
    r.out_local = static_cast<const uint32_t *>(s->out_local.p);
    r.out_bits = static_cast<const uint64_t *>(s->out_bits.p);
    r.out_start = static_cast<const uint32_t *>(s->out_start.p);
    r.n_out = s->meta.n_outliers;
    r.zero = static_cast<const uint32_t *>(ctx->dev_zero);
  }
  std::vector<BatchR<T>> ent;
  struct Launch { size_t off; int nf; uint32_t items; };
  std::vector<Launch> launches;
  for (int l = Kmax; l >= 1; --l) {
    Launch ln{ent.size(), 0, 0};
    for (int i = 0; i < n; ++i) {
      if (l > l_start[i]) continue;
      Level3Args La = level_args(ctx, ss[i]->meta, l, false);
      BatchR<T> e;
      std::memset(&e, 0, sizeof(e));
      e.L = La;
      e.gin = static_cast<const T *>(g[2 * i + (l & 1)].p);
      e.gout = l > 1 ? static_cast<T *>(g[2 * i + ((l - 1) & 1)].p) : static_cast<T *>(out[i]);
      e.in = in[i];
      for (int p = 0; p < 3; ++p) e.disc[p] = plans[i][La.pass_index[p]];
      e.two_eb = T(2.0 * ss[i]->meta.eb);
      e.item0 = ln.items;
      ent.push_back(e);
      ++ln.nf;
      ln.items += uint32_t(level3_wgs(La));
    }
    launches.push_back(ln);
  }
  // one upload: the head jobs (anchors, or a refinement's coarse grid
  // gathered from the resident field) as a head table, then the work lists;
  // one launch runs every head job
  const size_t heads_off = (sizeof(QueueTable) + 255) & ~size_t(255);
  const size_t ent_off = heads_off + ((size_t(n) * sizeof(HeadR<T>) + 255) & ~size_t(255));
  std::vector<char> up(ent_off + ent.size() * sizeof(BatchR<T>), 0);
  QueueTable &tab = *reinterpret_cast<QueueTable *>(up.data());
  tab.n_heads = uint32_t(n);
  tab.heads_off = uint32_t(heads_off);
  tab.ent_off = uint32_t(ent_off);
  for (int i = 0; i < n; ++i) {
    HeadR<T> &h = reinterpret_cast<HeadR<T> *>(up.data() + heads_off)[i];
    const Schedule &sc = ss[i]->meta.sched;
    const int ls = l_start[i];
    h.in = in[i];
    h.two_eb = T(2.0 * ss[i]->meta.eb);
    h.g = static_cast<T *>(g[2 * i + (ls & 1)].p);
    if (ls >= sc.K) {
      h.mode = 0;
      h.A = anchor3_args(sc);
    } else {
      h.mode = 1;
      h.field = static_cast<const T *>(out[i]);
      for (int j = 0; j < 3; ++j) {
        h.fd[j] = sc.dims3[j];
        h.gd[j] = ((sc.dims3[j] - 1) >> ls) + 1;
      }
      h.step = int64_t(1) << ls;
    }
  }
  std::memcpy(up.data() + ent_off, ent.data(), ent.size() * sizeof(BatchR<T>));
  DevBuf up_dev = dev_alloc(ctx, up.size());
  hip_check(ctx, hipMemcpyAsync(up_dev.p, up.data(), up.size(), hipMemcpyHostToDevice, ctx->stream), "upload");
  const BatchR<T> *ent_dev = reinterpret_cast<const BatchR<T> *>(static_cast<const char *>(up_dev.p) + ent_off);
  hip_check(ctx, launch_heads_retrieve(dtype, static_cast<const QueueTable *>(up_dev.p), ctx->stream),
            "head launch");
  for (const Launch &ln : launches)
    hip_check(ctx, launch_level3_retrieve_batch(dtype, interp, ent_dev + ln.off, ln.nf, ln.items, ctx->stream),
              "level kernel launch");
  hip_check(ctx, hipStreamSynchronize(ctx->stream), "retrieve");
  dev_free(ctx, up_dev);
  for (DevBuf &b : g) dev_free(ctx, b);
}

// ------------------------------------------------------- graph-replayed batches
//
// A batched retrieval of fused 3-D streams as queue launches: the head jobs
// (anchors, or coarse grids gathered for refinements) and one persistent
// launch per level slot, reading everything batch-specific from a table in
// device memory.  The launch sequence then depends only on the launch shape
// (dtype, interpolation, number of level slots and the grid class of each),
// so it is captured once into a HIP graph and replayed for every later batch
// of the same shape: a replay is one table upload and one graph launch.

constexpr size_t Q_HEADS = 2048;    // fields per queue batch
constexpr size_t Q_ENTRIES = 16384; // level work-list entries per queue batch
constexpr size_t Q_CLAIMS = 256;    // bytes of claim counters before the table
constexpr size_t Q_GRAPHS = 64;     // cached graphs (the cache is cleared beyond)

size_t queue_table_bytes() {
  const size_t h = std::max({sizeof(HeadR<float>), sizeof(HeadR<double>), sizeof(HeadC<float>),
                             sizeof(HeadC<double>)});
  const size_t e = std::max({sizeof(BatchR<float>), sizeof(BatchR<double>), sizeof(BatchC<float>),
                             sizeof(BatchC<double>)});
  // + 256: the entries start at the next 256-byte boundary after the heads
  return ((sizeof(QueueTable) + 255) & ~size_t(255)) + Q_HEADS * h + 256 + Q_ENTRIES * e;
}

// persistent grid of a level slot: a class of its item count
uint32_t queue_grid(const ipc_ctx *ctx, uint32_t items, size_t isz) {
  const uint32_t full = uint32_t(ctx->n_cu) * (ctx->per_cu_r ? ctx->per_cu_r : (isz == 4 ? 5u : 4u));
  if (items <= 16) return 16;
  if (items <= 128) return 128;
  return full;
}

// ... and of a compression slot (its kernel runs 4 workgroups per CU in
// float32, 2 in float64)
uint32_t queue_grid_c(const ipc_ctx *ctx, uint32_t items, size_t isz) {
  if (items <= 16) return 16;
  if (items <= 128) return 128;
  return uint32_t(ctx->n_cu) * (ctx->per_cu_c ? ctx->per_cu_c : (isz == 4 ? 4u : 2u));
}

// Fields above this many points make a batch run as direct launches in the
// automatic mode when the autotuner has no choice for it: there the launch
// overhead a replay saves is small against the work, and the persistent grid's
// claiming costs more (two 512^3 fields: 0.59 ms per field replayed, 0.52 ms
// direct; eight 256x384x384 float64 fields: 1.93 against 1.85 ms).
constexpr int64_t AUTO_GRAPH_POINTS = int64_t(1) << 22;

TuneKey tune_key(const StreamMeta &m) {
  return TuneKey{{m.sched.dims3[0], m.sched.dims3[1], m.sched.dims3[2]}, m.dtype, m.interp};
}

// whether a batch runs as graph replays, and the full-slot grid it uses
// (set in ctx->per_cu_* for the call)
bool batch_wants_graphs(ipc_ctx *ctx, const std::vector<const ipc_stream *> &ss, bool compress) {
  ctx->per_cu_r = ctx->per_cu_c = 0;
  if (ctx->batch_graphs == 0) return false;
  if (ctx->batch_graphs == 1) return true;
  // automatic: the autotuner's choice when every field of the batch has the
  // same tuned shape, else by the largest field
  const auto it = ctx->tuned_batch.find(tune_key(ss[0]->meta));
  bool same = it != ctx->tuned_batch.end();
  for (const ipc_stream *s : ss) same = same && !(tune_key(s->meta) < it->first) && !(it->first < tune_key(s->meta));
  if (same) {
    const BatchTune &b = it->second;
    ctx->per_cu_r = b.per_cu_r;
    ctx->per_cu_c = b.per_cu_c;
    return compress ? b.graphs_c != 0 : b.graphs_r != 0;
  }
  int64_t most = 0;
  for (const ipc_stream *s : ss) most = std::max(most, s->meta.sched.n_points);
  return most <= AUTO_GRAPH_POINTS;
}

bool queue_fits(const std::vector<const ipc_stream *> &ss) {
  if (ss.size() > Q_HEADS) return false;
  size_t ent = 0;
  int Kmax = 0;
  for (const ipc_stream *s : ss) {
    ent += size_t(s->meta.sched.K);
    Kmax = std::max(Kmax, s->meta.sched.K);
  }
  return ent <= Q_ENTRIES && Kmax <= QUEUE_LEVELS;
}

// false when the context's stream cannot be captured into a graph (nothing
// has run then but the table upload)
template <typename T>
bool retrieve_batch_queue(ipc_ctx *ctx, const std::vector<const ipc_stream *> &ss,
                          const std::vector<std::vector<int>> &plans, const std::vector<void *> &out,
                          const std::vector<int> &l_start) {
  const int n = int(ss.size());
  const int dtype = ss[0]->meta.dtype, interp = ss[0]->meta.interp;
  const size_t isz = sizeof(T);
  if (!ctx->ws_q) {
    ctx->ws_q_bytes = Q_CLAIMS + queue_table_bytes();
    hip_check(ctx, hipMalloc(&ctx->ws_q, ctx->ws_q_bytes), "queue table allocation");
    hip_check(ctx, hipHostMalloc(&ctx->host_q, queue_table_bytes(), hipHostMallocDefault),
              "pinned allocation");
  }
  uint32_t *claims = static_cast<uint32_t *>(ctx->ws_q);
  QueueTable *tab_dev = reinterpret_cast<QueueTable *>(static_cast<char *>(ctx->ws_q) + Q_CLAIMS);
  char *host = static_cast<char *>(ctx->host_q);
  QueueTable &tab = *reinterpret_cast<QueueTable *>(host);
  std::memset(&tab, 0, sizeof(tab));
  tab.n_heads = uint32_t(n);
  tab.heads_off = uint32_t((sizeof(QueueTable) + 255) & ~size_t(255));
  HeadR<T> *heads = reinterpret_cast<HeadR<T> *>(host + tab.heads_off);
  tab.ent_off = uint32_t(tab.heads_off + ((size_t(n) * sizeof(HeadR<T>) + 255) & ~size_t(255)));
  BatchR<T> *ent = reinterpret_cast<BatchR<T> *>(host + tab.ent_off);

  std::vector<DevBuf> g(2 * n);
  // the coarse grids go back to the cache once the stream has drained (also
  // when a step below fails after work was queued)
  struct Release {
    ipc_ctx *ctx;
    std::vector<DevBuf> &g;
    ~Release() {
      (void)hipStreamSynchronize(ctx->stream);
      for (DevBuf &b : g) dev_free(ctx, b);
    }
  } release{ctx, g};
  int Kmax = 0;
  for (int i = 0; i < n; ++i) {
    const ipc_stream *s = ss[i];
    const Schedule &sc = s->meta.sched;
    Kmax = std::max(Kmax, sc.K);
    size_t need[2] = {8, 8};
    for (int j = 1; j <= sc.K; ++j)
      need[j & 1] = std::max(need[j & 1], size_t(coarse_points(sc, j)) * isz);
    g[2 * i] = dev_alloc(ctx, need[0]);
    g[2 * i + 1] = dev_alloc(ctx, need[1]);
    HeadR<T> &h = heads[i];
    std::memset(&h, 0, sizeof(h));
    h.in = retrieve_in(ctx, s);
    h.two_eb = T(2.0 * s->meta.eb);
    const int ls = l_start[i];
    h.g = static_cast<T *>(g[2 * i + (ls & 1)].p);
    if (ls >= sc.K) {
      h.mode = 0;
      h.A = anchor3_args(sc);
    } else {
      h.mode = 1;
      h.field = static_cast<const T *>(out[i]);
      for (int j = 0; j < 3; ++j) {
        h.fd[j] = sc.dims3[j];
        h.gd[j] = ((sc.dims3[j] - 1) >> ls) + 1;
      }
      h.step = int64_t(1) << ls;
    }
  }
  std::vector<int> key = {dtype, interp, Kmax};
  size_t m = 0;
  for (int slot = 0; slot < Kmax; ++slot) {
    const int l = Kmax - slot;
    QueueLevel &q = tab.lev[slot];
    q.off = uint32_t(m);
    for (int i = 0; i < n; ++i) {
      if (l > l_start[i]) continue;
      Level3Args La = level_args(ctx, ss[i]->meta, l, false);
      BatchR<T> &e = ent[m++];
      std::memset(&e, 0, sizeof(e));
      e.L = La;
      e.gin = static_cast<const T *>(g[2 * i + (l & 1)].p);
      e.gout = l > 1 ? static_cast<T *>(g[2 * i + ((l - 1) & 1)].p) : static_cast<T *>(out[i]);
      e.in = heads[i].in;
      for (int p = 0; p < 3; ++p) e.disc[p] = plans[i][La.pass_index[p]];
      e.two_eb = heads[i].two_eb;
      e.item0 = q.items;
      ++q.nf;
      q.items += uint32_t(level3_wgs(La));
    }
    key.push_back(int(queue_grid(ctx, q.items, isz)));
  }
  const size_t bytes = tab.ent_off + m * sizeof(BatchR<T>);
  hip_check(ctx, hipMemcpyAsync(tab_dev, host, bytes, hipMemcpyHostToDevice, ctx->stream), "upload");

  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (ctx->graphs.size() >= Q_GRAPHS) {
      for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
      ctx->graphs.clear();
    }
    if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    hipError_t e = launch_queue_reset(claims, ctx->stream);
    if (e == hipSuccess) e = launch_heads_retrieve(dtype, tab_dev, ctx->stream);
    for (int slot = 0; slot < Kmax && e == hipSuccess; ++slot)
      e = launch_level3_retrieve_queue(dtype, interp, tab_dev, slot, claims, uint32_t(key[3 + slot]),
                                       ctx->stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
    if ((e != hipSuccess || ec != hipSuccess) && graph) (void)hipGraphDestroy(graph);
    hip_check(ctx, e, "queue launch capture");
    hip_check(ctx, ec, "end capture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(ctx, ei, "graph instantiate");
    it = ctx->graphs.emplace(key, exec).first;
    ++ctx->graphs_captured;
  }
  hip_check(ctx, hipGraphLaunch(it->second, ctx->stream), "graph launch");
  ++ctx->graph_replays;
  // the coarse grids and the staged table are reused by the next call
  hip_check(ctx, hipStreamSynchronize(ctx->stream), "retrieve");
  return true;
}

// batched retrieval of fused 3-D streams: queue launches from a captured
// graph when the context asks for them and the batch fits the table, else one
// direct launch per level
template <typename T>
void retrieve_batch_levels(ipc_ctx *ctx, const std::vector<const ipc_stream *> &ss,
                           const std::vector<std::vector<int>> &plans, const std::vector<void *> &out,
                           const std::vector<int> &l_start) {
  if (batch_wants_graphs(ctx, ss, false) && queue_fits(ss)) {
    if (retrieve_batch_queue<T>(ctx, ss, plans, out, l_start)) return;
    ctx->batch_graphs = 0;  // this stream cannot be captured: direct launches from now on
  }
  retrieve_batch_fused<T>(ctx, ss, plans, out, l_start);
}

// Batched compression of fused 3-D fields as queue launches replayed from a
// captured graph: one persistent launch per level slot whose workgroups claim
// (field, column segment) items from a device counter, the anchors of every
// field in one launch before them.  Everything a batch varies in (fields,
// outputs, bounds, work lists) sits in the device table, so the graph depends
// only on dtype, interpolation, level count and the grid classes.  The
// per-field row reductions, outlier indexes and the summary copy follow as
// direct launches.  Returns false (nothing launched but the table upload)
// when the context's stream cannot be captured.
template <typename T>
bool compress_batch_queue(ipc_ctx *ctx, std::vector<ipc_stream *> &ss, const void *const *fields,
                          const double *ebs, std::vector<char> &redo) {
  const int n = int(ss.size());
  const int dtype = ss[0]->meta.dtype, interp = ss[0]->meta.interp;
  const size_t isz = sizeof(T);
  if (!ctx->ws_q) {
    ctx->ws_q_bytes = Q_CLAIMS + queue_table_bytes();
    hip_check(ctx, hipMalloc(&ctx->ws_q, ctx->ws_q_bytes), "queue table allocation");
    hip_check(ctx, hipHostMalloc(&ctx->host_q, queue_table_bytes(), hipHostMallocDefault),
              "pinned allocation");
  }
  uint32_t *claims = static_cast<uint32_t *>(ctx->ws_q);
  QueueTable *tab_dev = reinterpret_cast<QueueTable *>(static_cast<char *>(ctx->ws_q) + Q_CLAIMS);
  char *host = static_cast<char *>(ctx->host_q);
  // the previous call's table upload has completed (its call synchronized)
  QueueTable &tab = *reinterpret_cast<QueueTable *>(host);
  std::memset(&tab, 0, sizeof(tab));
  tab.n_heads = uint32_t(n);
  tab.heads_off = uint32_t((sizeof(QueueTable) + 255) & ~size_t(255));
  HeadC<T> *heads = reinterpret_cast<HeadC<T> *>(host + tab.heads_off);
  tab.ent_off = uint32_t(tab.heads_off + ((size_t(n) * sizeof(HeadC<T>) + 255) & ~size_t(255)));
  BatchC<T> *ent = reinterpret_cast<BatchC<T> *>(host + tab.ent_off);

  // per-field summary blocks and record ranges (as compress_batch_fused)
  std::vector<size_t> sum_off(n + 1, 0), rec_off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const Schedule &sc = ss[i]->meta.sched;
    sum_off[i + 1] = sum_off[i] + ((summary_bytes(int(sc.passes.size())) + 255) & ~size_t(255));
    rec_off[i + 1] = rec_off[i] + std::max<size_t>(4096, size_t(sc.n_points / 1024));
  }
  char *summary = static_cast<char *>(ensure_ws(ctx, ctx->ws_summary, ctx->ws_summary_bytes, sum_off[n]));
  ensure_ws(ctx, ctx->ws_out, ctx->ws_out_cap, rec_off[n] * sizeof(OutlierRec));
  std::vector<PassArgs> args;
  std::vector<size_t> args_off(n);
  for (int i = 0; i < n; ++i) {
    args_off[i] = args.size();
    args.insert(args.end(), ss[i]->args.begin(), ss[i]->args.end());
  }
  DevBuf args_dev = dev_alloc(ctx, args.size() * sizeof(PassArgs));
  std::vector<DevBuf> g(2 * n);
  struct Release {
    ipc_ctx *ctx;
    std::vector<DevBuf> &g;
    DevBuf &args_dev;
    ~Release() {
      (void)hipStreamSynchronize(ctx->stream);
      for (DevBuf &b : g) dev_free(ctx, b);
      dev_free(ctx, args_dev);
    }
  } release{ctx, g, args_dev};
  hip_check(ctx, hipMemcpyAsync(args_dev.p, args.data(), args.size() * sizeof(PassArgs),
                                hipMemcpyHostToDevice, ctx->stream), "upload");
  hip_check(ctx, hipMemsetAsync(summary, 0, sum_off[n], ctx->stream), "memset");
  std::vector<CompressOut> o(n);
  int Kmax = 0;
  for (int i = 0; i < n; ++i) {
    const Schedule &sc = ss[i]->meta.sched;
    Kmax = std::max(Kmax, sc.K);
    size_t need[2] = {8, 8};
    for (int j = 1; j <= sc.K; ++j)
      need[j & 1] = std::max(need[j & 1], size_t(coarse_points(sc, j)) * isz);
    g[2 * i] = dev_alloc(ctx, need[0]);
    g[2 * i + 1] = dev_alloc(ctx, need[1]);
    char *sm = summary + sum_off[i];
    const int P = int(sc.passes.size());
    o[i].payload = static_cast<uint32_t *>(ss[i]->payload.p);
    o[i].masks = static_cast<uint32_t *>(ss[i]->masks.p);
    o[i].n_out = reinterpret_cast<unsigned long long *>(sm);
    o[i].maxabs_bits = reinterpret_cast<unsigned long long *>(sm + 8);
    o[i].sizes = reinterpret_cast<unsigned long long *>(sm + 16);
    o[i].errq = reinterpret_cast<uint32_t *>(sm + 16 + size_t(P) * 32 * 8);
    o[i].out_recs = static_cast<OutlierRec *>(ctx->ws_out) + rec_off[i];
    o[i].out_cap = rec_off[i + 1] - rec_off[i];
  }
  // level slots (level Kmax - slot) and every field's rows
  std::vector<LevelRows> lr(n);
  for (LevelRows &r : lr) std::memset(&r, 0, sizeof(r));
  uint32_t rows = 0;
  size_t m = 0;
  std::vector<int> key = {dtype + 16, interp, Kmax};  // 16 + dtype: compression graphs
  for (int slot = 0; slot < Kmax; ++slot) {
    const int l = Kmax - slot;
    QueueLevel &q = tab.lev[slot];
    q.off = uint32_t(m);
    for (int i = 0; i < n; ++i) {
      const Schedule &sc = ss[i]->meta.sched;
      if (l > sc.K) continue;
      Level3Args La = level_args(ctx, ss[i]->meta, l, true);
      La.row_base = rows;
      const uint32_t items = uint32_t(level3_wgs(La));
      LevelRows &r = lr[i];
      if (r.n >= MAX_LEVEL_LAUNCHES) {
        set_err(ctx, "too many levels for the fused kernels");
        throw Fail{IPC_EUNSUPPORTED};
      }
      r.row_base[r.n] = rows;
      r.n_rows[r.n] = items;
      for (int p = 0; p < 3; ++p) r.pass_index[r.n][p] = La.pass_index[p];
      ++r.n;
      rows += items;
      BatchC<T> &e = ent[m++];
      std::memset(&e, 0, sizeof(e));
      e.L = La;
      e.x = static_cast<const T *>(fields[i]);
      e.gin = static_cast<const T *>(g[2 * i + (l & 1)].p);
      e.gout = l > 1 ? static_cast<T *>(g[2 * i + ((l - 1) & 1)].p) : nullptr;
      e.o = o[i];
      e.eb = ebs[i];
      e.two_eb = T(2.0 * ebs[i]);
      e.inv = T(1.0 / (2.0 * ebs[i]));
      e.qmax = T(sizeof(T) == 4 ? QMAX_F32 : QMAX_F64);
      e.item0 = q.items;
      ++q.nf;
      q.items += items;
    }
    key.push_back(int(queue_grid_c(ctx, q.items, isz)));
  }
  uint32_t *rows_p = static_cast<uint32_t *>(
      ensure_ws(ctx, ctx->ws_rows, ctx->ws_rows_bytes, size_t(rows) * WG_ROW * 4));
  for (size_t k = 0; k < m; ++k) ent[k].o.wg_rows = rows_p;
  for (int i = 0; i < n; ++i) {
    o[i].wg_rows = rows_p;
    HeadC<T> &h = heads[i];
    std::memset(&h, 0, sizeof(h));
    const Schedule &sc = ss[i]->meta.sched;
    h.A = anchor3_args(sc);
    h.x = static_cast<const T *>(fields[i]);
    h.g = static_cast<T *>(g[2 * i + (sc.K & 1)].p);
    h.o = o[i];
    h.eb = ebs[i];
    h.two_eb = T(2.0 * ebs[i]);
    h.inv = T(1.0 / (2.0 * ebs[i]));
    h.qmax = T(sizeof(T) == 4 ? QMAX_F32 : QMAX_F64);
  }
  const size_t bytes = tab.ent_off + m * sizeof(BatchC<T>);
  hip_check(ctx, hipMemcpyAsync(tab_dev, host, bytes, hipMemcpyHostToDevice, ctx->stream), "upload");

  auto it = ctx->graphs.find(key);
  if (it == ctx->graphs.end()) {
    if (ctx->graphs.size() >= Q_GRAPHS) {
      for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
      ctx->graphs.clear();
    }
    if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    hipError_t e = launch_queue_reset(claims, ctx->stream);
    if (e == hipSuccess) e = launch_heads_compress(dtype, tab_dev, ctx->stream);
    for (int slot = 0; slot < Kmax && e == hipSuccess; ++slot)
      e = launch_level3_compress_queue(dtype, interp, tab_dev, slot, claims, uint32_t(key[3 + slot]),
                                       ctx->stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->stream, &graph);
    if ((e != hipSuccess || ec != hipSuccess) && graph) (void)hipGraphDestroy(graph);
    hip_check(ctx, e, "queue launch capture");
    hip_check(ctx, ec, "end capture");
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(ctx, ei, "graph instantiate");
    it = ctx->graphs.emplace(key, exec).first;
    ++ctx->graphs_captured;
  }
  hip_check(ctx, hipGraphLaunch(it->second, ctx->stream), "graph launch");
  ++ctx->graph_replays;
  // every field's rows -> errq, max |x^|, plane sizes in one launch
  std::vector<RowsJob> jobs;
  uint32_t most_rows = 0;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < lr[i].n; ++k) {
      RowsJob j;
      std::memset(&j, 0, sizeof(j));
      j.row_base = lr[i].row_base[k];
      j.n_rows = lr[i].n_rows[k];
      for (int p = 0; p < 3; ++p) j.pass_index[p] = lr[i].pass_index[k][p];
      j.errq = o[i].errq;
      j.maxabs_bits = o[i].maxabs_bits;
      j.sizes = o[i].sizes;
      most_rows = std::max(most_rows, j.n_rows);
      jobs.push_back(j);
    }
  DevBuf jobs_dev = dev_alloc(ctx, jobs.size() * sizeof(RowsJob));
  struct FreeJobs {
    ipc_ctx *ctx;
    DevBuf &b;
    ~FreeJobs() { dev_free(ctx, b); }
  } free_jobs{ctx, jobs_dev};
  hip_check(ctx, hipMemcpyAsync(jobs_dev.p, jobs.data(), jobs.size() * sizeof(RowsJob), hipMemcpyHostToDevice,
                                ctx->stream), "upload");
  hip_check(ctx, launch_rows_reduce_batch(static_cast<const RowsJob *>(jobs_dev.p), uint32_t(jobs.size()),
                                          most_rows, rows_p, ctx->stream),
            "row reduction launch");
  if (ctx->host_summary_bytes < sum_off[n]) {
    if (ctx->host_summary) (void)hipHostFree(ctx->host_summary);
    ctx->host_summary = nullptr;
    ctx->host_summary_bytes = 0;
    hip_check(ctx, hipHostMalloc(&ctx->host_summary, sum_off[n], hipHostMallocDefault), "pinned alloc");
    ctx->host_summary_bytes = sum_off[n];
  }
  char *hostp = static_cast<char *>(ctx->host_summary);
  hip_check(ctx, hipMemcpyAsync(hostp, summary, sum_off[n], hipMemcpyDeviceToHost, ctx->stream), "copy");
  hip_check(ctx, hipStreamSynchronize(ctx->stream), "compress");
  for (int i = 0; i < n; ++i) {
    uint64_t nout;
    std::memcpy(&nout, hostp + sum_off[i], 8);
    if (nout > o[i].out_cap) {
      redo[i] = 1;
      continue;
    }
    finish_stream(ss[i], hostp + sum_off[i], nout);
    // the outlier index of the fields that have outliers (as
    // compress_batch_fused)
    if (nout == 0) continue;
    ipc_stream *s = ss[i];
    const uint64_t nc = uint64_t(s->meta.sched.n_chunks);
    s->out_gchunk = dev_alloc(ctx, 8 * nout);
    s->out_local = dev_alloc(ctx, 4 * nout);
    s->out_bits = dev_alloc(ctx, 8 * nout);
    s->out_start = dev_alloc(ctx, 4 * (nc + 1));
    const size_t nb = (nc + 1 + 1023) / 1024;
    uint32_t *cnt = static_cast<uint32_t *>(
        ensure_ws(ctx, ctx->ws_cnt, ctx->ws_cnt_bytes, 4 * (nc + 1) + 4 * (nb + 1)));
    hip_check(ctx, launch_outlier_index_n(static_cast<const OutlierRec *>(o[i].out_recs), nout, o[i].n_out,
                                        static_cast<const PassArgs *>(args_dev.p) + args_off[i], nc,
                                        static_cast<uint32_t *>(s->out_start.p), cnt, cnt + (nc + 1),
                                        static_cast<uint64_t *>(s->out_gchunk.p),
                                        static_cast<uint32_t *>(s->out_local.p),
                                        static_cast<uint64_t *>(s->out_bits.p), ctx->stream),
              "outlier index launch");
  }
  return true;
}

// Compression of n fields on the one-pass-per-launch path (2-D, 1-D, other
// chunk shapes) with one launch per pass index over all of them: step i
// holds pass i of every field that has one.  Each field keeps its own
// working reconstruction, summary and outlier records.  Fields whose outliers
// overflow their record capacity are flagged in `redo`.
template <typename T>
void compress_batch_passes(ipc_ctx *ctx, std::vector<ipc_stream *> &ss, const void *const *fields,
                           const double *ebs, std::vector<char> &redo) {
  const int n = int(ss.size());
  const int dtype = ss[0]->meta.dtype, interp = ss[0]->meta.interp;
  std::vector<size_t> sum_off(n + 1, 0), rec_off(n + 1, 0), args_off(n);
  int Pmax = 0;
  std::vector<PassArgs> args;
  for (int i = 0; i < n; ++i) {
    const Schedule &sc = ss[i]->meta.sched;
    const int P = int(sc.passes.size());
    Pmax = std::max(Pmax, P);
    sum_off[i + 1] = sum_off[i] + ((summary_bytes(P) + 255) & ~size_t(255));
    rec_off[i + 1] = rec_off[i] + std::max<size_t>(4096, size_t(sc.n_points / 1024));
    args_off[i] = args.size();
    args.insert(args.end(), ss[i]->args.begin(), ss[i]->args.end());
  }
  char *summary = static_cast<char *>(ensure_ws(ctx, ctx->ws_summary, ctx->ws_summary_bytes, sum_off[n]));
  ensure_ws(ctx, ctx->ws_out, ctx->ws_out_cap, rec_off[n] * sizeof(OutlierRec));
  hip_check(ctx, hipMemsetAsync(summary, 0, sum_off[n], ctx->stream), "memset");
  std::vector<DevBuf> xh(n);
  DevBuf args_dev, ent_dev;
  auto release = [&] {
    for (DevBuf &b : xh) dev_free(ctx, b);
    dev_free(ctx, args_dev);
    dev_free(ctx, ent_dev);
  };
  try {
    args_dev = dev_alloc(ctx, args.size() * sizeof(PassArgs));
    hip_check(ctx, hipMemcpyAsync(args_dev.p, args.data(), args.size() * sizeof(PassArgs),
                                  hipMemcpyHostToDevice, ctx->stream), "upload");
    std::vector<CompressOut> o(n);
    for (int i = 0; i < n; ++i) {
      const Schedule &sc = ss[i]->meta.sched;
      xh[i] = dev_alloc(ctx, std::max<size_t>(8, size_t(sc.n_points) * sizeof(T)));
      char *sm = summary + sum_off[i];
      const int P = int(sc.passes.size());
      std::memset(&o[i], 0, sizeof(CompressOut));
      o[i].payload = static_cast<uint32_t *>(ss[i]->payload.p);
      o[i].masks = static_cast<uint32_t *>(ss[i]->masks.p);
      o[i].n_out = reinterpret_cast<unsigned long long *>(sm);
      o[i].maxabs_bits = reinterpret_cast<unsigned long long *>(sm + 8);
      o[i].sizes = reinterpret_cast<unsigned long long *>(sm + 16);
      o[i].errq = reinterpret_cast<uint32_t *>(sm + 16 + size_t(P) * 32 * 8);
      o[i].out_recs = static_cast<OutlierRec *>(ctx->ws_out) + rec_off[i];
      o[i].out_cap = rec_off[i + 1] - rec_off[i];
      o[i].wg_rows = nullptr;
    }
    // the work list of every step
    std::vector<PassBatchC<T>> ent;
    struct Launch { size_t off; int nf; uint32_t items; };
    std::vector<Launch> launches;
    for (int step = 0; step < Pmax; ++step) {
      Launch ln{ent.size(), 0, 0};
      for (int i = 0; i < n; ++i) {
        const int P = int(ss[i]->args.size());
        if (step >= P || ss[i]->args[size_t(step)].n_chunks == 0) continue;
        PassBatchC<T> e;
        std::memset(&e, 0, sizeof(e));
        e.a = ss[i]->args[size_t(step)];
        e.x = static_cast<const T *>(fields[i]);
        e.xh = static_cast<T *>(xh[i].p);
        e.o = o[i];
        e.eb = ebs[i];
        e.two_eb = T(2.0 * ebs[i]);
        e.inv = T(1.0 / (2.0 * ebs[i]));
        e.qmax = T(sizeof(T) == 4 ? QMAX_F32 : QMAX_F64);
        e.write_back = step + 1 < P ? 1 : 0;
        e.item0 = ln.items;
        ent.push_back(e);
        ++ln.nf;
        ln.items += uint32_t(e.a.n_chunks);
      }
      if (ln.nf) launches.push_back(ln);
    }
    ent_dev = dev_alloc(ctx, std::max<size_t>(1, ent.size()) * sizeof(PassBatchC<T>));
    hip_check(ctx, hipMemcpyAsync(ent_dev.p, ent.data(), ent.size() * sizeof(PassBatchC<T>),
                                  hipMemcpyHostToDevice, ctx->stream), "upload");
    for (const Launch &ln : launches)
      hip_check(ctx, launch_compress_pass_batch(dtype, interp,
                                                static_cast<PassBatchC<T> *>(ent_dev.p) + ln.off, ln.nf,
                                                ln.items, ctx->stream),
                "pass kernel launch");
    for (int i = 0; i < n; ++i) {
      ipc_stream *s = ss[i];
      const Schedule &sc = s->meta.sched;
      int64_t max_chunks = 0;
      for (const PassGeom &g : sc.passes) max_chunks = std::max(max_chunks, g.n_chunks);
      const PassArgs *ad = static_cast<const PassArgs *>(args_dev.p) + args_off[i];
      hip_check(ctx, launch_all_sizes(ad, int(sc.passes.size()), max_chunks, o[i].masks, o[i].sizes,
                                      ctx->stream),
                "sizes kernel launch");
      const uint64_t nc = uint64_t(sc.n_chunks);
      const size_t cap = size_t(o[i].out_cap);
      s->out_gchunk = dev_alloc(ctx, 8 * cap);
      s->out_local = dev_alloc(ctx, 4 * cap);
      s->out_bits = dev_alloc(ctx, 8 * cap);
      s->out_start = dev_alloc(ctx, 4 * (nc + 1));
      const size_t nb = (nc + 1 + 1023) / 1024;
      uint32_t *cnt = static_cast<uint32_t *>(
          ensure_ws(ctx, ctx->ws_cnt, ctx->ws_cnt_bytes, 4 * (nc + 1) + 4 * (nb + 1)));
      hip_check(ctx, launch_outlier_index(static_cast<const OutlierRec *>(o[i].out_recs), o[i].n_out, cap,
                                          ad, nc, static_cast<uint32_t *>(s->out_start.p), cnt,
                                          cnt + (nc + 1), static_cast<uint64_t *>(s->out_gchunk.p),
                                          static_cast<uint32_t *>(s->out_local.p),
                                          static_cast<uint64_t *>(s->out_bits.p), ctx->stream),
                "outlier index launch");
    }
    if (ctx->host_summary_bytes < sum_off[n]) {
      if (ctx->host_summary) (void)hipHostFree(ctx->host_summary);
      ctx->host_summary = nullptr;
      ctx->host_summary_bytes = 0;
      hip_check(ctx, hipHostMalloc(&ctx->host_summary, sum_off[n], hipHostMallocDefault), "pinned alloc");
      ctx->host_summary_bytes = sum_off[n];
    }
    char *hostp = static_cast<char *>(ctx->host_summary);
    hip_check(ctx, hipMemcpyAsync(hostp, summary, sum_off[n], hipMemcpyDeviceToHost, ctx->stream), "copy");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "compress");
    for (int i = 0; i < n; ++i) {
      uint64_t nout;
      std::memcpy(&nout, hostp + sum_off[i], 8);
      if (nout > o[i].out_cap) {
        redo[i] = 1;
        continue;
      }
      finish_stream(ss[i], hostp + sum_off[i], nout);
    }
  } catch (...) {
    (void)hipStreamSynchronize(ctx->stream);
    release();
    throw;
  }
  release();
}

// Retrieval of n streams on the one-pass-per-launch path: one launch per pass
// index over all of them, each stream from its own first pass `start[i]`
// (0, or the first changed pass of a refinement that recomputes in place).
template <typename T>
void retrieve_batch_passes(ipc_ctx *ctx, const std::vector<const ipc_stream *> &ss,
                           const std::vector<std::vector<int>> &plans, const std::vector<void *> &fields,
                           const std::vector<int> &start) {
  const int n = int(ss.size());
  const int dtype = ss[0]->meta.dtype, interp = ss[0]->meta.interp;
  int Pmax = 0;
  for (const ipc_stream *s : ss) Pmax = std::max(Pmax, int(s->args.size()));
  std::vector<PassBatchR<T>> ent;
  struct Launch { size_t off; int nf; uint32_t items; };
  std::vector<Launch> launches;
  for (int step = 0; step < Pmax; ++step) {
    Launch ln{ent.size(), 0, 0};
    for (int i = 0; i < n; ++i) {
      const ipc_stream *s = ss[i];
      if (step < start[i] || step >= int(s->args.size()) || s->args[size_t(step)].n_chunks == 0) continue;
      PassBatchR<T> e;
      std::memset(&e, 0, sizeof(e));
      e.a = s->args[size_t(step)];
      e.f = static_cast<T *>(fields[i]);
      e.in = retrieve_in(ctx, s);
      e.two_eb = T(2.0 * s->meta.eb);
      e.discard = plans[i][size_t(step)];
      e.item0 = ln.items;
      ent.push_back(e);
      ++ln.nf;
      ln.items += uint32_t(e.a.n_chunks);
    }
    if (ln.nf) launches.push_back(ln);
  }
  DevBuf ent_dev = dev_alloc(ctx, std::max<size_t>(1, ent.size()) * sizeof(PassBatchR<T>));
  try {
    hip_check(ctx, hipMemcpyAsync(ent_dev.p, ent.data(), ent.size() * sizeof(PassBatchR<T>),
                                  hipMemcpyHostToDevice, ctx->stream), "upload");
    for (const Launch &ln : launches)
      hip_check(ctx, launch_retrieve_pass_batch(dtype, interp,
                                                static_cast<PassBatchR<T> *>(ent_dev.p) + ln.off, ln.nf,
                                                ln.items, ctx->stream),
                "pass kernel launch");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "retrieve");
  } catch (...) {
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, ent_dev);
    throw;
  }
  dev_free(ctx, ent_dev);
}

// host copy of the chunk masks
void ensure_host_masks(ipc_ctx *ctx, ipc_stream *s) {
  if (s->host_masks_valid) return;
  StreamMeta &m = s->meta;
  m.masks.resize(size_t(m.sched.n_chunks));
  hip_check(ctx, hipMemcpyAsync(m.masks.data(), s->masks.p, m.masks.size() * 4, hipMemcpyDeviceToHost,
                                ctx->stream), "copy");
  hip_check(ctx, hipStreamSynchronize(ctx->stream), "copy");
  s->host_masks_valid = true;
}

// The raw payload in packed placement on the device: the stream's own buffer,
// or `tmp` filled from the slot placement (host masks must be valid)
const uint32_t *packed_payload(ipc_ctx *ctx, ipc_stream *s, DevBuf &tmp, DevBuf &tmp_off) {
  if (s->packed) return static_cast<const uint32_t *>(s->payload.p);
  const StreamMeta &m = s->meta;
  std::vector<uint64_t> off;
  packed_chunk_offsets(m, off);
  tmp_off = dev_alloc(ctx, off.size() * 8);
  tmp = dev_alloc(ctx, std::max<size_t>(4, m.payload_words * 4));
  hip_check(ctx, hipMemcpyAsync(tmp_off.p, off.data(), off.size() * 8, hipMemcpyHostToDevice, ctx->stream),
            "copy");
  for (const PassArgs &a : s->args)
    hip_check(ctx, launch_pack_payload(a, static_cast<const uint32_t *>(s->masks.p),
                                       static_cast<const uint64_t *>(tmp_off.p),
                                       static_cast<const uint32_t *>(s->payload.p),
                                       static_cast<uint32_t *>(tmp.p), ctx->stream),
              "pack kernel launch");
  // the offsets must outlive the launches: the caller synchronizes before
  // freeing them
  return static_cast<const uint32_t *>(tmp.p);
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

const char *ipc_status_string(ipc_status st) {
  switch (st) {
    case IPC_OK: return "ok";
    case IPC_EINVAL: return "invalid argument";
    case IPC_ENOMEM: return "out of memory";
    case IPC_ECORRUPT: return "corrupt stream";
    case IPC_EHIP: return "HIP runtime error";
    case IPC_ESTATE: return "object used with the wrong context or stream";
    case IPC_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

const char *ipc_last_error(const ipc_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

ipc_status ipc_ctx_set_profiling(ipc_ctx *ctx, int on, int only_pass) {
  if (!ctx) return IPC_EINVAL;
  ctx->profiling = on != 0;
  ctx->prof_only = only_pass;
  return IPC_OK;
}

ipc_status ipc_ctx_set_batch_graphs(ipc_ctx *ctx, int on) {
  if (!ctx) return IPC_EINVAL;
  ctx->batch_graphs = on == 0 ? 0 : (on == 2 ? 2 : 1);
  return IPC_OK;
}

ipc_status ipc_ctx_graph_stats(const ipc_ctx *ctx, uint64_t *captured, uint64_t *replays) {
  if (!ctx || !captured || !replays) return IPC_EINVAL;
  *captured = ctx->graphs_captured;
  *replays = ctx->graph_replays;
  return IPC_OK;
}

ipc_status ipc_ctx_pass_times(const ipc_ctx *ctx, float *ms, uint32_t capacity, uint32_t *n_out) {
  if (!ctx || !n_out) return IPC_EINVAL;
  *n_out = uint32_t(ctx->pass_ms.size());
  if (ms) {
    if (capacity < ctx->pass_ms.size()) return IPC_EINVAL;
    for (size_t k = 0; k < ctx->pass_ms.size(); ++k) ms[k] = ctx->pass_ms[k];
  }
  return IPC_OK;
}

ipc_status ipc_ctx_create(int device, void *hip_stream, ipc_ctx **out) {
  if (!out) return IPC_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return IPC_EINVAL;
  }
  ipc_ctx *c = new (std::nothrow) ipc_ctx();
  if (!c) return IPC_ENOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return IPC_EHIP;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
    c->n_cu = ncu;
  (void)hipGetLastError();
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreate(&c->owned) != hipSuccess) {  // blocking: see ipc_ctx::owned
      delete c;
      return IPC_EHIP;
    }
    c->stream = c->owned;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_copy, hipEventDisableTiming) != hipSuccess ||
      hipMalloc(&c->dev_zero, 256) != hipSuccess || hipMemset(c->dev_zero, 0, 256) != hipSuccess) {
    (void)hipGetLastError();
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev_copy) (void)hipEventDestroy(c->ev_copy);
    if (c->dev_zero) (void)hipFree(c->dev_zero);
    if (c->owned) (void)hipStreamDestroy(c->owned);
    delete c;
    return IPC_EHIP;
  }
  // with the device current: its copy of the no-allocation scratch
  c->scratch = device_scratch(device);
  *out = c;
  return IPC_OK;
}

ipc_status ipc_ctx_set_stream(ipc_ctx *ctx, void *hip_stream) {
  if (!ctx) return IPC_EINVAL;
  (void)hipStreamSynchronize(ctx->stream);
  if (hip_stream) {
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (!ctx->owned && hipStreamCreate(&ctx->owned) != hipSuccess) return IPC_EHIP;
    ctx->stream = ctx->owned;
  }
  return IPC_OK;
}

void ipc_ctx_destroy(ipc_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &kv : ctx->cache) (void)hipFree(kv.second);
  if (ctx->ws_xh) (void)hipFree(ctx->ws_xh);
  if (ctx->ws_summary) (void)hipFree(ctx->ws_summary);
  if (ctx->ws_out) (void)hipFree(ctx->ws_out);
  if (ctx->ws_cnt) (void)hipFree(ctx->ws_cnt);
  if (ctx->ws_rows) (void)hipFree(ctx->ws_rows);
  if (ctx->dev_zero) (void)hipFree(ctx->dev_zero);
  for (int i = 0; i < 2; ++i)
    if (ctx->ws_g[i]) (void)hipFree(ctx->ws_g[i]);
  if (ctx->ws_args) (void)hipFree(ctx->ws_args);
  for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  ctx->graphs.clear();
  if (ctx->ws_q) (void)hipFree(ctx->ws_q);
  if (ctx->host_q) (void)hipHostFree(ctx->host_q);
  if (ctx->host_summary) (void)hipHostFree(ctx->host_summary);
  for (hipEvent_t e : ctx->pev) (void)hipEventDestroy(e);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev_copy) (void)hipEventDestroy(ctx->ev_copy);
  if (ctx->owned) (void)hipStreamDestroy(ctx->owned);
  delete ctx;
}

ipc_status ipc_compress(ipc_ctx *ctx, const void *field_dev, const uint64_t *dims, int ndim,
                        int dtype, double abs_eb, const ipc_options *opts, ipc_stream **out) {
  TraceRange trace_range("ipc_compress");
  if (!out) return IPC_EINVAL;
  *out = nullptr;
  if (!ctx) return IPC_EINVAL;
  if (!field_dev || !dims || ndim < 1 || ndim > 3 || (dtype != IPC_F32 && dtype != IPC_F64) ||
      !(std::isfinite(abs_eb) && abs_eb > 0)) {
    set_err(ctx, "invalid argument to ipc_compress");
    return IPC_EINVAL;
  }
  int interp = opts ? opts->interp : IPC_CUBIC;
  if (interp != IPC_LINEAR && interp != IPC_CUBIC) {
    set_err(ctx, "interp must be IPC_LINEAR or IPC_CUBIC");
    return IPC_EINVAL;
  }
  ipc_stream *s = new (std::nothrow) ipc_stream();
  if (!s) return IPC_ENOMEM;
  s->ctx = ctx;
  ipc_status st = guarded(ctx, [&] {
    enter_device(ctx);
    setup_stream(ctx, s, dims, ndim, dtype, interp, abs_eb, opts);
    StreamMeta &m = s->meta;
    const Schedule &sc = m.sched;
    const int P = int(sc.passes.size());
    const size_t isz = dtype == IPC_F32 ? 4 : 8;
    const size_t nbytes = size_t(sc.n_points) * isz;
    const bool fused = fused3(sc) && !(opts && (opts->debug_flags & IPC_DEBUG_PER_PASS));
    void *xh = nullptr;
    if (fused)
      ensure_coarse(ctx, sc, isz);
    else
      xh = ensure_ws(ctx, ctx->ws_xh, ctx->ws_xh_bytes, nbytes);
    {
      const size_t had = ctx->ws_args_bytes;
      ensure_ws(ctx, ctx->ws_args, ctx->ws_args_bytes, s->args.size() * sizeof(PassArgs));
      if (ctx->ws_args_bytes != had) ctx->args_host.clear();  // a fresh allocation
    }
    // the pass table on the device: uploaded when it differs from the last one
    const size_t args_bytes = s->args.size() * sizeof(PassArgs);
    if (ctx->ws_args != ctx->args_dev_at || ctx->args_host.size() != s->args.size() ||
        std::memcmp(ctx->args_host.data(), s->args.data(), args_bytes) != 0) {
      hip_check(ctx, hipMemcpyAsync(ctx->ws_args, s->args.data(), args_bytes, hipMemcpyHostToDevice,
                                    ctx->stream), "upload");
      ctx->args_host = s->args;
      ctx->args_dev_at = ctx->ws_args;
    }
    int64_t max_chunks = 0;
    for (const PassGeom &g : sc.passes) max_chunks = std::max(max_chunks, g.n_chunks);
    // summary: n_out, maxabs bits, sizes [P][32] u64, errq [P][33] u32
    size_t sum_bytes = summary_bytes(P);
    char *summary = static_cast<char *>(ensure_ws(ctx, ctx->ws_summary, ctx->ws_summary_bytes, sum_bytes));
    size_t cap = std::max<size_t>(4096, size_t(sc.n_points / 1024));
    for (int attempt = 0; attempt < 2; ++attempt) {
      ensure_ws(ctx, ctx->ws_out, ctx->ws_out_cap, cap * sizeof(OutlierRec));
      size_t cap_recs = ctx->ws_out_cap / sizeof(OutlierRec);
      // (the fused path's anchor launch clears the summary itself)
      if (!fused) hip_check(ctx, hipMemsetAsync(summary, 0, sum_bytes, ctx->stream), "memset");
      unsigned long long *sizes = reinterpret_cast<unsigned long long *>(summary + 16);
      CompressOut o;
      o.payload = static_cast<uint32_t *>(s->payload.p);
      o.masks = static_cast<uint32_t *>(s->masks.p);
      o.n_out = reinterpret_cast<unsigned long long *>(summary);
      o.maxabs_bits = reinterpret_cast<unsigned long long *>(summary + 8);
      o.errq = reinterpret_cast<uint32_t *>(summary + 16 + size_t(P) * 32 * 8);
      o.out_recs = ctx->ws_out;
      o.out_cap = cap_recs;
      o.wg_rows = nullptr;
      o.sizes = sizes;
      hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
      prof_begin(ctx, size_t(P));
      if (fused) {
        const int K = sc.K;
        // level launches and their workgroup rows
        std::vector<Level3Args> las;
        LevelRows lr;
        std::memset(&lr, 0, sizeof(lr));
        uint32_t rows = 0;
        for (int l = K; l >= 1; --l) {
          Level3Args La = level_args(ctx, m, l, true);
          La.row_base = rows;
          if (lr.n >= MAX_LEVEL_LAUNCHES) {
            set_err(ctx, "too many levels for the fused kernels");
            throw Fail{IPC_EUNSUPPORTED};
          }
          lr.row_base[lr.n] = rows;
          lr.n_rows[lr.n] = uint32_t(level3_wgs(La));
          for (int p = 0; p < 3; ++p) lr.pass_index[lr.n][p] = La.pass_index[p];
          rows += lr.n_rows[lr.n];
          ++lr.n;
          las.push_back(La);
        }
        o.wg_rows = static_cast<uint32_t *>(
            ensure_ws(ctx, ctx->ws_rows, ctx->ws_rows_bytes, size_t(rows) * WG_ROW * 4));
        Level3Args A = anchor3_args(sc);
        prof_mark(ctx, 0, true);
        hip_check(ctx, launch_anchor3_compress(dtype, A, field_dev, ctx->ws_g[K & 1], abs_eb, o,
                                               reinterpret_cast<uint32_t *>(summary),
                                               uint32_t(sum_bytes / 4), ctx->stream),
                  "anchor kernel launch");
        prof_mark(ctx, 0, false);
        for (const Level3Args &La : las) {
          const int l = int(sc.passes[La.pass_index[2]].level);
          int pc = int(La.pass_index[2]);
          prof_mark(ctx, pc, true);
          hip_check(ctx, launch_level3_compress(dtype, interp, La, field_dev, ctx->ws_g[l & 1],
                                                l > 1 ? ctx->ws_g[(l - 1) & 1] : nullptr, abs_eb, o,
                                                ctx->stream),
                    "level kernel launch");
          prof_mark(ctx, pc, false);
        }
        hip_check(ctx, launch_rows_reduce(lr, o.wg_rows, o.errq, o.maxabs_bits, sizes, ctx->stream),
                  "row reduction launch");
      } else {
        for (int i = 0; i < P; ++i) {
          int wb = i + 1 < P ? 1 : 0;  // the last pass is read by nobody
          prof_mark(ctx, i, true);
          hip_check(ctx, launch_compress_pass(dtype, interp, s->args[i], field_dev, xh, wb, abs_eb,
                                              o, ctx->stream),
                    "compress kernel launch");
          prof_mark(ctx, i, false);
        }
      }
      if (!fused)
        hip_check(ctx, launch_all_sizes(static_cast<const PassArgs *>(ctx->ws_args), P, max_chunks,
                                        o.masks, sizes, ctx->stream),
                  "sizes kernel launch");
      hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
      if (ctx->host_summary_bytes < sum_bytes) {
        if (ctx->host_summary) (void)hipHostFree(ctx->host_summary);
        ctx->host_summary = nullptr;
        ctx->host_summary_bytes = 0;
        hip_check(ctx, hipHostMalloc(&ctx->host_summary, sum_bytes, hipHostMallocDefault), "pinned alloc");
        ctx->host_summary_bytes = sum_bytes;
      }
      char *hostp = static_cast<char *>(ctx->host_summary);
      hip_check(ctx, hipMemcpyAsync(hostp, summary, sum_bytes, hipMemcpyDeviceToHost, ctx->stream), "copy");
      hip_check(ctx, hipEventRecord(ctx->ev_copy, ctx->stream), "event");
      // the outlier index, sorted on the device (records stay there until a
      // serialization asks for them), queued behind the summary copy: it runs
      // while the host reads the summary, and only later work on the same
      // stream reads it.  (Issued after the wait instead, sized to the count
      // read there, its launches lengthened the call by their issue time.)
      {
        const uint64_t nc = uint64_t(sc.n_chunks);
        dev_free(ctx, s->out_gchunk);
        dev_free(ctx, s->out_local);
        dev_free(ctx, s->out_bits);
        dev_free(ctx, s->out_start);
        s->out_gchunk = dev_alloc(ctx, 8 * cap_recs);
        s->out_local = dev_alloc(ctx, 4 * cap_recs);
        s->out_bits = dev_alloc(ctx, 8 * cap_recs);
        s->out_start = dev_alloc(ctx, 4 * (nc + 1));
        const size_t nb = (nc + 1 + 1023) / 1024;
        uint32_t *cnt = static_cast<uint32_t *>(
            ensure_ws(ctx, ctx->ws_cnt, ctx->ws_cnt_bytes, 4 * (nc + 1) + 4 * (nb + 1)));
        hip_check(ctx, launch_outlier_index(static_cast<const OutlierRec *>(o.out_recs), o.n_out,
                                            cap_recs, static_cast<const PassArgs *>(ctx->ws_args),
                                            nc, static_cast<uint32_t *>(s->out_start.p), cnt,
                                            cnt + (nc + 1), static_cast<uint64_t *>(s->out_gchunk.p),
                                            static_cast<uint32_t *>(s->out_local.p),
                                            static_cast<uint64_t *>(s->out_bits.p), ctx->stream),
                  "outlier index launch");
      }
      hip_check(ctx, hipEventSynchronize(ctx->ev_copy), "compress");
      prof_end(ctx);
      uint64_t nout;
      std::memcpy(&nout, hostp, 8);
      if (nout > cap_recs) {
        cap = size_t(nout) + 1024;
        if (attempt == 0) continue;
        set_err(ctx, "outlier buffer overflow");
        throw Fail{IPC_EHIP};
      }
      finish_stream(s, hostp, nout);
      break;
    }
  });
  if (st == IPC_OK) st = finish_options(ctx, s, field_dev, opts);
  if (st != IPC_OK) {
    free_stream_bufs(s);
    delete s;
    return st;
  }
  *out = s;
  return IPC_OK;
}

ipc_status ipc_stream_size(const ipc_stream *s, uint64_t *bytes) {
  if (!s || !bytes) return IPC_EINVAL;
  *bytes = s->meta.serialized_bytes;
  return IPC_OK;
}

ipc_status ipc_stream_to_host(ipc_ctx *ctx, const ipc_stream *sc, void *dst, uint64_t capacity) {
  TraceRange trace_range("ipc_stream_to_host");
  if (!ctx || !sc || !dst) return IPC_EINVAL;
  if (sc->ctx != ctx) {
    set_err(ctx, "stream belongs to another context");
    return IPC_ESTATE;
  }
  ipc_stream *s = const_cast<ipc_stream *>(sc);
  if (capacity < s->meta.serialized_bytes) {
    set_err(ctx, "destination too small");
    return IPC_EINVAL;
  }
  return guarded(ctx, [&] {
    enter_device(ctx);
    StreamMeta &m = s->meta;
    ensure_host_masks(ctx, s);
    if (!s->host_outliers_valid) fetch_outliers(ctx, s);
    uint8_t *d = static_cast<uint8_t *>(dst);
    write_serialized_head(m, d);
    const uint64_t poff = payload_offset(m);
    const uint64_t pbytes = (m.coding ? m.coded_words : m.payload_words) * 4;
    DevBuf tmp, tmp_off;
    try {
      const void *src = m.coding ? s->coded.p : packed_payload(ctx, s, tmp, tmp_off);
      if (pbytes)
        // (the raw planes may sit in pinned host memory: the direction is inferred)
        hip_check(ctx, hipMemcpyAsync(d + poff, src, pbytes, hipMemcpyDefault, ctx->stream), "copy");
      hip_check(ctx, hipStreamSynchronize(ctx->stream), "copy");
    } catch (...) {
      dev_free(ctx, tmp);
      dev_free(ctx, tmp_off);
      throw;
    }
    dev_free(ctx, tmp);
    dev_free(ctx, tmp_off);
    std::memset(d + poff + pbytes, 0, size_t(pad8(pbytes) - pbytes));
  });
}

ipc_status ipc_stream_entropy_code(ipc_ctx *ctx, ipc_stream *s) {
  TraceRange trace_range("ipc_stream_entropy_code");
  if (!ctx || !s) return IPC_EINVAL;
  if (s->ctx != ctx) {
    set_err(ctx, "stream belongs to another context");
    return IPC_ESTATE;
  }
  if (s->meta.coding) return IPC_OK;
  return guarded(ctx, [&] {
    enter_device(ctx);
    StreamMeta &m = s->meta;
    ensure_host_masks(ctx, s);
    const uint64_t nb = n_blocks(m);
    DevBuf tmp, tmp_off, dblk, tabs, scratch, dwords, dtot, coded;
    auto release = [&] {
      for (DevBuf *b : {&tmp, &tmp_off, &dblk, &tabs, &scratch, &dwords, &dtot}) dev_free(ctx, *b);
    };
    try {
      device_blocks(ctx, m, dblk, tabs);
      const uint32_t *raw = packed_payload(ctx, s, tmp, tmp_off);
      scratch = dev_alloc(ctx, std::max<size_t>(4, m.payload_words * 4));
      dwords = dev_alloc(ctx, std::max<size_t>(1, nb));
      dtot = dev_alloc(ctx, std::max<size_t>(8, (nb + 1023) / 1024 * 8));
      EcBlock *blk = static_cast<EcBlock *>(dblk.p);
      uint8_t *words_d = static_cast<uint8_t *>(dwords.p);
      hip_check(ctx, launch_ec_encode(blk, nb, raw, static_cast<uint32_t *>(scratch.p), words_d, ctx->stream),
                "entropy encode launch");
      hip_check(ctx, launch_ec_offsets(words_d, nb, blk, static_cast<uint64_t *>(dtot.p), ctx->stream),
                "entropy offsets launch");
      std::vector<uint8_t> words(nb);
      if (nb)
        hip_check(ctx, hipMemcpyAsync(words.data(), words_d, nb, hipMemcpyDeviceToHost, ctx->stream), "copy");
      hip_check(ctx, hipStreamSynchronize(ctx->stream), "entropy encode");
      uint64_t tot = 0;
      for (uint8_t w : words) tot += w;
      coded = dev_alloc(ctx, std::max<size_t>(4, tot * 4));
      hip_check(ctx, launch_ec_gather(blk, nb, words_d, static_cast<const uint32_t *>(scratch.p),
                                      static_cast<uint32_t *>(coded.p), ctx->stream),
                "entropy gather launch");
      hip_check(ctx, hipStreamSynchronize(ctx->stream), "entropy gather");
      m.block_words = std::move(words);
      m.coded_words = tot;
      m.coding = 1;
      m.serialized_bytes = serialized_size(m);
      s->coded = coded;
      coded = DevBuf();
      s->tables = plan_tables(m);
    } catch (...) {
      (void)hipStreamSynchronize(ctx->stream);
      release();
      dev_free(ctx, coded);
      throw;
    }
    release();
  });
}

ipc_status ipc_stream_coding(const ipc_stream *s, int *coding) {
  if (!s || !coding) return IPC_EINVAL;
  *coding = s->meta.coding;
  return IPC_OK;
}

ipc_status ipc_stream_from_host(ipc_ctx *ctx, const void *src, uint64_t bytes, int device_resident,
                                ipc_stream **out) {
  TraceRange trace_range("ipc_stream_from_host");
  if (!out) return IPC_EINVAL;
  *out = nullptr;
  if (!ctx || !src) return IPC_EINVAL;
  ipc_stream *s = new (std::nothrow) ipc_stream();
  if (!s) return IPC_ENOMEM;
  s->ctx = ctx;
  ipc_status st = guarded(ctx, [&] {
    enter_device(ctx);
    const uint32_t *payload = nullptr;
    std::string e;
    if (!parse_serialized(static_cast<const uint8_t *>(src), bytes, s->meta, &payload, e)) {
      set_err(ctx, e);
      throw Fail{IPC_ECORRUPT};
    }
    if (!chunks_supported(s->meta.sched, e)) {
      set_err(ctx, e);
      throw Fail{IPC_EUNSUPPORTED};
    }
    StreamMeta &m = s->meta;
    s->host_masks_valid = true;
    s->packed = true;
    for (const PassGeom &p : m.sched.passes) s->args.push_back(make_args(m.sched, p));
    std::vector<uint64_t> off;
    packed_chunk_offsets(m, off);
    const size_t pbytes = std::max<size_t>(4, m.payload_words * 4);
    s->payload = dev_alloc(ctx, pbytes);
    s->masks = dev_alloc(ctx, std::max<size_t>(4, m.masks.size() * 4));
    s->chunk_off = dev_alloc(ctx, off.size() * 8);
    if (m.coding) {
      // stored blocks to the device, decoded there into the packed placement
      const uint64_t nb = m.block_words.size();
      s->coded = dev_alloc(ctx, std::max<size_t>(4, m.coded_words * 4));
      DevBuf dblk, tabs, dwords, dtot;
      auto release = [&] {
        for (DevBuf *b : {&dblk, &tabs, &dwords, &dtot}) dev_free(ctx, *b);
      };
      try {
        if (m.coded_words)
          hip_check(ctx, hipMemcpyAsync(s->coded.p, payload, m.coded_words * 4, hipMemcpyHostToDevice,
                                        ctx->stream), "upload");
        device_blocks(ctx, m, dblk, tabs);
        dwords = dev_alloc(ctx, std::max<size_t>(1, nb));
        dtot = dev_alloc(ctx, std::max<size_t>(8, (nb + 1023) / 1024 * 8));
        if (nb)
          hip_check(ctx, hipMemcpyAsync(dwords.p, m.block_words.data(), nb, hipMemcpyHostToDevice,
                                        ctx->stream), "upload");
        EcBlock *blk = static_cast<EcBlock *>(dblk.p);
        hip_check(ctx, launch_ec_offsets(static_cast<const uint8_t *>(dwords.p), nb, blk,
                                         static_cast<uint64_t *>(dtot.p), ctx->stream),
                  "entropy offsets launch");
        hip_check(ctx, launch_ec_decode(blk, nb, static_cast<const uint8_t *>(dwords.p),
                                        static_cast<const uint32_t *>(s->coded.p),
                                        static_cast<uint32_t *>(s->payload.p), ctx->stream),
                  "entropy decode launch");
        hip_check(ctx, hipStreamSynchronize(ctx->stream), "entropy decode");
      } catch (...) {
        (void)hipStreamSynchronize(ctx->stream);
        release();
        throw;
      }
      release();
    } else if (m.payload_words) {
      hip_check(ctx, hipMemcpyAsync(s->payload.p, payload, m.payload_words * 4, hipMemcpyHostToDevice,
                                    ctx->stream), "upload");
    }
    hip_check(ctx, hipMemcpyAsync(s->masks.p, m.masks.data(), m.masks.size() * 4, hipMemcpyHostToDevice, ctx->stream), "upload");
    hip_check(ctx, hipMemcpyAsync(s->chunk_off.p, off.data(), off.size() * 8, hipMemcpyHostToDevice, ctx->stream), "upload");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "upload");
    if (!device_resident) {
      // the raw planes move to pinned host memory that the kernels read in
      // place: a retrieval moves only the planes its plan loads over the bus
      void *hp = nullptr;
      if (hipHostMalloc(&hp, pbytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_err(ctx, "pinned host allocation of " + std::to_string(pbytes) + " bytes failed");
        throw Fail{IPC_ENOMEM};
      }
      hipError_t ce = hipMemcpy(hp, s->payload.p, pbytes, hipMemcpyDeviceToHost);
      if (ce != hipSuccess) {
        (void)hipHostFree(hp);
        hip_check(ctx, ce, "payload to host");
      }
      dev_free(ctx, s->payload);
      s->payload.p = hp;
      s->payload.bytes = pbytes;
      s->host_payload = true;
    }
    s->tables = plan_tables(m);
    upload_outliers(ctx, s);
  });
  if (st != IPC_OK) {
    free_stream_bufs(s);
    delete s;
    return st;
  }
  *out = s;
  return IPC_OK;
}

void ipc_stream_free(ipc_stream *s) {
  if (!s) return;
  if (s->ctx) (void)hipStreamSynchronize(s->ctx->stream);
  free_stream_bufs(s);
  delete s;
}

static ipc_status retrieve_common(ipc_ctx *ctx, const ipc_stream *s, const std::vector<int> &plan,
                                  double bound, uint32_t flags, float tplan, ipc_state **out,
                                  ipc_info *info) {
  ipc_state *stt = new (std::nothrow) ipc_state();
  if (!stt) return IPC_ENOMEM;
  stt->ctx = ctx;
  stt->stream = s;
  stt->plan = plan;
  stt->bound = bound;
  ipc_status st = guarded(ctx, [&] {
    enter_device(ctx);
    size_t isz = s->meta.dtype == IPC_F32 ? 4 : 8;
    stt->field = dev_alloc(ctx, size_t(s->meta.sched.n_points) * isz);
    hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
    run_retrieve(ctx, s, plan, 0, stt->field.p);
    hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
    // (waiting on the event instead returns a few us sooner, but the next
    // synchronization of the stream then takes longer: measured slower over
    // whole steps)
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "retrieve");
    prof_end(ctx);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    std::vector<int> none(plan.size(), 32);
    fill_info(s, plan, bound, flags, plane_bytes_between(s, plan, none), tplan, ms, info);
  });
  if (st != IPC_OK) {
    dev_free(ctx, stt->field);
    delete stt;
    return st;
  }
  *out = stt;
  return IPC_OK;
}

static bool valid_target(ipc_target t) {
  const int base = t.kind & ~IPC_TARGET_LEVEL_GROUPS;
  return (base == IPC_TARGET_EB || base == IPC_TARGET_BITRATE) && std::isfinite(t.value) &&
         t.value > 0;
}

ipc_status ipc_retrieve(ipc_ctx *ctx, const ipc_stream *s, ipc_target target, ipc_state **out,
                        ipc_info *info) {
  TraceRange trace_range("ipc_retrieve");
  if (!out) return IPC_EINVAL;
  *out = nullptr;
  if (!ctx || !s) return IPC_EINVAL;
  if (s->ctx != ctx) {
    set_err(ctx, "stream belongs to another context");
    return IPC_ESTATE;
  }
  if (!valid_target(target)) {
    set_err(ctx, "target value must be finite and > 0");
    return IPC_EINVAL;
  }
  auto t0 = std::chrono::steady_clock::now();
  PlanResult pr = plan_request(s->tables, target.kind, target.value, nullptr);
  float tplan = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return retrieve_common(ctx, s, pr.plan, pr.bound, pr.flags, tplan, out, info);
}

ipc_status ipc_retrieve_plan(ipc_ctx *ctx, const ipc_stream *s, const uint8_t *plan,
                             uint32_t n_passes, ipc_state **out, ipc_info *info) {
  TraceRange trace_range("ipc_retrieve_plan");
  if (!out) return IPC_EINVAL;
  *out = nullptr;
  if (!ctx || !s || !plan) return IPC_EINVAL;
  if (s->ctx != ctx) return IPC_ESTATE;
  if (n_passes != s->args.size()) {
    set_err(ctx, "plan has the wrong number of passes");
    return IPC_EINVAL;
  }
  std::vector<int> p(n_passes);
  for (uint32_t i = 0; i < n_passes; ++i) {
    if (plan[i] > 32 || ((!s->tables.progressive[i]) && plan[i] != 0)) {
      set_err(ctx, "plan entry out of range");
      return IPC_EINVAL;
    }
    p[i] = plan[i];
  }
  double b0 = plan_bound(s->tables, p, s->tables.maxabs);
  double bound = plan_bound(s->tables, p, 2.0 * (s->tables.maxabs + b0));
  return retrieve_common(ctx, s, p, bound, 0, 0.0f, out, info);
}

ipc_status ipc_retrieve_noalloc(ipc_ctx *ctx, const ipc_stream *s, ipc_target target,
                                void *field_dev, uint64_t capacity, ipc_info *info) {
  TraceRange trace_range("ipc_retrieve_noalloc");
  if (!ctx || !s || !field_dev) return IPC_EINVAL;
  if (s->ctx != ctx) {
    set_err(ctx, "stream belongs to another context");
    return IPC_ESTATE;
  }
  if (!valid_target(target)) {
    set_err(ctx, "target value must be finite and > 0");
    return IPC_EINVAL;
  }
  const Schedule &sc = s->meta.sched;
  const size_t isz = s->meta.dtype == IPC_F32 ? 4 : 8;
  if (capacity < uint64_t(sc.n_points) * isz) {
    set_err(ctx, "output capacity below the field's size");
    return IPC_EINVAL;
  }
  void *ws[2] = {nullptr, nullptr};
  if (fused3(sc)) {
    if (!ctx->scratch) {
      set_err(ctx, "the device's scratch array could not be resolved");
      return IPC_EHIP;
    }
    size_t need[2];
    coarse_need(sc, isz, need);
    const size_t off1 = (need[0] + 255) & ~size_t(255);
    if (off1 + need[1] > size_t(IPC_NOALLOC_SCRATCH_BYTES)) {
      set_err(ctx, "coarse grids need " + std::to_string(off1 + need[1]) +
                       " bytes, above the scratch of " +
                       std::to_string(size_t(IPC_NOALLOC_SCRATCH_BYTES)) + " bytes");
      return IPC_EINVAL;
    }
    ws[0] = ctx->scratch;
    ws[1] = static_cast<char *>(ctx->scratch) + off1;
  }
  auto t0 = std::chrono::steady_clock::now();
  PlanResult pr = plan_request(s->tables, target.kind, target.value, nullptr);
  float tplan = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  // per-pass timing would create events: off for this call
  struct ProfilingOff {
    ipc_ctx *c;
    bool was;
    ~ProfilingOff() { c->profiling = was; }
  } prof_off{ctx, ctx->profiling};
  ctx->profiling = false;
  return guarded(ctx, [&] {
    enter_device(ctx);
    hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
    run_retrieve(ctx, s, pr.plan, 0, field_dev, ws);
    hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "retrieve");
    prof_end(ctx);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    std::vector<int> none(pr.plan.size(), 32);
    fill_info(s, pr.plan, pr.bound, pr.flags, plane_bytes_between(s, pr.plan, none), tplan, ms, info);
  });
}

const void *ipc_state_field(const ipc_state *st) { return st ? st->field.p : nullptr; }

ipc_status ipc_stream_field_bytes(const ipc_stream *s, uint64_t *bytes) {
  if (!s || !bytes) return IPC_EINVAL;
  *bytes = uint64_t(s->meta.sched.n_points) * (s->meta.dtype == IPC_F32 ? 4u : 8u);
  return IPC_OK;
}

ipc_status ipc_state_field_bytes(const ipc_state *st, uint64_t *bytes) {
  if (!st || !bytes) return IPC_EINVAL;
  return ipc_stream_field_bytes(st->stream, bytes);
}

ipc_status ipc_state_copy_field(ipc_ctx *ctx, const ipc_state *st, void *dst_dev,
                                uint64_t capacity) {
  if (!ctx || !st || !dst_dev) return IPC_EINVAL;
  if (st->ctx != ctx) return IPC_ESTATE;
  uint64_t n = uint64_t(st->stream->meta.sched.n_points) * (st->stream->meta.dtype == IPC_F32 ? 4 : 8);
  if (capacity < n) {
    set_err(ctx, "destination too small");
    return IPC_EINVAL;
  }
  return guarded(ctx, [&] {
    enter_device(ctx);
    hip_check(ctx, hipMemcpyAsync(dst_dev, st->field.p, n, hipMemcpyDeviceToDevice, ctx->stream), "copy");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "copy");
  });
}

ipc_status ipc_stream_pass_info(const ipc_stream *s, uint32_t pass, ipc_pass_info *out) {
  if (!s || !out || pass >= s->args.size()) return IPC_EINVAL;
  const PassGeom &g = s->meta.sched.passes[pass];
  std::memset(out, 0, sizeof(*out));
  out->level = g.level;
  out->dim = g.dim;
  out->n_targets = uint64_t(g.n_targets);
  out->n_chunks = uint64_t(g.n_chunks);
  for (int k = 0; k < 32; ++k) out->plane_bytes[k] = uint64_t(s->tables.sizes[size_t(pass) * 32 + k]);
  for (int b = 0; b < 33; ++b) out->errq[b] = s->meta.errq[size_t(pass) * 33 + b];
  out->progressive = s->tables.progressive[pass];
  out->launch_pass = pass;
  if (fused3(s->meta.sched) && g.level >= 1)
    out->launch_pass = uint32_t(level_last_pass(s->meta.sched, g.level));
  return IPC_OK;
}

ipc_status ipc_stream_describe(const ipc_stream *s, ipc_stream_desc *out) {
  if (!s || !out) return IPC_EINVAL;
  std::memset(out, 0, sizeof(*out));
  const StreamMeta &m = s->meta;
  out->ndim = m.sched.D;
  out->dtype = m.dtype;
  for (int j = 0; j < m.sched.D && j < 3; ++j) out->dims[j] = uint64_t(m.sched.dims[j]);
  out->interp = m.interp;
  out->nonprog_levels = m.nonprog_levels;
  out->abs_eb = m.eb;
  out->n_passes = uint32_t(s->args.size());
  out->coding = m.coding;
  return IPC_OK;
}

ipc_status ipc_stream_passes(const ipc_stream *s, uint32_t *n_passes) {
  if (!s || !n_passes) return IPC_EINVAL;
  *n_passes = uint32_t(s->args.size());
  return IPC_OK;
}

ipc_status ipc_refine(ipc_ctx *ctx, ipc_state *st, ipc_target target, ipc_info *info) {
  TraceRange trace_range("ipc_refine");
  if (!ctx || !st) return IPC_EINVAL;
  if (st->ctx != ctx) {
    set_err(ctx, "state belongs to another context");
    return IPC_ESTATE;
  }
  if (!valid_target(target)) {
    set_err(ctx, "target value must be finite and > 0");
    return IPC_EINVAL;
  }
  const ipc_stream *s = st->stream;
  auto t0 = std::chrono::steady_clock::now();
  if ((target.kind & ~IPC_TARGET_LEVEL_GROUPS) == IPC_TARGET_EB && target.value >= st->bound) {
    fill_info(s, st->plan, st->bound, IPC_FLAG_NOOP, 0, 0.0f, 0.0f, info);
    return IPC_OK;
  }
  PlanResult pr = plan_request(s->tables, target.kind, target.value, st->plan.data());
  float tplan = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (pr.plan == st->plan) {
    fill_info(s, st->plan, st->bound, pr.flags | IPC_FLAG_NOOP, 0, tplan, 0.0f, info);
    return IPC_OK;
  }
  int s_min = -1;
  for (size_t i = 0; i < pr.plan.size(); ++i)
    if (pr.plan[i] < st->plan[i]) {
      s_min = int(i);
      break;
    }
  return guarded(ctx, [&] {
    enter_device(ctx);
    hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
    run_retrieve(ctx, s, pr.plan, s_min, st->field.p);
    hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "refine");
    prof_end(ctx);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    uint64_t read = plane_bytes_between(s, pr.plan, st->plan);
    st->plan = pr.plan;
    st->bound = pr.bound;
    fill_info(s, st->plan, st->bound, pr.flags, read, tplan, ms, info);
  });
}

ipc_status ipc_refine_additive(ipc_ctx *ctx, ipc_state *st, ipc_target target, ipc_info *info) {
  TraceRange trace_range("ipc_refine_additive");
  if (!ctx || !st) return IPC_EINVAL;
  if (st->ctx != ctx) {
    set_err(ctx, "state belongs to another context");
    return IPC_ESTATE;
  }
  if (!valid_target(target)) {
    set_err(ctx, "target value must be finite and > 0");
    return IPC_EINVAL;
  }
  const ipc_stream *s = st->stream;
  auto t0 = std::chrono::steady_clock::now();
  if ((target.kind & ~IPC_TARGET_LEVEL_GROUPS) == IPC_TARGET_EB && target.value >= st->bound) {
    fill_info(s, st->plan, st->bound, IPC_FLAG_NOOP, 0, 0.0f, 0.0f, info);
    return IPC_OK;
  }
  PlanResult pr = plan_request(s->tables, target.kind, target.value, st->plan.data());
  float tplan = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (pr.plan == st->plan) {
    fill_info(s, st->plan, st->bound, pr.flags | IPC_FLAG_NOOP, 0, tplan, 0.0f, info);
    return IPC_OK;
  }
  int s_min = -1;
  for (size_t i = 0; i < pr.plan.size(); ++i)
    if (pr.plan[i] < st->plan[i]) {
      s_min = int(i);
      break;
    }
  return guarded(ctx, [&] {
    enter_device(ctx);
    const size_t isz = s->meta.dtype == IPC_F32 ? 4 : 8;
    const uint64_t n = uint64_t(s->meta.sched.n_points);
    // the difference field lives in the per-pass working buffer
    void *delta = ensure_ws(ctx, ctx->ws_xh, ctx->ws_xh_bytes, size_t(n) * isz);
    const RetrieveIn in = retrieve_in(ctx, s);
    hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
    hip_check(ctx, hipMemsetAsync(delta, 0, size_t(n) * isz, ctx->stream), "memset");
    for (size_t i = size_t(s_min); i < s->args.size(); ++i)
      hip_check(ctx, launch_retrieve_pass(s->meta.dtype, s->meta.interp, s->args[i], delta, pr.plan[i],
                                          in, s->meta.eb, ctx->stream, st->plan[i]),
                "additive pass launch");
    hip_check(ctx, launch_add_delta(s->meta.dtype, st->field.p, delta, n, ctx->stream), "add launch");
    hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
    hip_check(ctx, hipStreamSynchronize(ctx->stream), "refine");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    uint64_t read = plane_bytes_between(s, pr.plan, st->plan);
    const double bound = plan_additive_bound(s->tables, pr.plan, st->plan, target.kind, target.value,
                                             pr.bound);
    st->plan = pr.plan;
    st->bound = bound;
    fill_info(s, st->plan, st->bound, pr.flags, read, tplan, ms, info);
  });
}

void ipc_state_free(ipc_state *st) {
  if (!st) return;
  if (st->ctx) (void)hipStreamSynchronize(st->ctx->stream);
  dev_free(st->ctx, st->field);
  delete st;
}

ipc_status ipc_plan_host(const void *stream_bytes, uint64_t nbytes, ipc_target target,
                         const uint8_t *limit, uint8_t *plan_out, uint32_t plan_capacity,
                         double *bound_out, uint32_t *flags_out, uint64_t *loaded_out) {
  if (!stream_bytes || !plan_out) return IPC_EINVAL;
  if (!valid_target(target)) return IPC_EINVAL;
  try {
    StreamMeta m;
    const uint32_t *payload = nullptr;
    std::string e;
    if (!parse_serialized(static_cast<const uint8_t *>(stream_bytes), nbytes, m, &payload, e))
      return IPC_ECORRUPT;
    PlanTables t = plan_tables(m);
    if (plan_capacity < uint32_t(t.P)) return IPC_EINVAL;
    std::vector<int> lim;
    if (limit) {
      lim.resize(t.P);
      for (int i = 0; i < t.P; ++i) {
        if (limit[i] > 32) return IPC_EINVAL;
        lim[i] = t.progressive[i] ? limit[i] : 0;
      }
    }
    PlanResult pr = plan_request(t, target.kind, target.value, limit ? lim.data() : nullptr);
    for (int i = 0; i < t.P; ++i) plan_out[i] = uint8_t(pr.plan[i]);
    if (bound_out) *bound_out = pr.bound;
    if (flags_out) *flags_out = pr.flags;
    if (loaded_out) *loaded_out = uint64_t(pr.loaded);
    return IPC_OK;
  } catch (...) {
    return IPC_ENOMEM;
  }
}

ipc_status ipc_compress_batch(ipc_ctx *ctx, uint32_t n, const void *const *fields_dev,
                              const uint64_t *dims, int ndim, int dtype, const double *abs_eb,
                              const ipc_options *opts, ipc_stream **out) {
  TraceRange trace_range("ipc_compress_batch");
  if (!out) return IPC_EINVAL;
  for (uint32_t i = 0; i < n; ++i) out[i] = nullptr;
  if (!ctx || n == 0 || !fields_dev || !dims || !abs_eb) return IPC_EINVAL;
  if (ndim < 1 || ndim > 3 || (dtype != IPC_F32 && dtype != IPC_F64)) {
    set_err(ctx, "invalid argument to ipc_compress_batch");
    return IPC_EINVAL;
  }
  int interp = opts ? opts->interp : IPC_CUBIC;
  // all fields on the fused 3-D path, or all on the one-pass-per-launch path
  bool fused = n > 1 && (interp == IPC_LINEAR || interp == IPC_CUBIC);
  bool passes = fused;
  for (uint32_t i = 0; i < n; ++i) {
    if (!fields_dev[i] || !(std::isfinite(abs_eb[i]) && abs_eb[i] > 0)) {
      set_err(ctx, "invalid field or error bound in ipc_compress_batch");
      return IPC_EINVAL;
    }
    const bool f = fused_dims(dims + size_t(i) * ndim, ndim, opts);
    fused = fused && f;
    passes = passes && !f;
  }
  auto undo = [&](uint32_t upto) {
    for (uint32_t j = 0; j < upto; ++j) {
      ipc_stream_free(out[j]);
      out[j] = nullptr;
    }
  };
  if (!fused && !passes) {
    // one call per field (a mix of paths, or one field)
    for (uint32_t i = 0; i < n; ++i) {
      ipc_status st = ipc_compress(ctx, fields_dev[i], dims + size_t(i) * ndim, ndim, dtype, abs_eb[i],
                                   opts, &out[i]);
      if (st != IPC_OK) {
        undo(i);
        return st;
      }
    }
    return IPC_OK;
  }
  std::vector<ipc_stream *> ss(n, nullptr);
  std::vector<char> redo(n, 0);
  ipc_status st = guarded(ctx, [&] {
    enter_device(ctx);
    for (uint32_t i = 0; i < n; ++i) {
      ss[i] = new ipc_stream();
      ss[i]->ctx = ctx;
      setup_stream(ctx, ss[i], dims + size_t(i) * ndim, ndim, dtype, interp, abs_eb[i], opts);
    }
    if (fused) {
      // queue launches from a captured graph when the context asks for them
      // and the batch fits the table; otherwise one direct launch per level
      std::vector<const ipc_stream *> cs(ss.begin(), ss.end());
      bool done = false;
      if (batch_wants_graphs(ctx, cs, true) && queue_fits(cs)) {
        done = dtype == IPC_F32 ? compress_batch_queue<float>(ctx, ss, fields_dev, abs_eb, redo)
                                : compress_batch_queue<double>(ctx, ss, fields_dev, abs_eb, redo);
        if (!done) ctx->batch_graphs = 0;  // this stream cannot be captured
      }
      if (!done) {
        if (dtype == IPC_F32)
          compress_batch_fused<float>(ctx, ss, fields_dev, abs_eb, redo);
        else
          compress_batch_fused<double>(ctx, ss, fields_dev, abs_eb, redo);
      }
    } else {
      if (dtype == IPC_F32)
        compress_batch_passes<float>(ctx, ss, fields_dev, abs_eb, redo);
      else
        compress_batch_passes<double>(ctx, ss, fields_dev, abs_eb, redo);
    }
  });
  if (st != IPC_OK) {
    for (ipc_stream *s : ss)
      if (s) {
        free_stream_bufs(s);
        delete s;
      }
    return st;
  }
  for (uint32_t i = 0; i < n; ++i) out[i] = ss[i];
  // fields whose outliers overflowed the batch's record capacity: again alone
  // (ipc_compress applies the options to them)
  for (uint32_t i = 0; i < n; ++i) {
    ipc_status st2 = IPC_OK;
    if (redo[i]) {
      ipc_stream_free(out[i]);
      out[i] = nullptr;
      st2 = ipc_compress(ctx, fields_dev[i], dims + size_t(i) * ndim, ndim, dtype, abs_eb[i], opts, &out[i]);
    } else {
      st2 = finish_options(ctx, out[i], fields_dev[i], opts);
    }
    if (st2 != IPC_OK) {
      undo(n);
      return st2;
    }
  }
  return IPC_OK;
}

ipc_status ipc_retrieve_batch(ipc_ctx *ctx, uint32_t n, const ipc_stream *const *streams,
                              const ipc_target *targets, ipc_state **out, ipc_info *info) {
  TraceRange trace_range("ipc_retrieve_batch");
  if (!out) return IPC_EINVAL;
  for (uint32_t i = 0; i < n; ++i) out[i] = nullptr;
  if (!ctx || n == 0 || !streams || !targets) return IPC_EINVAL;
  // all streams on the fused 3-D path, or all on the one-pass-per-launch
  // path, with one dtype and interpolation
  bool fused = n > 1, passes = n > 1;
  for (uint32_t i = 0; i < n; ++i) {
    const ipc_stream *s = streams[i];
    if (!s) return IPC_EINVAL;
    if (s->ctx != ctx) {
      set_err(ctx, "stream belongs to another context");
      return IPC_ESTATE;
    }
    if (!valid_target(targets[i])) {
      set_err(ctx, "target value must be finite and > 0");
      return IPC_EINVAL;
    }
    const bool same = s->meta.dtype == streams[0]->meta.dtype && s->meta.interp == streams[0]->meta.interp;
    const bool f = fused3(s->meta.sched);
    fused = fused && f && same;
    passes = passes && !f && same;
  }
  if (!fused && !passes) {
    for (uint32_t i = 0; i < n; ++i) {
      ipc_status st = ipc_retrieve(ctx, streams[i], targets[i], &out[i], info ? info + i : nullptr);
      if (st != IPC_OK) {
        for (uint32_t j = 0; j < i; ++j) {
          ipc_state_free(out[j]);
          out[j] = nullptr;
        }
        return st;
      }
    }
    return IPC_OK;
  }
  std::vector<const ipc_stream *> ss(streams, streams + n);
  std::vector<PlanResult> prs(n);
  std::vector<float> tplan(n);
  std::vector<std::vector<int>> plans(n);
  parallel_for(n, [&](size_t i) {
    auto t0 = std::chrono::steady_clock::now();
    prs[i] = plan_request(ss[i]->tables, targets[i].kind, targets[i].value, nullptr);
    tplan[i] = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    plans[i] = prs[i].plan;
  });
  std::vector<ipc_state *> sts(n, nullptr);
  ipc_status st = guarded(ctx, [&] {
    enter_device(ctx);
    std::vector<void *> fields(n);
    for (uint32_t i = 0; i < n; ++i) {
      sts[i] = new ipc_state();
      sts[i]->ctx = ctx;
      sts[i]->stream = ss[i];
      sts[i]->plan = plans[i];
      sts[i]->bound = prs[i].bound;
      const size_t isz = ss[i]->meta.dtype == IPC_F32 ? 4 : 8;
      sts[i]->field = dev_alloc(ctx, size_t(ss[i]->meta.sched.n_points) * isz);
      fields[i] = sts[i]->field.p;
    }
    hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
    if (fused) {
      std::vector<int> ls(n);
      for (uint32_t i = 0; i < n; ++i) ls[i] = ss[i]->meta.sched.K;
      if (ss[0]->meta.dtype == IPC_F32)
        retrieve_batch_levels<float>(ctx, ss, plans, fields, ls);
      else
        retrieve_batch_levels<double>(ctx, ss, plans, fields, ls);
    } else {
      std::vector<int> start(n, 0);
      if (ss[0]->meta.dtype == IPC_F32)
        retrieve_batch_passes<float>(ctx, ss, plans, fields, start);
      else
        retrieve_batch_passes<double>(ctx, ss, plans, fields, start);
    }
    hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
    hip_check(ctx, hipEventSynchronize(ctx->ev1), "retrieve");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    if (info)
      for (uint32_t i = 0; i < n; ++i) {
        std::vector<int> none(plans[i].size(), 32);
        fill_info(ss[i], plans[i], prs[i].bound, prs[i].flags, plane_bytes_between(ss[i], plans[i], none),
                  tplan[i], ms, info + i);
      }
  });
  if (st != IPC_OK) {
    for (ipc_state *t : sts)
      if (t) {
        dev_free(ctx, t->field);
        delete t;
      }
    return st;
  }
  for (uint32_t i = 0; i < n; ++i) out[i] = sts[i];
  return IPC_OK;
}

ipc_status ipc_autotune(ipc_ctx *ctx, const void *field_dev, const uint64_t *dims, int ndim,
                        int dtype, double abs_eb, const ipc_options *opts, int32_t *zseg_c,
                        int32_t *zseg_r, uint32_t capacity) {
  if (!ctx || !field_dev || !dims) return IPC_EINVAL;
  // a 2-D field's columns are one chunk row long: no column length to choose
  if (ndim != 3 || !fused_dims(dims, ndim, opts)) {
    set_err(ctx, "no tunable launches for this shape (3-D fields with the default chunks only)");
    return IPC_EUNSUPPORTED;
  }
  const bool prof = ctx->profiling;
  const int only = ctx->prof_only;
  ctx->profiling = true;
  ctx->prof_only = -1;
  const int cand[5] = {16, 8, 4, 2, 1};
  float best_c[32], best_r[32];
  int32_t zc[32], zr[32];
  for (int l = 0; l < 32; ++l) {
    best_c[l] = best_r[l] = 1e30f;
    zc[l] = zr[l] = 0;
  }
  ipc_status st = IPC_OK;
  int K = 0;
  // every candidate column length for every level at once, twice; the
  // fastest launch of each level wins (results do not depend on it)
  for (int rep = 0; rep < 2 && st == IPC_OK; ++rep)
    for (int c : cand) {
      ctx->forced_zseg = c;
      ipc_stream *s = nullptr;
      st = ipc_compress(ctx, field_dev, dims, ndim, dtype, abs_eb, opts, &s);
      if (st != IPC_OK) break;
      const Schedule &sc = s->meta.sched;
      K = sc.K;
      std::vector<float> tc = ctx->pass_ms;
      ipc_state *rs = nullptr;
      ipc_target t;
      t.kind = IPC_TARGET_EB;
      t.value = abs_eb;
      st = ipc_retrieve(ctx, s, t, &rs, nullptr);
      if (st != IPC_OK) {
        ipc_stream_free(s);
        break;
      }
      std::vector<float> tr = ctx->pass_ms;
      for (int l = 1; l <= sc.K && l < 32; ++l) {
        const size_t slot = size_t(level_last_pass(sc, l));
        if (slot < tc.size() && tc[slot] > 0 && tc[slot] < best_c[l]) {
          best_c[l] = tc[slot];
          zc[l] = c;
        }
        if (slot < tr.size() && tr[slot] > 0 && tr[slot] < best_r[l]) {
          best_r[l] = tr[slot];
          zr[l] = c;
        }
      }
      ipc_state_free(rs);
      ipc_stream_free(s);
    }
  ctx->forced_zseg = 0;
  ctx->profiling = prof;
  ctx->prof_only = only;
  if (st != IPC_OK) return st;
  int64_t d64[3] = {1, 1, 1};
  for (int j = 0; j < ndim; ++j) d64[3 - ndim + j] = int64_t(dims[j]);
  TuneKey k{{d64[0], d64[1], d64[2]}, dtype, opts ? opts->interp : IPC_CUBIC};
  TuneVal v;
  std::memcpy(v.zseg_c, zc, sizeof(zc));
  std::memcpy(v.zseg_r, zr, sizeof(zr));
  ctx->tuned[k] = v;
  for (uint32_t l = 0; l < capacity && l < 32; ++l) {
    if (zseg_c) zseg_c[l] = int(l) <= K ? zc[l] : 0;
    if (zseg_r) zseg_r[l] = int(l) <= K ? zr[l] : 0;
  }
  return IPC_OK;
}

ipc_status ipc_autotune_batch(ipc_ctx *ctx, const void *field_dev, const uint64_t *dims, int ndim,
                              int dtype, double abs_eb, const ipc_options *opts, uint32_t copies,
                              int32_t choice[4]) {
  if (!ctx || !field_dev || !dims || copies < 1 || copies > 64) return IPC_EINVAL;
  if (!fused_dims(dims, ndim, opts)) {
    set_err(ctx, "no batch schedule to choose for this shape (fused 3-D and 2-D fields only)");
    return IPC_EUNSUPPORTED;
  }
  const int saved = ctx->batch_graphs;
  // candidate schedules: direct launches (0), then graph replays with a full
  // queue slot of that many workgroups per CU
  const bool f32 = dtype == IPC_F32;
  const std::vector<int> cand_r = f32 ? std::vector<int>{0, 3, 4, 5} : std::vector<int>{0, 2, 3, 4};
  const std::vector<int> cand_c = f32 ? std::vector<int>{0, 2, 3, 4} : std::vector<int>{0, 1, 2};
  std::vector<const void *> fields(copies, field_dev);
  std::vector<uint64_t> dd(size_t(copies) * size_t(ndim));
  std::vector<double> ebs(copies, abs_eb);
  for (uint32_t i = 0; i < copies; ++i)
    for (int j = 0; j < ndim; ++j) dd[size_t(i) * ndim + j] = dims[j];
  int64_t d64[3] = {1, 1, 1};
  for (int j = 0; j < ndim; ++j) d64[3 - ndim + j] = int64_t(dims[j]);
  const TuneKey k{{d64[0], d64[1], d64[2]}, dtype, opts ? opts->interp : IPC_CUBIC};
  double best_r = 1e30, best_c = 1e30;
  int pick_r = 0, pick_c = 0;
  ipc_status st = IPC_OK;
  std::vector<ipc_stream *> ss(copies, nullptr);
  std::vector<ipc_state *> sts(copies, nullptr);
  std::vector<ipc_target> tg(copies);
  for (ipc_target &t : tg) {
    t.kind = IPC_TARGET_EB;
    t.value = abs_eb;
  }
  auto free_all = [&] {
    for (ipc_state *&x : sts) {
      if (x) ipc_state_free(x);
      x = nullptr;
    }
    for (ipc_stream *&x : ss) {
      if (x) ipc_stream_free(x);
      x = nullptr;
    }
  };
  // every candidate three times, in turns; a schedule is tried on the shape
  // as the automatic mode would run it (a forced entry in the table)
  for (int rep = 0; rep < 3 && st == IPC_OK; ++rep) {
    for (size_t ci = 0; ci < std::max(cand_r.size(), cand_c.size()) && st == IPC_OK; ++ci) {
      BatchTune bt;
      bt.graphs_c = ci < cand_c.size() && cand_c[ci] != 0;
      bt.per_cu_c = ci < cand_c.size() ? uint32_t(cand_c[ci]) : 0u;
      bt.graphs_r = ci < cand_r.size() && cand_r[ci] != 0;
      bt.per_cu_r = ci < cand_r.size() ? uint32_t(cand_r[ci]) : 0u;
      ctx->tuned_batch[k] = bt;
      ctx->batch_graphs = 2;
      auto t0 = std::chrono::steady_clock::now();
      st = ipc_compress_batch(ctx, copies, fields.data(), dd.data(), ndim, dtype, ebs.data(), opts, ss.data());
      auto t1 = std::chrono::steady_clock::now();
      if (st != IPC_OK) break;
      st = ipc_retrieve_batch(ctx, copies, ss.data(), tg.data(), sts.data(), nullptr);
      auto t2 = std::chrono::steady_clock::now();
      if (st != IPC_OK) break;
      const double tc = std::chrono::duration<double>(t1 - t0).count();
      const double tr = std::chrono::duration<double>(t2 - t1).count();
      if (ci < cand_c.size() && tc < best_c) {
        best_c = tc;
        pick_c = cand_c[ci];
      }
      if (ci < cand_r.size() && tr < best_r) {
        best_r = tr;
        pick_r = cand_r[ci];
      }
      free_all();
    }
  }
  free_all();
  ctx->batch_graphs = saved;
  if (st != IPC_OK) {
    ctx->tuned_batch.erase(k);
    return st;
  }
  BatchTune bt;
  bt.graphs_r = pick_r != 0;
  bt.per_cu_r = uint32_t(pick_r);
  bt.graphs_c = pick_c != 0;
  bt.per_cu_c = uint32_t(pick_c);
  ctx->tuned_batch[k] = bt;
  if (choice) {
    choice[0] = bt.graphs_c;
    choice[1] = int32_t(bt.per_cu_c);
    choice[2] = bt.graphs_r;
    choice[3] = int32_t(bt.per_cu_r);
  }
  return IPC_OK;
}

ipc_status ipc_autotune_set(ipc_ctx *ctx, const uint64_t *dims, int ndim, int dtype, int interp,
                            const int32_t *zseg_c, const int32_t *zseg_r, uint32_t n) {
  if (!ctx || !dims || ndim < 1 || ndim > 3 || !zseg_c || !zseg_r) return IPC_EINVAL;
  TuneVal v;
  std::memset(&v, 0, sizeof(v));
  for (uint32_t l = 0; l < n && l < 32; ++l) {
    if (zseg_c[l] < 0 || zseg_c[l] > 1024 || zseg_r[l] < 0 || zseg_r[l] > 1024) return IPC_EINVAL;
    v.zseg_c[l] = zseg_c[l];
    v.zseg_r[l] = zseg_r[l];
  }
  int64_t d64[3] = {1, 1, 1};
  for (int j = 0; j < ndim; ++j) d64[3 - ndim + j] = int64_t(dims[j]);
  ctx->tuned[TuneKey{{d64[0], d64[1], d64[2]}, dtype, interp}] = v;
  return IPC_OK;
}

ipc_status ipc_autotune_clear(ipc_ctx *ctx) {
  if (!ctx) return IPC_EINVAL;
  ctx->tuned.clear();
  ctx->tuned_batch.clear();
  return IPC_OK;
}

ipc_status ipc_serve_batch(ipc_ctx *ctx, uint32_t n, ipc_request *req) {
  TraceRange trace_range("ipc_serve_batch");
  if (!ctx || (n && !req)) return IPC_EINVAL;
  // plan every request; refinements that need nothing finish here
  struct Job {
    uint32_t r;
    const ipc_stream *s;
    ipc_state *st;
    PlanResult pr;
    int l_start;
    float tplan;
    uint64_t read;
    int s_min;  // first pass to recompute (0 for a new retrieval)
  };
  std::vector<Job> cand;  // requests that need a plan, in order
  std::vector<const ipc_state *> seen;
  for (uint32_t i = 0; i < n; ++i) {
    ipc_request &q = req[i];
    q.status = IPC_OK;
    std::memset(&q.info, 0, sizeof(q.info));
    if (q.refine && q.state) {
      if (std::find(seen.begin(), seen.end(), q.state) != seen.end()) {
        q.status = IPC_EINVAL;  // one request per state and batch
        continue;
      }
      seen.push_back(q.state);
    }
    const ipc_stream *s = q.refine ? (q.state ? q.state->stream : nullptr) : q.stream;
    if (!s || !valid_target(q.target) || (q.refine && q.state->ctx != ctx) || (!q.refine && q.state)) {
      q.status = IPC_EINVAL;
      continue;
    }
    if (s->ctx != ctx) {
      q.status = IPC_ESTATE;
      continue;
    }
    if (q.refine && (q.target.kind & ~IPC_TARGET_LEVEL_GROUPS) == IPC_TARGET_EB &&
        q.target.value >= q.state->bound) {
      fill_info(s, q.state->plan, q.state->bound, IPC_FLAG_NOOP, 0, 0.0f, 0.0f, &q.info);
      continue;
    }
    cand.push_back(Job{i, s, q.refine ? q.state : nullptr, PlanResult(), s->meta.sched.K, 0.0f, 0, 0});
  }
  // the plans, on several host threads
  ipc_status pst = IPC_OK;
  try {
    parallel_for(cand.size(), [&](size_t k) {
      Job &j = cand[k];
      const ipc_request &q = req[j.r];
      auto t0 = std::chrono::steady_clock::now();
      j.pr = plan_request(j.s->tables, q.target.kind, q.target.value, j.st ? j.st->plan.data() : nullptr);
      j.tplan = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
  } catch (...) {
    pst = IPC_ENOMEM;
  }
  if (pst != IPC_OK) {
    for (Job &j : cand) req[j.r].status = pst;
    return pst;
  }
  std::vector<Job> jobs;
  for (Job &j : cand) {
    ipc_request &q = req[j.r];
    const ipc_stream *s = j.s;
    if (j.st) {
      ipc_state *st = j.st;
      if (j.pr.plan == st->plan) {
        fill_info(s, st->plan, st->bound, j.pr.flags | IPC_FLAG_NOOP, 0, j.tplan, 0.0f, &q.info);
        continue;
      }
      int s_min = 0;
      while (s_min < int(j.pr.plan.size()) && j.pr.plan[s_min] >= st->plan[s_min]) ++s_min;
      j.read = plane_bytes_between(s, j.pr.plan, st->plan);
      j.s_min = s_min;
      j.l_start = s->meta.sched.passes[size_t(s_min)].level;
      if (s_min == 0) j.l_start = s->meta.sched.K;
    } else {
      std::vector<int> none(j.pr.plan.size(), 32);
      j.read = plane_bytes_between(s, j.pr.plan, none);
    }
    jobs.push_back(j);
  }
  if (jobs.empty()) return IPC_OK;
  // fused 3-D jobs of one dtype / interpolation share the level launches,
  // jobs on the one-pass-per-launch path of one dtype / interpolation share
  // the pass launches; the others run one at a time
  const ipc_stream *s0 = nullptr, *p0 = nullptr;
  std::vector<size_t> fused_idx, pass_idx, other_idx;
  auto same = [](const ipc_stream *a, const ipc_stream *b) {
    return a->meta.dtype == b->meta.dtype && a->meta.interp == b->meta.interp;
  };
  for (size_t k = 0; k < jobs.size(); ++k) {
    const ipc_stream *s = jobs[k].s;
    if (fused3(s->meta.sched)) {
      if (!s0) s0 = s;
      (same(s, s0) ? fused_idx : other_idx).push_back(k);
    } else {
      if (!p0) p0 = s;
      (same(s, p0) ? pass_idx : other_idx).push_back(k);
    }
  }
  std::vector<ipc_state *> fresh(jobs.size(), nullptr);  // new states of this call
  ipc_status st = guarded(ctx, [&] {
    enter_device(ctx);
    std::vector<const ipc_stream *> ss;
    std::vector<std::vector<int>> plans;
    std::vector<void *> fields;
    std::vector<int> ls;
    std::vector<const ipc_stream *> ps;
    std::vector<std::vector<int>> pplans;
    std::vector<void *> pfields;
    std::vector<int> pstart;
    for (size_t k : fused_idx) {
      Job &j = jobs[k];
      void *f;
      if (j.st) {
        f = j.st->field.p;
      } else {
        ipc_state *t = new ipc_state();
        t->ctx = ctx;
        t->stream = j.s;
        const size_t isz = j.s->meta.dtype == IPC_F32 ? 4 : 8;
        try {
          t->field = dev_alloc(ctx, size_t(j.s->meta.sched.n_points) * isz);
        } catch (...) {
          delete t;
          throw;
        }
        fresh[k] = t;
        f = t->field.p;
      }
      ss.push_back(j.s);
      plans.push_back(j.pr.plan);
      fields.push_back(f);
      ls.push_back(j.l_start);
    }
    for (size_t k : pass_idx) {
      Job &j = jobs[k];
      void *f;
      if (j.st) {
        f = j.st->field.p;
      } else {
        ipc_state *t = new ipc_state();
        t->ctx = ctx;
        t->stream = j.s;
        const size_t isz = j.s->meta.dtype == IPC_F32 ? 4 : 8;
        try {
          t->field = dev_alloc(ctx, size_t(j.s->meta.sched.n_points) * isz);
        } catch (...) {
          delete t;
          throw;
        }
        fresh[k] = t;
        f = t->field.p;
      }
      ps.push_back(j.s);
      pplans.push_back(j.pr.plan);
      pfields.push_back(f);
      pstart.push_back(j.s_min);
    }
    hip_check(ctx, hipEventRecord(ctx->ev0, ctx->stream), "event");
    if (!ss.empty()) {
      if (ss[0]->meta.dtype == IPC_F32)
        retrieve_batch_levels<float>(ctx, ss, plans, fields, ls);
      else
        retrieve_batch_levels<double>(ctx, ss, plans, fields, ls);
    }
    if (!ps.empty()) {
      if (ps[0]->meta.dtype == IPC_F32)
        retrieve_batch_passes<float>(ctx, ps, pplans, pfields, pstart);
      else
        retrieve_batch_passes<double>(ctx, ps, pplans, pfields, pstart);
    }
    hip_check(ctx, hipEventRecord(ctx->ev1, ctx->stream), "event");
    hip_check(ctx, hipEventSynchronize(ctx->ev1), "serve");
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    for (const std::vector<size_t> *idx : {&fused_idx, &pass_idx})
      for (size_t k : *idx) {
        Job &j = jobs[k];
        ipc_request &q = req[j.r];
        ipc_state *t = j.st ? j.st : fresh[k];
        t->plan = j.pr.plan;
        t->bound = j.pr.bound;
        if (!j.st) q.state = t;
        fill_info(j.s, t->plan, t->bound, j.pr.flags, j.read, j.tplan, ms, &q.info);
      }
  });
  if (st != IPC_OK) {
    for (const std::vector<size_t> *idx : {&fused_idx, &pass_idx})
      for (size_t k : *idx) {
        req[jobs[k].r].status = st;
        req[jobs[k].r].state = jobs[k].st;
      }
    for (ipc_state *t : fresh)
      if (t) {
        dev_free(ctx, t->field);
        delete t;
      }
    return st;
  }
  for (size_t k : other_idx) {
    Job &j = jobs[k];
    ipc_request &q = req[j.r];
    if (j.st) {
      q.status = ipc_refine(ctx, j.st, q.target, &q.info);
    } else {
      ipc_state *t = nullptr;
      q.status = retrieve_common(ctx, j.s, j.pr.plan, j.pr.bound, j.pr.flags, j.tplan, &t, &q.info);
      if (q.status == IPC_OK) q.state = t;
    }
  }
  return IPC_OK;
}

}  // extern "C"
