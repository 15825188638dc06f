// Queries that arrive in host memory (Section 5.2.1: the query batch is cut into chunks that are copied
// to the device, answered and copied back, with a chunk's copy overlapping the previous chunk's kernels
// and at most two chunks resident on the device; Sections 6.3.2-6.3.4 compare page-locked and pageable
// query arrays).
//
// Device memory of a call: two slots of (symbols, arguments, answers) of one chunk each, and one query
// scratch (binning buffers), shared by the chunks because their kernels run one after the other.
// Dependencies of chunk i in slot s = i mod 2:
//   copy-in(i)  after the kernels of chunk i-2 (they read slot s's inputs)
//   kernels(i)  after copy-in(i), the kernels of chunk i-1 (shared scratch, one chunk's kernels at a
//               time) and copy-out(i-2) (slot s's answers)
//   copy-out(i) after kernels(i)
// Page-locked host arrays: these nodes form one HIP graph (copy nodes need page-locked memory; each
// chunk's kernels are a child graph captured from the ordinary query path), instantiated once and kept
// for repeated calls with the same tree, arrays and sizes. Pageable host arrays: the host copies each
// chunk through two page-locked staging slots (queries in, answers out) on its own threads while the
// device works on the neighbouring chunks; the device side is the same three-stage pipeline on streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "wt_host.h"
#include "wt_internal.h"
#include "wt_query_dev.h"

namespace wt {

bool is_pinned(const void* p) {
  if (!p) return true;
  hipPointerAttribute_t attr;
  const hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeHost;
}

// Host memcpy split over a few threads (a single thread does not reach the host's memory bandwidth).
void par_copy(void* dst, const void* src, size_t bytes) {
  constexpr size_t kPiece = 4u << 20;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nt = std::min<size_t>(std::min<size_t>(8, hw), (bytes + kPiece - 1) / kPiece);
  if (nt <= 1) {
    std::memcpy(dst, src, bytes);
    return;
  }
  const size_t per = (bytes + nt - 1) / nt;
  std::vector<std::thread> th;
  for (size_t k = 1; k < nt; ++k) {
    const size_t a = k * per, b = std::min(bytes, a + per);
    if (a < b) th.emplace_back([=] { std::memcpy((char*)dst + a, (const char*)src + a, b - a); });
  }
  std::memcpy(dst, src, std::min(bytes, per));
  for (auto& x : th) x.join();
}

namespace {

constexpr uint64_t kDefaultChunk = 1ull << 22;

// Device buffers of one call: two slots and the shared scratch.
struct Slots {
  char* block = nullptr;
  uint32_t* sym[2];
  uint64_t* arg[2];
  char* out[2];
  char* scratch;
};

size_t slot_layout(uint64_t chunk, Slots* s, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  size_t o_sym[2], o_arg[2], o_out[2];
  for (int k = 0; k < 2; ++k) {
    o_sym[k] = take(4 * chunk);
    o_arg[k] = take(8 * chunk);
    o_out[k] = take(8 * chunk);
  }
  const size_t o_scr = take(query_scratch_bytes(chunk));
  if (s && base) {
    for (int k = 0; k < 2; ++k) {
      s->sym[k] = (uint32_t*)(base + o_sym[k]);
      s->arg[k] = (uint64_t*)(base + o_arg[k]);
      s->out[k] = base + o_out[k];
    }
    s->scratch = base + o_scr;
  }
  return off;
}

// An instantiated graph of a page-locked call, kept for repeated calls with the same arguments.
struct GraphKey {
  uint64_t tree;  // the tree's uid (a freed tree's address may come back for another tree)
  int kind;
  const void *sym, *arg, *out;
  uint64_t q, chunk;
  uint32_t version;
  bool operator==(const GraphKey& o) const {
    return tree == o.tree && kind == o.kind && sym == o.sym && arg == o.arg && out == o.out && q == o.q &&
           chunk == o.chunk && version == o.version;
  }
};

struct GraphCache {
  bool valid = false;
  GraphKey key{};
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  Slots slots{};
  int device = -1;
  void drop() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (slots.block) dev_free(slots.block, nullptr);
    exec = nullptr;
    graph = nullptr;
    slots = Slots{};
    valid = false;
  }
};

std::mutex g_cache_mu;
GraphCache g_cache;
uint32_t g_cache_version = 0;  // bumped by wt_query_host_release

// Page-locked staging of the pageable path (grown on demand, kept until wt_query_host_release).
struct Staging {
  char* in[2] = {nullptr, nullptr};
  char* out[2] = {nullptr, nullptr};
  size_t in_bytes = 0, out_bytes = 0;
  void drop() {
    for (int k = 0; k < 2; ++k) {
      if (in[k]) (void)hipHostFree(in[k]);
      if (out[k]) (void)hipHostFree(out[k]);
      in[k] = out[k] = nullptr;
    }
    in_bytes = out_bytes = 0;
  }
};
std::mutex g_stage_mu;
Staging g_stage;

struct Streams {
  hipStream_t in = nullptr, comp = nullptr, out = nullptr;
  hipEvent_t ev[8] = {};
  ~Streams() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (in) (void)hipStreamDestroy(in);
    if (comp) (void)hipStreamDestroy(comp);
    if (out) (void)hipStreamDestroy(out);
  }
  hipError_t init() {
    hipError_t e = hipStreamCreateWithFlags(&in, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&comp, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&out, hipStreamNonBlocking);
    for (int k = 0; k < 8 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
    return e;
  }
};

// Enqueues the device side of a call on the three streams: per chunk, copy-in on ss.in, the chunk's
// kernels on ss.comp, copy-out on ss.out, with the dependencies of the file header expressed by events.
// src_sym / src_arg / dst_out give the host addresses of chunk i (page-locked). Nothing here waits on the
// host, so the same sequence is recorded into the graph by stream capture.
template <typename SrcFn, typename DstFn>
wt_status enqueue_chunks(const wt_tree* t, int kind, uint64_t q, uint64_t chunk, const Slots& S, Streams& ss,
                         SrcFn src, DstFn dst) {
  const size_t ob = kind == 0 ? 4 : 8;
  hipEvent_t* e_in = ss.ev;
  hipEvent_t* e_k = ss.ev + 2;
  hipEvent_t* e_out = ss.ev + 4;
  const uint64_t nch = ceil_div(q, chunk);
  for (uint64_t i = 0; i < nch; ++i) {
    const int s = (int)(i & 1);
    const uint64_t a = i * chunk, m = std::min(chunk, q - a);
    const void* hsym = nullptr;
    const void* harg = nullptr;
    src(i, &hsym, &harg);
    // copy-in: slot s's inputs are free once the kernels of chunk i-2 are done
    if (i >= 2) WT_HIP(hipStreamWaitEvent(ss.in, e_k[s], 0));
    WT_HIP(hipMemcpyAsync(S.arg[s], harg, 8 * m, hipMemcpyHostToDevice, ss.in));
    if (kind != 0) WT_HIP(hipMemcpyAsync(S.sym[s], hsym, 4 * m, hipMemcpyHostToDevice, ss.in));
    WT_HIP(hipEventRecord(e_in[s], ss.in));
    // kernels: after the copy-in, the previous chunk's kernels (same stream) and the copy-out of chunk i-2
    WT_HIP(hipStreamWaitEvent(ss.comp, e_in[s], 0));
    if (i >= 2) WT_HIP(hipStreamWaitEvent(ss.comp, e_out[s], 0));
    const wt_status rc = query_run(t, kind, S.sym[s], S.arg[s], m, S.out[s], ss.comp, S.scratch);
    if (rc != WT_OK) return rc;
    WT_HIP(hipEventRecord(e_k[s], ss.comp));
    // copy-out after the kernels
    void* hout = dst(i);
    WT_HIP(hipStreamWaitEvent(ss.out, e_k[s], 0));
    WT_HIP(hipMemcpyAsync(hout, S.out[s], ob * m, hipMemcpyDeviceToHost, ss.out));
    WT_HIP(hipEventRecord(e_out[s], ss.out));
    (void)a;
  }
  return WT_OK;
}

// Graph of a page-locked call: the stream pipeline recorded by capture (fork from ss.comp into the two
// copy streams, join back at the end).
wt_status build_graph(const wt_tree* t, int kind, const uint32_t* h_sym, const uint64_t* h_arg, uint64_t q,
                      char* h_out, uint64_t chunk, const Slots& S, hipGraph_t* out) {
  Streams ss;
  WT_HIP(ss.init());
  const size_t ob = kind == 0 ? 4 : 8;
  WT_HIP(hipStreamBeginCapture(ss.comp, hipStreamCaptureModeThreadLocal));
  hipError_t he = hipEventRecord(ss.ev[6], ss.comp);
  if (he == hipSuccess) he = hipStreamWaitEvent(ss.in, ss.ev[6], 0);
  if (he == hipSuccess) he = hipStreamWaitEvent(ss.out, ss.ev[6], 0);
  wt_status rc = WT_OK;
  if (he == hipSuccess) {
    rc = enqueue_chunks(
        t, kind, q, chunk, S, ss,
        [&](uint64_t i, const void** hs, const void** ha) {
          *hs = h_sym ? (const void*)(h_sym + i * chunk) : nullptr;
          *ha = h_arg + i * chunk;
        },
        [&](uint64_t i) { return (void*)(h_out + i * chunk * ob); });
  }
  // join the copy streams back into the origin stream
  if (he == hipSuccess) he = hipEventRecord(ss.ev[7], ss.in);
  if (he == hipSuccess) he = hipStreamWaitEvent(ss.comp, ss.ev[7], 0);
  if (he == hipSuccess) he = hipEventRecord(ss.ev[6], ss.out);
  if (he == hipSuccess) he = hipStreamWaitEvent(ss.comp, ss.ev[6], 0);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(ss.comp, &g);
  if (rc != WT_OK || he != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    if (rc != WT_OK) return rc;
    return fail(WT_ERR_HIP, "wt_query_host: graph capture: %s", hipGetErrorString(he != hipSuccess ? he : ce));
  }
  *out = g;
  return WT_OK;
}

}  // namespace
}  // namespace wt

using namespace wt;

extern "C" wt_status wt_query_host(const wt_tree* t, int op, const uint32_t* h_sym, const uint64_t* h_arg, uint64_t q,
                                   void* h_out, const wt_host_opts* opts, wt_host_stats* stats, wt_stream_t stream) {
  clear_error();
  const auto t0 = std::chrono::steady_clock::now();
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (!t) return fail(WT_ERR_ARG, "wt_query_host: tree is NULL");
  if (op != WT_OP_ACCESS && op != WT_OP_RANK && op != WT_OP_SELECT)
    return fail(WT_ERR_ARG, "wt_query_host: op must be WT_OP_ACCESS, WT_OP_RANK or WT_OP_SELECT");
  if (q == 0) return WT_OK;
  const int kind = op;  // 0 access, 1 rank, 2 select
  if (!h_arg || !h_out || (kind != 0 && !h_sym)) return fail(WT_ERR_ARG, "wt_query_host: NULL buffer");
  uint64_t chunk = opts && opts->chunk ? opts->chunk : kDefaultChunk;
  if (chunk > (1ull << 28)) return fail(WT_ERR_ARG, "wt_query_host: chunk above 2^28 queries");
  chunk = std::min(chunk, q);
  const uint64_t nch = ceil_div(q, chunk);
  const size_t ob = kind == 0 ? 4 : 8;
  const bool pinned = is_pinned(h_arg) && (kind == 0 || is_pinned(h_sym)) && is_pinned(h_out);
  const bool use_graph = pinned && nch > 1 && !(opts && (opts->flags & WT_HOST_NO_GRAPH));
  hipStream_t st = (hipStream_t)stream;
  if (stats) {
    stats->chunks = (uint32_t)nch;
    stats->pinned = pinned;
    stats->graph = use_graph;
  }
  auto finish = [&]() {
    if (stats)
      stats->ms = (float)(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    return WT_OK;
  };

  if (use_graph) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    int dev = 0;
    WT_HIP(hipGetDevice(&dev));
    const GraphKey key{t->uid, kind, h_sym, h_arg, h_out, q, chunk, g_cache_version};
    if (!(g_cache.valid && g_cache.key == key && g_cache.device == dev)) {
      g_cache.drop();
      const size_t bytes = slot_layout(chunk, nullptr, nullptr);
      char* blk = (char*)dev_alloc(bytes, st);
      if (!blk) return fail(WT_ERR_OOM, "wt_query_host: %zu bytes of chunk buffers", bytes);
      WT_HIP(hipStreamSynchronize(st));  // the buffers are used from the graph's own streams
      g_cache.slots.block = blk;
      slot_layout(chunk, &g_cache.slots, blk);
      const wt_status rc = build_graph(t, kind, h_sym, h_arg, q, (char*)h_out, chunk, g_cache.slots, &g_cache.graph);
      if (rc != WT_OK) {
        g_cache.drop();
        return rc;
      }
      const hipError_t ie = hipGraphInstantiate(&g_cache.exec, g_cache.graph, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        g_cache.drop();
        return fail(WT_ERR_HIP, "wt_query_host: graph instantiation: %s", hipGetErrorString(ie));
      }
      g_cache.key = key;
      g_cache.device = dev;
      g_cache.valid = true;
    }
    WT_HIP(hipGraphLaunch(g_cache.exec, st));
    WT_HIP(hipStreamSynchronize(st));
    return finish();
  }

  // stream pipeline: page-locked arrays without a graph, or pageable arrays through the staging slots
  Streams ss;
  WT_HIP(ss.init());
  hipEvent_t* e_in = ss.ev;       // copy-in of slot s done
  hipEvent_t* e_k = ss.ev + 2;    // kernels of slot s done
  hipEvent_t* e_out = ss.ev + 4;  // copy-out of slot s done
  hipEvent_t e_start = ss.ev[6], e_end = ss.ev[7];
  Slots S{};
  const size_t bytes = slot_layout(chunk, nullptr, nullptr);
  S.block = (char*)dev_alloc(bytes, st);
  if (!S.block) return fail(WT_ERR_OOM, "wt_query_host: %zu bytes of chunk buffers", bytes);
  slot_layout(chunk, &S, S.block);
  // the work of the call starts after what the caller queued on `stream` (the buffer allocation)
  WT_HIP(hipEventRecord(e_start, st));
  WT_HIP(hipStreamWaitEvent(ss.in, e_start, 0));
  WT_HIP(hipStreamWaitEvent(ss.comp, e_start, 0));
  WT_HIP(hipStreamWaitEvent(ss.out, e_start, 0));
  const char* hs = (const char*)h_sym;
  const char* ha = (const char*)h_arg;
  char* ho = (char*)h_out;
  wt_status rc = WT_OK;
  if (pinned) {
    rc = enqueue_chunks(
        t, kind, q, chunk, S, ss,
        [&](uint64_t i, const void** s_, const void** a_) {
          *s_ = hs ? hs + i * chunk * 4 : nullptr;
          *a_ = ha + i * chunk * 8;
        },
        [&](uint64_t i) { return (void*)(ho + i * chunk * ob); });
  } else {
    std::lock_guard<std::mutex> stage_lock(g_stage_mu);
    const size_t need_in = 12 * chunk, need_out = 8 * chunk;
    if (g_stage.in_bytes < need_in || g_stage.out_bytes < need_out) {
      g_stage.drop();
      for (int k = 0; k < 2; ++k) {
        if (hipHostMalloc((void**)&g_stage.in[k], need_in, 0) != hipSuccess ||
            hipHostMalloc((void**)&g_stage.out[k], need_out, 0) != hipSuccess) {
          (void)hipGetLastError();
          g_stage.drop();
          dev_free(S.block, st);
          return fail(WT_ERR_OOM, "wt_query_host: page-locked staging of %zu bytes", 2 * (need_in + need_out));
        }
      }
      g_stage.in_bytes = need_in;
      g_stage.out_bytes = need_out;
    }
    // answers of chunk j: staging slot -> caller's array, once its copy-out is done
    auto drain = [&](uint64_t j) -> wt_status {
      const int s = (int)(j & 1);
      const uint64_t a = j * chunk, m = std::min(chunk, q - a);
      WT_HIP(hipEventSynchronize(e_out[s]));
      par_copy(ho + a * ob, g_stage.out[s], m * ob);
      return WT_OK;
    };
    for (uint64_t i = 0; i < nch && rc == WT_OK; ++i) {
      const int s = (int)(i & 1);
      const uint64_t a = i * chunk, m = std::min(chunk, q - a);
      // the host fills staging slot s once the copy-in of chunk i-2 has read it
      if (i >= 2) WT_HIP(hipEventSynchronize(e_in[s]));
      par_copy(g_stage.in[s], ha + a * 8, 8 * m);
      if (kind != 0) par_copy(g_stage.in[s] + 8 * chunk, hs + a * 4, 4 * m);
      if (i >= 2) WT_HIP(hipStreamWaitEvent(ss.in, e_k[s], 0));
      WT_HIP(hipMemcpyAsync(S.arg[s], g_stage.in[s], 8 * m, hipMemcpyHostToDevice, ss.in));
      if (kind != 0) WT_HIP(hipMemcpyAsync(S.sym[s], g_stage.in[s] + 8 * chunk, 4 * m, hipMemcpyHostToDevice, ss.in));
      WT_HIP(hipEventRecord(e_in[s], ss.in));
      WT_HIP(hipStreamWaitEvent(ss.comp, e_in[s], 0));
      if (i >= 2) WT_HIP(hipStreamWaitEvent(ss.comp, e_out[s], 0));
      rc = query_run(t, kind, S.sym[s], S.arg[s], m, S.out[s], ss.comp, S.scratch);
      if (rc != WT_OK) break;
      WT_HIP(hipEventRecord(e_k[s], ss.comp));
      // the staging slot of the answers is emptied (chunk i-2 drained) before chunk i's copy-out
      if (i >= 2) {
        rc = drain(i - 2);
        if (rc != WT_OK) break;
      }
      WT_HIP(hipStreamWaitEvent(ss.out, e_k[s], 0));
      WT_HIP(hipMemcpyAsync(g_stage.out[s], S.out[s], ob * m, hipMemcpyDeviceToHost, ss.out));
      WT_HIP(hipEventRecord(e_out[s], ss.out));
    }
    if (rc == WT_OK)
      for (uint64_t j = nch >= 2 ? nch - 2 : 0; j < nch && rc == WT_OK; ++j) rc = drain(j);
  }
  // everything of the call is done before the buffers go back to `stream`'s allocator
  WT_HIP(hipEventRecord(e_end, ss.in));
  WT_HIP(hipStreamWaitEvent(ss.out, e_end, 0));
  WT_HIP(hipEventRecord(e_end, ss.comp));
  WT_HIP(hipStreamWaitEvent(ss.out, e_end, 0));
  WT_HIP(hipEventRecord(e_end, ss.out));
  WT_HIP(hipStreamWaitEvent(st, e_end, 0));
  dev_free(S.block, st);
  WT_HIP(hipStreamSynchronize(st));
  if (rc != WT_OK) return rc;
  return finish();
}

extern "C" wt_status wt_query_host_release(void) {
  clear_error();
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    (void)hipDeviceSynchronize();
    g_cache.drop();
    ++g_cache_version;
  }
  std::lock_guard<std::mutex> g(g_stage_mu);
  g_stage.drop();
  return WT_OK;
}
