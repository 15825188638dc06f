// Serving loop over a resident forest with continuous batching.
//
// A trace of query batches (requests) is replayed on the server clock: a request becomes visible at
// its arrival time and is admitted, in arrival order, as soon as a slot (one stream) is free and its
// device buffers fit in what the memory budget has left (a first-fit arena carved once from device
// memory). When a slot frees up, the oldest waiting request takes it together with the waiting
// requests after it (in arrival order) while their total stays within the coalescing size: their
// queries are copied side by side into one device batch, answered by one run of the mixed-query
// kernels and copied back each to its own answer array, all on the slot's stream, so requests that
// arrive while others are on the GPU overlap with them; an event per slot is polled for completion.
// Latency = completion - arrival. With a simulated cost per query the same loop runs without a GPU
// (for tests of the scheduler).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

struct QTree;
size_t mixed_scratch_bytes(uint64_t q);
hipError_t mixed_enqueue(const QTree* qt, uint32_t ntrees, const uint32_t* d_tree, const uint8_t* d_op,
                         const uint32_t* d_sym, const uint64_t* d_arg, uint64_t q, uint64_t* d_out, char* sb,
                         uint32_t vshift, hipStream_t st);
wt_status forest_qtab(const wt_forest* f, hipStream_t st, const QTree** out);
uint32_t forest_count(const wt_forest* f);
uint32_t forest_vshift(const wt_forest* f);

namespace {

// First-fit allocator of byte ranges [0, size) (host bookkeeping only).
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t o2 = it->first + bytes;
        free_.erase(it);
        if (rest) free_[o2] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<uint32_t> reqs;  // the requests of the batch it runs
  size_t off = 0, bytes = 0;
  double sim_end = 0;
  // page-locked staging of batches within the coalescing size: the inputs packed in the device
  // layout (one copy up) and the answers (one copy down, then handed out to the requests)
  char* h_in = nullptr;
  uint64_t* h_ans = nullptr;
  bool staged = false;
};

// Bytes of the inputs of a batch of q queries in its device layout (tree, op, sym, arg).
size_t input_bytes(uint64_t q) {
  return round_up(4 * q, 256) + round_up(q, 256) + round_up(4 * q, 256) + round_up(8 * q, 256);
}

constexpr uint32_t kDefaultCoalesce = 16384;  // the size the mixed queries answer in one kernel
constexpr size_t kMaxGroup = 256;             // requests per coalesced batch

// Device bytes of one request: inputs, answers and the mixed-query scratch, each 256-byte aligned.
size_t request_bytes(uint64_t q) {
  return round_up(4 * q, 256) + round_up(q, 256) + round_up(4 * q, 256) + round_up(8 * q, 256) +
         round_up(8 * q, 256) + round_up(mixed_scratch_bytes(q), 256);
}

}  // namespace
}  // namespace wt

using namespace wt;

struct wt_server {
  const wt_forest* f = nullptr;
  std::vector<Slot> slots;
  uint64_t coalesce_q = wt::kDefaultCoalesce;
  char* arena_base = nullptr;
  size_t budget = 0;
  double sim_ns = 0;  // > 0: simulated execution, no GPU
  Arena arena;
};

extern "C" wt_status wt_server_create(const wt_forest* f, const wt_server_opts* opts, wt_server** out) {
  clear_error();
  if (!out) return fail(WT_ERR_ARG, "wt_server_create: out is NULL");
  *out = nullptr;
  uint32_t nslots = 8;  // measured: more slots than the 4 hardware queues still overlap copies better
  uint64_t budget = 4ull << 30;
  uint64_t coalesce = kDefaultCoalesce;
  double sim = 0;
  if (opts) {
    if (opts->slots) nslots = opts->slots;
    if (opts->mem_budget) budget = opts->mem_budget;
    if (opts->coalesce_q) coalesce = opts->coalesce_q;
    sim = opts->sim_ns_per_query;
  }
  if (nslots > 64) return fail(WT_ERR_ARG, "wt_server_create: at most 64 slots");
  if (!f && !(sim > 0)) return fail(WT_ERR_ARG, "wt_server_create: forest is NULL");
  wt_server* s = new wt_server();
  s->f = f;
  s->budget = budget;
  s->coalesce_q = coalesce;
  s->sim_ns = sim > 0 ? sim : 0;
  s->slots.resize(nslots);
  if (!s->sim_ns) {
    for (Slot& sl : s->slots) {
      hipError_t e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
      if (e != hipSuccess) {
        wt_server_destroy(s);
        return fail(WT_ERR_HIP, "wt_server_create: %s", hipGetErrorString(e));
      }
    }
    for (Slot& sl : s->slots) {
      if (hipHostMalloc((void**)&sl.h_in, input_bytes(coalesce), 0) != hipSuccess ||
          hipHostMalloc((void**)&sl.h_ans, 8 * coalesce, 0) != hipSuccess) {
        (void)hipGetLastError();
        wt_server_destroy(s);
        return fail(WT_ERR_OOM, "wt_server_create: page-locked staging of %llu queries per slot",
                    (unsigned long long)coalesce);
      }
    }
    s->arena_base = (char*)dev_alloc(budget, s->slots[0].st);
    if (!s->arena_base) {
      wt_server_destroy(s);
      return fail(WT_ERR_OOM, "wt_server_create: arena of %llu bytes", (unsigned long long)budget);
    }
    const hipError_t e = hipStreamSynchronize(s->slots[0].st);
    if (e != hipSuccess) {
      wt_server_destroy(s);
      return fail(WT_ERR_HIP, "wt_server_create: %s", hipGetErrorString(e));
    }
  }
  *out = s;
  return WT_OK;
}

extern "C" wt_status wt_server_destroy(wt_server* s) {
  clear_error();
  if (!s) return WT_OK;
  if (!s->sim_ns) (void)hipDeviceSynchronize();
  if (s->arena_base) dev_free(s->arena_base, nullptr);
  for (Slot& sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.h_in) (void)hipHostFree(sl.h_in);
    if (sl.h_ans) (void)hipHostFree(sl.h_ans);
  }
  if (!s->sim_ns) (void)hipDeviceSynchronize();
  delete s;
  return WT_OK;
}

extern "C" wt_status wt_server_run(wt_server* s, const wt_request* reqs, uint32_t count, wt_completion* comps,
                                   wt_serve_stats* stats) {
  clear_error();
  if (!s || (count && (!reqs || !comps))) return fail(WT_ERR_ARG, "wt_server_run: NULL argument");
  for (uint32_t i = 0; i < count; ++i) {
    if (i && reqs[i].arrival_s < reqs[i - 1].arrival_s)
      return fail(WT_ERR_ARG, "wt_server_run: requests must be sorted by arrival time (request %u)", i);
    if (reqs[i].q && !s->sim_ns && (!reqs[i].h_tree || !reqs[i].h_op || !reqs[i].h_arg || !reqs[i].h_out))
      return fail(WT_ERR_ARG, "wt_server_run: request %u has a NULL buffer", i);
    if (reqs[i].q >= (1ull << 32)) return fail(WT_ERR_ARG, "wt_server_run: request %u is too large", i);
  }
  const QTree* qt = nullptr;
  uint32_t ntrees = 0;
  if (!s->sim_ns) {
    const wt_status rc = forest_qtab(s->f, s->slots[0].st, &qt);
    if (rc != WT_OK) return rc;
    ntrees = forest_count(s->f);
  }
  s->arena.reset(s->budget);
  for (Slot& sl : s->slots) sl.busy = false;
  std::memset(comps, 0, sizeof(wt_completion) * count);
  const auto t0 = std::chrono::steady_clock::now();
  auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
  std::deque<uint32_t> pending;
  uint32_t next = 0, done = 0, in_flight = 0, peak_in_flight = 0, rejected = 0, batches = 0;
  wt_status err = WT_OK;
  while (done < count) {
    const double tnow = now();
    while (next < count && reqs[next].arrival_s <= tnow) pending.push_back(next++);
    bool progress = false;
    // completions
    for (uint32_t k = 0; k < s->slots.size(); ++k) {
      Slot& sl = s->slots[k];
      if (!sl.busy) continue;
      bool fin;
      if (s->sim_ns) {
        fin = tnow >= sl.sim_end;
      } else {
        const hipError_t e = hipEventQuery(sl.done);
        if (e != hipSuccess && e != hipErrorNotReady) {
          err = fail(WT_ERR_HIP, "wt_server_run: request %u: %s", sl.reqs.empty() ? 0u : sl.reqs[0],
                     hipGetErrorString(e));
          break;
        }
        fin = e == hipSuccess;
      }
      if (!fin) continue;
      if (sl.staged) {  // hand the answers out
        uint64_t at = 0;
        for (uint32_t r : sl.reqs) {
          if (reqs[r].q) std::memcpy(reqs[r].h_out, sl.h_ans + at, 8 * reqs[r].q);
          at += reqs[r].q;
        }
      }
      const double td = now();
      for (uint32_t r : sl.reqs) {
        comps[r].done_s = td;
        comps[r].status = WT_OK;
      }
      s->arena.release(sl.off, sl.bytes);
      sl.busy = false;
      in_flight -= (uint32_t)sl.reqs.size();
      done += (uint32_t)sl.reqs.size();
      progress = true;
    }
    if (err != WT_OK) break;
    // admission, in arrival order: the oldest waiting request and the ones after it while they coalesce
    while (!pending.empty()) {
      const uint32_t r = pending.front();
      const wt_request& R = reqs[r];
      if (request_bytes(R.q) > s->budget) {  // can never fit
        comps[r].arrival_s = R.arrival_s;
        comps[r].admit_s = comps[r].done_s = now();
        comps[r].status = WT_ERR_OOM;
        comps[r].slot = ~0u;
        pending.pop_front();
        ++rejected;
        ++done;
        progress = true;
        continue;
      }
      uint32_t k = 0;
      while (k < s->slots.size() && s->slots[k].busy) ++k;
      if (k == s->slots.size()) break;
      // the group: consecutive waiting requests (no rejected one among them) within the coalescing size
      size_t ng = 1;
      uint64_t total = R.q;
      bool any_sym = R.h_sym != nullptr;
      if (R.q <= s->coalesce_q) {
        while (ng < pending.size() && ng < kMaxGroup) {
          const wt_request& X = reqs[pending[ng]];
          if (total + X.q > s->coalesce_q) break;
          total += X.q;
          any_sym = any_sym || X.h_sym != nullptr;
          ++ng;
        }
      }
      const size_t need = request_bytes(total);
      size_t off = 0;
      if (!s->arena.alloc(need, &off)) break;
      Slot& sl = s->slots[k];
      const double tadm = now();
      sl.busy = true;
      sl.reqs.assign(pending.begin(), pending.begin() + (long)ng);
      sl.off = off;
      sl.bytes = need;
      for (uint32_t x : sl.reqs) {
        comps[x].arrival_s = reqs[x].arrival_s;
        comps[x].admit_s = tadm;
        comps[x].slot = k;
        comps[x].status = WT_ERR_STATE;  // until it completes
      }
      if (s->sim_ns) {
        sl.sim_end = tadm + s->sim_ns * 1e-9 * (double)total;
      } else {
        hipError_t e = hipSuccess;
        if (total) {
          char* b = s->arena_base + off;
          uint32_t* d_tree = (uint32_t*)b;
          uint8_t* d_op = (uint8_t*)(b + round_up(4 * total, 256));
          uint32_t* d_sym = (uint32_t*)((char*)d_op + round_up(total, 256));
          uint64_t* d_arg = (uint64_t*)((char*)d_sym + round_up(4 * total, 256));
          uint64_t* d_out = (uint64_t*)((char*)d_arg + round_up(8 * total, 256));
          char* scratch = (char*)d_out + round_up(8 * total, 256);
          // each request's queries side by side (the answers of an all-access request ignore its
          // symbols, so a request without symbols leaves its part of d_sym unwritten); a batch within
          // the coalescing size is packed into the slot's page-locked staging first: one copy each way
          sl.staged = total <= s->coalesce_q;
          uint64_t at = 0;
          if (sl.staged) {
            char* hb = sl.h_in;
            const size_t o_op = (char*)d_op - b, o_sym = (char*)d_sym - b, o_arg = (char*)d_arg - b;
            for (uint32_t x : sl.reqs) {
              const wt_request& X = reqs[x];
              if (!X.q) continue;
              std::memcpy(hb + 4 * at, X.h_tree, 4 * X.q);
              std::memcpy(hb + o_op + at, X.h_op, X.q);
              if (X.h_sym) std::memcpy(hb + o_sym + 4 * at, X.h_sym, 4 * X.q);
              std::memcpy(hb + o_arg + 8 * at, X.h_arg, 8 * X.q);
              at += X.q;
            }
            e = hipMemcpyAsync(b, hb, input_bytes(total), hipMemcpyHostToDevice, sl.st);
          } else {
            for (uint32_t x : sl.reqs) {
              const wt_request& X = reqs[x];
              if (!X.q) continue;
              if (e == hipSuccess) e = hipMemcpyAsync(d_tree + at, X.h_tree, 4 * X.q, hipMemcpyHostToDevice, sl.st);
              if (e == hipSuccess) e = hipMemcpyAsync(d_op + at, X.h_op, X.q, hipMemcpyHostToDevice, sl.st);
              if (e == hipSuccess && X.h_sym)
                e = hipMemcpyAsync(d_sym + at, X.h_sym, 4 * X.q, hipMemcpyHostToDevice, sl.st);
              if (e == hipSuccess) e = hipMemcpyAsync(d_arg + at, X.h_arg, 8 * X.q, hipMemcpyHostToDevice, sl.st);
              at += X.q;
            }
          }
          if (e == hipSuccess)
            e = mixed_enqueue(qt, ntrees, d_tree, d_op, any_sym ? d_sym : nullptr, d_arg, total, d_out, scratch,
                              forest_vshift(s->f), sl.st);
          if (sl.staged) {
            if (e == hipSuccess) e = hipMemcpyAsync(sl.h_ans, d_out, 8 * total, hipMemcpyDeviceToHost, sl.st);
          } else {
            at = 0;
            for (uint32_t x : sl.reqs) {
              const wt_request& X = reqs[x];
              if (!X.q) continue;
              if (e == hipSuccess) e = hipMemcpyAsync(X.h_out, d_out + at, 8 * X.q, hipMemcpyDeviceToHost, sl.st);
              at += X.q;
            }
          }
        } else {
          sl.staged = false;
        }
        if (e == hipSuccess) e = hipEventRecord(sl.done, sl.st);
        if (e != hipSuccess) {
          err = fail(WT_ERR_HIP, "wt_server_run: request %u: %s", r, hipGetErrorString(e));
          break;
        }
      }
      pending.erase(pending.begin(), pending.begin() + (long)ng);
      in_flight += (uint32_t)ng;
      ++batches;
      peak_in_flight = std::max(peak_in_flight, in_flight);
      progress = true;
    }
    if (err != WT_OK) break;
    if (!progress) std::this_thread::yield();
  }
  if (err != WT_OK) {
    if (!s->sim_ns) (void)hipDeviceSynchronize();
    return err;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    std::vector<double> lat;
    double first = count ? reqs[0].arrival_s : 0, last = 0;
    uint64_t qsum = 0;
    for (uint32_t i = 0; i < count; ++i) {
      if (comps[i].status != WT_OK) continue;
      lat.push_back(comps[i].done_s - comps[i].arrival_s);
      last = std::max(last, comps[i].done_s);
      qsum += reqs[i].q;
    }
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
      if (lat.empty()) return 0.0;
      const size_t i = std::min(lat.size() - 1, (size_t)(p * (double)(lat.size() - 1) + 0.5));
      return lat[i];
    };
    stats->requests = count;
    stats->rejected = rejected;
    stats->peak_in_flight = peak_in_flight;
    stats->batches = batches;
    stats->queries = qsum;
    stats->peak_bytes = s->arena.peak();
    stats->makespan_s = last > first ? last - first : 0;
    stats->qps = stats->makespan_s > 0 ? (double)qsum / stats->makespan_s : 0;
    stats->lat_p50_s = pct(0.50);
    stats->lat_p99_s = pct(0.99);
    double m = 0;
    for (double x : lat) m += x;
    stats->lat_mean_s = lat.empty() ? 0 : m / (double)lat.size();
    stats->lat_max_s = lat.empty() ? 0 : lat.back();
  }
  return WT_OK;
}
