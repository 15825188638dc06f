// Autotuner of the L2 block size |L2| and the select sample interval s (Sections 4.1 and 4.2 leave
// both as parameters) per shape bucket of a forest: for every occupied bucket, the bucket's longest
// sequence (a prefix of at most max_probe_n symbols) is built with every candidate pair and answers a
// batch of each query kind; the pair with the least build time per symbol plus the query time of the
// expected number of queries per symbol wins, among the pairs whose directory and samples stay within
// the space cap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

void tune_bucket(uint64_t n, uint64_t sigma, uint32_t* nb, uint32_t* sb);

__device__ __forceinline__ uint64_t tune_mix(uint64_t x) {  // SplitMix64 finaliser
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// Probe queries: positions uniform in [0, n), symbols drawn from the sequence, k uniform in
// [1, count(symbol)] (counts from the built tree's cumulative histogram).
template <typename E>
__global__ void k_tune_queries(const E* __restrict__ S, uint64_t n, const uint64_t* __restrict__ cum, uint64_t q,
                               uint64_t* __restrict__ pos, uint32_t* __restrict__ sym, uint64_t* __restrict__ k) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= q) return;
  const uint64_t a = tune_mix(3 * j), b = tune_mix(3 * j + 1), c = tune_mix(3 * j + 2);
  pos[j] = a % n;
  const uint32_t s = (uint32_t)S[b % n];
  sym[j] = s;
  const uint64_t cnt = cum[s + 1] - cum[s];
  k[j] = 1 + c % cnt;
}

}  // namespace wt

using namespace wt;

extern "C" wt_status wt_autotune(const wt_seq_desc* h_descs, uint32_t count, uint32_t sym_bytes,
                                 const wt_tune_opts* opts, wt_stream_t stream, wt_tune_table* out,
                                 wt_tune_report* report) {
  clear_error();
  if (!h_descs || !out || count == 0) return fail(WT_ERR_ARG, "wt_autotune: NULL argument or no sequences");
  if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4)
    return fail(WT_ERR_ARG, "wt_autotune: sym_bytes must be 1, 2 or 4");
  uint64_t max_probe = 1ull << 22;
  uint32_t nq = 1u << 16;
  double qps = 1.0 / 64.0, cap = 0.10;
  if (opts) {
    if (opts->max_probe_n) max_probe = opts->max_probe_n;
    if (opts->queries) nq = opts->queries;
    if (opts->queries_per_symbol > 0) qps = opts->queries_per_symbol;
    if (opts->space_cap > 0) cap = opts->space_cap;
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::memset(out, 0, sizeof(*out));
  if (report) std::memset(report, 0, sizeof(*report));
  hipStream_t st = (hipStream_t)stream;
  // representative of every occupied bucket: its longest sequence
  int rep[WT_TUNE_NB][WT_TUNE_SB];
  for (auto& r : rep)
    for (int& x : r) x = -1;
  for (uint32_t j = 0; j < count; ++j) {
    const wt_seq_desc& d = h_descs[j];
    if (d.n == 0 || d.sigma < 2) continue;
    if (!d.d_sym) return fail(WT_ERR_ARG, "wt_autotune: sequence %u: d_sym is NULL", j);
    uint32_t nb, sb;
    tune_bucket(d.n, d.sigma, &nb, &sb);
    if (rep[nb][sb] < 0 || h_descs[rep[nb][sb]].n < d.n) rep[nb][sb] = (int)j;
  }
  static const uint32_t kL2[] = {256, 512, 1024};
  static const uint32_t kS[] = {1024, 4096, 16384};
  const uint64_t qmax = nq;
  char* qb = (char*)dev_alloc(qmax * (8 + 4 + 8 + 8), st);
  if (!qb) return fail(WT_ERR_OOM, "wt_autotune: query buffers");
  uint64_t* d_pos = (uint64_t*)qb;
  uint64_t* d_k = d_pos + qmax;
  uint64_t* d_out = d_k + qmax;
  uint32_t* d_sym = (uint32_t*)(d_out + qmax);
  hipEvent_t e[8];
  for (auto& x : e) WT_HIP(hipEventCreate(&x));
  struct Cleanup {
    hipEvent_t* e;
    char* qb;
    hipStream_t st;
    ~Cleanup() {
      for (int i = 0; i < 8; ++i) (void)hipEventDestroy(e[i]);
      dev_free(qb, st);
    }
  } cleanup{e, qb, st};
  uint32_t tuned = 0, probes = 0;
  for (uint32_t nb = 0; nb < WT_TUNE_NB; ++nb) {
    for (uint32_t sb = 0; sb < WT_TUNE_SB; ++sb) {
      if (rep[nb][sb] < 0) continue;
      const wt_seq_desc& d = h_descs[rep[nb][sb]];
      const uint64_t n = std::min<uint64_t>(d.n, max_probe);
      const uint64_t q = std::min<uint64_t>(qmax, std::max<uint64_t>(n, 1));
      double best = 1e300;
      uint32_t bl2 = 512, bs = 4096;
      for (uint32_t l2 : kL2) {
        for (uint32_t s : kS) {
          const double space = 16.0 / l2 + 64.0 / s + 64.0 / 65536.0;
          if (space > cap) continue;
          wt_build_opts bo{l2, s, 0, 0};
          wt_tree* t = nullptr;
          WT_HIP(hipEventRecord(e[0], st));
          wt_status rc = wt_build(d.d_sym, n, sym_bytes, d.sigma, &bo, stream, &t);
          if (rc != WT_OK) return rc;
          WT_HIP(hipEventRecord(e[1], st));
          const uint32_t g = (uint32_t)ceil_div(q, 256);
          if (sym_bytes == 1)
            hipLaunchKernelGGL(k_tune_queries<uint8_t>, dim3(g), dim3(256), 0, st, (const uint8_t*)d.d_sym, n,
                               (const uint64_t*)t->dev.cum, q, d_pos, d_sym, d_k);
          else if (sym_bytes == 2)
            hipLaunchKernelGGL(k_tune_queries<uint16_t>, dim3(g), dim3(256), 0, st, (const uint16_t*)d.d_sym, n,
                               (const uint64_t*)t->dev.cum, q, d_pos, d_sym, d_k);
          else
            hipLaunchKernelGGL(k_tune_queries<uint32_t>, dim3(g), dim3(256), 0, st, (const uint32_t*)d.d_sym, n,
                               (const uint64_t*)t->dev.cum, q, d_pos, d_sym, d_k);
          // warm-up pass, then the timed pass of each kind
          for (int rep_i = 0; rep_i < 2 && rc == WT_OK; ++rep_i) {
            if (rc == WT_OK) rc = hipEventRecord(e[2], st) == hipSuccess ? WT_OK : WT_ERR_HIP;
            if (rc == WT_OK) rc = wt_access(t, d_pos, q, (uint32_t*)d_out, stream);
            if (rc == WT_OK) rc = hipEventRecord(e[3], st) == hipSuccess ? WT_OK : WT_ERR_HIP;
            if (rc == WT_OK) rc = wt_rank(t, d_sym, d_pos, q, d_out, stream);
            if (rc == WT_OK) rc = hipEventRecord(e[4], st) == hipSuccess ? WT_OK : WT_ERR_HIP;
            if (rc == WT_OK) rc = wt_select(t, d_sym, d_k, q, d_out, stream);
            if (rc == WT_OK) rc = hipEventRecord(e[5], st) == hipSuccess ? WT_OK : WT_ERR_HIP;
          }
          if (rc == WT_OK && hipStreamSynchronize(st) != hipSuccess) rc = WT_ERR_HIP;
          float bms = 0, ams = 0, rms = 0, sms = 0;
          (void)hipEventElapsedTime(&bms, e[0], e[1]);
          (void)hipEventElapsedTime(&ams, e[2], e[3]);
          (void)hipEventElapsedTime(&rms, e[3], e[4]);
          (void)hipEventElapsedTime(&sms, e[4], e[5]);
          wt_free(t);
          if (rc != WT_OK) return fail(rc, "wt_autotune: probe failed");
          ++probes;
          const double cost = (double)bms / (double)n + qps * (double)(ams + rms + sms) / (3.0 * (double)q);
          if (cost < best) {
            best = cost;
            bl2 = l2;
            bs = s;
          }
        }
      }
      out->l2_bits[nb][sb] = bl2;
      out->sample_rate[nb][sb] = bs;
      if (report) report->cost_ns_per_symbol[nb][sb] = (float)(best * 1e6);
      ++tuned;
    }
  }
  if (report) {
    report->buckets = tuned;
    report->probes = probes;
    report->total_ms =
        (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return WT_OK;
}
