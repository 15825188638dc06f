// Batched access / rank / select on gfx950: one lane per query, persistent grid-stride loop.
//
// Large batches are first binned by where their answers lie (access and rank by position, select by
// the rank of the wanted occurrence in symbol order, cum[c] + k - 1): a counting pass into 2^16
// buckets, a scan and a scatter put the queries in bucket order, the traversal reads them in that
// order and writes every answer to its query's index. Queries that are close in the key touch the
// same lines of bits, L2 counts and samples at every level (each traversal keeps the order inside a
// node), so the cache lines a wave fetches are shared instead of fetched once per query.
//
// Per level a query needs the node entry (start position and precomputed rank0, indexed by code
// prefix), then one binary rank (Section 4.1, Algorithm 1: L1 + L2 + popcount of the words of one
// L2 block, read as 16-byte vectors) or one binary select (Section 4.2, Algorithm 2: samples ->
// binary search over L1 -> binary search over L2 -> word scan -> in-word select).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wt_host.h"
#include "wt_internal.h"
#include "wt_query_dev.h"

namespace wt {

// perm: NULL, or the query index of every (binned) slot j; the answer of slot j goes to out[perm[j]].
template <int L2S>
__global__ __launch_bounds__(kQT) void k_access(QArgs a, const uint64_t* __restrict__ pos, uint64_t q,
                                                uint32_t* __restrict__ out, const uint32_t* __restrict__ perm) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT)
    out[perm ? perm[j] : j] = access_one<L2S>(a, s_meta, pos[j]);
}

template <int L2S>
__global__ __launch_bounds__(kQT) void k_rank(QArgs a, const uint32_t* __restrict__ sym,
                                              const uint64_t* __restrict__ pos, uint64_t q,
                                              uint64_t* __restrict__ out, const uint32_t* __restrict__ perm) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT)
    out[perm ? perm[j] : j] = rank_one<L2S>(a, s_meta, sym[j], pos[j]);
}

template <int L2S>
__global__ __launch_bounds__(kQT, 8) void k_select(QArgs a, const uint32_t* __restrict__ sym,
                                                const uint64_t* __restrict__ kin, uint64_t q,
                                                uint64_t* __restrict__ out, const uint32_t* __restrict__ perm) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT)
    out[perm ? perm[j] : j] = select_one<L2S>(a, s_meta, sym[j], kin[j]);
}

// ---------------------------------------------------------------- locality binning

constexpr uint32_t kSortBuckets = 1u << 16;

__global__ void k_sort_zero(uint32_t* __restrict__ p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

__device__ __forceinline__ uint64_t sort_key(const QArgs& a, int kind, uint32_t c, uint64_t x) {
  if (kind != 2) return min(x, a.n);  // access, rank: the position
  if (x == 0 || c >= a.sigma) return a.n;
  const uint64_t lo = a.d.cum[c], cnt = a.d.cum[c + 1] - lo;
  return x > cnt ? a.n : lo + x - 1;  // select: rank of the occurrence in symbol order
}

// Lanes of a wave with the same bucket as their left neighbour form a run; the run's first lane acts
// for it (one atomic per run: already-ordered batches do not serialise on a bucket counter).
struct WaveRun {
  uint32_t head;  // lane of the run's first lane
  uint32_t len;   // run length (meaningful in the head lane)
};

__device__ __forceinline__ WaveRun wave_run(uint32_t b, bool in) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t prev = __shfl_up(b, 1, 64);
  const bool prev_in = __shfl_up((uint32_t)in, 1, 64) != 0u;
  const bool head = in && (lane == 0 || !prev_in || prev != b);
  const uint64_t heads = __ballot(head);
  const uint64_t act = __ballot(in);
  WaveRun r;
  const uint64_t upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  r.head = upto ? 63u - (uint32_t)__clzll(upto) : lane;
  const uint64_t after = heads & ~((2ull << lane) - 1ull) & (lane == 63 ? 0ull : ~0ull);
  const uint32_t next = after ? (uint32_t)__ffsll((unsigned long long)after) - 1u : 64u;
  const uint32_t last_in = act ? 64u - (uint32_t)__clzll(act) : 0u;  // one past the last active lane
  r.len = min(next, last_in) - lane;
  return r;
}

template <int KIND>
__global__ __launch_bounds__(kQT) void k_sort_count(QArgs a, const uint32_t* __restrict__ sym,
                                                    const uint64_t* __restrict__ arg, uint64_t q, uint32_t shift,
                                                    uint32_t* __restrict__ bucket, uint32_t* __restrict__ cnt) {
  const uint64_t stride = (uint64_t)gridDim.x * kQT;
  for (uint64_t j0 = (uint64_t)blockIdx.x * kQT; j0 < q; j0 += stride) {
    const uint64_t j = j0 + threadIdx.x;
    const bool in = j < q;
    uint32_t b = 0;
    if (in) {
      b = (uint32_t)min<uint64_t>(sort_key(a, KIND, KIND ? sym[j] : 0u, arg[j]) >> shift, kSortBuckets - 1);
      bucket[j] = b;
    }
    const WaveRun r = wave_run(b, in);
    if (in && r.head == (threadIdx.x & 63u)) atomicAdd(&cnt[b], r.len);
  }
}

// In place exclusive scan of the bucket counts (one block).
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ cnt) {
  __shared__ uint32_t s_w[16];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < kSortBuckets; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t x = cnt[i];
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(inc, off, 64);
      if ((int)lane >= off) inc += y;
    }
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      pre += w < wv ? s_w[w] : 0u;
      tot += s_w[w];
    }
    cnt[i] = carry + pre + inc - x;
    carry += tot;
    __syncthreads();
  }
}

template <int KIND>
__global__ __launch_bounds__(kQT) void k_sort_scatter(uint64_t q, const uint32_t* __restrict__ bucket,
                                                      const uint32_t* __restrict__ sym,
                                                      const uint64_t* __restrict__ arg, uint32_t* __restrict__ cursor,
                                                      uint32_t* __restrict__ perm, uint32_t* __restrict__ ssym,
                                                      uint64_t* __restrict__ sarg) {
  const uint64_t stride = (uint64_t)gridDim.x * kQT;
  const uint32_t lane = threadIdx.x & 63u;
  for (uint64_t j0 = (uint64_t)blockIdx.x * kQT; j0 < q; j0 += stride) {
    const uint64_t j = j0 + threadIdx.x;
    const bool in = j < q;
    const uint32_t b = in ? bucket[j] : 0u;
    const WaveRun r = wave_run(b, in);
    uint32_t base = 0;
    if (in && r.head == lane) base = atomicAdd(&cursor[b], r.len);
    base = __shfl(base, (int)r.head, 64);
    if (in) {
      const uint32_t s = base + (lane - r.head);
      perm[s] = (uint32_t)j;
      if (KIND) ssym[s] = sym[j];
      sarg[s] = arg[j];
    }
  }
}

constexpr uint64_t kSortMinQ = 1ull << 16;

// Bins the batch on st (kind 0 access, 1 rank, 2 select); false when the batch is too small to pay.
wt_status sort_batch(const wt_tree* t, const QArgs& a, int kind, const uint32_t* sym, const uint64_t* arg,
                            uint64_t q, hipStream_t st, SortBufs& sb, bool& binned) {
  binned = false;
  if (q < kSortMinQ || q >= (1ull << 32)) return WT_OK;
  const size_t o_b = round_up(4ull * kSortBuckets, 256), o_p = o_b + round_up(4 * q, 256),
               o_s = o_p + round_up(4 * q, 256), o_a = o_s + round_up(4 * q, 256), bytes = o_a + 8 * q;
  sb.block = (char*)dev_alloc(bytes, st);
  if (!sb.block) return fail(WT_ERR_OOM, "query binning: scratch allocation of %zu bytes failed", bytes);
  sb.cnt = (uint32_t*)sb.block;
  sb.bucket = (uint32_t*)(sb.block + o_b);
  sb.perm = (uint32_t*)(sb.block + o_p);
  sb.ssym = (uint32_t*)(sb.block + o_s);
  sb.sarg = (uint64_t*)(sb.block + o_a);
  uint32_t bits = 0;
  while ((1ull << bits) < a.n + 1) ++bits;
  const uint32_t shift = bits > 16 ? bits - 16 : 0;
  const uint32_t grid = query_grid(q);
  hipLaunchKernelGGL(k_sort_zero, dim3(kSortBuckets / 256), dim3(256), 0, st, sb.cnt, kSortBuckets);
  if (kind == 0) {
    hipLaunchKernelGGL(k_sort_count<0>, dim3(grid), dim3(kQT), 0, st, a, sym, arg, q, shift, sb.bucket, sb.cnt);
  } else if (kind == 1) {
    hipLaunchKernelGGL(k_sort_count<1>, dim3(grid), dim3(kQT), 0, st, a, sym, arg, q, shift, sb.bucket, sb.cnt);
  } else {
    hipLaunchKernelGGL(k_sort_count<2>, dim3(grid), dim3(kQT), 0, st, a, sym, arg, q, shift, sb.bucket, sb.cnt);
  }
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, sb.cnt);
  if (kind == 0) {
    hipLaunchKernelGGL(k_sort_scatter<0>, dim3(grid), dim3(kQT), 0, st, q, (const uint32_t*)sb.bucket, sym, arg,
                       sb.cnt, sb.perm, sb.ssym, sb.sarg);
  } else {
    hipLaunchKernelGGL(k_sort_scatter<1>, dim3(grid), dim3(kQT), 0, st, q, (const uint32_t*)sb.bucket, sym, arg,
                       sb.cnt, sb.perm, sb.ssym, sb.sarg);
  }
  WT_HIP(hipGetLastError());
  binned = true;
  (void)t;
  return WT_OK;
}

}  // namespace wt

using namespace wt;

extern "C" wt_status wt_access(const wt_tree* t, const uint64_t* d_pos, uint64_t q, uint32_t* d_out,
                               wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_access: tree is NULL");
  if (q == 0) return WT_OK;
  if (!d_pos || !d_out) return fail(WT_ERR_ARG, "wt_access: NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  const QArgs a = make_args(t);
  const uint32_t grid = query_grid(q);
  SortBufs sb;
  bool binned;
  const wt_status rc = sort_batch(t, a, 0, nullptr, d_pos, q, st, sb, binned);
  if (rc != WT_OK) return rc;
  if (binned) {
    WT_DISPATCH_L2(t->l2_bits, k_access, a, (const uint64_t*)sb.sarg, q, d_out, (const uint32_t*)sb.perm);
    dev_free(sb.block, st);
  } else {
    WT_DISPATCH_L2(t->l2_bits, k_access, a, d_pos, q, d_out, (const uint32_t*)nullptr);
  }
  WT_HIP(hipGetLastError());
  return WT_OK;
}

extern "C" wt_status wt_rank(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_pos, uint64_t q,
                             uint64_t* d_out, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_rank: tree is NULL");
  if (q == 0) return WT_OK;
  if (!d_sym || !d_pos || !d_out) return fail(WT_ERR_ARG, "wt_rank: NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  const QArgs a = make_args(t);
  const uint32_t grid = query_grid(q);
  SortBufs sb;
  bool binned;
  const wt_status rc = sort_batch(t, a, 1, d_sym, d_pos, q, st, sb, binned);
  if (rc != WT_OK) return rc;
  if (binned) {
    WT_DISPATCH_L2(t->l2_bits, k_rank, a, (const uint32_t*)sb.ssym, (const uint64_t*)sb.sarg, q, d_out,
                   (const uint32_t*)sb.perm);
    dev_free(sb.block, st);
  } else {
    WT_DISPATCH_L2(t->l2_bits, k_rank, a, d_sym, d_pos, q, d_out, (const uint32_t*)nullptr);
  }
  WT_HIP(hipGetLastError());
  return WT_OK;
}

extern "C" wt_status wt_select(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_k, uint64_t q,
                               uint64_t* d_out, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_select: tree is NULL");
  if (q == 0) return WT_OK;
  if (!d_sym || !d_k || !d_out) return fail(WT_ERR_ARG, "wt_select: NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  const QArgs a = make_args(t);
  const uint32_t grid = query_grid(q);
  SortBufs sb;
  bool binned;
  const wt_status rc = sort_batch(t, a, 2, d_sym, d_k, q, st, sb, binned);
  if (rc != WT_OK) return rc;
  if (binned) {
    WT_DISPATCH_L2(t->l2_bits, k_select, a, (const uint32_t*)sb.ssym, (const uint64_t*)sb.sarg, q, d_out,
                   (const uint32_t*)sb.perm);
    dev_free(sb.block, st);
  } else {
    WT_DISPATCH_L2(t->l2_bits, k_select, a, d_sym, d_k, q, d_out, (const uint32_t*)nullptr);
  }
  WT_HIP(hipGetLastError());
  return WT_OK;
}
