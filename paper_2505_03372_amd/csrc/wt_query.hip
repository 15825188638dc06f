// Batched access / rank / select on gfx950: one lane per query, persistent grid-stride loop.
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

template <int L2S>
__global__ __launch_bounds__(kQT) void k_access(QArgs a, const uint64_t* __restrict__ pos, uint64_t q,
                                                uint32_t* __restrict__ out) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT)
    out[j] = access_one<L2S>(a, s_meta, pos[j]);
}

template <int L2S>
__global__ __launch_bounds__(kQT) void k_rank(QArgs a, const uint32_t* __restrict__ sym,
                                              const uint64_t* __restrict__ pos, uint64_t q,
                                              uint64_t* __restrict__ out) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT)
    out[j] = rank_one<L2S>(a, s_meta, sym[j], pos[j]);
}

template <int L2S>
__global__ __launch_bounds__(kQT) void k_select(QArgs a, const uint32_t* __restrict__ sym,
                                                const uint64_t* __restrict__ kin, uint64_t q,
                                                uint64_t* __restrict__ out) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT)
    out[j] = select_one<L2S>(a, s_meta, sym[j], kin[j]);
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
  WT_DISPATCH_L2(t->l2_bits, k_access, a, d_pos, q, d_out);
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
  WT_DISPATCH_L2(t->l2_bits, k_rank, a, d_sym, d_pos, q, d_out);
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
  WT_DISPATCH_L2(t->l2_bits, k_select, a, d_sym, d_k, q, d_out);
  WT_HIP(hipGetLastError());
  return WT_OK;
}
