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

// Algorithm 5 (top-down): the bit of the element picks the child; its position in the child is its
// rank among the equal bits of the node. Stops once the node covers at most two symbols.
template <int L2S>
__global__ __launch_bounds__(kQT) void k_access(QArgs a, const uint64_t* __restrict__ pos, uint64_t q,
                                                uint32_t* __restrict__ out) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT) {
    const uint64_t i = pos[j];
    uint32_t res;
    if (i >= a.n) {
      res = 0xFFFFFFFFu;
    } else {
      uint32_t s = 0, e = a.sigma;
      uint64_t p = 0, x = i;
      for (uint32_t l = 0; l < a.L; ++l) {
        const uint32_t width = e - s;
        const NodeQ nd = a.d.nodes[(1ull << l) - 1 + p];
        const LevelMeta& m = s_meta[l];
        const uint64_t y = nd.start + x;
        if (width <= 2) {
          if (width == 2) s += (uint32_t)(a.d.bits[m.bits + (y >> 6)] >> (y & 63)) & 1u;
          break;
        }
        uint32_t bit;
        const uint64_t r0 = y - rank1_at<L2S>(a.d, m, y, bit);
        const uint32_t half = (uint32_t)pow2_below(width);
        if (!bit) {
          x = r0 - nd.r0;
          e = s + half;
          p = 2 * p;
        } else {
          x = x - (r0 - nd.r0);
          s += half;
          p = 2 * p + 1;
        }
      }
      res = s;
    }
    out[j] = res;
  }
}

// Algorithm 6 (top-down along the symbol's path): the count of the symbol's side before the position.
template <int L2S>
__global__ __launch_bounds__(kQT) void k_rank(QArgs a, const uint32_t* __restrict__ sym,
                                              const uint64_t* __restrict__ pos, uint64_t q,
                                              uint64_t* __restrict__ out) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT) {
    const uint32_t c = sym[j];
    const uint64_t i = pos[j];
    uint64_t res;
    if (i > a.n) {
      res = ~0ull;
    } else if (c >= a.sigma) {
      res = 0;
    } else {
      uint32_t s = 0, e = a.sigma;
      uint64_t p = 0, x = i;
      for (uint32_t l = 0; l < a.L; ++l) {
        if (e - s <= 1 || x == 0) break;
        const NodeQ nd = a.d.nodes[(1ull << l) - 1 + p];
        const uint64_t y = nd.start + x;
        uint32_t bit;
        const uint64_t r0 = y - rank1_at<L2S>(a.d, s_meta[l], y, bit);
        const uint32_t split = s + (uint32_t)pow2_below(e - s);
        if (c < split) {
          x = r0 - nd.r0;
          e = split;
          p = 2 * p;
        } else {
          x = x - (r0 - nd.r0);
          s = split;
          p = 2 * p + 1;
        }
      }
      res = x;
    }
    out[j] = res;
  }
}

// Algorithms 7 and 8 (bottom-up from the symbol's leaf): the k-th occurrence inside the current node
// is the (rank-at-node-start + k)-th bit equal to the node's side in the parent level.
template <int L2S>
__global__ __launch_bounds__(kQT) void k_select(QArgs a, const uint32_t* __restrict__ sym,
                                                const uint64_t* __restrict__ kin, uint64_t q,
                                                uint64_t* __restrict__ out) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT) {
    const uint32_t c = sym[j];
    const uint64_t k = kin[j];
    uint64_t res;
    if (k == 0) {
      res = ~0ull;
    } else if (c >= a.sigma) {
      res = a.n;
    } else if (k > a.d.cum[c + 1] - a.d.cum[c]) {
      res = a.n;
    } else if (a.L == 0) {
      res = k - 1;
    } else {
      uint32_t len;
      const uint32_t code = encode_sym(c, a.sigma, a.L, a.pow2, &len);
      uint64_t r = k;
      for (int l = (int)len - 1; l >= 0; --l) {
        const uint64_t p = l ? (uint64_t)(code >> (a.L - l)) : 0ull;
        const uint32_t b = (code >> (a.L - 1 - l)) & 1u;
        const NodeQ nd = a.d.nodes[(1ull << l) - 1 + p];
        const uint64_t target = b ? (nd.start - nd.r0) + r : nd.r0 + r;
        const uint64_t at = select_at<L2S>(a.d, s_meta[l], b, target, a.sshift);
        r = at - nd.start + 1;
      }
      res = r - 1;
    }
    out[j] = res;
  }
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
