// Huffman-shaped tree (the Huffman variant named as a next step in the thesis's Conclusion): the
// level-wise tree over an optimal length-limited prefix code of the symbol counts.
//
// Host: code lengths by package-merge (Larmore and Hirschberg) from the histogram, canonical codes
// with the longer codes on the left (so a node's elements start at the count of the symbols ordered
// before it, as with the reduced codes of Section 5.1), and the tables the queries read.
// Device: the symbols rewritten as left-aligned codes (with the ones of code bit L - 1 per tile of the
// first level), and the node table from the codes in rank order. The level passes are the tree's own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "wt_build_dev.h"
#include "wt_host.h"
#include "wt_huff.h"
#include "wt_internal.h"

namespace wt {

uint32_t huff_limit(uint64_t m) {
  uint32_t lg = 0;
  while ((1ull << lg) < m) ++lg;
  return std::min<uint32_t>(WT_MAX_LEVELS, std::max<uint32_t>(lg, 1) + 8);
}

void huff_code(const uint64_t* hist, uint64_t sigma, HuffCode& hc) {
  hc = HuffCode{};
  hc.hcode.assign(sigma, 0ull);
  // occurring symbols, lightest first (ties: smaller symbol first)
  std::vector<std::pair<uint64_t, uint32_t>> lv;
  for (uint64_t c = 0; c < sigma; ++c)
    if (hist[c]) lv.emplace_back(hist[c], (uint32_t)c);
  std::sort(lv.begin(), lv.end());
  const uint64_t m = lv.size();
  hc.m = m;
  if (m == 0) return;
  if (m == 1) {  // a lone symbol: no level; access answers it
    hc.sym.push_back(lv[0].second);
    hc.cumr = {0ull, lv[0].first};
    hc.depth.push_back(m << 32);
    return;
  }
  const uint32_t D = huff_limit(m);
  // package-merge: list of depth d = the symbols merged (by weight, a symbol before an equal-weight
  // package) with the consecutive pairs of the list of depth d + 1; sym_item[d] marks its symbols
  std::vector<std::vector<uint8_t>> sym_item(D + 1);
  std::vector<uint64_t> deeper, here;
  for (uint32_t d = D; d >= 1; --d) {
    here.clear();
    std::vector<uint8_t>& mark = sym_item[d];
    const size_t npk = d == D ? 0 : deeper.size() / 2;
    size_t i = 0, k = 0;
    while (i < m || k < npk) {
      const bool take_sym = i < m && (k == npk || lv[i].first <= deeper[2 * k] + deeper[2 * k + 1]);
      if (take_sym) {
        here.push_back(lv[i++].first);
        mark.push_back(1);
      } else {
        here.push_back(deeper[2 * k] + deeper[2 * k + 1]);
        ++k;
        mark.push_back(0);
      }
    }
    deeper.swap(here);
  }
  // the first 2m - 2 items of depth 1; a package taken at depth d takes its pair at depth d + 1
  std::vector<uint32_t> len(m, 0);
  uint64_t take = 2 * m - 2;
  for (uint32_t d = 1; d <= D && take; ++d) {
    const std::vector<uint8_t>& mark = sym_item[d];
    uint64_t syms = 0;
    for (uint64_t x = 0; x < take && x < mark.size(); ++x) syms += mark[x];
    for (uint64_t j = 0; j < syms; ++j) ++len[j];  // the `syms` lightest symbols
    take = 2 * (take - syms);
  }
  uint32_t L = 0;
  for (uint32_t x : len) L = std::max(L, x);
  hc.L = L;
  // canonical order: length descending, symbol ascending
  std::vector<uint64_t> ord(m);
  for (uint64_t j = 0; j < m; ++j) ord[j] = j;
  std::sort(ord.begin(), ord.end(), [&](uint64_t a, uint64_t b) {
    if (len[a] != len[b]) return len[a] > len[b];
    return lv[a].second < lv[b].second;
  });
  hc.sym.resize(m);
  hc.code_r.resize(m);
  hc.cumr.assign(m + 1, 0ull);
  uint64_t v = 0;
  for (uint64_t r = 0; r < m; ++r) {
    const uint64_t j = ord[r];
    const uint32_t c = lv[j].second;
    hc.sym[r] = c;
    hc.code_r[r] = (uint32_t)v;
    hc.hcode[c] = ((uint64_t)len[j] << 32) | v;
    hc.cumr[r + 1] = hc.cumr[r] + lv[j].first;
    v += 1ull << (L - len[j]);
  }
  // per depth d: I_d (internal prefixes [0, I_d)) and F_d (first rank of a code of length <= d)
  hc.depth.assign(L + 1, 0ull);
  hc.depth[0] = (m << 32) | 1ull;
  for (uint32_t d = 1; d <= L; ++d) {
    uint64_t F = 0;
    while (F < m && len[ord[F]] > d) ++F;
    const uint64_t I = F < m ? (uint64_t)(hc.code_r[F] >> (L - d)) : (1ull << d);
    hc.depth[d] = (F << 32) | I;
  }
}

// ---------------------------------------------------------------- device

// Symbols -> left-aligned codes of the first level (one block per tile of EC elements), and the ones
// of code bit L - 1 of every tile (the tile counts of level 0). 16-byte loads of the symbols when the
// array is aligned; the code table is staged in LDS for alphabets up to kEncLds symbols.
constexpr uint32_t kEncLds = 8192;

template <typename E, typename EC>
__global__ __launch_bounds__(kBT) void k_huff_encode(const E* __restrict__ in, uint64_t n, uint32_t sigma,
                                                     const uint64_t* __restrict__ hcode, uint32_t L, uint32_t aligned,
                                                     EC* __restrict__ out, uint64_t* __restrict__ cnt0) {
  __shared__ uint32_t s_w[kBT / 64];
  __shared__ uint32_t s_code[kEncLds];
  constexpr uint32_t T = kTileBytes / sizeof(EC);
  constexpr uint32_t V = 16 / sizeof(E);  // symbols per 16-byte load
  const bool lds = sigma <= kEncLds;
  if (lds) {
    for (uint32_t c = threadIdx.x; c < sigma; c += kBT) s_code[c] = (uint32_t)hcode[c];
    __syncthreads();
  }
  auto code_of = [&](uint32_t s) -> uint32_t {
    if (s >= sigma) s = 0;  // out of range: the build has already failed; keep the index valid
    return lds ? s_code[s] : (uint32_t)hcode[s];
  };
  const uint64_t t0 = (uint64_t)blockIdx.x * T;
  const uint32_t cnt = (uint32_t)min<uint64_t>((uint64_t)T, n - t0);
  uint32_t ones = 0;
  if (aligned) {
    for (uint32_t j = threadIdx.x * V; j < cnt; j += kBT * V) {
      E v[V];
      if (j + V <= cnt) {
        const uint4 x = *reinterpret_cast<const uint4*>(in + t0 + j);
        __builtin_memcpy(v, &x, 16);
      } else {
#pragma unroll
        for (uint32_t e = 0; e < V; ++e) v[e] = j + e < cnt ? in[t0 + j + e] : (E)0;
      }
      EC o[V];
#pragma unroll
      for (uint32_t e = 0; e < V; ++e) {
        const uint32_t code = code_of((uint32_t)v[e]);
        o[e] = (EC)code;
        ones += (j + e < cnt) ? ((code >> (L - 1)) & 1u) : 0u;
      }
      if (j + V <= cnt) {
        __builtin_memcpy(out + t0 + j, o, sizeof(o));
      } else {
#pragma unroll
        for (uint32_t e = 0; e < V; ++e)
          if (j + e < cnt) out[t0 + j + e] = o[e];
      }
    }
  } else {
    for (uint32_t j = threadIdx.x; j < cnt; j += kBT) {
      const uint32_t code = code_of((uint32_t)in[t0 + j]);
      out[t0 + j] = (EC)code;
      ones += (code >> (L - 1)) & 1u;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ones += __shfl_xor(ones, off, 64);
  if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = ones;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < kBT / 64; ++w) tot += s_w[w];
    cnt0[blockIdx.x] = tot;
  }
}

// First index in [lo, hi) of the ascending array a whose value is >= v.
__device__ __forceinline__ uint64_t lower_bound_u32(const uint32_t* __restrict__ a, uint64_t lo, uint64_t hi,
                                                    uint64_t v) {
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if ((uint64_t)a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Heap entry h (level l, code prefix p): the ranks [s, e) of the codes with prefix p; a node exists
// when it holds two codes or more (one code with prefix p is a leaf at or above level l). Its left
// child ends at the first code whose bit l is 1. The same outputs as the reduced tree's node walk.
__global__ __launch_bounds__(kBT) void k_node_walk_huff(uint32_t L, uint64_t m, uint64_t nheap,
                                                        const uint32_t* __restrict__ code_r,
                                                        const uint64_t* __restrict__ cumr, NodeB* __restrict__ ntb,
                                                        uint64_t* __restrict__ zeros) {
  const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nheap) return;
  const uint32_t l = 63u - (uint32_t)__clzll(h + 1);
  const uint64_t p = h + 1 - (1ull << l);
  const uint64_t lo = p << (L - l), hi = (p + 1) << (L - l);
  const uint64_t s = lower_bound_u32(code_r, 0, m, lo);
  const uint64_t e = lower_bound_u32(code_r, s, m, hi);
  NodeB b;
  if (e - s >= 2) {
    const uint64_t mm = lower_bound_u32(code_r, s, e, (2 * p + 1) << (L - l - 1));
    b.start = cumr[s];
    b.end = cumr[e];
    b.off0 = cumr[mm];  // left-child end, turned into off0/off1 by the node-final kernel
    b.off1 = 0;
    zeros[h] = cumr[mm] - cumr[s];
  } else {
    b.start = kNoNode;
    b.end = 0;
    b.off0 = 0;
    b.off1 = 0;
    zeros[h] = 0;
  }
  ntb[h] = b;
}

template <typename E, typename EC>
static hipError_t launch_encode(const void* in, uint64_t n, uint32_t sigma, const uint64_t* hcode, uint32_t L,
                                void* out, uint64_t* cnt0, hipStream_t st) {
  const uint64_t nt = ceil_div(n, kTileBytes / sizeof(EC));
  if (nt == 0) return hipSuccess;
  const uint32_t aligned = ((uintptr_t)in & 15u) == 0;
  hipLaunchKernelGGL((k_huff_encode<E, EC>), dim3((uint32_t)nt), dim3(kBT), 0, st, (const E*)in, n, sigma, hcode, L,
                     aligned, (EC*)out, cnt0);
  return hipGetLastError();
}

hipError_t huff_encode(const void* d_sym, uint32_t w, uint64_t n, uint32_t sigma, const uint64_t* d_hcode,
                       uint32_t L, void* d_out, uint32_t wc, uint64_t* cnt0, hipStream_t st) {
  if (w == 1) {
    if (wc == 1) return launch_encode<uint8_t, uint8_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
    if (wc == 2) return launch_encode<uint8_t, uint16_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
    return launch_encode<uint8_t, uint32_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
  }
  if (w == 2) {
    if (wc == 1) return launch_encode<uint16_t, uint8_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
    if (wc == 2) return launch_encode<uint16_t, uint16_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
    return launch_encode<uint16_t, uint32_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
  }
  if (wc == 1) return launch_encode<uint32_t, uint8_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
  if (wc == 2) return launch_encode<uint32_t, uint16_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
  return launch_encode<uint32_t, uint32_t>(d_sym, n, sigma, d_hcode, L, d_out, cnt0, st);
}

hipError_t huff_node_walk(uint32_t L, uint64_t m, uint64_t nheap, const uint32_t* d_code_r, const uint64_t* d_cumr,
                          NodeB* ntb, uint64_t* zeros, hipStream_t st) {
  if (nheap == 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_walk_huff, dim3((uint32_t)ceil_div(nheap, kBT)), dim3(kBT), 0, st, L, m, nheap, d_code_r,
                     d_cumr, ntb, zeros);
  return hipGetLastError();
}

}  // namespace wt
