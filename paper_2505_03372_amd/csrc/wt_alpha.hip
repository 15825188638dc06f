// Alphabet extraction: wt_build with sigma = 0.
//
// The thesis's construction (Section 5.1) works on the minimal alphabet, the distinct values of the
// sequence numbered in increasing order; Section 6.3.1 measures the build both with the alphabet
// extracted from the sequence and with it passed by the caller. Here the extraction is a front end of
// the declared-alphabet build:
//   1. the largest value (u32 sequences; u8/u16 cover their whole range),
//   2. a presence bit per value (LDS words for ranges up to 2^19 values, else global words, each set
//      with an atomic OR only when a read shows it still clear),
//   3. the number of values present before every 64-value word (exclusive scan of the popcounts),
//      which is the code of the word's first value, and sigma = the number of distinct values,
//   4. the value of every code (the sorted distinct values), and the sequence rewritten as codes,
//   5. the declared-alphabet build over the codes with that sigma.
// The tree keeps the presence words (value -> code: the word's count plus a popcount below the bit)
// and the value of every code. Query symbols are mapped to codes before the traversal (a value that
// does not occur maps to sigma, i.e. it is absent: rank 0, select n) and access answers are mapped
// back to values, so every answer is in the caller's values.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

constexpr int kAT = 256;
constexpr uint64_t kALdsWords = 8192;  // 64 KiB of presence bits in LDS: values below 2^19

__global__ __launch_bounds__(kAT) void k_alpha_fill(uint64_t* __restrict__ p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kAT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kAT) p[i] = 0;
}

template <typename E>
__global__ __launch_bounds__(kAT) void k_alpha_max(const E* __restrict__ s, uint64_t n, uint32_t* __restrict__ mx) {
  uint32_t m = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kAT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kAT)
    m = max(m, (uint32_t)s[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
  if ((threadIdx.x & 63u) == 0) atomicMax(mx, m);
}

// Presence bits of every value of s (every value is below 64 nw).
template <typename E>
__global__ __launch_bounds__(kAT) void k_alpha_presence(const E* __restrict__ s, uint64_t n, AWord* __restrict__ aw,
                                                        uint64_t nw) {
  __shared__ unsigned long long s_bits[kALdsWords];
  const bool lds = nw <= kALdsWords;  // uniform over the launch
  if (lds) {
    for (uint64_t w = threadIdx.x; w < nw; w += kAT) s_bits[w] = 0;
    __syncthreads();
  }
  for (uint64_t i = (uint64_t)blockIdx.x * kAT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kAT) {
    const uint32_t v = (uint32_t)s[i];
    const unsigned long long bit = 1ull << (v & 63u);
    if (lds) {
      if (!(s_bits[v >> 6] & bit)) atomicOr(&s_bits[v >> 6], bit);
    } else {
      unsigned long long* p = reinterpret_cast<unsigned long long*>(&aw[v >> 6].bits);
      if (!(*p & bit)) atomicOr(p, bit);
    }
  }
  if (lds) {
    __syncthreads();
    for (uint64_t w = threadIdx.x; w < nw; w += kAT)
      if (s_bits[w]) atomicOr(reinterpret_cast<unsigned long long*>(&aw[w].bits), s_bits[w]);
  }
}

__global__ __launch_bounds__(kAT) void k_alpha_count(const AWord* __restrict__ aw, uint64_t nw,
                                                     uint64_t* __restrict__ cnt) {
  for (uint64_t w = (uint64_t)blockIdx.x * kAT + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * kAT)
    cnt[w] = (uint64_t)__popcll(aw[w].bits);
}

// Codes of the words' first values; total = distinct values.
__global__ __launch_bounds__(kAT) void k_alpha_pre(AWord* __restrict__ aw, uint64_t nw, const uint64_t* __restrict__ pre,
                                                   const uint64_t* __restrict__ cnt, uint64_t* __restrict__ total) {
  for (uint64_t w = (uint64_t)blockIdx.x * kAT + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * kAT) {
    aw[w].pre = (uint32_t)pre[w];
    aw[w].pad = 0;
    if (w == nw - 1) *total = pre[w] + cnt[w];
  }
}

// alpha[code] = value.
__global__ __launch_bounds__(kAT) void k_alpha_list(const AWord* __restrict__ aw, uint64_t nw,
                                                    uint32_t* __restrict__ alpha) {
  for (uint64_t w = (uint64_t)blockIdx.x * kAT + threadIdx.x; w < nw; w += (uint64_t)gridDim.x * kAT) {
    uint64_t b = aw[w].bits;
    uint32_t r = aw[w].pre;
    while (b) {
      const uint32_t j = (uint32_t)__ffsll((unsigned long long)b) - 1u;
      alpha[r++] = (uint32_t)(64 * w + j);
      b &= b - 1;
    }
  }
}

__device__ __forceinline__ uint32_t alpha_code(const AWord& a, uint32_t v) {
  return a.pre + (uint32_t)__popcll(a.bits & ((1ull << (v & 63u)) - 1ull));
}

// The sequence as codes (every value is present).
template <typename E>
__global__ __launch_bounds__(kAT) void k_alpha_remap(const E* __restrict__ s, uint64_t n, const AWord* __restrict__ aw,
                                                     E* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * kAT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kAT) {
    const uint32_t v = (uint32_t)s[i];
    out[i] = (E)alpha_code(aw[v >> 6], v);
  }
}

// Query symbols as codes; values that do not occur become `absent` (= sigma).
__global__ __launch_bounds__(kAT) void k_alpha_map(const AWord* __restrict__ aw, uint64_t nw, uint32_t absent,
                                                   const uint32_t* __restrict__ in, uint64_t q,
                                                   uint32_t* __restrict__ out) {
  for (uint64_t j = (uint64_t)blockIdx.x * kAT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kAT) {
    const uint32_t v = in[j];
    uint32_t c = absent;
    if ((uint64_t)(v >> 6) < nw) {
      const AWord a = aw[v >> 6];
      if ((a.bits >> (v & 63u)) & 1ull) c = alpha_code(a, v);
    }
    out[j] = c;
  }
}

// Access answers (codes) back to values; the out-of-range sentinel stays.
__global__ __launch_bounds__(kAT) void k_alpha_unmap(const uint32_t* __restrict__ alpha, uint32_t sigma,
                                                     uint32_t* __restrict__ out, uint64_t q) {
  for (uint64_t j = (uint64_t)blockIdx.x * kAT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kAT) {
    const uint32_t x = out[j];
    if (x < sigma) out[j] = alpha[x];
  }
}

static uint32_t grid_for(uint64_t n) { return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(ceil_div(n, kAT), 1), 8192); }

wt_status alpha_map_syms(const wt_tree* t, const uint32_t* d_sym, uint64_t q, hipStream_t st, const uint32_t** mapped,
                         void** scratch, uint32_t* buf) {
  *mapped = d_sym;
  *scratch = nullptr;
  if (!t->amap || q == 0) return WT_OK;
  uint32_t* m = buf ? buf : (uint32_t*)dev_alloc(q * 4, st);
  if (!m) return fail(WT_ERR_OOM, "symbol mapping: allocation of %llu bytes failed", (unsigned long long)(q * 4));
  hipLaunchKernelGGL(k_alpha_map, dim3(grid_for(q)), dim3(kAT), 0, st, t->amap, t->amap_words, (uint32_t)t->sigma,
                     d_sym, q, m);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (!buf) dev_free(m, st);
    return fail(WT_ERR_HIP, "symbol mapping: %s", hipGetErrorString(e));
  }
  *mapped = m;
  *scratch = buf ? nullptr : m;
  return WT_OK;
}

wt_status alpha_unmap_access(const wt_tree* t, uint32_t* d_out, uint64_t q, hipStream_t st) {
  if (!t->alpha || q == 0) return WT_OK;
  hipLaunchKernelGGL(k_alpha_unmap, dim3(grid_for(q)), dim3(kAT), 0, st, t->alpha, (uint32_t)t->sigma, d_out, q);
  WT_HIP(hipGetLastError());
  return WT_OK;
}

namespace {

template <typename E>
hipError_t launch_presence(const void* s, uint64_t n, AWord* aw, uint64_t nw, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(ceil_div(n, (uint64_t)kAT * 64), 4096);
  hipLaunchKernelGGL(k_alpha_presence<E>, dim3(grid), dim3(kAT), 0, st, (const E*)s, n, aw, nw);
  return hipGetLastError();
}

template <typename E>
hipError_t launch_remap(const void* s, uint64_t n, const AWord* aw, void* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_alpha_remap<E>, dim3(grid_for(n)), dim3(kAT), 0, st, (const E*)s, n, aw, (E*)out);
  return hipGetLastError();
}

}  // namespace
}  // namespace wt

using namespace wt;

extern "C" wt_status wt_build(const void* d_sym, uint64_t n, uint32_t sym_bytes, uint64_t sigma,
                              const wt_build_opts* opts, wt_stream_t stream, wt_tree** out) {
  clear_error();
  if (sigma != 0) return build_tree(d_sym, n, sym_bytes, sigma, opts, stream, out);
  if (!out) return fail(WT_ERR_ARG, "wt_build: out is NULL");
  *out = nullptr;
  if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4)
    return fail(WT_ERR_ARG, "wt_build: sym_bytes must be 1, 2 or 4 (got %u)", sym_bytes);
  if (n && !d_sym) return fail(WT_ERR_ARG, "wt_build: d_sym is NULL");
  if (n >= (1ull << 40)) return fail(WT_ERR_ARG, "wt_build: n too large");
  const wt_status orc = check_build_opts(opts);
  if (orc != WT_OK) return orc;
  hipStream_t st = (hipStream_t)stream;

  // device buffers released on every exit: the scratch always, the map unless a tree takes it
  struct Bufs {
    hipStream_t st;
    void* scratch = nullptr;
    void* aw = nullptr;
    void* alpha = nullptr;
    ~Bufs() {
      if (scratch) dev_free(scratch, st);
      if (aw) dev_free(aw, st);
      if (alpha) dev_free(alpha, st);
    }
  } B{st};

  // 1. value range
  uint64_t nw = sym_bytes == 4 ? 1 : (1ull << (8 * sym_bytes)) / 64;
  const size_t o_seq = 0, o_small = round_up(std::max<uint64_t>(n, 1) * sym_bytes, 256);
  B.scratch = dev_alloc(o_small + 256, st);
  if (!B.scratch) return fail(WT_ERR_OOM, "wt_build: scratch allocation failed");
  char* sb = (char*)B.scratch;
  uint64_t* small = (uint64_t*)(sb + o_small);  // [0]: largest value, [1]: distinct values
  hipLaunchKernelGGL(k_alpha_fill, dim3(1), dim3(kAT), 0, st, small, 2ull);
  uint32_t maxv = 0;
  if (sym_bytes == 4 && n) {
    hipLaunchKernelGGL(k_alpha_max<uint32_t>, dim3(grid_for(n)), dim3(kAT), 0, st, (const uint32_t*)d_sym, n,
                       (uint32_t*)small);
    WT_HIP(hipGetLastError());
    WT_HIP(hipMemcpyAsync(&maxv, small, 4, hipMemcpyDeviceToHost, st));
    WT_HIP(hipStreamSynchronize(st));
    nw = (uint64_t)maxv / 64 + 1;
  }
  // 2. presence words
  B.aw = dev_alloc(nw * sizeof(AWord), st);
  if (!B.aw) return fail(WT_ERR_OOM, "wt_build: alphabet map allocation of %llu bytes failed",
                         (unsigned long long)(nw * sizeof(AWord)));
  AWord* aw = (AWord*)B.aw;
  hipLaunchKernelGGL(k_alpha_fill, dim3(grid_for(2 * nw)), dim3(kAT), 0, st, (uint64_t*)aw, 2 * nw);
  hipError_t he = sym_bytes == 1   ? launch_presence<uint8_t>(d_sym, n, aw, nw, st)
                  : sym_bytes == 2 ? launch_presence<uint16_t>(d_sym, n, aw, nw, st)
                                   : launch_presence<uint32_t>(d_sym, n, aw, nw, st);
  if (he != hipSuccess) return fail(WT_ERR_HIP, "wt_build: alphabet presence: %s", hipGetErrorString(he));
  // 3. codes of the words' first values and the number of distinct values
  const uint64_t nparts = ceil_div(nw, 4096) + 1;
  uint64_t* cs = (uint64_t*)dev_alloc((2 * nw + nparts) * 8, st);
  if (!cs) return fail(WT_ERR_OOM, "wt_build: alphabet scan allocation failed");
  hipLaunchKernelGGL(k_alpha_count, dim3(grid_for(nw)), dim3(kAT), 0, st, (const AWord*)aw, nw, cs);
  he = exclusive_scan_u64(cs, nw, cs + nw, cs + 2 * nw, st);
  if (he == hipSuccess) {
    hipLaunchKernelGGL(k_alpha_pre, dim3(grid_for(nw)), dim3(kAT), 0, st, aw, nw, (const uint64_t*)(cs + nw),
                       (const uint64_t*)cs, small + 1);
    he = hipGetLastError();
  }
  uint64_t distinct = 0;
  if (he == hipSuccess) he = hipMemcpyAsync(&distinct, small + 1, 8, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  dev_free(cs, st);
  if (he != hipSuccess) return fail(WT_ERR_HIP, "wt_build: alphabet scan: %s", hipGetErrorString(he));
  if (distinct > WT_MAX_SIGMA)
    return fail(WT_ERR_ARG, "wt_build: %llu distinct symbols exceed %llu", (unsigned long long)distinct,
                (unsigned long long)WT_MAX_SIGMA);
  // an empty sequence has no symbol: a one-symbol alphabet that no query value maps to
  const uint64_t sig = std::max<uint64_t>(distinct, 1);
  // 4. value of every code, sequence as codes
  B.alpha = dev_alloc(sig * 4, st);
  if (!B.alpha) return fail(WT_ERR_OOM, "wt_build: alphabet allocation failed");
  if (distinct == 0) {
    const uint32_t zero = 0;
    WT_HIP(hipMemcpyAsync(B.alpha, &zero, 4, hipMemcpyHostToDevice, st));
  }
  hipLaunchKernelGGL(k_alpha_list, dim3(grid_for(nw)), dim3(kAT), 0, st, (const AWord*)aw, nw, (uint32_t*)B.alpha);
  he = sym_bytes == 1   ? launch_remap<uint8_t>(d_sym, n, aw, sb + o_seq, st)
       : sym_bytes == 2 ? launch_remap<uint16_t>(d_sym, n, aw, sb + o_seq, st)
                        : launch_remap<uint32_t>(d_sym, n, aw, sb + o_seq, st);
  if (he != hipSuccess) return fail(WT_ERR_HIP, "wt_build: alphabet remap: %s", hipGetErrorString(he));
  // 5. the declared-alphabet build over the codes
  wt_tree* t = nullptr;
  const wt_status rc = build_tree(n ? sb + o_seq : nullptr, n, sym_bytes, sig, opts, stream, &t);
  if (rc != WT_OK) return rc;
  if (sym_bytes < 4) {
    uint32_t last = 0;
    if (distinct) WT_HIP(hipMemcpy(&last, (const uint32_t*)B.alpha + (distinct - 1), 4, hipMemcpyDeviceToHost));
    maxv = last;
  }
  t->alpha_block = B.aw;
  t->amap = aw;
  t->amap_words = nw;
  t->alpha = (const uint32_t*)B.alpha;
  t->max_symbol = maxv;
  B.aw = nullptr;
  B.alpha = nullptr;
  *out = t;
  return WT_OK;
}
