// Construction of the level-wise wavelet tree on gfx950 (Section 5.1, Algorithm 4).
//
// Pipeline on one stream, no host synchronisation until the end:
//   k_init        level metadata and cleared counters
//   k_hist        histogram + out-of-range flag + per-tile ones of level 0 (codes computed on the fly)
//   scan          cumulative histogram (exclusive prefix sums, Section 5: node boundaries)
//   k_node_walk   every node (by code prefix) -> its symbol range -> left-child size
//   scan + k_node_final
//                 precomputed node-start ranks and per-node partition offsets, derived from
//                 the histogram alone, plus the level sizes
//   per level l:  k_tile_scan  exclusive prefix of the ones per tile (= L1 values at tile starts)
//                 k_level      one pass over level l: 64-bit bit words, L1/L2 entries, select
//                              samples, and the stable 0/1 partition into level l + 1 (replacing the
//                              thesis's radix sort by the bits above the level), plus the ones per
//                              tile of level l + 1
//
// Partition rule: the level-(l+1) position of the level-l element at position p with bit b in node
// N is off_b[N] + rank_b(p), where off0[N] = start(N) - R0[N] and
// off1[N] = start(N) + zeros(N) - (start(N) - R0[N]). R0[N] (rank0 at the node start) equals the
// number of occurrences of the symbols left of N whose bit at this level is 0, so it is known
// before the level is built.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "wt_build_dev.h"
#include "wt_host.h"
#include "wt_huff.h"
#include "wt_internal.h"

namespace wt {

// ---------------------------------------------------------------- single-tree kernels

__global__ __launch_bounds__(kBT) void k_scan_reduce(const uint64_t* __restrict__ in, uint64_t n,
                                                     uint64_t* __restrict__ part) {
  scan_reduce_body(in, n, part, blockIdx.x);
}

// Single block: exclusive scan of np partial sums in place.
__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t* __restrict__ part, uint64_t np) {
  scan_partials_body(part, np);
}

__global__ __launch_bounds__(kBT) void k_scan_down(const uint64_t* __restrict__ in, uint64_t n,
                                                   const uint64_t* __restrict__ part, uint64_t* __restrict__ out) {
  scan_down_body(in, n, part, out, blockIdx.x);
}

// out[i] = sum of in[0, i) for i in [0, n); `part` needs ceil(n / kScanChunk) entries.
hipError_t exclusive_scan_u64(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* part,
                                     hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t nb = ceil_div(n, kScanChunk);
  hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(kBT), 0, st, in, n, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, part, nb);
  hipLaunchKernelGGL(k_scan_down, dim3((uint32_t)nb), dim3(kBT), 0, st, in, n, (const uint64_t*)part, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- init

struct InitArgs {
  LevelMeta meta[WT_MAX_LEVELS];
  uint32_t L;
};

__global__ void k_init_meta(InitArgs a, LevelMeta* __restrict__ meta) {
  const uint32_t l = threadIdx.x;
  if (l < a.L) meta[l] = a.meta[l];
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  fill_body(p, n, v, blockIdx.x, gridDim.x);
}

template <typename E, uint32_t kWords>
__global__ __launch_bounds__(kHT) void k_hist_dense(const E* __restrict__ sym, uint64_t n, uint32_t sigma, uint32_t L,
                                                    uint32_t aligned, uint64_t* __restrict__ hist,
                                                    uint64_t* __restrict__ tile_cnt0, uint32_t* __restrict__ err) {
  hist_dense_body<E, kWords>(sym, n, sigma, L, aligned, hist, tile_cnt0, err, blockIdx.x, gridDim.x);
}

template <typename E>
__global__ __launch_bounds__(kHT) void k_hist_gcount(const E* __restrict__ sym, uint64_t n, uint32_t sigma, uint32_t L,
                                                     uint32_t aligned, uint64_t* __restrict__ gcnt,
                                                     uint64_t* __restrict__ tile_cnt0, uint32_t* __restrict__ err) {
  hist_group_count_body<E>(sym, n, sigma, L, aligned, gcnt, tile_cnt0, err, blockIdx.x, gridDim.x);
}

template <typename E>
__global__ __launch_bounds__(kHT) void k_hist_gscatter(const E* __restrict__ sym, uint64_t n, uint32_t sigma,
                                                       uint32_t aligned, const uint64_t* __restrict__ goff,
                                                       E* __restrict__ dst) {
  hist_group_scatter_body<E>(sym, n, sigma, aligned, goff, dst, blockIdx.x, gridDim.x);
}

template <typename E>
__global__ __launch_bounds__(kHT) void k_hist_wcount(const E* __restrict__ src, const uint64_t* __restrict__ goff,
                                                     uint64_t nblk1, uint32_t sigma, uint64_t* __restrict__ hist) {
  hist_window_count_body<E>(src, goff, nblk1, sigma, hist, blockIdx.x);
}

__global__ void k_node_walk(uint32_t sigma, uint64_t nheap, const uint64_t* __restrict__ cum,
                            NodeB* __restrict__ ntb, uint64_t* __restrict__ zeros) {
  node_walk_body(sigma, nheap, cum, ntb, zeros, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ void k_node_final(uint64_t nheap, const uint64_t* __restrict__ zs, NodeB* __restrict__ ntb,
                             NodeQ* __restrict__ ntq, LevelMeta* __restrict__ meta) {
  node_final_body(nheap, zs, ntb, ntq, meta, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kBT) void k_tile_reduce(const LevelMeta* __restrict__ meta, uint32_t l,
                                                     uint32_t tshift, const uint64_t* __restrict__ cnt,
                                                     uint64_t* __restrict__ chunk) {
  tile_reduce_body(meta, l, tshift, cnt, chunk, blockIdx.x);
}

__global__ __launch_bounds__(kBT) void k_tile_scan(LevelMeta* __restrict__ meta, uint32_t l, uint32_t tshift,
                                                   const uint64_t* __restrict__ cnt,
                                                   const uint64_t* __restrict__ chunk, uint64_t* __restrict__ pre,
                                                   uint64_t* __restrict__ L1, uint16_t* __restrict__ L2) {
  tile_scan_body(meta, l, tshift, cnt, chunk, pre, L1, L2, blockIdx.x);
}



// ---------------------------------------------------------------- wavelet matrix

// Bit-reversal of the low L bits of x (L >= 1).
__device__ __forceinline__ uint32_t rev_low(uint32_t x, uint32_t L) { return __brev(x) >> (32u - L); }

// Ones of every level of a wavelet matrix from the cumulative histogram: level l holds every element,
// and its bit is bit k = L-1-l of the symbol, set on the ranges [(2j+1) 2^k, (2j+2) 2^k) of symbols.
// Grid (blocks, L): each block adds its share of the ranges of level blockIdx.y.
__global__ __launch_bounds__(kBT) void k_wm_ones(const uint64_t* __restrict__ cum, uint32_t sigma, uint32_t L,
                                                 uint64_t* __restrict__ ones) {
  __shared__ uint64_t s_w[kBT / 64];
  const uint32_t l = blockIdx.y, k = L - 1 - l;
  const uint64_t step = 1ull << k;
  const uint64_t nr = sigma > step ? ((uint64_t)sigma - step + 2 * step - 1) >> (k + 1) : 0ull;
  uint64_t sum = 0;
  for (uint64_t j = (uint64_t)blockIdx.x * kBT + threadIdx.x; j < nr; j += (uint64_t)gridDim.x * kBT) {
    const uint64_t a = (2 * j + 1) << k, b = min<uint64_t>((2 * j + 2) << k, sigma);
    sum += cum[b] - cum[a];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (uint32_t w = 0; w < kBT / 64; ++w) t += s_w[w];
    if (t) atomic_add_u64(ones + l, t);
  }
}

// Node table of the level passes (one node per level: zeros to [0, Z_l), ones from Z_l) and the level
// sizes (every level holds all n elements).
__global__ void k_wm_final(uint64_t n, uint32_t L, const uint64_t* __restrict__ ones, NodeB* __restrict__ ntb,
                           LevelMeta* __restrict__ meta) {
  const uint32_t l = threadIdx.x;
  if (l >= L) return;
  NodeB b;
  b.start = 0;
  b.end = n;
  b.off0 = 0;
  b.off1 = n - ones[l];
  ntb[l] = b;
  meta[l].n = n;
}

// rc[rev_L(c)] = count of c (0 for the reversed codes of no symbol), for the 2^L codes.
__global__ __launch_bounds__(kBT) void k_wm_rcount(const uint64_t* __restrict__ hist, uint32_t sigma, uint32_t L,
                                                   uint64_t* __restrict__ rc) {
  const uint64_t nc = 1ull << L;
  for (uint64_t c = (uint64_t)blockIdx.x * kBT + threadIdx.x; c < nc; c += (uint64_t)gridDim.x * kBT)
    rc[rev_low((uint32_t)c, L)] = c < sigma ? hist[c] : 0ull;
}

// start[c] = elements whose reversed code is below rev_L(c) (exclusive scan rs of rc).
__global__ __launch_bounds__(kBT) void k_wm_starts(const uint64_t* __restrict__ rs, uint32_t sigma, uint32_t L,
                                                   uint64_t* __restrict__ wstart) {
  for (uint64_t c = (uint64_t)blockIdx.x * kBT + threadIdx.x; c < sigma; c += (uint64_t)gridDim.x * kBT)
    wstart[c] = rs[rev_low((uint32_t)c, L)];
}

// ---------------------------------------------------------------- nodes by position (narrow codes)

// flag[h] = 1 for a non-empty node (heap entry h), flag[nheap] = 0.
__global__ __launch_bounds__(kBT) void k_ns_flag(const NodeB* __restrict__ ntb, uint64_t nheap, uint64_t* __restrict__ flag) {
  const uint64_t h = (uint64_t)blockIdx.x * kBT + threadIdx.x;
  if (h < nheap) flag[h] = (ntb[h].start != kNoNode && ntb[h].end > ntb[h].start) ? 1ull : 0ull;
  else if (h == nheap) flag[h] = 0;
}

// The non-empty nodes in heap order (= position order within a level), at the exclusive scan of the flags.
__global__ __launch_bounds__(kBT) void k_ns_scatter(const NodeB* __restrict__ ntb, uint64_t nheap,
                                                    const uint64_t* __restrict__ idx, NodeS* __restrict__ ns) {
  const uint64_t h = (uint64_t)blockIdx.x * kBT + threadIdx.x;
  if (h >= nheap || idx[h + 1] == idx[h]) return;
  const uint32_t l = 63u - (uint32_t)__clzll(h + 1);
  NodeS e;
  e.start = ntb[h].start;
  e.pfx = (uint32_t)(h + 1 - (1ull << l));
  e.pad = 0;
  ns[idx[h]] = e;
}

// Per tile of level l (2^tshift elements): the node holding its first element, as an index from the
// level's first entry of the position list (the last entry starting at or before the tile).
__global__ __launch_bounds__(kBT) void k_tile_first(const LevelMeta* __restrict__ meta, uint32_t l, uint32_t tshift,
                                                    const NodeS* __restrict__ ns, const uint64_t* __restrict__ idx,
                                                    uint32_t* __restrict__ tfirst) {
  const uint64_t t = (uint64_t)blockIdx.x * kBT + threadIdx.x;
  const uint64_t x = t << tshift;
  if (x >= meta[l].n) return;
  const uint64_t lo = idx[(1ull << l) - 1], hi = idx[(2ull << l) - 1];
  uint64_t a = lo, b = hi - 1;
  while (a < b) {
    const uint64_t mid = (a + b + 1) >> 1;
    if (ns[mid].start <= x) a = mid;
    else b = mid - 1;
  }
  tfirst[t] = (uint32_t)(a - lo);
}

// ---------------------------------------------------------------- host orchestration

namespace {

struct Prof {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> ev;
  std::vector<wt_prof_entry> ent;
  hipError_t begin(const char* name, int level) {
    if (!on) return hipSuccess;
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    ev.push_back(a);
    ev.push_back(b);
    wt_prof_entry p{};
    std::strncpy(p.kernel, name, sizeof(p.kernel) - 1);
    p.level = level;
    ent.push_back(p);
    return hipEventRecord(a, st);
  }
  hipError_t end() {
    if (!on) return hipSuccess;
    return hipEventRecord(ev.back(), st);
  }
  void collect(std::vector<wt_prof_entry>& out) {
    for (size_t i = 0; i < ent.size(); ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) ent[i].ms = ms;
    }
    out = ent;
  }
  ~Prof() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

struct Scratch {
  void* block = nullptr;
  hipStream_t st = nullptr;
  ~Scratch() {
    if (block) dev_free(block, st);
  }
};

// Buffers of the histogram phase; gcnt, goff and seq only for alphabets above kHDenseMax.
struct HistBufs {
  uint64_t* hist;
  uint64_t* cnt0;
  uint32_t* err;
  uint64_t* gcnt;  // windows x blocks + 1 (radix step)
  uint64_t* goff;  // its exclusive scan
  uint64_t* part;  // scan partials
  void* seq;       // n symbols in window order
};

// Entries of gcnt for an alphabet above kHDenseMax (0 otherwise).
inline uint64_t hist_gcnt_entries(uint64_t n, uint32_t w, uint64_t sigma) {
  if (sigma <= kHDenseMax || n == 0) return 0;
  const uint64_t ntiles = ceil_div(n, tile_elems(w));
  const uint64_t G = ceil_div(sigma, 1ull << kHWinShift);
  return G * hist_dense_blocks(ntiles, hist_tiles_per_block(ntiles)) + 1;
}

template <typename E>
hipError_t launch_hist(const void* d_sym, uint64_t n, uint32_t sigma, uint32_t L, const HistBufs& hb, hipStream_t st) {
  using TL = Tile<E>;
  const uint64_t ntiles = ceil_div(n, TL::T);
  if (ntiles == 0) return hipSuccess;
  const uint32_t aligned = ((uintptr_t)d_sym & 15u) == 0;
  const uint32_t grid = (uint32_t)hist_dense_blocks(ntiles, hist_tiles_per_block(ntiles));
  if (sigma <= kHDenseMax) {
    if (sigma + 1 <= kHSmallWords)
      hipLaunchKernelGGL((k_hist_dense<E, kHSmallWords>), dim3(grid), dim3(kHT), 0, st, (const E*)d_sym, n, sigma,
                         L, aligned, hb.hist, hb.cnt0, hb.err);
    else
      hipLaunchKernelGGL((k_hist_dense<E, kHBigWords>), dim3(grid), dim3(kHT), 0, st, (const E*)d_sym, n, sigma, L,
                         aligned, hb.hist, hb.cnt0, hb.err);
    return hipGetLastError();
  }
  const uint64_t G = ceil_div(sigma, 1ull << kHWinShift);
  hipLaunchKernelGGL(k_hist_gcount<E>, dim3(grid), dim3(kHT), 0, st, (const E*)d_sym, n, sigma, L, aligned, hb.gcnt,
                     hb.cnt0, hb.err);
  hipError_t he = exclusive_scan_u64(hb.gcnt, G * grid + 1, hb.goff, hb.part, st);
  if (he != hipSuccess) return he;
  hipLaunchKernelGGL(k_hist_gscatter<E>, dim3(grid), dim3(kHT), 0, st, (const E*)d_sym, n, sigma, aligned,
                     (const uint64_t*)hb.goff, (E*)hb.seq);
  hipLaunchKernelGGL(k_hist_wcount<E>, dim3((uint32_t)ceil_div(n, kHWinChunk)), dim3(kHT), 0, st,
                     (const E*)hb.seq, (const uint64_t*)hb.goff, (uint64_t)grid, sigma, hb.hist);
  return hipGetLastError();
}

// Histogram of d_sym on its own, copied to the host, with the symbol-range check: the first step of a
// Huffman-shaped build, whose levels depend on the counts. Scratch of its own.
wt_status huff_prepass(const void* d_sym, uint64_t n, uint32_t w, uint64_t sigma, hipStream_t st,
                       std::vector<uint64_t>& hist) {
  hist.assign(sigma, 0ull);
  if (n == 0) return WT_OK;
  const size_t o_err = round_up((sigma + 1) * 8, 256);
  const size_t o_hs = o_err + 256;
  const size_t so = o_hs + hist_add_scratch_bytes(n, w, sigma);
  Scratch S;
  S.st = st;
  S.block = dev_alloc(so, st);
  if (!S.block) return fail(WT_ERR_OOM, "wt_build: scratch allocation of %zu bytes failed", so);
  char* sb = (char*)S.block;
  uint64_t* h = (uint64_t*)sb;
  uint32_t* err = (uint32_t*)(sb + o_err);
  hipLaunchKernelGGL(k_fill_u64, dim3(64), dim3(kBT), 0, st, h, sigma + 1, 0ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, (uint64_t*)err, 8ull, 0ull);
  WT_HIP(hipGetLastError());
  WT_HIP(hist_add(d_sym, n, w, sigma, h, err, sb + o_hs, st));
  uint32_t bad = 0;
  WT_HIP(hipMemcpyAsync(hist.data(), h, sigma * 8, hipMemcpyDeviceToHost, st));
  WT_HIP(hipMemcpyAsync(&bad, err, 4, hipMemcpyDeviceToHost, st));
  WT_HIP(hipStreamSynchronize(st));
  if (bad) return fail(WT_ERR_SYMBOL_RANGE, "wt_build: a symbol is >= sigma (%llu)", (unsigned long long)sigma);
  return WT_OK;
}

template <typename E, typename EO = E, bool kPos = false>
hipError_t launch_level(const LevelArgs& a, uint64_t n, hipStream_t st) {
  using TL = Tile<E>;
  const uint64_t nt = ceil_div(n, TL::T);
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL((k_level<E, false, EO, kPos>), dim3((uint32_t)nt), dim3(kBT), 0, st, a, ForestGrid{});
  return hipGetLastError();
}

// Level pass for input width wi, output width wo (bytes) and the node lookup of the level.
hipError_t launch_level_w(const LevelArgs& a, uint64_t n, uint32_t wi, uint32_t wo, hipStream_t st) {
  if (a.pos_node) {
    if (wi == 1) return launch_level<uint8_t, uint8_t, true>(a, n, st);
    if (wi == 2) return wo == 1 ? launch_level<uint16_t, uint8_t, true>(a, n, st)
                                : launch_level<uint16_t, uint16_t, true>(a, n, st);
    return wo == 1 ? launch_level<uint32_t, uint8_t, true>(a, n, st) : launch_level<uint32_t, uint16_t, true>(a, n, st);
  }
  if (wi == 1) return launch_level<uint8_t>(a, n, st);
  if (wi == 2) return wo == 1 ? launch_level<uint16_t, uint8_t>(a, n, st) : launch_level<uint16_t>(a, n, st);
  return wo == 1 ? launch_level<uint32_t, uint8_t>(a, n, st)
                 : wo == 2 ? launch_level<uint32_t, uint16_t>(a, n, st) : launch_level<uint32_t>(a, n, st);
}

}  // namespace

TreePlan plan_tree(uint64_t n, uint32_t w, uint64_t sigma, uint32_t L, uint32_t l2_bits, uint32_t srate,
                   bool matrix, bool huff) {
  TreePlan p{};
  p.n = n;
  p.sigma = sigma;
  p.L = L;
  p.w = w;
  p.l2_bits = l2_bits;
  p.srate = srate;
  p.tile = tile_elems(w);
  // capacity: whole tiles plus one L2 block of slack (queries read the whole L2 block at i = n_l),
  // rounded to 128-byte lines so every level starts on a line. A level pass writes every bit word of
  // its last tile, and a level of narrowed 1-byte codes has the longest tiles (kTileBytes elements).
  const uint64_t cap_bits = round_up(round_up(std::max<uint64_t>(n, 1), tile_elems(1)) + 2048, 1024);
  p.words_per_level = cap_bits / 64;
  p.l1_per_level = round_up(ceil_div(n, kL1Bits) + 1, 16);
  // + one group of slack: a select reads up to 40 entries from the vector of its first candidate
  p.l2_per_level = round_up(ceil_div(n, l2_bits) + 1 + 64, 64);
  p.smp_per_level = round_up(n / srate + 1, 16);
  p.nheap = L ? ((1ull << L) - 1) : 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  // level metadata, then one more entry holding the build's symbol-range flag (read back with them)
  p.off_meta = take(sizeof(LevelMeta) * (WT_MAX_LEVELS + 1));
  p.off_cum = take((sigma + 1) * sizeof(uint64_t));
  p.off_nodes = take(matrix ? sizeof(NodeQ) : std::max<uint64_t>(p.nheap, 1) * sizeof(NodeQ));
  p.off_wstart = take(matrix ? std::max<uint64_t>(sigma, 1) * sizeof(uint64_t) : 0);
  p.off_huff = take(huff ? huff_table_bytes(sigma) : 0);
  p.off_bits = take((size_t)L * p.words_per_level * sizeof(uint64_t));
  p.off_l1 = take((size_t)L * p.l1_per_level * sizeof(uint64_t));
  p.off_l2 = take((size_t)L * p.l2_per_level * sizeof(uint16_t));
  p.off_smp = take((size_t)L * p.smp_per_level * sizeof(uint64_t));
  p.total = off;
  return p;
}

// Scratch of hist_add: tile counts it also makes (not used), and for alphabets above the dense
// histogram the window counts, their scan and the symbols in window order.
size_t hist_add_scratch_bytes(uint64_t n, uint32_t w, uint64_t sigma) {
  const uint64_t ntiles = ceil_div(std::max<uint64_t>(n, 1), tile_elems(w));
  const uint64_t gcnt_n = hist_gcnt_entries(n, w, sigma);
  return round_up((ntiles + 1) * 8, 256) + 2 * round_up(gcnt_n * 8, 256) +
         round_up((ceil_div(std::max<uint64_t>(gcnt_n, 1), kScanChunk) + 1) * 8, 256) +
         round_up(gcnt_n ? n * w : 0, 256);
}

hipError_t hist_add(const void* d_sym, uint64_t n, uint32_t w, uint64_t sigma, uint64_t* hist, uint32_t* err,
                    char* sb, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t ntiles = ceil_div(n, tile_elems(w));
  const uint64_t gcnt_n = hist_gcnt_entries(n, w, sigma);
  const size_t o_gcnt = round_up((ntiles + 1) * 8, 256);
  const size_t o_goff = o_gcnt + round_up(gcnt_n * 8, 256);
  const size_t o_part = o_goff + round_up(gcnt_n * 8, 256);
  const size_t o_seq = o_part + round_up((ceil_div(std::max<uint64_t>(gcnt_n, 1), kScanChunk) + 1) * 8, 256);
  // the level-0 tile counts the histogram kernels also make (bit 0 of the symbols) are not used
  const HistBufs hb{hist, (uint64_t*)sb, err, (uint64_t*)(sb + o_gcnt), (uint64_t*)(sb + o_goff),
                    (uint64_t*)(sb + o_part), sb + o_seq};
  if (w == 1) return launch_hist<uint8_t>(d_sym, n, (uint32_t)sigma, 1, hb, st);
  if (w == 2) return launch_hist<uint16_t>(d_sym, n, (uint32_t)sigma, 1, hb, st);
  return launch_hist<uint32_t>(d_sym, n, (uint32_t)sigma, 1, hb, st);
}

hipError_t init_levels(const TreePlan& P, LevelMeta* d_meta, LevelMeta* h_meta, hipStream_t st) {
  InitArgs ia{};
  ia.L = P.L;
  for (uint32_t l = 0; l < P.L; ++l) {
    LevelMeta& mm = ia.meta[l];
    mm.bits = (uint64_t)l * P.words_per_level;
    mm.l1 = (uint64_t)l * P.l1_per_level;
    mm.l2 = (uint64_t)l * P.l2_per_level;
    mm.smp = (uint64_t)l * P.smp_per_level;
    mm.smp_cap = P.smp_per_level;
    h_meta[l] = mm;
  }
  hipLaunchKernelGGL(k_init_meta, dim3(1), dim3(64), 0, st, ia, d_meta);
  return hipGetLastError();
}

hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)std::min<uint64_t>(ceil_div(n, kBT), 4096)), dim3(kBT), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t node_tables(uint32_t sigma, uint64_t nheap, const uint64_t* cum, NodeB* ntb, uint64_t* z, uint64_t* zs,
                       uint64_t* part, NodeQ* nodes, LevelMeta* meta, hipStream_t st) {
  if (nheap == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)ceil_div(nheap, kBT);
  hipLaunchKernelGGL(k_node_walk, dim3(nb), dim3(kBT), 0, st, sigma, nheap, cum, ntb, z);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, z + nheap, 1ull, 0ull);
  hipError_t he = hipGetLastError();
  if (he != hipSuccess) return he;
  he = exclusive_scan_u64(z, nheap + 1, zs, part, st);
  if (he != hipSuccess) return he;
  hipLaunchKernelGGL(k_node_final, dim3(nb), dim3(kBT), 0, st, nheap, (const uint64_t*)zs, ntb, nodes, meta);
  return hipGetLastError();
}

}  // namespace wt

using namespace wt;

wt_status wt::check_build_opts(const wt_build_opts* opts) {
  const uint32_t l2_bits = opts && opts->l2_bits ? opts->l2_bits : 512;
  const uint32_t srate = opts && opts->sample_rate ? opts->sample_rate : 4096;
  if (l2_bits != 256 && l2_bits != 512 && l2_bits != 1024 && l2_bits != 2048)
    return fail(WT_ERR_ARG, "wt_build: l2_bits must be 256, 512, 1024 or 2048");
  if (srate < 512 || srate > (1u << 20) || (srate & (srate - 1)))
    return fail(WT_ERR_ARG, "wt_build: sample_rate must be a power of two in [512, 2^20]");
  return WT_OK;
}

// The build of wt_build for a declared alphabet (sigma >= 1); wt_build (wt_alpha.hip) first extracts
// the alphabet when sigma = 0.
wt_status wt::build_tree(const void* d_sym, uint64_t n, uint32_t sym_bytes, uint64_t sigma, const wt_build_opts* opts,
                         wt_stream_t stream, wt_tree** out, NodeB* ntb_out) {
  if (!out) return fail(WT_ERR_ARG, "wt_build: out is NULL");
  *out = nullptr;
  if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4)
    return fail(WT_ERR_ARG, "wt_build: sym_bytes must be 1, 2 or 4 (got %u)", sym_bytes);
  if (n && !d_sym) return fail(WT_ERR_ARG, "wt_build: d_sym is NULL");
  if (sigma == 0) return fail(WT_ERR_ARG, "wt_build: sigma must be >= 1 (declared alphabet size)");
  if (sigma > WT_MAX_SIGMA) return fail(WT_ERR_ARG, "wt_build: sigma %llu exceeds %llu",
                                        (unsigned long long)sigma, (unsigned long long)WT_MAX_SIGMA);
  if (sym_bytes < 4 && sigma > (1ull << (8 * sym_bytes)))
    return fail(WT_ERR_ARG, "wt_build: sigma %llu does not fit %u-byte symbols", (unsigned long long)sigma,
                sym_bytes);
  if (n >= (1ull << 40)) return fail(WT_ERR_ARG, "wt_build: n too large");
  const wt_status orc = check_build_opts(opts);
  if (orc != WT_OK) return orc;
  uint32_t l2_bits = 512, srate = 4096, flags = 0;
  if (opts) {
    if (opts->l2_bits) l2_bits = opts->l2_bits;
    if (opts->sample_rate) srate = opts->sample_rate;
    flags = opts->flags;
  }

  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  WT_HIP(hipGetDevice(&dev));

  uint32_t L = 0;
  while ((1ull << L) < sigma) ++L;
  const bool matrix = (flags & WT_BUILD_MATRIX) != 0;
  const bool huff = (flags & WT_BUILD_HUFFMAN) != 0;
  if (huff && matrix) return fail(WT_ERR_ARG, "wt_build: WT_BUILD_HUFFMAN and WT_BUILD_MATRIX do not combine");
  // Huffman-shaped: the counts fix the codes and so the levels; the first level pass then reads the
  // symbols rewritten as codes of wc bytes
  HuffCode hc;
  std::vector<uint64_t> hh;
  uint32_t wc = sym_bytes;
  if (huff) {
    const wt_status hr = huff_prepass(d_sym, n, sym_bytes, sigma, st, hh);
    if (hr != WT_OK) return hr;
    huff_code(hh.data(), sigma, hc);
    L = hc.L;
    wc = L <= 8 ? 1u : L <= 16 ? 2u : 4u;
  }
  // a wavelet matrix uses the plain L-bit symbols as codes, whatever sigma; a Huffman-shaped tree its
  // canonical codes (no reduced-code step)
  const uint32_t pow2 = matrix || huff || (sigma & (sigma - 1)) == 0;
  const TreePlan P = plan_tree(n, wc, sigma, L, l2_bits, srate, matrix, huff);

  wt_tree* t = new wt_tree();
  t->n = n;
  t->sigma = sigma;
  t->L = L;
  t->w = sym_bytes;
  t->l2_bits = l2_bits;
  t->srate = srate;
  t->pow2 = pow2;
  t->matrix = matrix ? 1u : 0u;
  t->huff = huff ? 1u : 0u;
  t->device = dev;
  t->block_bytes = P.total;
  t->block = dev_alloc(P.total, st);
  if (!t->block) {
    delete t;
    return fail(WT_ERR_OOM, "wt_build: tree allocation of %zu bytes failed", P.total);
  }
  char* base = (char*)t->block;
  t->dev.meta = (LevelMeta*)(base + P.off_meta);
  t->dev.cum = (uint64_t*)(base + P.off_cum);
  t->dev.nodes = (NodeQ*)(base + P.off_nodes);
  t->dev.bits = (uint64_t*)(base + P.off_bits);
  t->dev.L1 = (uint64_t*)(base + P.off_l1);
  t->dev.L2 = (uint16_t*)(base + P.off_l2);
  t->dev.smp = (uint64_t*)(base + P.off_smp);
  t->dev.wstart = matrix ? (uint64_t*)(base + P.off_wstart) : nullptr;
  if (huff) {
    t->dev.hcode = (const uint64_t*)(base + P.off_huff);
    t->dev.hsym = (const uint32_t*)(base + P.off_huff + huff_hsym_off(sigma));
    t->dev.hdepth = (const uint64_t*)(base + P.off_huff + huff_hdepth_off(sigma));
  }
  t->bytes_bits = (size_t)L * P.words_per_level * 8;
  t->bytes_l1 = (size_t)L * P.l1_per_level * 8;
  t->bytes_l2 = (size_t)L * P.l2_per_level * 2;
  t->bytes_smp = (size_t)L * P.smp_per_level * 8;
  t->bytes_nodes = matrix ? std::max<uint64_t>(sigma, 1) * 8 : (size_t)std::max<uint64_t>(P.nheap, 1) * sizeof(NodeQ);
  t->bytes_cum = (sigma + 1) * 8;

  auto bail = [&](wt_status s) {
    dev_free(t->block, st);
    delete t;
    return s;
  };

  // scratch: ping-pong sequences, histogram, tile counts and prefixes, build node table, scan partials
  const uint32_t T = P.tile;
  const uint64_t ntiles = ceil_div(std::max<uint64_t>(n, 1), T);
  const uint64_t seq_elems = round_up(std::max<uint64_t>(n, 1), T);
  const uint64_t hist_n = sigma + 1;
  const uint64_t part_n = ceil_div(std::max<uint64_t>(hist_n, P.nheap + 1), kScanChunk) + 1;
  size_t so = 0;
  auto take = [&](size_t bytes) {
    const size_t o = so;
    so = round_up(so + bytes, 256);
    return o;
  };
  const size_t o_seq0 = take(L > 1 ? seq_elems * wc : 0);
  const size_t o_seq1 = take(L > 2 ? seq_elems * wc : 0);
  const size_t o_enc = take(huff && L > 0 ? seq_elems * wc : 0);  // Huffman: the symbols as codes
  const size_t o_code_r = take(huff ? hc.m * 4 : 0);
  const size_t o_cumr = take(huff ? (hc.m + 1) * 8 : 0);
  const size_t o_hist = take(hist_n * 8);
  const uint64_t nchunks = ceil_div(ntiles, kChunkTiles);
  const uint64_t cstride = (ntiles + 1) + (nchunks + 1);  // per level: tile counts, then chunk counts
  const size_t o_cnt = take((size_t)std::max<uint32_t>(L, 1) * cstride * 8);
  const size_t o_pre = take((size_t)std::max<uint32_t>(L, 1) * (ntiles + 1) * 8);
  // the matrix: one build node per level; z / zs hold the counts by reversed code and their scan
  const size_t o_ntb = take(std::max<uint64_t>(matrix ? L : P.nheap, 1) * sizeof(NodeB));
  const size_t o_z = take((P.nheap + 1) * 8);
  const size_t o_zs = take((P.nheap + 1) * 8);
  const size_t o_wones = take(WT_MAX_LEVELS * 8);
  const size_t o_ns = take(std::max<uint64_t>(P.nheap, 1) * sizeof(NodeS));
  const size_t o_tfirst = take(ntiles * 4);
  const uint64_t gcnt_n = huff ? 0 : hist_gcnt_entries(n, sym_bytes, sigma);
  const size_t o_part = take(std::max<uint64_t>(part_n, ceil_div(gcnt_n, kScanChunk) + 1) * 8);
  const size_t o_gcnt = take(gcnt_n * 8);
  const size_t o_goff = take(gcnt_n * 8);
  const size_t o_err = take(64);
  Scratch S;
  S.st = st;
  S.block = dev_alloc(so, st);
  if (!S.block) return bail(fail(WT_ERR_OOM, "wt_build: scratch allocation of %zu bytes failed", so));
  char* sb = (char*)S.block;
  void* seq[2] = {sb + o_seq0, sb + o_seq1};
  uint64_t* hist = (uint64_t*)(sb + o_hist);
  uint64_t* tcnt = (uint64_t*)(sb + o_cnt);
  uint64_t* tpre = (uint64_t*)(sb + o_pre);
  NodeB* ntb = (NodeB*)(sb + o_ntb);
  uint64_t* z = (uint64_t*)(sb + o_z);
  uint64_t* zs = (uint64_t*)(sb + o_zs);
  uint64_t* part = (uint64_t*)(sb + o_part);
  uint32_t* err = (uint32_t*)(t->dev.meta + WT_MAX_LEVELS);
  (void)o_err;
  uint64_t* wones = (uint64_t*)(sb + o_wones);
  NodeS* ns = (NodeS*)(sb + o_ns);
  uint32_t* tfirst = (uint32_t*)(sb + o_tfirst);

  // Carried code width per level: level l + 1 needs only the code bits below level l (L - 1 - l of
  // them), so the sequence narrows to 2 and then 1 byte as levels consume bits. Once a level writes
  // codes without their prefix bits (fewer than L bits), nodes are found by position from that level on.
  const bool narrow = (flags & WT_BUILD_WIDE) == 0 && ((flags & WT_BUILD_NARROW) != 0 || n >= WT_NARROW_MIN_N);
  uint32_t wl[WT_MAX_LEVELS + 1];
  bool posm[WT_MAX_LEVELS] = {};
  bool any_pos = false;
  wl[0] = wc;
  {
    bool lost = false;
    for (uint32_t l = 0; l < L; ++l) {
      uint32_t wo = wl[l];
      if (narrow && l + 1 < L) {
        const uint32_t need = L - 1 - l;
        wo = std::min<uint32_t>(wo, need <= 8 ? 1u : need <= 16 ? 2u : 4u);
      }
      wl[l + 1] = wo;
      const bool drops = 8 * wo < L;
      posm[l] = !matrix && l > 0 && (lost || drops);
      any_pos = any_pos || posm[l];
      lost = lost || drops;
    }
  }

  Prof prof;
  prof.on = (flags & WT_BUILD_PROFILE) != 0;
  prof.st = st;
  hipError_t he = hipSuccess;
#define WT_STEP(x)                                                             \
  do {                                                                         \
    he = (x);                                                                  \
    if (he != hipSuccess)                                                      \
      return bail(fail(WT_ERR_HIP, "wt_build: %s: %s", #x, hipGetErrorString(he))); \
  } while (0)

  // metadata and cleared counters
  InitArgs ia{};
  ia.L = L;
  for (uint32_t l = 0; l < L; ++l) {
    LevelMeta& mm = ia.meta[l];
    mm.n = 0;
    mm.ones = 0;
    mm.bits = (uint64_t)l * P.words_per_level;
    mm.l1 = (uint64_t)l * P.l1_per_level;
    mm.l2 = (uint64_t)l * P.l2_per_level;
    mm.smp = (uint64_t)l * P.smp_per_level;
    mm.smp_cap = P.smp_per_level;
    t->hmeta[l] = mm;
  }
  WT_STEP(prof.begin("init", -1));
  hipLaunchKernelGGL(k_init_meta, dim3(1), dim3(64), 0, st, ia, t->dev.meta);
  hipLaunchKernelGGL(k_fill_u64, dim3(64), dim3(kBT), 0, st, hist, hist_n, 0ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(256), dim3(kBT), 0, st, tcnt, (uint64_t)std::max<uint32_t>(L, 1) * cstride,
                     0ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, (uint64_t*)err, 8ull, 0ull);
  if (matrix) hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, wones, (uint64_t)WT_MAX_LEVELS, 0ull);
  WT_STEP(hipGetLastError());
  WT_STEP(prof.end());

  WT_STEP(prof.begin("hist", -1));
  if (huff) {
    // the histogram is known; the code tables go with the tree, the codes in rank order and their
    // counts to the node walk (host vectors live until the build's final synchronisation)
    if (sigma) WT_STEP(hipMemcpyAsync(hist, hh.data(), sigma * 8, hipMemcpyHostToDevice, st));
    WT_STEP(hipMemcpyAsync((void*)t->dev.hcode, hc.hcode.data(), sigma * 8, hipMemcpyHostToDevice, st));
    if (hc.m) WT_STEP(hipMemcpyAsync((void*)t->dev.hsym, hc.sym.data(), hc.m * 4, hipMemcpyHostToDevice, st));
    if (!hc.depth.empty())
      WT_STEP(hipMemcpyAsync((void*)t->dev.hdepth, hc.depth.data(), hc.depth.size() * 8, hipMemcpyHostToDevice, st));
    if (hc.m > 1) {
      WT_STEP(hipMemcpyAsync(sb + o_code_r, hc.code_r.data(), hc.m * 4, hipMemcpyHostToDevice, st));
      WT_STEP(hipMemcpyAsync(sb + o_cumr, hc.cumr.data(), (hc.m + 1) * 8, hipMemcpyHostToDevice, st));
    }
  } else {
    const HistBufs hb{hist, tcnt, err, (uint64_t*)(sb + o_gcnt), (uint64_t*)(sb + o_goff), part, seq[0]};
    if (sym_bytes == 1) WT_STEP(launch_hist<uint8_t>(d_sym, n, (uint32_t)sigma, L, hb, st));
    else if (sym_bytes == 2) WT_STEP(launch_hist<uint16_t>(d_sym, n, (uint32_t)sigma, L, hb, st));
    else WT_STEP(launch_hist<uint32_t>(d_sym, n, (uint32_t)sigma, L, hb, st));
  }
  WT_STEP(prof.end());

  WT_STEP(prof.begin("cum_hist", -1));
  WT_STEP(exclusive_scan_u64(hist, hist_n, t->dev.cum, part, st));
  WT_STEP(prof.end());

  if (matrix) {
    // level sizes, the one node of every level, and every symbol's start below the last level
    WT_STEP(prof.begin("nodes", -1));
    if (L > 0) {
      const uint32_t nbo = (uint32_t)std::min<uint64_t>(ceil_div(sigma, 2ull * kBT * 8), 256);
      hipLaunchKernelGGL(k_wm_ones, dim3(std::max(nbo, 1u), L), dim3(kBT), 0, st, (const uint64_t*)t->dev.cum,
                         (uint32_t)sigma, L, wones);
      hipLaunchKernelGGL(k_wm_final, dim3(1), dim3(64), 0, st, n, L, (const uint64_t*)wones, ntb, t->dev.meta);
      const uint64_t nc = 1ull << L;
      const uint32_t nbc = (uint32_t)std::min<uint64_t>(ceil_div(nc, kBT), 4096);
      hipLaunchKernelGGL(k_wm_rcount, dim3(nbc), dim3(kBT), 0, st, (const uint64_t*)hist, (uint32_t)sigma, L, z);
      WT_STEP(hipGetLastError());
      WT_STEP(exclusive_scan_u64(z, nc, zs, part, st));
      hipLaunchKernelGGL(k_wm_starts, dim3(nbc), dim3(kBT), 0, st, (const uint64_t*)zs, (uint32_t)sigma, L,
                         t->dev.wstart);
    } else {
      hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, t->dev.wstart, 1ull, 0ull);
    }
    WT_STEP(hipGetLastError());
    WT_STEP(prof.end());
  } else if (L > 0) {
    WT_STEP(prof.begin("nodes", -1));
    const uint32_t nb = (uint32_t)ceil_div(P.nheap, kBT);
    if (huff)
      WT_STEP(huff_node_walk(L, hc.m, P.nheap, (const uint32_t*)(sb + o_code_r), (const uint64_t*)(sb + o_cumr), ntb,
                             z, st));
    else
      hipLaunchKernelGGL(k_node_walk, dim3(nb), dim3(kBT), 0, st, (uint32_t)sigma, P.nheap,
                         (const uint64_t*)t->dev.cum, ntb, z);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, z + P.nheap, 1ull, 0ull);
    WT_STEP(hipGetLastError());
    WT_STEP(exclusive_scan_u64(z, P.nheap + 1, zs, part, st));
    hipLaunchKernelGGL(k_node_final, dim3(nb), dim3(kBT), 0, st, P.nheap, (const uint64_t*)zs, ntb, t->dev.nodes,
                       t->dev.meta);
    WT_STEP(hipGetLastError());
    if (ntb_out) WT_STEP(hipMemcpyAsync(ntb_out, ntb, P.nheap * sizeof(NodeB), hipMemcpyDeviceToDevice, st));
    if (any_pos) {
      // the non-empty nodes of every level in position order (z, zs are free again)
      const uint32_t nbf = (uint32_t)ceil_div(P.nheap + 1, kBT);
      hipLaunchKernelGGL(k_ns_flag, dim3(nbf), dim3(kBT), 0, st, (const NodeB*)ntb, P.nheap, z);
      WT_STEP(hipGetLastError());
      WT_STEP(exclusive_scan_u64(z, P.nheap + 1, zs, part, st));
      hipLaunchKernelGGL(k_ns_scatter, dim3(nb), dim3(kBT), 0, st, (const NodeB*)ntb, P.nheap, (const uint64_t*)zs, ns);
      WT_STEP(hipGetLastError());
    }
    WT_STEP(prof.end());
  }

  if (huff && L > 0) {
    // symbols -> codes, and the ones per tile of level 0 (code bit L - 1)
    WT_STEP(prof.begin("encode", -1));
    WT_STEP(huff_encode(d_sym, sym_bytes, n, (uint32_t)sigma, t->dev.hcode, L, sb + o_enc, wc, tcnt, st));
    WT_STEP(prof.end());
  }

  uint32_t l2shift = 0, sshift = 0;
  while ((1u << l2shift) < l2_bits) ++l2shift;
  while ((1u << sshift) < srate) ++sshift;

  for (uint32_t l = 0; l < L; ++l) {
    uint64_t* cnt_l = tcnt + (size_t)l * cstride;
    uint64_t* chunk_l = cnt_l + ntiles + 1;
    uint64_t* pre_l = tpre + (size_t)l * (ntiles + 1);
    uint32_t tshift = 0;  // tiles of level l: kTileBytes of its element width
    while ((1u << tshift) < tile_elems(wl[l])) ++tshift;
    WT_STEP(prof.begin("tile_scan", (int)l));
    hipLaunchKernelGGL(k_tile_reduce, dim3((uint32_t)nchunks), dim3(kBT), 0, st, (const LevelMeta*)t->dev.meta, l,
                       tshift, (const uint64_t*)cnt_l, chunk_l);
    hipLaunchKernelGGL(k_tile_scan, dim3((uint32_t)(nchunks + 1)), dim3(kBT), 0, st, t->dev.meta, l, tshift,
                       (const uint64_t*)cnt_l, (const uint64_t*)chunk_l, pre_l, t->dev.L1, t->dev.L2);
    if (posm[l])
      hipLaunchKernelGGL(k_tile_first, dim3((uint32_t)ceil_div(ceil_div(n, 1ull << tshift), kBT)), dim3(kBT), 0, st,
                         (const LevelMeta*)t->dev.meta, l, tshift, (const NodeS*)ns, (const uint64_t*)zs, tfirst);
    WT_STEP(hipGetLastError());
    WT_STEP(prof.end());
    LevelArgs a{};
    a.in = l == 0 ? (huff ? (const void*)(sb + o_enc) : d_sym) : seq[(l - 1) & 1];
    a.out = (l + 1 < L) ? seq[l & 1] : nullptr;
    a.bits = t->dev.bits;
    a.L1 = t->dev.L1;
    a.L2 = t->dev.L2;
    a.smp = t->dev.smp;
    a.meta = t->dev.meta;
    a.pre = pre_l;
    a.cnt_next = (l + 1 < L) ? tcnt + (size_t)(l + 1) * cstride : nullptr;
    a.ntb = matrix ? ntb + l : ntb + ((1ull << l) - 1);
    a.l = l;
    a.L = L;
    a.sigma = (uint32_t)sigma;
    a.pow2 = pow2;
    a.l2shift = l2shift;
    a.sshift = sshift;
    a.encode = (l == 0 && !pow2) ? 1u : 0u;
    a.in_vec = (l == 0 && !huff) ? 0u : 1u;
    a.in_aligned = (l == 0 && !huff) ? (((uintptr_t)d_sym & 15u) == 0) : 1u;
    a.matrix = matrix ? 1u : 0u;
    a.pos_node = posm[l] ? 1u : 0u;
    a.ns = ns;
    a.ns_idx = zs;
    a.tfirst = tfirst;
    a.err = err;
    WT_STEP(prof.begin("level", (int)l));
    WT_STEP(launch_level_w(a, n, wl[l], wl[l + 1], st));
    WT_STEP(prof.end());
  }

  // read back level sizes and the range flag (one copy: the flag sits after the level entries)
  std::vector<LevelMeta> rb(WT_MAX_LEVELS + 1);
  WT_STEP(hipMemcpyAsync(rb.data(), t->dev.meta, sizeof(LevelMeta) * (WT_MAX_LEVELS + 1), hipMemcpyDeviceToHost, st));
  WT_STEP(hipStreamSynchronize(st));
#undef WT_STEP
  uint32_t rb_err = 0;
  std::memcpy(&rb_err, &rb[WT_MAX_LEVELS], sizeof(rb_err));
  if (rb_err & 1u)
    return bail(fail(WT_ERR_SYMBOL_RANGE, "wt_build: a symbol is >= sigma (%llu)", (unsigned long long)sigma));
  if (rb_err & 2u)
    return bail(fail(WT_ERR_STATE, "wt_build: internal error: the level pass placed an element outside its tile"));
  for (uint32_t l = 0; l < L; ++l) t->hmeta[l] = rb[l];
  if (prof.on) prof.collect(t->prof);
  *out = t;
  return WT_OK;
}
