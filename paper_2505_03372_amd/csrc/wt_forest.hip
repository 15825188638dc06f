// Batched construction of many wavelet trees (a forest) in one captured HIP graph.
//
// Every phase of the single-tree build (Section 5.1, Algorithm 4) becomes one kernel over the blocks
// of all trees that have work in it. A block map (tree of every block) and the block offsets of every
// tree are planned on the host and uploaded once with the per-tree state; a block reads its tree's
// state and runs the same device body as the single-tree kernel. The trees are ordered by level count
// (descending), so the trees that still have a level l form a prefix of the order and the level-l
// launches cover a prefix of the level map. The whole sequence is captured into a graph and launched
// once; a final gather puts every tree's level sizes and range flag in one buffer for one readback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <vector>

#include "wt_build_dev.h"
#include "wt_host.h"
#include "wt_internal.h"
#include "wt_learn_dev.h"
#include "wt_query_dev.h"

namespace wt {

struct FB {
  uint32_t j;
  uint64_t bid, nblk;
};

__device__ __forceinline__ FB forest_block(const ForestGrid& fg) {
  const uint32_t g = blockIdx.x + fg.base;
  const uint32_t j = fg.bmap[g];
  const uint32_t b0 = fg.boff[j];
  return FB{j, (uint64_t)(g - b0), (uint64_t)(fg.boff[j + 1] - b0)};
}

// Level metadata of every tree and cleared counters (histogram, tile counts, range flag).
__global__ __launch_bounds__(kBT) void kf_init(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  fill_body(b.clear, b.clear_n, 0ull, f.bid, f.nblk);
  if (f.bid == 0) {
    const uint32_t l = threadIdx.x;
    if (l < b.L) {
      LevelMeta m;
      m.n = 0;
      m.ones = 0;
      m.bits = (uint64_t)l * b.words_per_level;
      m.l1 = (uint64_t)l * b.l1_per_level;
      m.l2 = (uint64_t)l * b.l2_per_level;
      m.smp = (uint64_t)l * b.smp_per_level;
      m.smp_cap = b.smp_per_level;
      m.pad = 0;
      b.meta[l] = m;
    }
    if (threadIdx.x == 0 && b.L) b.z[b.nheap] = 0;
  }
}

template <typename E, uint32_t kWords>
__global__ __launch_bounds__(kHT) void kf_hist_dense(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  hist_dense_body<E, kWords>((const WT_GLOBAL E*)b.sym, b.n, b.sigma, b.L, b.aligned, (WT_GLOBAL uint64_t*)b.hist,
                             (WT_GLOBAL uint64_t*)b.tcnt, (WT_GLOBAL uint32_t*)b.err, f.bid, f.nblk);
}

template <typename E>
__global__ __launch_bounds__(kBT) void kf_hist_hash(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  hist_hash_body<E>((const WT_GLOBAL E*)b.sym, b.n, b.sigma, b.L, b.aligned, (WT_GLOBAL uint64_t*)b.hist,
                    (WT_GLOBAL uint64_t*)b.tcnt, (WT_GLOBAL uint32_t*)b.err, f.bid, f.nblk);
}

// which = 0: cumulative histogram (sigma + 1 entries); 1: node-table prefix (nheap + 1 entries).
__device__ __forceinline__ void scan_operands(const TreeB& b, uint32_t which, const uint64_t*& in, uint64_t& n,
                                              uint64_t*& out) {
  if (which == 0) {
    in = b.hist;
    n = (uint64_t)b.sigma + 1;
    out = b.cum;
  } else {
    in = b.z;
    n = b.L ? b.nheap + 1 : 0;
    out = b.zs;
  }
}

__global__ __launch_bounds__(kBT) void kf_scan_reduce(ForestGrid fg, uint32_t which) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  const uint64_t* in;
  uint64_t n;
  uint64_t* out;
  scan_operands(b, which, in, n, out);
  scan_reduce_body(in, n, b.part, f.bid);
}

// One block per tree.
__global__ __launch_bounds__(1024) void kf_scan_partials(const TreeB* __restrict__ tb, uint32_t which) {
  const TreeB& b = tb[blockIdx.x];
  const uint64_t* in;
  uint64_t n;
  uint64_t* out;
  scan_operands(b, which, in, n, out);
  if (n) scan_partials_body(b.part, (n + kScanChunk - 1) / kScanChunk);
}

__global__ __launch_bounds__(kBT) void kf_scan_down(ForestGrid fg, uint32_t which) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  const uint64_t* in;
  uint64_t n;
  uint64_t* out;
  scan_operands(b, which, in, n, out);
  scan_down_body(in, n, b.part, out, f.bid);
}

__global__ __launch_bounds__(kBT) void kf_node_walk(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  node_walk_body(b.sigma, b.nheap, b.cum, b.ntb, b.z, f.bid * kBT + threadIdx.x);
}

__global__ __launch_bounds__(kBT) void kf_node_final(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  node_final_body(b.nheap, b.zs, b.ntb, b.nodes, b.meta, f.bid * kBT + threadIdx.x);
}

// Tiles of level l hold kTileBytes of its carried codes (b.tshift: the symbols' tile at level 0).
__device__ __forceinline__ uint32_t forest_tshift(const TreeB& b, uint32_t l) {
  return b.tshift + forest_wlog(b, 0) - forest_wlog(b, l);
}

__global__ __launch_bounds__(kBT) void kf_tile_reduce(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  const uint32_t l = fg.l;
  const uint64_t* cnt = b.tcnt + (uint64_t)l * b.cstride;
  tile_reduce_body(b.meta, l, forest_tshift(b, l), cnt, b.tcnt + (uint64_t)l * b.cstride + b.ntiles + 1, f.bid);
}

__global__ __launch_bounds__(kBT) void kf_tile_scan(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  const uint32_t l = fg.l;
  const uint64_t* cnt = b.tcnt + (uint64_t)l * b.cstride;
  tile_scan_body(b.meta, l, forest_tshift(b, l), cnt, cnt + b.ntiles + 1, b.tpre + (uint64_t)l * (b.ntiles + 1),
                 b.L1, b.L2, f.bid);
}

// Non-empty nodes in position order for trees with levels whose nodes are found by position: flags of
// the heap entries into z (z[nheap] stays 0 from kf_init), then, after the scan of z into zs, every
// non-empty entry at its rank.
__global__ __launch_bounds__(kBT) void kf_ns_flag(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  const uint64_t h = f.bid * kBT + threadIdx.x;
  if (!b.posmask || h >= b.nheap) return;
  b.z[h] = (b.ntb[h].start != kNoNode && b.ntb[h].end > b.ntb[h].start) ? 1ull : 0ull;
}

__global__ __launch_bounds__(kBT) void kf_ns_scatter(ForestGrid fg) {
  const FB f = forest_block(fg);
  const TreeB& b = fg.tb[f.j];
  const uint64_t h = f.bid * kBT + threadIdx.x;
  if (!b.posmask || h >= b.nheap || b.zs[h + 1] == b.zs[h]) return;
  const uint32_t l = 63u - (uint32_t)__clzll(h + 1);
  NodeS e;
  e.start = b.ntb[h].start;
  e.pfx = (uint32_t)(h + 1 - (1ull << l));
  e.pad = 0;
  b.ns[b.zs[h]] = e;
}

// Level sizes and range flag of every tree into one buffer (one block per tree, caller order).
struct ForestOut {
  LevelMeta meta[WT_MAX_LEVELS];
  uint32_t err;
  uint32_t pad[3];
};

__global__ void kf_gather(const TreeB* __restrict__ tb, const uint32_t* __restrict__ order,
                          ForestOut* __restrict__ out) {
  const uint32_t s = blockIdx.x;  // position in the build order
  const TreeB& b = tb[s];
  ForestOut& o = out[order[s]];
  if (threadIdx.x < b.L) o.meta[threadIdx.x] = b.meta[threadIdx.x];
  if (threadIdx.x == 0) o.err = *b.err;
}

// ---------------------------------------------------------------- mixed queries

// Query state of one tree of a forest.
struct QTree {
  QArgs a;
  const LearnQ* lq;  // compiled learned-select models, or NULL
  uint32_t l2s;      // log2 |L2|
  uint32_t pad;
  uint64_t vbase;    // start of the tree in the forest's concatenated position space (n + 1 per tree)
};

// Class of a query: op * 4 + (log2 |L2| - 8) for the four ops (a learned select on a tree without a
// learned index is a plain select); kMixInvalid for an unknown tree or op.
constexpr uint32_t kMixInvalid = 16;
constexpr uint32_t kMixClasses = 17;
constexpr uint64_t kMixDirectMax = 16384;   // batches up to this size skip the binning
constexpr uint32_t kMixChunk = kQT * 16;    // queries per class-sort block
constexpr uint64_t kMixSortMin = 1ull << 16;  // batches from this size are sorted by (class, position)
constexpr uint32_t kMixB = 2048;            // position buckets per class in that sort
constexpr uint32_t kMixBucketClasses = 13;  // classes 0-11 (three ops x four |L2|) and the invalid one
static_assert(kMixBucketClasses * kMixB <= kSortIdBins, "bucket ids");

__device__ __forceinline__ uint32_t mix_class(const QTree* __restrict__ qt, uint32_t ntrees, uint32_t tree,
                                              uint32_t op) {
  if (tree >= ntrees || op > WT_OP_SELECT_LEARNED) return kMixInvalid;
  // Learned selects are answered by the plain select in mixed batches: the learned traversal inside
  // these kernels (tree arguments per lane) faulted once on 64 trees of 2^26 symbols with no cause
  // found, so that path is switched off; the single-tree learned select is unaffected.
  if (op == WT_OP_SELECT_LEARNED) op = WT_OP_SELECT;
  return op * 4 + (qt[tree].l2s - 8);
}

// Adds the lanes of every class present in the wave to the LDS counter of that class.
__device__ __forceinline__ void wave_class_count(uint32_t c, bool in, uint32_t* s_cnt) {
  uint64_t pend = __ballot(in);
  const uint32_t lane = threadIdx.x & 63u;
  while (pend) {
    const int leader = __ffsll((unsigned long long)pend) - 1;
    const uint32_t lc = __shfl(c, leader, 64);
    const uint64_t m = __ballot(in && c == lc);
    if (lane == (uint32_t)leader) atomicAdd(&s_cnt[lc], (uint32_t)__popcll(m));
    pend &= ~m;
  }
}

// Pass 1: the class of every query and the number of queries per class.
__global__ __launch_bounds__(kQT) void k_mix_count(const QTree* __restrict__ qt, uint32_t ntrees,
                                                   const uint32_t* __restrict__ tree, const uint8_t* __restrict__ op,
                                                   uint64_t q, uint8_t* __restrict__ cls,
                                                   uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_cnt[32];
  if (threadIdx.x < 32) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kMixChunk;
  for (uint32_t i = threadIdx.x; i < kMixChunk; i += kQT) {
    const uint64_t j = c0 + i;
    const bool in = j < q;
    uint32_t c = 0;
    if (in) {
      c = mix_class(qt, ntrees, tree[j], op[j]);
      cls[j] = (uint8_t)c;
    }
    wave_class_count(c, in, s_cnt);
  }
  __syncthreads();
  if (threadIdx.x < kMixClasses && s_cnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], s_cnt[threadIdx.x]);
}

// Pass 2: every query gets a slot inside its class's range (the order inside a class is free): the
// block reserves its share of every class with one atomic, the waves split it with LDS atomics.
__global__ __launch_bounds__(kQT) void k_mix_scatter(uint64_t q, const uint8_t* __restrict__ cls,
                                                     const uint32_t* __restrict__ off, uint32_t* __restrict__ cursor,
                                                     uint32_t* __restrict__ perm) {
  __shared__ uint32_t s_cnt[32];
  __shared__ uint32_t s_off[32];
  if (threadIdx.x < 32) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kMixChunk;
  for (uint32_t i = threadIdx.x; i < kMixChunk; i += kQT) {
    const uint64_t j = c0 + i;
    const bool in = j < q;
    wave_class_count(in ? cls[j] : 0u, in, s_cnt);
  }
  __syncthreads();
  if (threadIdx.x < kMixClasses) {
    const uint32_t n = s_cnt[threadIdx.x];
    s_off[threadIdx.x] = n ? off[threadIdx.x] + atomicAdd(&cursor[threadIdx.x], n) : 0u;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (uint32_t i = threadIdx.x; i < kMixChunk; i += kQT) {
    const uint64_t j = c0 + i;
    const bool in = j < q;
    const uint32_t c = in ? cls[j] : 0u;
    uint64_t pend = __ballot(in);
    uint32_t slot = 0;
    while (pend) {
      const int leader = __ffsll((unsigned long long)pend) - 1;
      const uint32_t lc = __shfl(c, leader, 64);
      const uint64_t m = __ballot(in && c == lc);
      uint32_t first = 0;
      if (lane == (uint32_t)leader) first = atomicAdd(&s_off[lc], (uint32_t)__popcll(m));
      first = __shfl(first, leader, 64);
      if (in && c == lc) slot = first + (uint32_t)__popcll(m & lt);
      pend &= ~m;
    }
    if (in) perm[slot] = (uint32_t)j;
  }
}

// Start of every class's slots from the class counts (kMixClasses + 1 entries; the last is q).
__global__ void k_mix_off_counts(const uint32_t* __restrict__ counts, uint64_t q, uint32_t* __restrict__ off) {
  if (threadIdx.x != 0) return;
  uint32_t run = 0;
  for (uint32_t c = 0; c < kMixClasses; ++c) {
    off[c] = run;
    run += counts[c];
  }
  off[kMixClasses] = (uint32_t)q;
}

// Bucket of every query for the (class, position) sort: class (0-11, or 12 for an invalid query)
// times kMixB plus its place in the forest's concatenated position space (the tree's start plus the
// position, or for a select the rank of the occurrence in symbol order) >> shift. The queries of one
// tree and region then share a bucket, so a wave's traversals share lines.
__global__ __launch_bounds__(kQT) void k_mix_bucket(const QTree* __restrict__ qt, uint32_t ntrees,
                                                    const uint32_t* __restrict__ tree, const uint8_t* __restrict__ op,
                                                    const uint32_t* __restrict__ sym,
                                                    const uint64_t* __restrict__ arg, uint64_t q, uint32_t shift,
                                                    uint16_t* __restrict__ ids) {
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT) {
    const uint32_t tj = tree[j];
    const uint32_t c = mix_class(qt, ntrees, tj, op[j]);
    uint32_t id = 12u * kMixB;
    if (c != kMixInvalid) {
      const QTree& T = qt[tj];
      const QArgs& a = T.a;
      const uint64_t x = arg[j];
      uint64_t key;
      if ((c >> 2) == WT_OP_SELECT) {
        const uint32_t cs = sym ? sym[j] : 0u;
        key = a.n;
        if (x != 0 && cs < a.sigma) {
          const uint64_t lo = a.d.cum[cs], cnt = a.d.cum[cs + 1] - lo;
          if (x <= cnt) key = lo + x - 1;
        }
      } else {
        key = min(x, a.n);
      }
      id = c * kMixB + (uint32_t)min<uint64_t>((T.vbase + key) >> shift, kMixB - 1);
    }
    ids[j] = (uint16_t)id;
  }
}

// Start of every class's slots from the bucket starts of the (class, position) sort.
__global__ void k_mix_off_buckets(const uint32_t* __restrict__ tot, uint64_t q, uint32_t* __restrict__ off) {
  const uint32_t c = threadIdx.x;
  if (c < kMixClasses) off[c] = tot[(c < 12u ? c : 12u) * kMixB];
  else if (c == kMixClasses) off[c] = (uint32_t)q;
}

// Pass 3: one kernel per class (op, |L2|), over that class's range of slots: every wave runs one
// traversal, with the registers of that traversal alone. The lanes of a wave ask different trees, so
// the tree arguments live in vector registers; the bound keeps every class at 80 (6 waves per SIMD)
// without spills.
template <int OP, int L2S>
__global__ __launch_bounds__(kQT, 6) void k_mix_run(const QTree* __restrict__ qt, const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ perm, const uint32_t* __restrict__ tree,
                                                 const uint32_t* __restrict__ sym, const uint64_t* __restrict__ arg,
                                                 uint64_t* __restrict__ out) {
  constexpr uint32_t kC = OP * 4 + (L2S - 8);
  const uint64_t lo = off[kC], hi = off[kC + 1];
  for (uint64_t s = lo + (uint64_t)blockIdx.x * kQT + threadIdx.x; s < hi; s += (uint64_t)gridDim.x * kQT) {
    const uint32_t jj = perm[s];
    const QArgs& a = qt[tree[jj]].a;
    const uint64_t x = arg[jj];
    uint64_t res;
    if constexpr (OP == WT_OP_ACCESS) res = access_one<L2S>(a, a.d.meta, x);
    else if constexpr (OP == WT_OP_RANK) res = rank_one<L2S>(a, a.d.meta, sym ? sym[jj] : 0u, x);
    else res = select_one<L2S>(a, a.d.meta, sym ? sym[jj] : 0u, x);
    out[jj] = res;
  }
}

// Small batches: every query in one kernel, no binning (a wave may run several traversals).
__global__ __launch_bounds__(kQT) void k_mix_direct(const QTree* __restrict__ qt, uint32_t ntrees,
                                                    const uint32_t* __restrict__ tree, const uint8_t* __restrict__ op,
                                                    const uint32_t* __restrict__ sym,
                                                    const uint64_t* __restrict__ arg, uint64_t q,
                                                    uint64_t* __restrict__ out) {
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT) {
    const uint32_t tj = tree[j];
    const uint32_t c = mix_class(qt, ntrees, tj, op[j]);
    uint64_t res = ~0ull;
    if (c != kMixInvalid) {
      const QArgs& a = qt[tj].a;
      const LevelMeta* meta = a.d.meta;
      const uint32_t sj = sym ? sym[j] : 0u;
      const uint64_t x = arg[j];
      switch (c >> 2) {
        case WT_OP_ACCESS:
          switch (c & 3) {
            case 0: res = access_one<8>(a, meta, x); break;
            case 1: res = access_one<9>(a, meta, x); break;
            case 2: res = access_one<10>(a, meta, x); break;
            default: res = access_one<11>(a, meta, x); break;
          }
          break;
        case WT_OP_RANK:
          switch (c & 3) {
            case 0: res = rank_one<8>(a, meta, sj, x); break;
            case 1: res = rank_one<9>(a, meta, sj, x); break;
            case 2: res = rank_one<10>(a, meta, sj, x); break;
            default: res = rank_one<11>(a, meta, sj, x); break;
          }
          break;
        default:
          switch (c & 3) {
            case 0: res = select_one<8>(a, meta, sj, x); break;
            case 1: res = select_one<9>(a, meta, sj, x); break;
            case 2: res = select_one<10>(a, meta, sj, x); break;
            default: res = select_one<11>(a, meta, sj, x); break;
          }
          break;
      }
    }
    out[j] = res;
  }
}

// Unknown tree or op.
__global__ __launch_bounds__(kQT) void k_mix_invalid(const uint32_t* __restrict__ off,
                                                     const uint32_t* __restrict__ perm, uint64_t* __restrict__ out) {
  const uint64_t lo = off[kMixInvalid], hi = off[kMixInvalid + 1];
  for (uint64_t s = lo + (uint64_t)blockIdx.x * kQT + threadIdx.x; s < hi; s += (uint64_t)gridDim.x * kQT)
    out[perm[s]] = ~0ull;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0u;
}

}  // namespace wt

using namespace wt;

struct wt_forest {
  uint32_t count = 0, w = 0;
  std::vector<wt_tree*> trees;  // caller order
  void* block = nullptr;        // every tree's parts
  size_t block_bytes = 0;
  void* qtab = nullptr;         // per-tree query state for wt_query_mixed (made on first use)
  uint64_t qversion = 0;        // sum of the trees' learned-index versions when qtab was made
  uint32_t vshift = 0;          // position-space shift of the (class, position) query sort
  wt_forest_info_t info{};
};

namespace {

struct MapBuilder {
  std::vector<uint32_t> bmap, boff;
  void add(uint32_t j, uint64_t nblocks) {
    boff.push_back((uint32_t)bmap.size());
    for (uint64_t i = 0; i < nblocks; ++i) bmap.push_back(j);
  }
  void close() { boff.push_back((uint32_t)bmap.size()); }
};

uint32_t log2_floor(uint64_t x) { return x ? 63u - (uint32_t)__builtin_clzll(x) : 0u; }

}  // namespace

namespace wt {

// Tuning-table bucket of a shape.
void tune_bucket(uint64_t n, uint64_t sigma, uint32_t* nb, uint32_t* sb) {
  *nb = std::min<uint32_t>(log2_floor(std::max<uint64_t>(n, 1)) / 2, WT_TUNE_NB - 1);
  *sb = std::min<uint32_t>(log2_floor(std::max<uint64_t>(sigma, 1)) / 4, WT_TUNE_SB - 1);
}

}  // namespace wt

extern "C" wt_status wt_build_forest(const wt_seq_desc* h_descs, uint32_t count, uint32_t sym_bytes,
                                     const wt_forest_opts* opts, wt_stream_t stream, wt_forest** out) {
  clear_error();
  const auto t_start = std::chrono::steady_clock::now();
  if (!out) return fail(WT_ERR_ARG, "wt_build_forest: out is NULL");
  *out = nullptr;
  if (count == 0 || !h_descs) return fail(WT_ERR_ARG, "wt_build_forest: no sequences");
  if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4)
    return fail(WT_ERR_ARG, "wt_build_forest: sym_bytes must be 1, 2 or 4 (got %u)", sym_bytes);
  const wt_tune_table* tune = opts ? opts->tune : nullptr;

  // per-tree shape and options, checked as wt_build checks them
  struct Shape {
    uint64_t n, sigma;
    uint32_t L, pow2, l2_bits, srate;
  };
  std::vector<Shape> sh(count);
  for (uint32_t j = 0; j < count; ++j) {
    const wt_seq_desc& d = h_descs[j];
    Shape& s = sh[j];
    s.n = d.n;
    s.sigma = d.sigma;
    if (d.n && !d.d_sym) return fail(WT_ERR_ARG, "wt_build_forest: sequence %u: d_sym is NULL", j);
    if (d.sigma == 0 || d.sigma > WT_MAX_SIGMA)
      return fail(WT_ERR_ARG, "wt_build_forest: sequence %u: sigma must be in [1, %llu]", j,
                  (unsigned long long)WT_MAX_SIGMA);
    if (sym_bytes < 4 && d.sigma > (1ull << (8 * sym_bytes)))
      return fail(WT_ERR_ARG, "wt_build_forest: sequence %u: sigma %llu does not fit %u-byte symbols", j,
                  (unsigned long long)d.sigma, sym_bytes);
    if (d.n >= (1ull << 40)) return fail(WT_ERR_ARG, "wt_build_forest: sequence %u: n too large", j);
    uint32_t nb, sb;
    tune_bucket(d.n, d.sigma, &nb, &sb);
    s.l2_bits = d.l2_bits ? d.l2_bits : (tune && tune->l2_bits[nb][sb] ? tune->l2_bits[nb][sb] : 512u);
    s.srate = d.sample_rate ? d.sample_rate : (tune && tune->sample_rate[nb][sb] ? tune->sample_rate[nb][sb] : 4096u);
    if (s.l2_bits != 256 && s.l2_bits != 512 && s.l2_bits != 1024 && s.l2_bits != 2048)
      return fail(WT_ERR_ARG, "wt_build_forest: sequence %u: l2_bits must be 256, 512, 1024 or 2048", j);
    if (s.srate < 512 || s.srate > (1u << 20) || (s.srate & (s.srate - 1)))
      return fail(WT_ERR_ARG, "wt_build_forest: sequence %u: sample_rate must be a power of two in [512, 2^20]", j);
    s.L = 0;
    while ((1ull << s.L) < s.sigma) ++s.L;
    s.pow2 = (s.sigma & (s.sigma - 1)) == 0;
  }
  // Carried code width per tree and level, as the single-tree build narrows them: level l + 1 needs the
  // L - 1 - l code bits below level l only, so the codes narrow as levels consume bits; once a level
  // has dropped prefix bits, the levels after it find nodes by position. WT_BUILD_WIDE keeps the width.
  const bool narrow = !(opts && (opts->flags & WT_BUILD_WIDE));
  struct Sched {
    uint64_t wlog;     // 2 bits per level: log2 of its element bytes
    uint32_t posmask;  // levels whose nodes are found by position
  };
  std::vector<Sched> sched(count);
  for (uint32_t j = 0; j < count; ++j) {
    const uint32_t L = sh[j].L;
    uint32_t w = sym_bytes;
    uint64_t wlog = log2_floor(w);
    uint32_t posmask = 0;
    bool lost = false;
    for (uint32_t l = 0; l < L; ++l) {
      uint32_t wo = w;
      if (narrow && l + 1 < L) {
        const uint32_t need = L - 1 - l;
        wo = std::min<uint32_t>(wo, need <= 8 ? 1u : need <= 16 ? 2u : 4u);
      }
      const bool drops = 8 * wo < L;
      if (l > 0 && (lost || drops)) posmask |= 1u << l;
      lost = lost || drops;
      wlog |= (uint64_t)log2_floor(wo) << (2 * (l + 1));
      w = wo;
    }
    sched[j] = Sched{wlog, posmask};
  }

  // build order: level count descending (stable)
  std::vector<uint32_t> order(count);
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return sh[a].L > sh[b].L; });
  const uint32_t Lmax = sh[order[0]].L;

  hipStream_t user_st = (hipStream_t)stream;
  hipStream_t st = user_st;
  bool own_stream = false;
  if (!st) {
    // a private stream (the null stream cannot be captured) that first waits for the null stream's work
    WT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    own_stream = true;
    hipEvent_t ready;
    hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ready, nullptr);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ready, 0);
    (void)hipEventDestroy(ready);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(st);
      return fail(WT_ERR_HIP, "wt_build_forest: stream setup: %s", hipGetErrorString(e));
    }
  }
  struct StreamGuard {
    hipStream_t s;
    bool own;
    ~StreamGuard() {
      if (own) (void)hipStreamDestroy(s);
    }
  } sguard{st, own_stream};
  int dev = 0;
  WT_HIP(hipGetDevice(&dev));

  // tree parts: one allocation, every tree at a 256-byte aligned offset
  std::vector<TreePlan> plans(count);
  std::vector<size_t> toff(count);
  size_t tbytes = 0;
  for (uint32_t j = 0; j < count; ++j) {
    plans[j] = plan_tree(sh[j].n, sym_bytes, sh[j].sigma, sh[j].L, sh[j].l2_bits, sh[j].srate);
    toff[j] = tbytes;
    tbytes = round_up(tbytes + plans[j].total, 256);
  }
  // scratch of every tree
  struct SOff {
    size_t seq0, seq1, clear, tpre, ntb, z, zs, part, ns;
    uint64_t hist_n, clear_n, ntiles, nchunks, cstride, part_n;
  };
  std::vector<SOff> so(count);
  size_t sbytes = 0;
  auto take = [&](size_t bytes) {
    const size_t o = sbytes;
    sbytes = round_up(sbytes + bytes, 256);
    return o;
  };
  const uint32_t T = tile_elems(sym_bytes);
  for (uint32_t j = 0; j < count; ++j) {
    const TreePlan& P = plans[j];
    SOff& o = so[j];
    const uint64_t n = sh[j].n, L = sh[j].L;
    o.ntiles = ceil_div(std::max<uint64_t>(n, 1), T);
    const uint64_t seq_elems = round_up(std::max<uint64_t>(n, 1), T);
    o.hist_n = sh[j].sigma + 1;
    o.nchunks = ceil_div(o.ntiles, kChunkTiles);
    o.cstride = (o.ntiles + 1) + (o.nchunks + 1);
    o.clear_n = o.hist_n + std::max<uint64_t>(L, 1) * o.cstride + 8;  // hist | tile counts | err
    o.part_n = ceil_div(std::max<uint64_t>(o.hist_n, P.nheap + 1), kScanChunk) + 1;
    o.seq0 = take(L > 1 ? seq_elems * sym_bytes : 0);
    o.seq1 = take(L > 2 ? seq_elems * sym_bytes : 0);
    o.clear = take(o.clear_n * 8);
    o.tpre = take(std::max<uint64_t>(L, 1) * (o.ntiles + 1) * 8);
    o.ntb = take(std::max<uint64_t>(P.nheap, 1) * sizeof(NodeB));
    o.z = take((P.nheap + 1) * 8);
    o.zs = take((P.nheap + 1) * 8);
    o.part = take(o.part_n * 8);
    o.ns = take(sched[j].posmask ? P.nheap * sizeof(NodeS) : 0);
  }

  wt_forest* f = new wt_forest();
  f->count = count;
  f->w = sym_bytes;
  f->block_bytes = tbytes;
  f->block = dev_alloc(tbytes, st);
  if (!f->block) {
    delete f;
    return fail(WT_ERR_OOM, "wt_build_forest: allocation of %zu bytes for the trees failed", tbytes);
  }
  auto bail = [&](wt_status s) {
    for (wt_tree* t : f->trees) delete t;
    dev_free(f->block, st);
    delete f;
    return s;
  };
  void* sblock = dev_alloc(sbytes, st);
  if (!sblock) return bail(fail(WT_ERR_OOM, "wt_build_forest: scratch allocation of %zu bytes failed", sbytes));
  struct Free {
    void* p;
    hipStream_t s;
    ~Free() {
      if (p) dev_free(p, s);
    }
  } sfree{sblock, st};

  // per-tree state (build order) and block maps
  std::vector<TreeB> tb(count);
  MapBuilder m_init, m_hist_small, m_hist_big, m_hist_hash, m_scan_c, m_scan_z, m_node, m_tile;
  MapBuilder m_level[3];  // level passes over 1-, 2- and 4-byte codes: tiles of kTileBytes per tree
  bool any_pos = false;
  uint64_t all_tiles = 0;
  for (uint32_t j = 0; j < count; ++j) all_tiles += sh[j].n ? ceil_div(sh[j].n, T) : 0;
  // histogram blocks of a quarter of the single-tree size: most of a forest's trees get one block,
  // and shorter blocks for the long ones leave a shorter tail behind the last full round of blocks
  const uint64_t hist_tpb = std::max<uint64_t>(ceil_div(all_tiles, 4 * kHTargetBlocks), kHMinTiles);
  std::vector<uint32_t> active(Lmax + 1, 0);  // trees with more than l levels
  for (uint32_t s = 0; s < count; ++s) {
    const uint32_t j = order[s];
    const TreePlan& P = plans[j];
    const SOff& o = so[j];
    char* base = (char*)f->block + toff[j];
    char* sb = (char*)sblock;
    TreeB& b = tb[s];
    std::memset(&b, 0, sizeof(b));
    b.sym = h_descs[j].d_sym;
    b.n = sh[j].n;
    b.sigma = (uint32_t)sh[j].sigma;
    b.L = sh[j].L;
    b.pow2 = sh[j].pow2;
    b.aligned = ((uintptr_t)h_descs[j].d_sym & 15u) == 0;
    b.l2shift = log2_floor(sh[j].l2_bits);
    b.sshift = log2_floor(sh[j].srate);
    b.tshift = log2_floor(T);
    b.meta = (LevelMeta*)(base + P.off_meta);
    b.cum = (uint64_t*)(base + P.off_cum);
    b.nodes = (NodeQ*)(base + P.off_nodes);
    b.bits = (uint64_t*)(base + P.off_bits);
    b.L1 = (uint64_t*)(base + P.off_l1);
    b.L2 = (uint16_t*)(base + P.off_l2);
    b.smp = (uint64_t*)(base + P.off_smp);
    b.words_per_level = P.words_per_level;
    b.l1_per_level = P.l1_per_level;
    b.l2_per_level = P.l2_per_level;
    b.smp_per_level = P.smp_per_level;
    b.seq[0] = sb + o.seq0;
    b.seq[1] = sb + o.seq1;
    b.clear = (uint64_t*)(sb + o.clear);
    b.clear_n = o.clear_n;
    b.hist = b.clear;
    b.tcnt = b.clear + o.hist_n;
    b.err = (uint32_t*)(b.clear + o.hist_n + std::max<uint64_t>(b.L, 1) * o.cstride);
    b.tpre = (uint64_t*)(sb + o.tpre);
    b.ntb = (NodeB*)(sb + o.ntb);
    b.z = (uint64_t*)(sb + o.z);
    b.zs = (uint64_t*)(sb + o.zs);
    b.part = (uint64_t*)(sb + o.part);
    b.ntiles = o.ntiles;
    b.nchunks = o.nchunks;
    b.cstride = o.cstride;
    b.nheap = P.nheap;
    b.wlog = sched[j].wlog;
    b.posmask = sched[j].posmask;
    b.ns = sched[j].posmask ? (NodeS*)(sb + o.ns) : nullptr;
    any_pos = any_pos || sched[j].posmask != 0;
    for (uint32_t l = 0; l < b.L; ++l) active[l] = s + 1;

    const uint64_t ntiles_n = b.n ? ceil_div(b.n, T) : 0;
    m_init.add(s, std::min<uint64_t>(64, ceil_div(o.clear_n, (uint64_t)kBT * 16)));
    // histogram: dense (small or large LDS) in long tile ranges, or the hashed count for alphabets
    // above 2^16 (eight tiles per block, strided)
    const int hk = b.sigma + 1 <= kHSmallWords ? 0 : (b.sigma <= kHDenseMax ? 1 : 2);
    const uint64_t hdense = hist_dense_blocks(ntiles_n, hist_tpb);
    m_hist_small.add(s, hk == 0 ? hdense : 0);
    m_hist_big.add(s, hk == 1 ? hdense : 0);
    m_hist_hash.add(s, hk == 2 ? ceil_div(ntiles_n, 8) : 0);
    m_scan_c.add(s, ceil_div(o.hist_n, kScanChunk));
    m_scan_z.add(s, b.L ? ceil_div(P.nheap + 1, kScanChunk) : 0);
    m_node.add(s, b.L ? ceil_div(P.nheap, kBT) : 0);
    m_tile.add(s, b.L ? o.nchunks + 1 : 0);
    for (uint32_t k = 0; k < 3; ++k)
      m_level[k].add(s, b.L && (1u << k) <= sym_bytes ? ceil_div(b.n, tile_elems(1u << k)) : 0);
  }
  for (MapBuilder* m : {&m_init, &m_hist_small, &m_hist_big, &m_hist_hash, &m_scan_c, &m_scan_z, &m_node, &m_tile,
                        &m_level[0], &m_level[1], &m_level[2]})
    m->close();

  // one upload: tree states, build order, every map
  std::vector<char> hbuf;
  auto put = [&](const void* p, size_t bytes) {
    const size_t o = round_up(hbuf.size(), 256);
    hbuf.resize(o + std::max<size_t>(bytes, 1));
    if (bytes) std::memcpy(hbuf.data() + o, p, bytes);
    return o;
  };
  const size_t u_tb = put(tb.data(), tb.size() * sizeof(TreeB));
  const size_t u_order = put(order.data(), order.size() * 4);
  struct MapOff {
    size_t bmap, boff;
  };
  auto put_map = [&](const MapBuilder& m) { return MapOff{put(m.bmap.data(), m.bmap.size() * 4), put(m.boff.data(), m.boff.size() * 4)}; };
  const MapOff u_init = put_map(m_init), u_hs = put_map(m_hist_small), u_hb = put_map(m_hist_big),
               u_hh = put_map(m_hist_hash),
               u_sc = put_map(m_scan_c), u_sz = put_map(m_scan_z), u_node = put_map(m_node),
               u_tile = put_map(m_tile);
  const MapOff u_level[3] = {put_map(m_level[0]), put_map(m_level[1]), put_map(m_level[2])};
  const size_t u_out = round_up(hbuf.size(), 256);
  const size_t plan_bytes = u_out + (size_t)count * sizeof(ForestOut);
  void* dplan = dev_alloc(plan_bytes, st);
  if (!dplan) return bail(fail(WT_ERR_OOM, "wt_build_forest: plan allocation failed"));
  Free pfree{dplan, st};
  char* dp = (char*)dplan;
  WT_HIP(hipMemcpyAsync(dp, hbuf.data(), hbuf.size(), hipMemcpyHostToDevice, st));
  const TreeB* d_tb = (const TreeB*)(dp + u_tb);
  auto grid_of = [&](const MapOff& u, uint32_t l = 0, uint32_t base = 0) {
    ForestGrid g;
    g.tb = d_tb;
    g.bmap = (const uint32_t*)(dp + u.bmap);
    g.boff = (const uint32_t*)(dp + u.boff);
    g.l = l;
    g.base = base;
    return g;
  };
  ForestOut* d_out = (ForestOut*)(dp + u_out);
  const auto t_plan = std::chrono::steady_clock::now();

  // capture the build
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t nk = 0;
  WT_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  auto launch = [&](auto kernel, uint64_t blocks, uint32_t threads, size_t lds, auto... args) {
    if (blocks == 0) return;
    hipLaunchKernelGGL(kernel, dim3((uint32_t)blocks), dim3(threads), lds, st, args...);
    ++nk;
  };
  launch(kf_init, m_init.bmap.size(), kBT, 0, grid_of(u_init));
  auto launch_hist = [&](auto e) {
    using E = decltype(e);
    launch(kf_hist_dense<E, kHSmallWords>, m_hist_small.bmap.size(), kHT, 0, grid_of(u_hs));
    launch(kf_hist_dense<E, kHBigWords>, m_hist_big.bmap.size(), kHT, 0, grid_of(u_hb));
    launch(kf_hist_hash<E>, m_hist_hash.bmap.size(), kBT, 0, grid_of(u_hh));
  };
  if (sym_bytes == 1) launch_hist(uint8_t{});
  else if (sym_bytes == 2) launch_hist(uint16_t{});
  else launch_hist(uint32_t{});
  launch(kf_scan_reduce, m_scan_c.bmap.size(), kBT, 0, grid_of(u_sc), 0u);
  launch(kf_scan_partials, count, 1024, 0, d_tb, 0u);
  launch(kf_scan_down, m_scan_c.bmap.size(), kBT, 0, grid_of(u_sc), 0u);
  launch(kf_node_walk, m_node.bmap.size(), kBT, 0, grid_of(u_node));
  launch(kf_scan_reduce, m_scan_z.bmap.size(), kBT, 0, grid_of(u_sz), 1u);
  launch(kf_scan_partials, active.empty() ? 0 : (Lmax ? active[0] : 0), 1024, 0, d_tb, 1u);
  launch(kf_scan_down, m_scan_z.bmap.size(), kBT, 0, grid_of(u_sz), 1u);
  launch(kf_node_final, m_node.bmap.size(), kBT, 0, grid_of(u_node));
  if (any_pos) {
    // non-empty nodes in position order (z and zs are free again)
    launch(kf_ns_flag, m_node.bmap.size(), kBT, 0, grid_of(u_node));
    launch(kf_scan_reduce, m_scan_z.bmap.size(), kBT, 0, grid_of(u_sz), 1u);
    launch(kf_scan_partials, active.empty() ? 0 : (Lmax ? active[0] : 0), 1024, 0, d_tb, 1u);
    launch(kf_scan_down, m_scan_z.bmap.size(), kBT, 0, grid_of(u_sz), 1u);
    launch(kf_ns_scatter, m_node.bmap.size(), kBT, 0, grid_of(u_node));
  }
  // one level-pass launch per run of trees (in build order) with the same code widths and node lookup
  auto launch_level = [&](uint32_t wi, uint32_t wo, bool pos, uint64_t nb, const ForestGrid& g) {
#define WT_LV(E, EO)                                                      \
  do {                                                                    \
    if (pos) launch(k_level<E, true, EO, true>, nb, kBT, 0, LevelArgs{}, g);  \
    else launch(k_level<E, true, EO, false>, nb, kBT, 0, LevelArgs{}, g);     \
  } while (0)
    if (wi == 0) WT_LV(uint8_t, uint8_t);
    else if (wi == 1) {
      if (wo == 0) WT_LV(uint16_t, uint8_t);
      else WT_LV(uint16_t, uint16_t);
    } else {
      if (wo == 0) WT_LV(uint32_t, uint8_t);
      else if (wo == 1) WT_LV(uint32_t, uint16_t);
      else WT_LV(uint32_t, uint32_t);
    }
#undef WT_LV
  };
  auto level_class = [&](uint32_t s, uint32_t l) {
    const TreeB& b = tb[s];
    return (uint32_t)((b.wlog >> (2 * l)) & 15u) | (((b.posmask >> l) & 1u) << 4);  // input, output width, lookup
  };
  for (uint32_t l = 0; l < Lmax; ++l) {
    const uint32_t A = active[l];
    launch(kf_tile_reduce, m_tile.boff[A], kBT, 0, grid_of(u_tile, l));
    launch(kf_tile_scan, m_tile.boff[A], kBT, 0, grid_of(u_tile, l));
    for (uint32_t s0 = 0; s0 < A;) {
      const uint32_t c = level_class(s0, l);
      uint32_t s1 = s0 + 1;
      while (s1 < A && level_class(s1, l) == c) ++s1;
      const uint32_t wi = c & 3u, wo = (c >> 2) & 3u;
      const MapBuilder& m = m_level[wi];
      launch_level(wi, wo, (c >> 4) != 0, (uint64_t)m.boff[s1] - m.boff[s0], grid_of(u_level[wi], l, m.boff[s0]));
      s0 = s1;
    }
  }
  launch(kf_gather, count, 64, 0, d_tb, (const uint32_t*)(dp + u_order), d_out);
  hipError_t he = hipGetLastError();
  const hipError_t ce = hipStreamEndCapture(st, &graph);
  if (he == hipSuccess) he = ce;
  if (he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (he != hipSuccess) {
    if (exec) (void)hipGraphExecDestroy(exec);
    return bail(fail(WT_ERR_HIP, "wt_build_forest: graph capture: %s", hipGetErrorString(he)));
  }
  const auto t_cap = std::chrono::steady_clock::now();
  hipEvent_t e0, e1;
  WT_HIP(hipEventCreate(&e0));
  WT_HIP(hipEventCreate(&e1));
  WT_HIP(hipEventRecord(e0, st));
  he = hipGraphLaunch(exec, st);
  if (he == hipSuccess) he = hipEventRecord(e1, st);
  std::vector<ForestOut> ho(count);
  if (he == hipSuccess) he = hipMemcpyAsync(ho.data(), d_out, count * sizeof(ForestOut), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  float gms = 0.f;
  if (he == hipSuccess) (void)hipEventElapsedTime(&gms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(exec);
  if (he != hipSuccess) return bail(fail(WT_ERR_HIP, "wt_build_forest: graph launch: %s", hipGetErrorString(he)));

  for (uint32_t j = 0; j < count; ++j) {
    if (ho[j].err & 1u)
      return bail(fail(WT_ERR_SYMBOL_RANGE, "wt_build_forest: sequence %u has a symbol >= sigma (%llu)", j,
                       (unsigned long long)sh[j].sigma));
    if (ho[j].err & 2u)
      return bail(fail(WT_ERR_STATE, "wt_build_forest: internal error: a level pass placed an element of sequence "
                       "%u outside its tile", j));
  }
  uint64_t symbols = 0;
  for (uint32_t j = 0; j < count; ++j) {
    const TreePlan& P = plans[j];
    char* base = (char*)f->block + toff[j];
    wt_tree* t = new wt_tree();
    t->n = sh[j].n;
    t->sigma = sh[j].sigma;
    t->L = sh[j].L;
    t->w = sym_bytes;
    t->l2_bits = sh[j].l2_bits;
    t->srate = sh[j].srate;
    t->pow2 = sh[j].pow2;
    t->device = dev;
    t->borrowed = true;
    t->block = nullptr;
    t->block_bytes = P.total;
    t->dev.meta = (LevelMeta*)(base + P.off_meta);
    t->dev.cum = (uint64_t*)(base + P.off_cum);
    t->dev.nodes = (NodeQ*)(base + P.off_nodes);
    t->dev.bits = (uint64_t*)(base + P.off_bits);
    t->dev.L1 = (uint64_t*)(base + P.off_l1);
    t->dev.L2 = (uint16_t*)(base + P.off_l2);
    t->dev.smp = (uint64_t*)(base + P.off_smp);
    t->bytes_bits = (size_t)t->L * P.words_per_level * 8;
    t->bytes_l1 = (size_t)t->L * P.l1_per_level * 8;
    t->bytes_l2 = (size_t)t->L * P.l2_per_level * 2;
    t->bytes_smp = (size_t)t->L * P.smp_per_level * 8;
    t->bytes_nodes = (size_t)std::max<uint64_t>(P.nheap, 1) * sizeof(NodeQ);
    t->bytes_cum = (t->sigma + 1) * 8;
    for (uint32_t l = 0; l < t->L; ++l) t->hmeta[l] = ho[j].meta[l];
    f->trees.push_back(t);
    symbols += t->n;
  }
  const auto t_end = std::chrono::steady_clock::now();
  auto ms = [](auto a, auto b) { return (float)std::chrono::duration<double, std::milli>(b - a).count(); };
  f->info.trees = count;
  f->info.levels_max = Lmax;
  f->info.symbols = symbols;
  f->info.bytes_trees = tbytes;
  f->info.bytes_scratch = sbytes;
  f->info.graph_kernels = nk;
  f->info.plan_ms = ms(t_start, t_plan);
  f->info.capture_ms = ms(t_plan, t_cap);
  f->info.graph_ms = gms;
  f->info.total_ms = ms(t_start, t_end);
  *out = f;
  return WT_OK;
}

extern "C" wt_status wt_forest_tree(const wt_forest* f, uint32_t j, wt_tree** out) {
  clear_error();
  if (!f || !out) return fail(WT_ERR_ARG, "wt_forest_tree: NULL argument");
  if (j >= f->count) return fail(WT_ERR_ARG, "wt_forest_tree: tree %u >= %u", j, f->count);
  *out = f->trees[j];
  return WT_OK;
}

extern "C" wt_status wt_forest_info(const wt_forest* f, wt_forest_info_t* out) {
  clear_error();
  if (!f || !out) return fail(WT_ERR_ARG, "wt_forest_info: NULL argument");
  *out = f->info;
  return WT_OK;
}

extern "C" wt_status wt_forest_free(wt_forest* f) {
  clear_error();
  if (!f) return WT_OK;
  WT_HIP(hipDeviceSynchronize());
  for (wt_tree* t : f->trees) {
    if (t->learn) dev_free(t->learn, nullptr);
    delete t;
  }
  if (f->qtab) dev_free(f->qtab, nullptr);
  dev_free(f->block, nullptr);
  WT_HIP(hipDeviceSynchronize());
  delete f;
  return WT_OK;
}

namespace wt {

// Scratch of one mixed batch. Class sort (2048 < q < 2^16): class offsets, counts and cursors,
// classes, slots. (class, position) sort: class offsets, bucket ids, sort passes, bucket starts,
// slots. Nothing for the unbinned path.
struct MixLayout {
  size_t off = 0, counts = 0, cls = 0, ids = 0, sort = 0, tot = 0, perm = 0, total = 0;
};
MixLayout mix_layout(uint64_t q) {
  MixLayout L;
  if (q <= kMixDirectMax) return L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = round_up(o + bytes, 256);
    return at;
  };
  L.off = take(4 * (kMixClasses + 1));
  if (q < kMixSortMin) {
    L.counts = take(4 * 64);
    L.cls = take(q);
  } else {
    L.ids = take(2 * q);
    L.sort = take(sort_ids_bytes(q));
    L.tot = take(4 * kSortIdBins);
  }
  L.perm = take(4 * q);
  L.total = o;
  return L;
}

size_t mixed_scratch_bytes(uint64_t q) { return mix_layout(q).total; }

// Enqueues one mixed batch on st (scratch: mixed_scratch_bytes(q) bytes of device memory; vshift:
// forest_vshift of the forest).
hipError_t mixed_enqueue(const QTree* qt, uint32_t ntrees, const uint32_t* d_tree, const uint8_t* d_op,
                         const uint32_t* d_sym, const uint64_t* d_arg, uint64_t q, uint64_t* d_out, char* sb,
                         uint32_t vshift, hipStream_t st) {
  if (q <= kMixDirectMax) {
    hipLaunchKernelGGL(k_mix_direct, dim3((uint32_t)ceil_div(q, kQT)), dim3(kQT), 0, st, qt, ntrees, d_tree, d_op,
                       d_sym, d_arg, q, d_out);
    return hipGetLastError();
  }
  const MixLayout L = mix_layout(q);
  uint32_t* off = (uint32_t*)(sb + L.off);
  uint32_t* perm = (uint32_t*)(sb + L.perm);
  if (q < kMixSortMin) {
    uint32_t* counts = (uint32_t*)(sb + L.counts);
    uint32_t* cursor = counts + 32;
    const uint32_t nchunk = (uint32_t)ceil_div(q, kMixChunk);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, counts, 64u);
    hipLaunchKernelGGL(k_mix_count, dim3(nchunk), dim3(kQT), 0, st, qt, ntrees, d_tree, d_op, q,
                       (uint8_t*)(sb + L.cls), counts);
    hipLaunchKernelGGL(k_mix_off_counts, dim3(1), dim3(64), 0, st, (const uint32_t*)counts, q, off);
    hipLaunchKernelGGL(k_mix_scatter, dim3(nchunk), dim3(kQT), 0, st, q, (const uint8_t*)(sb + L.cls),
                       (const uint32_t*)off, cursor, perm);
  } else {
    uint16_t* ids = (uint16_t*)(sb + L.ids);
    uint32_t* tot = (uint32_t*)(sb + L.tot);
    hipLaunchKernelGGL(k_mix_bucket, dim3((uint32_t)std::min<uint64_t>(ceil_div(q, kQT), 4096)), dim3(kQT), 0, st, qt,
                       ntrees, d_tree, d_op, d_sym, d_arg, q, vshift, ids);
    sort_ids_enqueue(ids, q, sb + L.sort, tot, perm, st);
    hipLaunchKernelGGL(k_mix_off_buckets, dim3(1), dim3(64), 0, st, (const uint32_t*)tot, q, off);
  }
  // the class sizes stay on the device: every class kernel is launched and finds its own range
  const uint32_t grid = (uint32_t)std::min<uint64_t>(ceil_div(q, kQT), 2048);
  const uint32_t* po = off;
  const uint32_t* pm = perm;
#define WT_MIX(OP, S) \
  hipLaunchKernelGGL((k_mix_run<OP, S>), dim3(grid), dim3(kQT), 0, st, qt, po, pm, d_tree, d_sym, d_arg, d_out)
  WT_MIX(0, 8); WT_MIX(0, 9); WT_MIX(0, 10); WT_MIX(0, 11);
  WT_MIX(1, 8); WT_MIX(1, 9); WT_MIX(1, 10); WT_MIX(1, 11);
  WT_MIX(2, 8); WT_MIX(2, 9); WT_MIX(2, 10); WT_MIX(2, 11);
#undef WT_MIX
  hipLaunchKernelGGL(k_mix_invalid, dim3(std::min<uint32_t>(grid, 64)), dim3(kQT), 0, st, po, pm, d_out);
  return hipGetLastError();
}

uint32_t forest_count(const wt_forest* f) { return f->count; }
uint32_t forest_vshift(const wt_forest* f) { return f->vshift; }

// Query table of a forest, rebuilt when a tree's learned index changed since it was made.
wt_status forest_qtab(const wt_forest* fc, hipStream_t st, const QTree** out) {
  wt_forest* f = const_cast<wt_forest*>(fc);
  uint64_t ver = 0;
  for (const wt_tree* t : f->trees) ver += t->learn_version;
  if (!f->qtab || ver != f->qversion) {
    std::vector<QTree> hq(f->count);
    uint64_t vb = 0;
    for (uint32_t j = 0; j < f->count; ++j) {
      const wt_tree* t = f->trees[j];
      std::memset(&hq[j], 0, sizeof(QTree));
      hq[j].vbase = vb;
      vb += t->n + 1;
      hq[j].a = make_args(t);
      hq[j].lq = t->learn && t->nmodels ? (const LearnQ*)((const char*)t->learn + (size_t)t->nmodels * learn_model_bytes())
                                        : nullptr;
      hq[j].l2s = log2_floor(t->l2_bits);
    }
    uint32_t bits = 0;
    while ((1ull << bits) < vb) ++bits;
    f->vshift = bits > 11 ? bits - 11 : 0;  // kMixB = 2^11 buckets over the whole space
    if (!f->qtab) {
      f->qtab = dev_alloc(f->count * sizeof(QTree), st);
      if (!f->qtab) return fail(WT_ERR_OOM, "query table allocation failed");
    }
    WT_HIP(hipMemcpyAsync(f->qtab, hq.data(), f->count * sizeof(QTree), hipMemcpyHostToDevice, st));
    WT_HIP(hipStreamSynchronize(st));
    f->qversion = ver;
  }
  *out = (const QTree*)f->qtab;
  return WT_OK;
}

}  // namespace wt

extern "C" wt_status wt_query_mixed(const wt_forest* f, const uint32_t* d_tree, const uint8_t* d_op,
                                    const uint32_t* d_sym, const uint64_t* d_arg, uint64_t q, uint64_t* d_out,
                                    wt_stream_t stream) {
  clear_error();
  if (!f) return fail(WT_ERR_ARG, "wt_query_mixed: forest is NULL");
  if (q == 0) return WT_OK;
  if (!d_tree || !d_op || !d_arg || !d_out) return fail(WT_ERR_ARG, "wt_query_mixed: NULL buffer");
  if (q >= (1ull << 32)) return fail(WT_ERR_ARG, "wt_query_mixed: at most 2^32 - 1 queries per call");
  hipStream_t st = (hipStream_t)stream;
  const QTree* qt = nullptr;
  const wt_status rc = forest_qtab(f, st, &qt);
  if (rc != WT_OK) return rc;
  const size_t bytes = mixed_scratch_bytes(q);
  char* sb = nullptr;
  if (bytes) {
    sb = (char*)dev_alloc(bytes, st);
    if (!sb) return fail(WT_ERR_OOM, "wt_query_mixed: scratch allocation of %zu bytes failed", bytes);
  }
  const hipError_t he = mixed_enqueue(qt, f->count, d_tree, d_op, d_sym, d_arg, q, d_out, sb, f->vshift, st);
  if (sb) dev_free(sb, st);
  if (he != hipSuccess) return fail(WT_ERR_HIP, "wt_query_mixed: %s", hipGetErrorString(he));
  return WT_OK;
}
