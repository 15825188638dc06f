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

#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

constexpr int kBT = 256;         // threads per block (4 waves)
constexpr int kHashSlots = 4096; // LDS count cache for large alphabets

template <typename E>
struct Tile {
  static constexpr int EV = 16 / (int)sizeof(E);         // elements per 16-byte vector
  static constexpr int NCH = kTileBytes / (kBT * 16);     // vectors per thread
  static constexpr int T = kBT * NCH * EV;               // elements per tile
  static constexpr int W = T / 64;                       // bit words per tile
  static constexpr int G = 64 / EV;                      // lanes whose vectors form one word
  static constexpr int TSHIFT = __builtin_ctz((unsigned)T);
  static_assert((1 << TSHIFT) == T, "tile");
  static_assert(T % 512 == 0 && kL1Bits % T == 0, "tiles cover whole L2 blocks and divide L1 blocks");
};

// ---------------------------------------------------------------- block scans

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  return x;
}

// Exclusive scan over the block (blockDim.x threads, multiple of 64, at most 1024); s_w holds one
// entry per wave. Returns the exclusive prefix and the block total.
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t x, uint32_t* s_w, uint32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t inc = wave_incl_scan_u32(x);
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const uint32_t v = s_w[i];
    pre += (i < wv) ? v : 0u;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return pre + inc - x;
}

__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t x, uint64_t* s_w, uint64_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t inc = wave_incl_scan_u64(x);
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
  for (int i = 0; i < nw; ++i) {
    const uint64_t v = s_w[i];
    pre += (i < wv) ? v : 0ull;
    tot += v;
  }
  __syncthreads();
  total = tot;
  return pre + inc - x;
}

// ---------------------------------------------------------------- generic u64 exclusive scan

constexpr int kScanPer = 16;
constexpr int kScanChunk = kBT * kScanPer;  // elements per block

__global__ __launch_bounds__(kBT) void k_scan_reduce(const uint64_t* __restrict__ in, uint64_t n,
                                                     uint64_t* __restrict__ part) {
  __shared__ uint64_t s_w[kBT / 64];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i)
    if (b0 + i < n) s += in[b0 + i];
  uint64_t tot;
  block_excl_scan_u64(s, s_w, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of np partial sums in place.
__global__ __launch_bounds__(1024) void k_scan_partials(uint64_t* __restrict__ part, uint64_t np) {
  __shared__ uint64_t s_w[16];
  uint64_t carry = 0;
  for (uint64_t base = 0; base < np; base += 1024) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t x = i < np ? part[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_excl_scan_u64(x, s_w, tot);
    if (i < np) part[i] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(kBT) void k_scan_down(const uint64_t* __restrict__ in, uint64_t n,
                                                   const uint64_t* __restrict__ part, uint64_t* __restrict__ out) {
  __shared__ uint64_t s_w[kBT / 64];
  const uint64_t b0 = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = (b0 + i < n) ? in[b0 + i] : 0;
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan_u64(s, s_w, tot) + part[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (b0 + i < n) out[b0 + i] = run;
    run += v[i];
  }
}

// out[i] = sum of in[0, i) for i in [0, n); `part` needs ceil(n / kScanChunk) entries.
static hipError_t exclusive_scan_u64(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* part,
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
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- loads

// Loads elements [q0, q0 + EV) of a tile into v; elements at or beyond cnt read as 0. `vec` says the
// 16 bytes starting at q0 may be read as one vector (aligned and inside the buffer).
template <typename E>
__device__ __forceinline__ void load16(const E* __restrict__ base, uint32_t q0, uint32_t cnt, bool vec,
                                       E (&v)[16 / sizeof(E)]) {
  constexpr int EV = 16 / (int)sizeof(E);
  if (vec) {
    const uint4 x = *reinterpret_cast<const uint4*>(base + q0);
    __builtin_memcpy(v, &x, 16);
    if (q0 + EV > cnt) {
#pragma unroll
      for (int e = 0; e < EV; ++e)
        if (q0 + e >= cnt) v[e] = 0;
    }
  } else {
#pragma unroll
    for (int e = 0; e < EV; ++e) v[e] = (q0 + e < cnt) ? base[q0 + e] : (E)0;
  }
}

// ---------------------------------------------------------------- histogram (Section 5.1.1)

// Ones per tile are accumulated per chunk of kChunkTiles tiles as well, so a level's tile prefix
// needs one launch: block b adds the chunk sums before it to the scan of its own chunk.
constexpr int kChunkShift = 10;
constexpr uint64_t kChunkTiles = 1ull << kChunkShift;

// Persistent grid over whole tiles. Small alphabets count into LDS replicas (one per group of
// threads, assigned round-robin; replicas are padded by one counter so equal symbols of different
// replicas fall into different banks); large alphabets use an LDS cache of claimed symbols with
// global atomics for the rest. Also records, per level-0 tile, the number of ones (code bit L-1).
template <typename E, bool kSmall>
__global__ __launch_bounds__(kBT) void k_hist(const E* __restrict__ sym, uint64_t n, uint32_t sigma, uint32_t L,
                                              uint32_t pow2, uint32_t aligned, uint32_t nrep,
                                              uint64_t* __restrict__ hist, uint64_t* __restrict__ tile_cnt0,
                                              uint32_t* __restrict__ err) {
  using TL = Tile<E>;
  extern __shared__ uint32_t s_h[];
  __shared__ uint32_t s_w[kBT / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t stride = sigma + 1;
  const uint32_t hsize = kSmall ? nrep * stride : 2u * kHashSlots;
  for (uint32_t i = tid; i < hsize; i += kBT) s_h[i] = 0;
  __syncthreads();
  uint32_t* my_h = s_h + (kSmall ? (tid % nrep) * stride : 0u);
  uint32_t* s_keys = s_h;
  uint32_t* s_cnts = s_h + kHashSlots;
  const uint64_t ntiles = (n + TL::T - 1) >> TL::TSHIFT;
  uint32_t bad = 0;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t t0 = t << TL::TSHIFT;
    const uint32_t cnt = (uint32_t)min<uint64_t>(TL::T, n - t0);
    uint32_t ones = 0;
#pragma unroll 1
    for (int k = 0; k < TL::NCH; ++k) {
      const uint32_t q0 = (uint32_t)(k * kBT + tid) * TL::EV;
      E v[TL::EV];
      load16<E>(sym + t0, q0, cnt, aligned && (q0 + TL::EV <= cnt), v);
#pragma unroll
      for (int e = 0; e < TL::EV; ++e) {
        const uint32_t s = (uint32_t)v[e];
        const bool in = q0 + e < cnt;
        if (in && s >= sigma) bad = 1;
        if (in && s < sigma) {
          if (L) {
            uint32_t len;
            const uint32_t code = encode_sym(s, sigma, L, pow2, &len);
            ones += (code >> (L - 1)) & 1u;
          }
          if (kSmall) {
            atomicAdd(&my_h[s], 1u);
          } else {
            const uint32_t h = (s * 2654435761u) >> (32 - 12);
            const uint32_t old = atomicCAS(&s_keys[h], 0u, s + 1u);
            if (old == 0u || old == s + 1u) atomicAdd(&s_cnts[h], 1u);
            else atomicAdd((unsigned long long*)&hist[s], 1ull);
          }
        }
      }
    }
    uint32_t tot;
    block_excl_scan_u32(ones, s_w, tot);
    if (tid == 0) tile_cnt0[t] = tot;
  }
  if (bad) atomicOr(err, 1u);
  __syncthreads();
  if (kSmall) {
    for (uint32_t s = tid; s < sigma; s += kBT) {
      uint64_t c = 0;
      for (uint32_t r = 0; r < nrep; ++r) c += s_h[r * stride + s];
      if (c) atomicAdd((unsigned long long*)&hist[s], (unsigned long long)c);
    }
  } else {
    for (uint32_t h = tid; h < (uint32_t)kHashSlots; h += kBT) {
      const uint32_t key = s_keys[h];
      if (key) atomicAdd((unsigned long long*)&hist[key - 1u], (unsigned long long)s_cnts[h]);
    }
  }
}

// ---------------------------------------------------------------- node tables

// Heap entry h (level l = floor(lg(h+1)), code prefix p = h + 1 - 2^l): follow p from the root with
// the split rule of the reduced tree (left child = the largest power of two strictly below the
// width). A prefix that reaches a leaf before level l names no node at level l.
__global__ void k_node_walk(uint32_t sigma, uint64_t nheap, const uint64_t* __restrict__ cum,
                            NodeB* __restrict__ ntb, uint64_t* __restrict__ zeros) {
  const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nheap) return;
  const uint32_t l = 63u - (uint32_t)__clzll(h + 1);
  const uint64_t p = h + 1 - (1ull << l);
  uint64_t s = 0, e = sigma;
  bool exists = true;
  for (int i = (int)l - 1; i >= 0; --i) {
    if (e - s <= 1) {
      exists = false;
      break;
    }
    const uint64_t half = pow2_below(e - s);
    if ((p >> i) & 1) s += half;
    else e = s + half;
  }
  if (exists && e - s <= 1) exists = false;
  if (exists) {
    const uint64_t m = s + pow2_below(e - s);
    NodeB b;
    b.start = cum[s];
    b.end = cum[e];
    b.off0 = cum[m];  // left-child end, turned into off0/off1 by k_node_final
    b.off1 = 0;
    ntb[h] = b;
    zeros[h] = cum[m] - cum[s];
  } else {
    NodeB b;
    b.start = kNoNode;
    b.end = 0;
    b.off0 = 0;
    b.off1 = 0;
    ntb[h] = b;
    zeros[h] = 0;
  }
}

// zs = exclusive prefix sums of the left-child sizes in heap order, so the rank0 at a node start is
// zs[h] - zs[first entry of the level].
__global__ void k_node_final(uint64_t nheap, const uint64_t* __restrict__ zs, NodeB* __restrict__ ntb,
                             NodeQ* __restrict__ ntq, LevelMeta* __restrict__ meta) {
  const uint64_t h = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nheap) return;
  const uint32_t l = 63u - (uint32_t)__clzll(h + 1);
  const uint64_t base = (1ull << l) - 1;
  NodeB b = ntb[h];
  NodeQ q;
  if (b.start == kNoNode) {
    q.start = kNoNode;
    q.r0 = kNoNode;
    ntq[h] = q;
    return;
  }
  const uint64_t r0 = zs[h] - zs[base];
  const uint64_t mid = b.off0;
  q.start = b.start;
  q.r0 = r0;
  ntq[h] = q;
  b.off0 = b.start - r0;
  b.off1 = mid - b.start + r0;
  ntb[h] = b;
  atomicMax((unsigned long long*)&meta[l].n, (unsigned long long)b.end);
}

// ---------------------------------------------------------------- per-level tile prefix

// Sum of the ones of every chunk of kChunkTiles tiles of level l.
__global__ __launch_bounds__(kBT) void k_tile_reduce(const LevelMeta* __restrict__ meta, uint32_t l,
                                                     uint32_t tshift, const uint64_t* __restrict__ cnt,
                                                     uint64_t* __restrict__ chunk) {
  __shared__ uint64_t s_w[kBT / 64];
  const uint64_t nl = meta[l].n;
  const uint64_t nt = (nl + (1ull << tshift) - 1) >> tshift;
  const uint64_t b = blockIdx.x;
  if ((b << kChunkShift) >= nt) return;
  constexpr int kPer = (int)(kChunkTiles / kBT);
  const uint64_t i0 = (b << kChunkShift) + (uint64_t)threadIdx.x * kPer;
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) sum += (i0 + i < nt) ? cnt[i0 + i] : 0ull;
  uint64_t tot;
  block_excl_scan_u64(sum, s_w, tot);
  if (threadIdx.x == 0) chunk[b] = tot;
}

// Exclusive prefix of the ones per tile of level l (tile size 2^tshift). Block b scans the tiles of
// chunk b (4 per thread) after adding the sums of the chunks before it. Levels with no element get
// their sentinel L1/L2 entries here; otherwise the block of the last tile writes them.
__global__ __launch_bounds__(kBT) void k_tile_scan(LevelMeta* __restrict__ meta, uint32_t l, uint32_t tshift,
                                                   const uint64_t* __restrict__ cnt,
                                                   const uint64_t* __restrict__ chunk, uint64_t* __restrict__ pre,
                                                   uint64_t* __restrict__ L1, uint16_t* __restrict__ L2) {
  __shared__ uint64_t s_w[kBT / 64];
  const LevelMeta m = meta[l];
  const uint64_t nl = m.n;
  const uint64_t nt = (nl + (1ull << tshift) - 1) >> tshift;
  const uint64_t b = blockIdx.x;
  if (nl == 0) {
    if (b == 0 && threadIdx.x == 0) {
      pre[0] = 0;
      meta[l].ones = 0;
      L1[m.l1] = 0;
      L2[m.l2] = 0;
    }
    return;
  }
  if ((b << kChunkShift) > nt) return;
  uint64_t before = 0;
  for (uint64_t c = threadIdx.x; c < b; c += kBT) before += chunk[c];
  uint64_t tot;
  block_excl_scan_u64(before, s_w, tot);
  before = tot;
  constexpr int kPer = (int)(kChunkTiles / kBT);
  const uint64_t i0 = (b << kChunkShift) + (uint64_t)threadIdx.x * kPer;
  uint64_t v[kPer];
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    v[i] = (i0 + i < nt) ? cnt[i0 + i] : 0ull;
    sum += v[i];
  }
  uint64_t run = before + block_excl_scan_u64(sum, s_w, tot);
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    if (i0 + i <= nt) pre[i0 + i] = run;
    run += v[i];
  }
}

// ---------------------------------------------------------------- level pass

struct LevelArgs {
  const void* in;  // level-l sequence (codes; symbols at level 0)
  void* out;       // level-(l+1) sequence
  uint64_t* bits;
  uint64_t* L1;
  uint16_t* L2;
  uint64_t* smp;
  LevelMeta* meta;
  const uint64_t* pre;    // exclusive ones before each tile of this level
  uint64_t* cnt_next;     // ones per tile of level l + 1 (accumulated)
  const NodeB* ntb;       // node table of this level, indexed by code prefix
  uint32_t l, L, sigma, pow2;
  uint32_t l2shift, sshift;
  uint32_t encode;      // level 0 of a reduced alphabet: turn symbols into codes
  uint32_t in_vec;      // the input may be read with 16-byte vectors everywhere (padded and aligned)
  uint32_t in_aligned;  // the input base is 16-byte aligned (vectors only inside the sequence)
};

// Adds, for the lanes in `cls`, their next-level ones (the bit `nbit`, or `cnt_lane` when nbit is
// unused) per destination tile to a running per-wave (tile, count) pair, flushing it to the global
// tile counter when the tile changes. Destinations increase with the processing order, so each tile
// is flushed about once per wave, and a tile counter sees few writers.
__device__ __forceinline__ void count_next(uint64_t cls, uint64_t dt, uint32_t nbit, uint32_t lane,
                                           uint64_t& cur_tile, uint32_t& cur_c, uint64_t* __restrict__ cnt,
                                           uint32_t cnt_lane) {
  const uint32_t mine = nbit + cnt_lane;
  while (cls) {
    const int leader = __ffsll((unsigned long long)cls) - 1;
    const uint64_t ldt = __shfl(dt, leader, 64);
    const bool in = ((cls >> lane) & 1ull) && dt == ldt;
    const uint64_t same = __ballot(in);
    uint32_t c1 = in ? mine : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c1 += __shfl_xor(c1, off, 64);
    if (ldt == cur_tile) {
      cur_c += c1;
    } else {
      if (cur_c && lane == 0) atomicAdd((unsigned long long*)&cnt[cur_tile], (unsigned long long)cur_c);
      cur_tile = ldt;
      cur_c = c1;
    }
    cls &= ~same;
  }
}

// Tile-local rank1 at x in [0, T]: ones in the words before x / 64 plus the low bits of that word.
__device__ __forceinline__ uint32_t r1loc(const uint64_t* __restrict__ sw, const uint32_t* __restrict__ sp,
                                          uint32_t x) {
  const uint32_t wi = x >> 6, bi = x & 63u;
  return sp[wi] + popc64(sw[wi] & ((1ull << bi) - 1ull));
}

struct Seg {
  uint32_t a, z, zs, pad;  // tile-local segment [a, z) and its zeros
  uint64_t d0, d1;         // level-(l+1) destinations of its first zero and first one
};
constexpr int kSegMax = 128;  // node segments per tile handled by the vector write-out
static_assert(2 * kSegMax <= kBT, "one thread per run in the run prefix");

// A lane meets the node of its element at tile position q: the node's segment [sa, sz) of the tile,
// its zeros zs and the tile-local rank1 R1a at its start. The lane holding the segment's first
// element records the segment's two runs.
__device__ __forceinline__ void enter_node(const NodeB nb, uint32_t q, uint64_t t0, uint32_t cnt, uint64_t G0,
                                           uint64_t G1, const uint64_t* s_words, const uint32_t* s_wpre,
                                           Seg* s_seg, uint32_t* s_nseg, uint32_t& sa, uint32_t& zs,
                                           uint32_t& R1a) {
  sa = (uint32_t)(nb.start > t0 ? min(nb.start - t0, (uint64_t)cnt) : 0ull);
  const uint32_t sz = (uint32_t)(nb.end > t0 ? min(nb.end - t0, (uint64_t)cnt) : 0ull);
  R1a = r1loc(s_words, s_wpre, sa);
  zs = (sz - r1loc(s_words, s_wpre, sz)) - (sa - R1a);
  if (q == sa) {
    const uint32_t idx = atomicAdd(s_nseg, 1u);
    if (idx < (uint32_t)kSegMax) {
      Seg g;
      g.a = sa;
      g.z = sz;
      g.zs = zs;
      g.pad = 0;
      g.d0 = nb.off0 + G0 + (sa - R1a);
      g.d1 = nb.off1 + G1 + R1a;
      s_seg[idx] = g;
    }
  }
}

// Element e of a 16-byte vector of E (e a compile-time constant after unrolling).
template <typename E>
__device__ __forceinline__ uint32_t vec_elem(const uint4& x, uint32_t e) {
  constexpr uint32_t per = 4 / sizeof(E);  // elements per dword
  const uint32_t d = e / per;
  const uint32_t dw = d < 2 ? (d == 0 ? x.x : x.y) : (d == 2 ? x.z : x.w);
  if constexpr (sizeof(E) == 4) return dw;
  else return (dw >> ((e % per) * 8 * sizeof(E))) & ((1u << (8 * sizeof(E))) - 1u);
}

// Element e of the 128-bit value (lo, hi) for a run-time e, by shifting (no indexed access, which
// would put the vector in scratch memory).
template <typename E>
__device__ __forceinline__ uint32_t elem128(uint64_t lo, uint64_t hi, uint32_t e) {
  const uint32_t sh = e * 8u * (uint32_t)sizeof(E);
  const uint64_t v = sh < 64 ? (sh ? (lo >> sh) | (hi << (64 - sh)) : lo) : (hi >> (sh - 64));
  return (uint32_t)v & (uint32_t)((1ull << (8 * sizeof(E))) - 1ull);
}

// One block per tile of T elements of level l:
//  1. coalesced 16-byte loads (NCH per thread, kept in registers); each vector gives EV bits and G
//     neighbouring lanes OR them into one 64-bit word of the level;
//  2. block scan of the word popcounts -> tile-local rank1 at every word;
//  3. bit words, L2 entries (ones since the enclosing L1 block start), the L1 entry when the tile
//     starts an L1 block, select samples where the global one/zero count crosses a multiple of s;
//  4. stable partition into level l + 1: every element goes to off_b[node] + rank_b(position).
//     a. staged in LDS in destination order: a node segment of the tile keeps its slot range and is
//        reordered zeros first (each lane walks its own vectors with a running rank);
//     b. runs (segment, bit) are contiguous in the destination: each lane writes one aligned
//        16-byte chunk of a run (element stores only at run edges), and the next level's ones per
//        destination tile are counted on the way.
template <typename E>
__global__ __launch_bounds__(kBT) void k_level(LevelArgs a) {
  using TL = Tile<E>;
  constexpr int T = TL::T, W = TL::W, EV = TL::EV, G = TL::G, NCH = TL::NCH;
  __shared__ __align__(16) E s_stage[T + 16 / sizeof(E) + 4];  // + slack for the 20-byte chunk reads
  __shared__ uint64_t s_words[W + 1];  // entry W: 0, so ranks are defined at x = T
  __shared__ uint32_t s_wpre[W + 1];   // entry W: ones of the tile
  __shared__ uint32_t s_w[kBT / 64];
  __shared__ Seg s_seg[kSegMax];
  __shared__ uint32_t s_cp[2 * kSegMax + 1];
  __shared__ uint32_t s_nseg;
  __shared__ uint64_t s_node[2];  // node of the tile's first and last element
  __shared__ uint64_t s_dst[2];   // single-node tile: destinations of its first zero and first one
  __shared__ uint32_t s_nc[4];    // single-node tile: next-level ones per (run, destination tile)

  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t l = a.l, L = a.L;
  const LevelMeta m = a.meta[l];
  const uint64_t nl = m.n;
  const uint64_t t = blockIdx.x;
  const uint64_t t0 = t << TL::TSHIFT;
  if (t0 >= nl) return;
  // independent scalars first, so their latency overlaps the tile loads
  const bool last = l + 1 >= L;
  const uint64_t G1 = a.pre[t];  // ones of the level before the tile
  const uint64_t l1val = a.pre[t & ~(uint64_t)((kL1Bits / T) - 1)];
  const uint64_t n_next = last ? 0ull : a.meta[l + 1].n;
  const uint32_t cnt = (uint32_t)min<uint64_t>((uint64_t)T, nl - t0);
  const uint32_t bsh = L - 1 - l;
  if (tid == 0) s_nseg = 0;

  // 1. load, encode (level 0 of a reduced alphabet), bit words
  const E* in = reinterpret_cast<const E*>(a.in) + t0;
  uint4 vx[NCH];
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
    E v[EV];
    load16<E>(in, q0, cnt, a.in_vec || (a.in_aligned && q0 + EV <= cnt), v);
    if (a.encode) {
#pragma unroll
      for (int e = 0; e < EV; ++e) {
        uint32_t s = (uint32_t)v[e];
        if (s >= a.sigma) s = 0;  // out-of-range input: the build reports an error; keep indices valid
        uint32_t len;
        v[e] = (E)encode_sym(s, a.sigma, L, a.pow2, &len);
      }
    }
    __builtin_memcpy(&vx[k], v, 16);
  }
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
    uint32_t mask = 0;
#pragma unroll
    for (int e = 0; e < EV; ++e)
      if (q0 + e < cnt) mask |= ((vec_elem<E>(vx[k], e) >> bsh) & 1u) << e;
    uint64_t word = (uint64_t)mask << ((tid % G) * EV);
#pragma unroll
    for (int off = 1; off < G; off <<= 1) word |= __shfl_xor(word, off, 64);
    if (tid % G == 0) s_words[k * (kBT / G) + tid / G] = word;
    if (q0 < cnt && q0 + EV > cnt - 1) {
      const uint32_t cx = elem128<E>(((uint64_t)vx[k].y << 32) | vx[k].x, ((uint64_t)vx[k].w << 32) | vx[k].z,
                                     cnt - 1 - q0);
      s_node[1] = l ? ((uint64_t)cx >> (L - l)) & ((1ull << l) - 1ull) : 0ull;
    }
    if (q0 == 0) s_node[0] = l ? ((uint64_t)vec_elem<E>(vx[k], 0) >> (L - l)) & ((1ull << l) - 1ull) : 0ull;
  }
  if (tid < 4) s_nc[tid] = 0;
  __syncthreads();
  // a tile inside one node (the rule at shallow levels) takes the fast path: two runs, no segments
  const bool single = s_node[0] == s_node[1];
  if (single && !last && tid == 0) {
    const NodeB nb = a.ntb[s_node[0]];
    s_dst[0] = nb.off0 + (t0 - G1);
    s_dst[1] = nb.off1 + G1;
  }

  // 2. tile-local rank1 at every word
  uint32_t tile_ones;
  {
    const uint32_t pc = (tid < (uint32_t)W) ? popc64(s_words[tid]) : 0u;
    const uint32_t ex = block_excl_scan_u32(pc, s_w, tile_ones);
    if (tid < (uint32_t)W) s_wpre[tid] = ex;
    if (tid == 0) {
      s_wpre[W] = tile_ones;
      s_words[W] = 0;
    }
  }
  __syncthreads();

  // 3. bits and directory
  const uint64_t G0 = t0 - G1;  // zeros of the level before the tile
  if (tid < (uint32_t)W) {
    const uint64_t word = s_words[tid];
    const uint64_t gw = ((uint64_t)t * W) + tid;
    a.bits[m.bits + gw] = word;
    const uint32_t q = tid * 64u;
    if (q < cnt) {
      const uint64_t ones_before = G1 + s_wpre[tid];
      const uint32_t l2w_shift = a.l2shift - 6;
      if ((gw & ((1ull << l2w_shift) - 1)) == 0) a.L2[m.l2 + (gw >> l2w_shift)] = (uint16_t)(ones_before - l1val);
      const uint32_t sh = a.sshift;
      const uint32_t pc = popc64(word);
      const uint64_t k1 = (ones_before + pc) >> sh;
      if (k1 > (ones_before >> sh)) {
        const uint32_t r = (uint32_t)((k1 << sh) - ones_before);
        a.smp[m.smp + k1 - 1] = t0 + q + select_in_word(word, r);
      }
      const uint32_t vb = min(64u, cnt - q);
      const uint64_t zw = ~word & (vb == 64u ? ~0ull : ((1ull << vb) - 1ull));
      const uint64_t zeros_before = t0 + q - ones_before;
      const uint64_t k0 = (zeros_before + popc64(zw)) >> sh;
      if (k0 > (zeros_before >> sh)) {
        const uint32_t r = (uint32_t)((k0 << sh) - zeros_before);
        a.smp[m.smp + m.smp_cap - k0] = t0 + q + select_in_word(zw, r);
      }
    }
  }
  if (tid == 0) {
    if ((t0 & (kL1Bits - 1)) == 0) a.L1[m.l1 + (t0 >> kL1Shift)] = G1;
    if (t0 + cnt == nl) {
      // last tile: total ones and the sentinel L1/L2 entries that make rank defined at i = n_l
      const uint64_t total = G1 + tile_ones;
      a.meta[l].ones = total;
      a.L1[m.l1 + ((nl + kL1Bits - 1) >> kL1Shift)] = total;
      const uint64_t j = (nl + (1ull << a.l2shift) - 1) >> a.l2shift;
      const uint64_t blk = (j << a.l2shift) >> kL1Shift;
      const uint64_t lv = ((blk << kL1Shift) >= nl) ? total : a.pre[blk << (kL1Shift - TL::TSHIFT)];
      a.L2[m.l2 + j] = (uint16_t)(total - lv);
    }
  }
  if (last) return;

  // 4a. staging
  const uint32_t nbsh = L - 2 - l;
  const uint64_t pmask = (1ull << l) - 1ull;
  if (single) {
    // zeros fill slots [0, Z), ones [Z, cnt)
    const uint32_t Z = cnt - tile_ones;
#pragma unroll 1
    for (int k = 0; k < NCH; ++k) {
      const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
      if (q0 < cnt) {
        // vector k without indexed access (an indexed register array would go to scratch)
        uint4 x = vx[0];
#pragma unroll
        for (int kk = 1; kk < NCH; ++kk)
          if (k == kk) x = vx[kk];
        uint32_t r1 = r1loc(s_words, s_wpre, q0);
        uint32_t r0 = q0 - r1;
        const uint32_t nv = min((uint32_t)EV, cnt - q0);
#pragma unroll
        for (int e = 0; e < EV; ++e) {
          if ((uint32_t)e < nv) {
            const uint32_t code = vec_elem<E>(x, e);
            const uint32_t b = (code >> bsh) & 1u;
            s_stage[b ? Z + r1 : r0] = (E)code;
            r1 += b;
            r0 += 1u - b;
          }
        }
      }
    }
    __syncthreads();
    // 4b. write-out of the two runs, one 16-byte destination chunk per lane; the next level's ones
    //     are counted per (run, destination tile): a run of at most T elements touches two tiles
    const uint64_t d0 = s_dst[0], d1 = s_dst[1];
    char* outb = reinterpret_cast<char*>(a.out);
    const uint32_t* st32 = reinterpret_cast<const uint32_t*>(s_stage);
    const uint32_t len0 = d0 < n_next ? (uint32_t)min<uint64_t>(Z, n_next - d0) : 0u;
    const uint32_t len1 = d1 < n_next ? (uint32_t)min<uint64_t>(cnt - Z, n_next - d1) : 0u;
    const uint32_t C0 = len0 ? (uint32_t)(((d0 + len0 - 1) * sizeof(E) >> 4) - ((d0 * sizeof(E)) >> 4) + 1) : 0u;
    const uint32_t C1 = len1 ? (uint32_t)(((d1 + len1 - 1) * sizeof(E) >> 4) - ((d1 * sizeof(E)) >> 4) + 1) : 0u;
    constexpr uint32_t kTileB = (uint32_t)T * (uint32_t)sizeof(E);  // bytes of a destination tile
    uint32_t cnt4[4] = {0u, 0u, 0u, 0u};                          // (run, first / second tile)
    for (uint32_t c = tid; c < C0 + C1; c += kBT) {
      const bool bb = c >= C0;
      const uint64_t d = bb ? d1 : d0;
      const uint32_t len = bb ? len1 : len0;
      const uint32_t slot0 = bb ? Z : 0u;
      const uint64_t db = d * sizeof(E), de = (d + len) * sizeof(E);
      const uint64_t cb = ((db >> 4) + (bb ? c - C0 : c)) << 4;
      const uint64_t blo = max(db, cb), bhi = min(de, cb + 16);
      const uint32_t src = slot0 * (uint32_t)sizeof(E) + (uint32_t)(blo - db);
      uint32_t nb = 0;
      if (blo == cb && bhi == cb + 16) {
        const uint32_t dw = src >> 2, sh = src & 3u;
        const uint32_t x0 = st32[dw], x1 = st32[dw + 1], x2 = st32[dw + 2], x3 = st32[dw + 3], x4 = st32[dw + 4];
        uint4 y;
        y.x = __builtin_amdgcn_alignbyte(x1, x0, sh);
        y.y = __builtin_amdgcn_alignbyte(x2, x1, sh);
        y.z = __builtin_amdgcn_alignbyte(x3, x2, sh);
        y.w = __builtin_amdgcn_alignbyte(x4, x3, sh);
        *reinterpret_cast<uint4*>(outb + cb) = y;
        // next-level bits of the 16/w elements: one bit per element, popcount per dword
        constexpr uint32_t kLow = sizeof(E) == 1 ? 0x01010101u : (sizeof(E) == 2 ? 0x00010001u : 1u);
        nb = __popc((y.x >> nbsh) & kLow) + __popc((y.y >> nbsh) & kLow) + __popc((y.z >> nbsh) & kLow) +
             __popc((y.w >> nbsh) & kLow);
      } else {
        const uint32_t s0 = src / (uint32_t)sizeof(E);
        E* oe = reinterpret_cast<E*>(outb);
        const uint64_t e0 = blo / sizeof(E), e1 = bhi / sizeof(E);
        for (uint64_t e = e0; e < e1; ++e) {
          const E v = s_stage[s0 + (uint32_t)(e - e0)];
          oe[e] = v;
          nb += ((uint32_t)v >> nbsh) & 1u;
        }
      }
      const uint32_t sub = (uint32_t)(cb / kTileB - db / kTileB);  // 0 or 1
      cnt4[(bb ? 2 : 0) + sub] += nb;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint32_t v = cnt4[r];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0 && v) atomicAdd(&s_nc[r], v);
    }
    __syncthreads();
    if (tid < 4) {
      const uint32_t c = s_nc[tid];
      const uint64_t d = (tid < 2) ? d0 : d1;
      if (c && d < n_next)
        atomicAdd((unsigned long long*)&a.cnt_next[(d >> TL::TSHIFT) + (tid & 1u)], (unsigned long long)c);
    }
    return;
  }
  {
    uint64_t curN = ~0ull;
    uint32_t sa = 0, zs = 0, R1a = 0;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
      if (q0 < cnt) {
        uint32_t r1 = r1loc(s_words, s_wpre, q0);
        const uint32_t nv = min((uint32_t)EV, cnt - q0);
        const uint64_t lo = ((uint64_t)vx[k].y << 32) | vx[k].x, hi = ((uint64_t)vx[k].w << 32) | vx[k].z;
        const uint32_t cf = vec_elem<E>(vx[k], 0), cl = elem128<E>(lo, hi, nv - 1);
        const uint64_t Nf = l ? ((uint64_t)cf >> (L - l)) & pmask : 0ull;
        const uint64_t Nl = l ? ((uint64_t)cl >> (L - l)) & pmask : 0ull;
        if (Nf == Nl) {
          // the whole vector lies in one node
          if (Nf != curN) enter_node(a.ntb[Nf], q0, t0, cnt, G0, G1, s_words, s_wpre, s_seg, &s_nseg, sa, zs, R1a), curN = Nf;
          const uint32_t b0 = R1a, b1 = sa + zs - R1a;  // slot = b0 + rank0 or b1 + rank1 (tile-local)
#pragma unroll
          for (int e = 0; e < EV; ++e) {
            if ((uint32_t)e < nv) {
              const uint32_t code = vec_elem<E>(vx[k], e);
              const uint32_t b = (code >> bsh) & 1u;
              const uint32_t q = q0 + e;
              const uint32_t slot = b ? b1 + r1 : b0 + (q - r1);
              s_stage[min(slot, (uint32_t)T - 1u)] = (E)code;
              r1 += b;
            }
          }
        } else {
          for (uint32_t e = 0; e < nv; ++e) {
            const uint32_t code = elem128<E>(lo, hi, e);
            const uint32_t b = (code >> bsh) & 1u;
            const uint32_t q = q0 + e;
            const uint64_t N = l ? ((uint64_t)code >> (L - l)) & pmask : 0ull;
            if (N != curN) enter_node(a.ntb[N], q, t0, cnt, G0, G1, s_words, s_wpre, s_seg, &s_nseg, sa, zs, R1a), curN = N;
            const uint32_t slot = b ? sa + zs + (r1 - R1a) : sa + ((q - r1) - (sa - R1a));
            s_stage[min(slot, (uint32_t)T - 1u)] = (E)code;
            r1 += b;
          }
        }
      }
    }
  }
  __syncthreads();
  const uint32_t nseg = s_nseg;
  uint64_t cur_tile = ~0ull;
  uint32_t cur_c = 0;
  char* outb = reinterpret_cast<char*>(a.out);

  if (nseg <= (uint32_t)kSegMax) {
    // 4b. runs (segment, bit) -> their 16-byte destination chunks, prefix over runs
    {
      const uint32_t r = tid;
      uint32_t nch = 0;
      if (r < 2 * nseg) {
        const Seg g = s_seg[r >> 1];
        const uint32_t bb = r & 1u;
        const uint64_t d = bb ? g.d1 : g.d0;
        const uint32_t len = d < n_next ? (uint32_t)min<uint64_t>(bb ? g.z - g.a - g.zs : g.zs, n_next - d) : 0u;
        if (len) nch = (uint32_t)(((d + len - 1) * sizeof(E) >> 4) - ((d * sizeof(E)) >> 4) + 1);
      }
      uint32_t total;
      const uint32_t ex = block_excl_scan_u32(nch, s_w, total);
      if (r < 2 * nseg) s_cp[r] = ex;
      if (tid == 0) s_cp[2 * nseg] = total;
    }
    __syncthreads();
    const uint32_t nrun = 2 * nseg;
    const uint32_t C = s_cp[nrun];
    const uint32_t* st32 = reinterpret_cast<const uint32_t*>(s_stage);
    // 4c. write-out: one 16-byte destination chunk per lane
    for (uint32_t c0 = 0; c0 < C; c0 += kBT) {
      const uint32_t c = c0 + tid;
      const bool active = c < C;
      uint32_t nb1 = 0;
      uint64_t chunk = 0;
      if (active) {
        uint32_t lo = 0, hi = nrun - 1;  // largest run with cp <= c
        while (lo < hi) {
          const uint32_t mid = (lo + hi + 1) >> 1;
          if (s_cp[mid] <= c) lo = mid;
          else hi = mid - 1;
        }
        const Seg g = s_seg[lo >> 1];
        const uint32_t bb = lo & 1u;
        const uint64_t d = bb ? g.d1 : g.d0;
        const uint32_t len = (uint32_t)min<uint64_t>(bb ? g.z - g.a - g.zs : g.zs, n_next - d);
        const uint32_t slot0 = bb ? g.a + g.zs : g.a;
        const uint64_t db = d * sizeof(E), de = (d + len) * sizeof(E);
        chunk = (db >> 4) + (c - s_cp[lo]);
        const uint64_t cb = chunk << 4;
        const uint64_t blo = max(db, cb), bhi = min(de, cb + 16);
        const uint32_t src = slot0 * (uint32_t)sizeof(E) + (uint32_t)(blo - db);  // LDS byte of blo
        if (blo == cb && bhi == cb + 16) {
          const uint32_t dw = src >> 2, sh = src & 3u;
          const uint32_t x0 = st32[dw], x1 = st32[dw + 1], x2 = st32[dw + 2], x3 = st32[dw + 3],
                         x4 = st32[dw + 4];
          uint4 y;
          y.x = __builtin_amdgcn_alignbyte(x1, x0, sh);
          y.y = __builtin_amdgcn_alignbyte(x2, x1, sh);
          y.z = __builtin_amdgcn_alignbyte(x3, x2, sh);
          y.w = __builtin_amdgcn_alignbyte(x4, x3, sh);
          *reinterpret_cast<uint4*>(outb + cb) = y;
#pragma unroll
          for (int e = 0; e < EV; ++e) nb1 += (vec_elem<E>(y, e) >> nbsh) & 1u;
        } else {
          const uint32_t s0 = src / (uint32_t)sizeof(E);
          E* oe = reinterpret_cast<E*>(outb);
          const uint64_t e0 = blo / sizeof(E), e1 = bhi / sizeof(E);
          for (uint64_t e = e0; e < e1; ++e) {
            const E v = s_stage[s0 + (uint32_t)(e - e0)];
            oe[e] = v;
            nb1 += ((uint32_t)v >> nbsh) & 1u;
          }
        }
      }
      const uint64_t dt = (chunk << 4) / ((uint64_t)T * sizeof(E));
      count_next(__ballot(active), dt, 0u, lane, cur_tile, cur_c, a.cnt_next, nb1);
    }
  } else {
    // 4b'. many small nodes in this tile: element stores in slot order, destination per slot
    const uint32_t wv = tid >> 6;
    constexpr uint32_t kPerWave = T / (kBT / 64);
    uint64_t curN = ~0ull, D0 = 0, D1 = 0;
    uint32_t sa = 0, zs = 0;
    for (uint32_t base = wv * kPerWave; base < (wv + 1) * kPerWave; base += 64) {
      if (base >= cnt) break;
      const uint32_t j = base + lane;
      bool cont = false;
      uint64_t dest = 0;
      uint32_t nbit = 0;
      if (j < cnt) {
        const uint32_t code = (uint32_t)s_stage[j];
        const uint64_t N = l ? ((uint64_t)code >> (L - l)) & pmask : 0ull;
        if (N != curN) {
          const NodeB nb = a.ntb[N];
          sa = (uint32_t)(nb.start > t0 ? min(nb.start - t0, (uint64_t)cnt) : 0ull);
          const uint32_t sz = (uint32_t)(nb.end > t0 ? min(nb.end - t0, (uint64_t)cnt) : 0ull);
          const uint32_t R1a = r1loc(s_words, s_wpre, sa);
          zs = (sz - r1loc(s_words, s_wpre, sz)) - (sa - R1a);
          D0 = nb.off0 + G0 + (sa - R1a);
          D1 = nb.off1 + G1 + R1a;
          curN = N;
        }
        dest = (j < sa + zs) ? D0 + (j - sa) : D1 + (j - sa - zs);
        cont = dest < n_next;
        if (cont) {
          reinterpret_cast<E*>(outb)[dest] = (E)code;
          nbit = (code >> nbsh) & 1u;
        }
      }
      count_next(__ballot(cont), dest >> TL::TSHIFT, nbit, lane, cur_tile, cur_c, a.cnt_next, 0u);
    }
  }
  if (lane == 0 && cur_c) atomicAdd((unsigned long long*)&a.cnt_next[cur_tile], (unsigned long long)cur_c);
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

template <typename E>
hipError_t launch_hist(const void* d_sym, uint64_t n, uint32_t sigma, uint32_t L, uint32_t pow2, uint64_t* hist,
                       uint64_t* cnt0, uint32_t* err, hipStream_t st) {
  using TL = Tile<E>;
  const uint64_t ntiles = ceil_div(n, TL::T);
  if (ntiles == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>(ntiles, 2048);
  const uint32_t aligned = ((uintptr_t)d_sym & 15u) == 0;
  if (sigma <= 16384) {
    const uint32_t nrep = std::max<uint32_t>(1u, std::min<uint32_t>(32u, 16383u / (sigma + 1)));
    const size_t lds = (size_t)nrep * (sigma + 1) * sizeof(uint32_t);
    hipLaunchKernelGGL((k_hist<E, true>), dim3(grid), dim3(kBT), lds, st, (const E*)d_sym, n, sigma, L, pow2,
                       aligned, nrep, hist, cnt0, err);
  } else {
    const size_t lds = 2ull * kHashSlots * sizeof(uint32_t);
    hipLaunchKernelGGL((k_hist<E, false>), dim3(grid), dim3(kBT), lds, st, (const E*)d_sym, n, sigma, L, pow2,
                       aligned, 1u, hist, cnt0, err);
  }
  return hipGetLastError();
}

template <typename E>
hipError_t launch_level(const LevelArgs& a, uint64_t n, hipStream_t st) {
  using TL = Tile<E>;
  const uint64_t nt = ceil_div(n, TL::T);
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL((k_level<E>), dim3((uint32_t)nt), dim3(kBT), 0, st, a);
  return hipGetLastError();
}

}  // namespace

TreePlan plan_tree(uint64_t n, uint32_t w, uint64_t sigma, uint32_t L, uint32_t l2_bits, uint32_t srate) {
  TreePlan p{};
  p.n = n;
  p.sigma = sigma;
  p.L = L;
  p.w = w;
  p.l2_bits = l2_bits;
  p.srate = srate;
  p.tile = tile_elems(w);
  // capacity: whole tiles plus one L2 block of slack (queries read the whole L2 block at i = n_l),
  // rounded to 128-byte lines so every level starts on a line
  const uint64_t cap_bits = round_up(round_up(std::max<uint64_t>(n, 1), p.tile) + 2048, 1024);
  p.words_per_level = cap_bits / 64;
  p.l1_per_level = round_up(ceil_div(n, kL1Bits) + 1, 16);
  p.l2_per_level = round_up(ceil_div(n, l2_bits) + 1, 64);
  p.smp_per_level = round_up(n / srate + 1, 16);
  p.nheap = L ? ((1ull << L) - 1) : 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  p.off_meta = take(sizeof(LevelMeta) * WT_MAX_LEVELS);
  p.off_cum = take((sigma + 1) * sizeof(uint64_t));
  p.off_nodes = take(std::max<uint64_t>(p.nheap, 1) * sizeof(NodeQ));
  p.off_bits = take((size_t)L * p.words_per_level * sizeof(uint64_t));
  p.off_l1 = take((size_t)L * p.l1_per_level * sizeof(uint64_t));
  p.off_l2 = take((size_t)L * p.l2_per_level * sizeof(uint16_t));
  p.off_smp = take((size_t)L * p.smp_per_level * sizeof(uint64_t));
  p.total = off;
  return p;
}

}  // namespace wt

using namespace wt;

extern "C" wt_status wt_build(const void* d_sym, uint64_t n, uint32_t sym_bytes, uint64_t sigma,
                              const wt_build_opts* opts, wt_stream_t stream, wt_tree** out) {
  clear_error();
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
  uint32_t l2_bits = 512, srate = 4096, flags = 0;
  if (opts) {
    if (opts->l2_bits) l2_bits = opts->l2_bits;
    if (opts->sample_rate) srate = opts->sample_rate;
    flags = opts->flags;
  }
  if (l2_bits != 256 && l2_bits != 512 && l2_bits != 1024 && l2_bits != 2048)
    return fail(WT_ERR_ARG, "wt_build: l2_bits must be 256, 512, 1024 or 2048");
  if (srate < 512 || srate > (1u << 20) || (srate & (srate - 1)))
    return fail(WT_ERR_ARG, "wt_build: sample_rate must be a power of two in [512, 2^20]");

  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  WT_HIP(hipGetDevice(&dev));

  uint32_t L = 0;
  while ((1ull << L) < sigma) ++L;
  const uint32_t pow2 = (sigma & (sigma - 1)) == 0;
  const TreePlan P = plan_tree(n, sym_bytes, sigma, L, l2_bits, srate);

  wt_tree* t = new wt_tree();
  t->n = n;
  t->sigma = sigma;
  t->L = L;
  t->w = sym_bytes;
  t->l2_bits = l2_bits;
  t->srate = srate;
  t->pow2 = pow2;
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
  t->bytes_bits = (size_t)L * P.words_per_level * 8;
  t->bytes_l1 = (size_t)L * P.l1_per_level * 8;
  t->bytes_l2 = (size_t)L * P.l2_per_level * 2;
  t->bytes_smp = (size_t)L * P.smp_per_level * 8;
  t->bytes_nodes = (size_t)std::max<uint64_t>(P.nheap, 1) * sizeof(NodeQ);
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
  const size_t o_seq0 = take(L > 1 ? seq_elems * sym_bytes : 0);
  const size_t o_seq1 = take(L > 2 ? seq_elems * sym_bytes : 0);
  const size_t o_hist = take(hist_n * 8);
  const uint64_t nchunks = ceil_div(ntiles, kChunkTiles);
  const uint64_t cstride = (ntiles + 1) + (nchunks + 1);  // per level: tile counts, then chunk counts
  const size_t o_cnt = take((size_t)std::max<uint32_t>(L, 1) * cstride * 8);
  const size_t o_pre = take((size_t)std::max<uint32_t>(L, 1) * (ntiles + 1) * 8);
  const size_t o_ntb = take(std::max<uint64_t>(P.nheap, 1) * sizeof(NodeB));
  const size_t o_z = take((P.nheap + 1) * 8);
  const size_t o_zs = take((P.nheap + 1) * 8);
  const size_t o_part = take(part_n * 8);
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
  uint32_t* err = (uint32_t*)(sb + o_err);

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
  WT_STEP(hipGetLastError());
  WT_STEP(prof.end());

  WT_STEP(prof.begin("hist", -1));
  if (sym_bytes == 1) WT_STEP(launch_hist<uint8_t>(d_sym, n, (uint32_t)sigma, L, pow2, hist, tcnt, err, st));
  else if (sym_bytes == 2) WT_STEP(launch_hist<uint16_t>(d_sym, n, (uint32_t)sigma, L, pow2, hist, tcnt, err, st));
  else WT_STEP(launch_hist<uint32_t>(d_sym, n, (uint32_t)sigma, L, pow2, hist, tcnt, err, st));
  WT_STEP(prof.end());

  WT_STEP(prof.begin("cum_hist", -1));
  WT_STEP(exclusive_scan_u64(hist, hist_n, t->dev.cum, part, st));
  WT_STEP(prof.end());

  if (L > 0) {
    WT_STEP(prof.begin("nodes", -1));
    const uint32_t nb = (uint32_t)ceil_div(P.nheap, kBT);
    hipLaunchKernelGGL(k_node_walk, dim3(nb), dim3(kBT), 0, st, (uint32_t)sigma, P.nheap,
                       (const uint64_t*)t->dev.cum, ntb, z);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, z + P.nheap, 1ull, 0ull);
    WT_STEP(hipGetLastError());
    WT_STEP(exclusive_scan_u64(z, P.nheap + 1, zs, part, st));
    hipLaunchKernelGGL(k_node_final, dim3(nb), dim3(kBT), 0, st, P.nheap, (const uint64_t*)zs, ntb, t->dev.nodes,
                       t->dev.meta);
    WT_STEP(hipGetLastError());
    WT_STEP(prof.end());
  }

  uint32_t l2shift = 0, sshift = 0;
  while ((1u << l2shift) < l2_bits) ++l2shift;
  while ((1u << sshift) < srate) ++sshift;
  uint32_t tshift = 0;
  while ((1u << tshift) < T) ++tshift;

  for (uint32_t l = 0; l < L; ++l) {
    uint64_t* cnt_l = tcnt + (size_t)l * cstride;
    uint64_t* chunk_l = cnt_l + ntiles + 1;
    uint64_t* pre_l = tpre + (size_t)l * (ntiles + 1);
    WT_STEP(prof.begin("tile_scan", (int)l));
    hipLaunchKernelGGL(k_tile_reduce, dim3((uint32_t)nchunks), dim3(kBT), 0, st, (const LevelMeta*)t->dev.meta, l,
                       tshift, (const uint64_t*)cnt_l, chunk_l);
    hipLaunchKernelGGL(k_tile_scan, dim3((uint32_t)(nchunks + 1)), dim3(kBT), 0, st, t->dev.meta, l, tshift,
                       (const uint64_t*)cnt_l, (const uint64_t*)chunk_l, pre_l, t->dev.L1, t->dev.L2);
    WT_STEP(hipGetLastError());
    WT_STEP(prof.end());
    LevelArgs a{};
    a.in = l == 0 ? d_sym : seq[(l - 1) & 1];
    a.out = (l + 1 < L) ? seq[l & 1] : nullptr;
    a.bits = t->dev.bits;
    a.L1 = t->dev.L1;
    a.L2 = t->dev.L2;
    a.smp = t->dev.smp;
    a.meta = t->dev.meta;
    a.pre = pre_l;
    a.cnt_next = (l + 1 < L) ? tcnt + (size_t)(l + 1) * cstride : nullptr;
    a.ntb = ntb + ((1ull << l) - 1);
    a.l = l;
    a.L = L;
    a.sigma = (uint32_t)sigma;
    a.pow2 = pow2;
    a.l2shift = l2shift;
    a.sshift = sshift;
    a.encode = (l == 0 && !pow2) ? 1u : 0u;
    a.in_vec = (l == 0) ? 0u : 1u;
    a.in_aligned = (l == 0) ? (((uintptr_t)d_sym & 15u) == 0) : 1u;
    WT_STEP(prof.begin("level", (int)l));
    if (sym_bytes == 1) WT_STEP(launch_level<uint8_t>(a, n, st));
    else if (sym_bytes == 2) WT_STEP(launch_level<uint16_t>(a, n, st));
    else WT_STEP(launch_level<uint32_t>(a, n, st));
    WT_STEP(prof.end());
  }

  // read back level sizes and the range flag
  struct Readback {
    LevelMeta meta[WT_MAX_LEVELS];
    uint32_t err;
  };
  Readback rb{};
  if (L) WT_STEP(hipMemcpyAsync(rb.meta, t->dev.meta, sizeof(LevelMeta) * L, hipMemcpyDeviceToHost, st));
  WT_STEP(hipMemcpyAsync(&rb.err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  WT_STEP(hipStreamSynchronize(st));
#undef WT_STEP
  if (rb.err) return bail(fail(WT_ERR_SYMBOL_RANGE, "wt_build: a symbol is >= sigma (%llu)", (unsigned long long)sigma));
  for (uint32_t l = 0; l < L; ++l) t->hmeta[l] = rb.meta[l];
  if (prof.on) prof.collect(t->prof);
  *out = t;
  return WT_OK;
}
