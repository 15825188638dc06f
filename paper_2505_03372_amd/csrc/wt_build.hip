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
  static constexpr int EV = 16 / (int)sizeof(E);  // elements per 16-byte vector
  static constexpr int NCH = 4;                   // vectors per thread
  static constexpr int T = kBT * NCH * EV;        // elements per tile
  static constexpr int W = T / 64;                // bit words per tile
  static constexpr int G = 64 / EV;               // lanes whose vectors form one word
  static constexpr int TSHIFT = sizeof(E) == 1 ? 14 : (sizeof(E) == 2 ? 13 : 12);
  static_assert((1 << TSHIFT) == T, "tile");
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

// Persistent grid over whole tiles. Small alphabets count into LDS replicas (one per group of
// threads, assigned round-robin); large alphabets use an LDS cache of claimed symbols with global
// atomics for the rest. Also records, per level-0 tile, the number of ones (code bit L-1).
template <typename E, bool kSmall>
__global__ __launch_bounds__(kBT) void k_hist(const E* __restrict__ sym, uint64_t n, uint32_t sigma, uint32_t L,
                                              uint32_t pow2, uint32_t aligned, uint32_t nrep,
                                              uint64_t* __restrict__ hist, uint64_t* __restrict__ tile_cnt0,
                                              uint32_t* __restrict__ err) {
  using TL = Tile<E>;
  extern __shared__ uint32_t s_h[];
  __shared__ uint32_t s_w[kBT / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t hsize = kSmall ? nrep * sigma : 2u * kHashSlots;
  for (uint32_t i = tid; i < hsize; i += kBT) s_h[i] = 0;
  __syncthreads();
  uint32_t* my_h = s_h + (kSmall ? (tid % nrep) * sigma : 0u);
  uint32_t* s_keys = s_h;
  uint32_t* s_cnts = s_h + kHashSlots;
  const uint64_t ntiles = (n + TL::T - 1) >> TL::TSHIFT;
  uint32_t bad = 0;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t t0 = t << TL::TSHIFT;
    const uint32_t cnt = (uint32_t)min<uint64_t>(TL::T, n - t0);
    uint32_t ones = 0;
#pragma unroll
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
      for (uint32_t r = 0; r < nrep; ++r) c += s_h[r * sigma + s];
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

// Single block: exclusive prefix of the ones per tile of level l (tile size 2^tshift), the level's
// total ones, and the sentinel L1/L2 entries that make rank defined at i = n_l.
__global__ __launch_bounds__(1024) void k_tile_scan(LevelMeta* __restrict__ meta, uint32_t l, uint32_t tshift,
                                                    const uint64_t* __restrict__ cnt, uint64_t* __restrict__ pre,
                                                    uint64_t* __restrict__ L1, uint16_t* __restrict__ L2,
                                                    uint32_t l2shift) {
  __shared__ uint64_t s_w[16];
  const LevelMeta m = meta[l];
  const uint64_t nl = m.n;
  const uint64_t nt = (nl + (1ull << tshift) - 1) >> tshift;
  const uint64_t per = (nt + 1023) / 1024;
  const uint64_t i0 = (uint64_t)threadIdx.x * per;
  const uint64_t i1 = min(i0 + per, nt);
  uint64_t s = 0;
  for (uint64_t i = i0; i < i1; ++i) s += cnt[i];
  uint64_t total;
  uint64_t run = block_excl_scan_u64(s, s_w, total);
  for (uint64_t i = i0; i < i1; ++i) {
    pre[i] = run;
    run += cnt[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    pre[nt] = total;
    meta[l].ones = total;
    L1[m.l1 + ((nl + kL1Bits - 1) >> kL1Shift)] = total;
    const uint64_t j = (nl + (1ull << l2shift) - 1) >> l2shift;
    const uint64_t blk = (j << l2shift) >> kL1Shift;
    const uint64_t l1val = ((blk << kL1Shift) >= nl) ? total : pre[blk << (kL1Shift - tshift)];
    L2[m.l2 + j] = (uint16_t)(total - l1val);
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
  const uint64_t* pre;  // exclusive ones before each tile of this level
  uint64_t* cnt_next;   // ones per tile of level l + 1 (accumulated)
  const NodeB* ntb;     // node table of this level, indexed by code prefix
  uint32_t l, L, sigma, pow2;
  uint32_t l2shift, sshift;
  uint32_t encode;  // level 0 of a reduced alphabet: turn symbols into codes
  uint32_t in_vec;      // the input may be read with 16-byte vectors everywhere (padded and aligned)
  uint32_t in_aligned;  // the input base is 16-byte aligned (vectors only inside the sequence)
};

__device__ __forceinline__ uint32_t r1loc(const uint64_t* __restrict__ sw, const uint32_t* __restrict__ sp,
                                          uint32_t x) {
  const uint32_t wi = x >> 6, bi = x & 63u;
  return sp[wi] + popc64(sw[wi] & ((1ull << bi) - 1ull));
}

// One block per tile of T elements of level l:
//  1. coalesced 16-byte loads (4 per thread); element q of the tile sits in vector q / EV;
//  2. bit words: each vector gives EV bits, G neighbouring lanes OR them into one 64-bit word;
//  3. block scan of the word popcounts -> tile-local rank1 at every word;
//  4. bit words, L2 entries (ones since the enclosing L1 block start), the L1 entry when the tile
//     starts an L1 block, select samples where the global one/zero count crosses a multiple of s;
//  5. stable partition staged in LDS: within the tile every node segment is reordered zeros-first
//     (slot = segment start + tile-local rank of the element among its bit inside the segment), so
//     the slot range of a segment equals its position range and slots are ordered by destination;
//  6. write-out in slot order, 64 consecutive slots per wave instruction (contiguous destinations
//     inside each run), and per-destination-tile counts of the next level's ones.
template <typename E>
__global__ __launch_bounds__(kBT) void k_level(LevelArgs a) {
  using TL = Tile<E>;
  constexpr int T = TL::T, W = TL::W, EV = TL::EV, G = TL::G, NCH = TL::NCH;
  __shared__ uint64_t s_words[W + 1];
  __shared__ uint32_t s_wpre[W + 1];
  __shared__ E s_stage[T];
  __shared__ uint32_t s_w[kBT / 64];

  const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const uint32_t l = a.l, L = a.L;
  const LevelMeta m = a.meta[l];
  const uint64_t nl = m.n;
  const uint64_t t = blockIdx.x;
  const uint64_t t0 = t << TL::TSHIFT;
  if (t0 >= nl) return;
  const uint32_t cnt = (uint32_t)min<uint64_t>((uint64_t)T, nl - t0);
  const uint32_t bsh = L - 1 - l;
  const uint64_t pmask = (1ull << l) - 1ull;

  // 1. load
  E v[NCH][EV];
  const E* in = reinterpret_cast<const E*>(a.in) + t0;
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
    load16<E>(in, q0, cnt, a.in_vec || (a.in_aligned && q0 + EV <= cnt), v[k]);
  }
  if (a.encode) {
#pragma unroll
    for (int k = 0; k < NCH; ++k)
#pragma unroll
      for (int e = 0; e < EV; ++e) {
        uint32_t s = (uint32_t)v[k][e];
        if (s >= a.sigma) s = 0;  // out-of-range input: the build reports an error; keep indices valid
        uint32_t len;
        v[k][e] = (E)encode_sym(s, a.sigma, L, a.pow2, &len);
      }
  }

  // 2. bit words
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
    uint32_t mask = 0;
#pragma unroll
    for (int e = 0; e < EV; ++e)
      if (q0 + e < cnt) mask |= (((uint32_t)v[k][e] >> bsh) & 1u) << e;
    uint64_t word = (uint64_t)mask << ((tid % G) * EV);
#pragma unroll
    for (int off = 1; off < G; off <<= 1) word |= __shfl_xor(word, off, 64);
    if (tid % G == 0) s_words[k * (kBT / G) + tid / G] = word;
  }
  if (tid == 0) s_words[W] = 0;
  __syncthreads();

  // 3. tile-local rank1 at every word
  {
    const uint32_t pc = (tid < (uint32_t)W) ? popc64(s_words[tid]) : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan_u32(pc, s_w, tot);
    if (tid < (uint32_t)W) s_wpre[tid] = ex;
    if (tid == 0) s_wpre[W] = tot;
  }
  __syncthreads();

  // 4. bits and directory
  const uint64_t G1 = a.pre[t];  // ones of the level before the tile
  const uint64_t G0 = t0 - G1;   // zeros of the level before the tile
  if (tid < (uint32_t)W) {
    const uint64_t word = s_words[tid];
    const uint64_t gw = ((uint64_t)t * W) + tid;
    a.bits[m.bits + gw] = word;
    const uint32_t q = tid * 64u;
    if (q < cnt) {
      const uint64_t ones_before = G1 + s_wpre[tid];
      const uint32_t l2w_shift = a.l2shift - 6;
      if ((gw & ((1ull << l2w_shift) - 1)) == 0) {
        const uint64_t l1val = a.pre[t & ~(uint64_t)((kL1Bits / T) - 1)];
        a.L2[m.l2 + (gw >> l2w_shift)] = (uint16_t)(ones_before - l1val);
      }
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
  if (tid == 0 && (t0 & (kL1Bits - 1)) == 0) a.L1[m.l1 + (t0 >> kL1Shift)] = G1;
  if (l + 1 >= L) return;

  // 5. stable partition of each node segment of the tile into LDS
  {
    uint64_t curN = ~0ull;
    uint32_t base0 = 0, base1 = 0;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
      uint32_t r1 = r1loc(s_words, s_wpre, min(q0, cnt));
#pragma unroll
      for (int e = 0; e < EV; ++e) {
        const uint32_t q = q0 + e;
        if (q >= cnt) continue;
        const uint32_t code = (uint32_t)v[k][e];
        const uint32_t b = (code >> bsh) & 1u;
        const uint64_t N = l ? ((uint64_t)code >> (L - l)) & pmask : 0ull;
        if (N != curN) {
          const NodeB nb = a.ntb[N];
          const uint64_t sa = nb.start > t0 ? min(nb.start - t0, (uint64_t)cnt) : 0ull;
          const uint64_t sz = nb.end > t0 ? min(nb.end - t0, (uint64_t)cnt) : 0ull;
          const uint32_t R1a = r1loc(s_words, s_wpre, (uint32_t)sa);
          const uint32_t R1z = r1loc(s_words, s_wpre, (uint32_t)sz);
          const uint32_t R0a = (uint32_t)sa - R1a;
          const uint32_t zs = ((uint32_t)sz - R1z) - R0a;
          base0 = R1a;
          base1 = zs + R0a;
          curN = N;
        }
        uint32_t slot = b ? base1 + r1 : base0 + (q - r1);
        slot = min(slot, (uint32_t)T - 1u);
        s_stage[slot] = (E)code;
        r1 += b;
      }
    }
  }
  __syncthreads();

  // 6. write-out in slot order
  {
    const uint64_t n_next = a.meta[l + 1].n;
    const uint32_t nbsh = L - 2 - l;
    E* out = reinterpret_cast<E*>(a.out);
    uint64_t curN = ~0ull, D0 = 0, D1 = 0;
    uint64_t cur_tile = ~0ull;
    uint32_t cur_c = 0;
    constexpr uint32_t kPerWave = T / (kBT / 64);
    for (uint32_t j0 = wv * kPerWave; j0 < (wv + 1) * kPerWave; j0 += 64) {
      if (j0 >= cnt) break;
      const uint32_t j = j0 + lane;
      bool cont = false;
      uint64_t dest = 0;
      uint32_t nbit = 0;
      if (j < cnt) {
        const uint32_t code = (uint32_t)s_stage[j];
        const uint32_t b = (code >> bsh) & 1u;
        const uint64_t N = l ? ((uint64_t)code >> (L - l)) & pmask : 0ull;
        if (N != curN) {
          const NodeB nb = a.ntb[N];
          const uint64_t sa = nb.start > t0 ? min(nb.start - t0, (uint64_t)cnt) : 0ull;
          const uint64_t sz = nb.end > t0 ? min(nb.end - t0, (uint64_t)cnt) : 0ull;
          const uint32_t R1a = r1loc(s_words, s_wpre, (uint32_t)sa);
          const uint32_t R1z = r1loc(s_words, s_wpre, (uint32_t)sz);
          const uint32_t R0a = (uint32_t)sa - R1a;
          const uint32_t zs = ((uint32_t)sz - R1z) - R0a;
          D0 = nb.off0 + G0 - R1a;
          D1 = nb.off1 + G1 - (zs + R0a);
          curN = N;
        }
        dest = (uint64_t)j + (b ? D1 : D0);
        cont = dest < n_next;
        if (cont) {
          out[dest] = (E)code;
          nbit = (code >> nbsh) & 1u;
        }
      }
      // ones of the next level per destination tile; destinations increase with the slot
      const uint64_t dt = dest >> TL::TSHIFT;
      uint64_t pend = __ballot(cont);
      while (pend) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const uint64_t ldt = __shfl(dt, leader, 64);
        const bool same = cont && dt == ldt;
        const uint64_t sm = __ballot(same);
        const uint32_t c1 = (uint32_t)__popcll(__ballot(same && nbit));
        if (ldt == cur_tile) {
          cur_c += c1;
        } else {
          if (cur_tile != ~0ull && cur_c && lane == 0)
            atomicAdd((unsigned long long*)&a.cnt_next[cur_tile], (unsigned long long)cur_c);
          cur_tile = ldt;
          cur_c = c1;
        }
        pend &= ~sm;
      }
    }
    if (cur_tile != ~0ull && cur_c && lane == 0)
      atomicAdd((unsigned long long*)&a.cnt_next[cur_tile], (unsigned long long)cur_c);
  }
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
    const uint32_t nrep = std::max<uint32_t>(1u, std::min<uint32_t>(32u, 16384u / sigma));
    const size_t lds = (size_t)nrep * sigma * sizeof(uint32_t);
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
  const size_t o_cnt = take((size_t)std::max<uint32_t>(L, 1) * (ntiles + 1) * 8);
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
  hipLaunchKernelGGL(k_fill_u64, dim3(256), dim3(kBT), 0, st, tcnt, (uint64_t)std::max<uint32_t>(L, 1) * (ntiles + 1),
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
    uint64_t* cnt_l = tcnt + (size_t)l * (ntiles + 1);
    uint64_t* pre_l = tpre + (size_t)l * (ntiles + 1);
    WT_STEP(prof.begin("tile_scan", (int)l));
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, t->dev.meta, l, tshift, (const uint64_t*)cnt_l, pre_l,
                       t->dev.L1, t->dev.L2, l2shift);
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
    a.cnt_next = (l + 1 < L) ? tcnt + (size_t)(l + 1) * (ntiles + 1) : nullptr;
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
