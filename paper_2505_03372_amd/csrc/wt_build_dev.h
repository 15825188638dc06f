// Device code of the level-wise construction (Section 5.1, Algorithm 4), shared by the single-tree
// build and the batched forest build: every phase is a device body over a block index, called by a
// kernel of one tree (block index = blockIdx.x) or by a forest kernel that maps its blocks to trees.
#pragma once

#include <hip/hip_runtime.h>

#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

// Device memory. The compiler infers it for pointers passed as kernel arguments, not for pointers
// read from device memory (per-tree state of a forest build), whose accesses would otherwise all be
// flat accesses: the level pass and the histogram take their pointers in this address space.
#define WT_GLOBAL __attribute__((address_space(1)))

template <typename T, typename U>
__device__ __forceinline__ T* pcast(U* p) {
  return (T*)p;
}
template <typename T, typename U>
__device__ __forceinline__ WT_GLOBAL T* pcast(WT_GLOBAL U* p) {
  return (WT_GLOBAL T*)p;
}

// 16-byte and struct accesses that keep the pointer's address space (HIP's uint4 and the tree
// structs are classes whose copies take generic references).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename P>
__device__ __forceinline__ void st16(P p, const uint4& y) {
  u32x4 x;
  __builtin_memcpy(&x, &y, 16);
  *pcast<u32x4>(p) = x;
}

template <typename P>
__device__ __forceinline__ LevelMeta ld_meta(P p) {
  LevelMeta m;
  m.n = p->n;
  m.ones = p->ones;
  m.bits = p->bits;
  m.l1 = p->l1;
  m.l2 = p->l2;
  m.smp = p->smp;
  m.smp_cap = p->smp_cap;
  m.pad = p->pad;
  return m;
}

template <typename P>
__device__ __forceinline__ NodeB ld_node(P p) {
  NodeB b;
  b.start = p->start;
  b.end = p->end;
  b.off0 = p->off0;
  b.off1 = p->off1;
  return b;
}

template <typename P>
__device__ __forceinline__ void atomic_add_u64(P p, uint64_t v) {
  (void)__hip_atomic_fetch_add(pcast<unsigned long long>(p), (unsigned long long)v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

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

__device__ __forceinline__ void scan_reduce_body(const uint64_t* __restrict__ in, uint64_t n,
                                                 uint64_t* __restrict__ part, uint64_t bid) {
  __shared__ uint64_t s_w[kBT / 64];
  // only the chunk's sum is needed, so the loads go in the coalesced order
  const uint64_t b0 = bid * kScanChunk + threadIdx.x;
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const uint64_t j = b0 + (uint64_t)i * kBT;
    if (j < n) s += in[j];
  }
  uint64_t tot;
  block_excl_scan_u64(s, s_w, tot);
  if (threadIdx.x == 0) part[bid] = tot;
}

// Single block: exclusive scan of np partial sums in place.
__device__ __forceinline__ void scan_partials_body(uint64_t* __restrict__ part, uint64_t np) {
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

// The chunk goes through LDS (each thread's run of kScanPer padded by one slot against bank
// conflicts), so the global loads and stores are coalesced while every thread scans its own run.
__device__ __forceinline__ void scan_down_body(const uint64_t* __restrict__ in, uint64_t n,
                                               const uint64_t* __restrict__ part, uint64_t* __restrict__ out,
                                               uint64_t bid) {
  constexpr uint32_t R = kScanPer + 1;
  __shared__ uint64_t s_w[kBT / 64];
  __shared__ uint64_t s_v[kBT * R];
  const uint32_t tid = threadIdx.x;
  const uint64_t c0 = bid * kScanChunk;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const uint32_t j = (uint32_t)i * kBT + tid;
    s_v[(j / kScanPer) * R + j % kScanPer] = c0 + j < n ? in[c0 + j] : 0ull;
  }
  __syncthreads();
  uint64_t v[kScanPer];
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = s_v[tid * R + i];
    s += v[i];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan_u64(s, s_w, tot) + part[bid];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    s_v[tid * R + i] = run;
    run += v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const uint32_t j = (uint32_t)i * kBT + tid;
    if (c0 + j < n) out[c0 + j] = s_v[(j / kScanPer) * R + j % kScanPer];
  }
}

// ---------------------------------------------------------------- fill

__device__ __forceinline__ void fill_body(uint64_t* __restrict__ p, uint64_t n, uint64_t v, uint64_t bid,
                                          uint64_t nblk) {
  for (uint64_t i = bid * blockDim.x + threadIdx.x; i < n; i += nblk * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------- loads

// Loads elements [q0, q0 + EV) of a tile into v; elements at or beyond cnt read as 0. `vec` says the
// 16 bytes starting at q0 may be read as one vector (aligned and inside the buffer). A vector that
// lies inside the tile but starts off a 16-byte boundary is read as the two aligned 16-byte blocks it
// spans (both hold bytes of the sequence, so neither leaves its pages) and funnel-shifted. `base`
// must be the same for every lane of the wave (tile offsets q0 * sizeof(E) are multiples of 16, so the
// misalignment is then wave-uniform and picks its shift with scalar branches).
// The 16 bytes starting m bytes (0 < m < 16, wave-uniform) into the aligned pair of blocks x0, x1.
__device__ __forceinline__ void funnel16(const u32x4& x0, const u32x4& x1, uint32_t m, uint32_t (&y)[4]) {
  const uint32_t d[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
  const uint32_t mu = (uint32_t)__builtin_amdgcn_readfirstlane((int)m);
  const uint32_t sh = mu & 3u;
  switch (mu >> 2) {
#define WT_FUNNEL(K)                                                                     \
  case K:                                                                                \
    for (int i = 0; i < 4; ++i) y[i] = __builtin_amdgcn_alignbyte(d[i + K + 1], d[i + K], sh); \
    break;
    WT_FUNNEL(0)
    WT_FUNNEL(1)
    WT_FUNNEL(2)
    default:
      for (int i = 0; i < 4; ++i) y[i] = __builtin_amdgcn_alignbyte(d[i + 4], d[i + 3], sh);
      break;
#undef WT_FUNNEL
  }
}

template <typename E, typename P>
__device__ __forceinline__ void load16(P base, uint32_t q0, uint32_t cnt, bool vec, E (&v)[16 / sizeof(E)]) {
  constexpr int EV = 16 / (int)sizeof(E);
  if (vec) {
    const u32x4 x = *pcast<const u32x4>(base + q0);
    __builtin_memcpy(v, &x, 16);
    if (q0 + EV > cnt) {
#pragma unroll
      for (int e = 0; e < EV; ++e)
        if (q0 + e >= cnt) v[e] = 0;
    }
    return;
  }
  const uint32_t m = (uint32_t)((uintptr_t)(base + q0) & 15u);
  if (q0 + EV <= cnt && m != 0) {
    const auto blk = pcast<const u32x4>(pcast<const char>(base + q0) - m);
    const u32x4 x0 = blk[0], x1 = blk[1];
    uint32_t y[4];
    funnel16(x0, x1, m, y);
    __builtin_memcpy(v, y, 16);
    return;
  }
#pragma unroll
  for (int e = 0; e < EV; ++e) v[e] = (q0 + e < cnt) ? base[q0 + e] : (E)0;
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

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t udot2_u16(uint32_t a, uint32_t w, uint32_t c) {
  u16x2 x, y;
  __builtin_memcpy(&x, &a, 4);
  __builtin_memcpy(&y, &w, 4);
  return __builtin_amdgcn_udot2(x, y, c, false);
}

// Bit `bsh` of every element of a 16-byte vector of E, as a mask (element e -> bit e). For bytes
// and halfwords the selected bits, still at offset bsh inside their lanes, are weighted by powers of
// two in a dot product, which sums to the mask shifted left by bsh.
template <typename E>
__device__ __forceinline__ uint32_t vec_bits(const uint4& x, uint32_t bsh) {
  if constexpr (sizeof(E) == 1) {
    const uint32_t M = 0x01010101u << bsh;
    const uint32_t lo = __builtin_amdgcn_udot4(x.x & M, 0x08040201u,
                                               __builtin_amdgcn_udot4(x.y & M, 0x80402010u, 0u, false), false);
    const uint32_t hi = __builtin_amdgcn_udot4(x.z & M, 0x08040201u,
                                               __builtin_amdgcn_udot4(x.w & M, 0x80402010u, 0u, false), false);
    return ((hi << 8) | lo) >> bsh;
  } else if constexpr (sizeof(E) == 2) {
    const uint32_t M = 0x00010001u << bsh;
    uint32_t d = udot2_u16(x.w & M, 0x00800040u, 0u);
    d = udot2_u16(x.z & M, 0x00200010u, d);
    d = udot2_u16(x.y & M, 0x00080004u, d);
    d = udot2_u16(x.x & M, 0x00020001u, d);
    return d >> bsh;
  } else {
    return ((x.x >> bsh) & 1u) | (((x.y >> bsh) & 1u) << 1) | (((x.z >> bsh) & 1u) << 2) | (((x.w >> bsh) & 1u) << 3);
  }
}

// Number of elements of a 16-byte vector of E whose bit `bsh` is set.
template <typename E>
__device__ __forceinline__ uint32_t vec_count_bit(const uint4& x, uint32_t bsh) {
  if constexpr (sizeof(E) == 1) {
    const uint32_t M = 0x01010101u << bsh;
    uint32_t d = __builtin_amdgcn_udot4(x.x & M, 0x01010101u, 0u, false);
    d = __builtin_amdgcn_udot4(x.y & M, 0x01010101u, d, false);
    d = __builtin_amdgcn_udot4(x.z & M, 0x01010101u, d, false);
    d = __builtin_amdgcn_udot4(x.w & M, 0x01010101u, d, false);
    return d >> bsh;
  } else if constexpr (sizeof(E) == 2) {
    const uint32_t M = 0x00010001u << bsh;
    uint32_t d = udot2_u16(x.x & M, 0x00010001u, 0u);
    d = udot2_u16(x.y & M, 0x00010001u, d);
    d = udot2_u16(x.z & M, 0x00010001u, d);
    d = udot2_u16(x.w & M, 0x00010001u, d);
    return d >> bsh;
  } else {
    return ((x.x >> bsh) & 1u) + ((x.y >> bsh) & 1u) + ((x.z >> bsh) & 1u) + ((x.w >> bsh) & 1u);
  }
}

// ---------------------------------------------------------------- histogram (Section 5.1.1)

// Ones per tile are accumulated per chunk of kChunkTiles tiles as well, so a level's tile prefix
// needs one launch: block b adds the chunk sums before it to the scan of its own chunk.
constexpr int kChunkShift = 10;
constexpr uint64_t kChunkTiles = 1ull << kChunkShift;

// Histogram blocks: kHT threads, a contiguous range of tiles each (kHG tiles in flight, one per
// group of kBT threads). Alphabets up to kHDenseMax are counted densely in LDS: kHSmallWords
// counters (replicated for small alphabets, one replica per group of lanes) or, in the large-LDS
// variant, windows of kHBigWords symbols (two passes over the block's tiles for 2^16 symbols).
// Each block adds its nonzero counts to the global histogram once, so a block's range is made long
// (hundreds of thousands of symbols) to amortise that flush.
constexpr int kHT = 1024;
constexpr int kHG = kHT / kBT;
constexpr uint32_t kHSmallWords = 8192;   // 32 KB
constexpr uint32_t kHBigWords = 32768;    // 128 KB
constexpr uint32_t kHDenseMax = 65536;
constexpr uint32_t kHMaxRep = 32;

// Tiles per dense-histogram block: at least kHMinTiles, about kHTargetBlocks blocks for a long
// sequence (several blocks per compute unit).
constexpr uint64_t kHMinTiles = 8;
constexpr uint64_t kHTargetBlocks = 1024;
__host__ __device__ inline uint64_t hist_tiles_per_block(uint64_t total_tiles) {
  const uint64_t t = (total_tiles + kHTargetBlocks - 1) / kHTargetBlocks;
  return t > kHMinTiles ? t : kHMinTiles;
}
__host__ __device__ inline uint64_t hist_dense_blocks(uint64_t ntiles, uint64_t tpb) {
  return (ntiles + tpb - 1) / tpb;
}

// Alphabets above kHDenseMax: an LDS cache of claimed symbols (open addressing, no eviction) with
// global atomics for the symbols that find no slot; kBT threads, blocks strided over the tiles.
template <typename E, typename PS, typename PH, typename PE>
__device__ __forceinline__ void hist_hash_body(PS sym, uint64_t n, uint32_t sigma, uint32_t L, uint32_t aligned,
                                               PH hist, PH tile_cnt0, PE err, uint64_t bid, uint64_t nblk) {
  using TL = Tile<E>;
  __shared__ uint32_t s_keys[kHashSlots];
  __shared__ uint32_t s_cnts[kHashSlots];
  __shared__ uint32_t s_w[kBT / 64];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < (uint32_t)kHashSlots; i += kBT) s_keys[i] = 0, s_cnts[i] = 0;
  __syncthreads();
  const uint64_t ntiles = (n + TL::T - 1) >> TL::TSHIFT;
  uint32_t bad = 0;
  for (uint64_t t = bid; t < ntiles; t += nblk) {
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
          // the level-0 bit of a symbol's code is the symbol's own bit L - 1 (reduced codes keep
          // the first 2^(L-1) symbols in the left subtree)
          ones += (s >> (L - 1)) & 1u;
          const uint32_t h = (s * 2654435761u) >> (32 - 12);
          const uint32_t old = atomicCAS(&s_keys[h], 0u, s + 1u);
          if (old == 0u || old == s + 1u) atomicAdd(&s_cnts[h], 1u);
          else atomic_add_u64(hist + s, 1ull);
        }
      }
    }
    uint32_t tot;
    block_excl_scan_u32(ones, s_w, tot);
    if (tid == 0 && tot) atomic_add_u64(tile_cnt0 + t, tot);
  }
  if (bad) (void)__hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (uint32_t h = tid; h < (uint32_t)kHashSlots; h += kBT) {
    const uint32_t key = s_keys[h];
    if (key) atomic_add_u64(hist + (key - 1u), s_cnts[h]);
  }
}

// Alphabets up to kHDenseMax (sigma + 1 <= kWords for the small variant): block bid of nblk takes
// tiles [ntiles * bid / nblk, ntiles * (bid + 1) / nblk). Also adds, per level-0 tile, its ones
// (code bit L - 1) to tile_cnt0 (cleared beforehand), one atomic per wave and tile.
template <typename E, uint32_t kWords, typename PS, typename PH, typename PE>
__device__ __forceinline__ void hist_dense_body(PS sym, uint64_t n, uint32_t sigma, uint32_t L, uint32_t aligned,
                                                PH hist, PH tile_cnt0, PE err, uint64_t bid, uint64_t nblk) {
  using TL = Tile<E>;
  constexpr int EV = TL::EV, NCH = TL::NCH;
  __shared__ uint32_t s_h[kWords];
  const uint32_t tid = threadIdx.x, grp = tid / kBT, gt = tid % kBT, lane = tid & 63u;
  const uint32_t win = min(sigma, kWords);
  const uint32_t nrep = sigma + 1 <= kWords ? max(1u, min(kHMaxRep, kWords / (sigma + 1))) : 1u;
  const uint32_t stride = nrep > 1 ? sigma + 1 : win;
  uint32_t* my_h = s_h + (lane % nrep) * stride;
  const uint64_t ntiles = (n + TL::T - 1) >> TL::TSHIFT;
  const uint64_t tb = ntiles * bid / nblk, te = ntiles * (bid + 1) / nblk;
  const uint64_t nit = (te - tb + kHG - 1) / kHG;
  const uint32_t lsh = L ? L - 1 : 0;
  // sigma covers every value of E (u8 with 256 symbols, u16 with 2^16): counted in one window
  const bool full = sizeof(E) < 4 && sigma == (1u << (8 * sizeof(E))) && win == sigma;
  uint32_t bad = 0;
  for (uint32_t w0 = 0; w0 < sigma; w0 += win) {
    const uint32_t wn = min(win, sigma - w0);
    for (uint32_t i = tid; i < nrep * stride; i += kHT) s_h[i] = 0;
    __syncthreads();
    const bool first = w0 == 0;
    for (uint64_t it = 0; it < nit; ++it) {
      const uint64_t t = tb + it * kHG + grp;
      if (t < te) {  // uniform over the group's waves
        const uint64_t t0 = t << TL::TSHIFT;
        const uint32_t cnt = (uint32_t)min<uint64_t>(TL::T, n - t0);
        uint32_t ones = 0;
        // a whole vector of a whole tile: no bounds, and the level-0 ones by a dot product (a symbol
        // >= sigma fails the build, so counting its bit changes nothing that is kept)
        auto count_vec_full = [&](const uint4& x) {
#pragma unroll
          for (int e = 0; e < EV; ++e) {
            const uint32_t s = vec_elem<E>(x, e);
            const uint32_t r = s - w0;
            if (r < wn) atomicAdd(&my_h[r], 1u);
            if (first) bad |= s >= sigma ? 1u : 0u;
          }
          if (first) ones += vec_count_bit<E>(x, lsh);
        };
        auto count_vec = [&](const uint4& x, uint32_t q0) {
#pragma unroll
          for (int e = 0; e < EV; ++e) {
            const uint32_t s = vec_elem<E>(x, e);
            if (q0 + e < cnt) {
              const uint32_t r = s - w0;
              if (r < wn) atomicAdd(&my_h[r], 1u);
              if (first) {
                bad |= s >= sigma ? 1u : 0u;
                ones += s < sigma ? (s >> lsh) & 1u : 0u;
              }
            }
          }
        };
        if (full && aligned && cnt == (uint32_t)TL::T) {
          // every value of E is a symbol (one window, nothing out of range): per element only the
          // counter address and the add; the level-0 ones per vector by a dot product
          u32x4 vx[NCH];
#pragma unroll
          for (int k = 0; k < NCH; ++k) vx[k] = *pcast<const u32x4>(sym + t0 + (uint32_t)(k * kBT + gt) * EV);
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            uint4 x;
            __builtin_memcpy(&x, &vx[k], 16);
#pragma unroll
            for (int e = 0; e < EV; ++e) atomicAdd(&my_h[vec_elem<E>(x, e)], 1u);
            ones += vec_count_bit<E>(x, lsh);
          }
        } else if (aligned && cnt == (uint32_t)TL::T) {
          // whole aligned tile: every vector in flight at once, kept packed (4 registers each)
          u32x4 vx[NCH];
#pragma unroll
          for (int k = 0; k < NCH; ++k) vx[k] = *pcast<const u32x4>(sym + t0 + (uint32_t)(k * kBT + gt) * EV);
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            uint4 x;
            __builtin_memcpy(&x, &vx[k], 16);
            count_vec_full(x);
          }
        } else if (sizeof(E) < 4 && !aligned && cnt == (uint32_t)TL::T && ((uintptr_t)(sym + t0) & 15u) != 0) {
          // whole tile of a u8/u16 sequence that starts off a 16-byte boundary (forest trees at
          // arbitrary offsets): the two aligned blocks of every vector in flight at once, then
          // funnel-shifted (every vector of the tile has the same misalignment; both blocks hold
          // bytes of the tile). Not compiled for u32, whose dense count would lose occupancy.
          const uint32_t m = (uint32_t)((uintptr_t)(sym + t0) & 15u);
          u32x4 va[NCH], vb[NCH];
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            const auto blk = pcast<const u32x4>(pcast<const char>(sym + t0 + (uint32_t)(k * kBT + gt) * EV) - m);
            va[k] = blk[0];
            vb[k] = blk[1];
          }
#pragma unroll
          for (int k = 0; k < NCH; ++k) {
            uint32_t y[4];
            funnel16(va[k], vb[k], m, y);
            uint4 x;
            __builtin_memcpy(&x, y, 16);
            if (full) {
#pragma unroll
              for (int e = 0; e < EV; ++e) atomicAdd(&my_h[vec_elem<E>(x, e)], 1u);
              ones += vec_count_bit<E>(x, lsh);
            } else {
              count_vec_full(x);
            }
          }
        } else {
          // ragged last tile: one vector at a time
#pragma unroll 1
          for (int k = 0; k < NCH; ++k) {
            const uint32_t q0 = (uint32_t)(k * kBT + gt) * EV;
            E v[EV];
            load16<E>(sym + t0, q0, cnt, aligned && (q0 + EV <= cnt), v);
            uint4 x;
            __builtin_memcpy(&x, v, 16);
            count_vec(x, q0);
          }
        }
        if (first && L) {
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) ones += __shfl_xor(ones, off, 64);
          if (lane == 0 && ones) atomic_add_u64(tile_cnt0 + t, (uint64_t)ones);
        }
      }
    }
    __syncthreads();
    for (uint32_t r = tid; r < wn; r += kHT) {
      uint32_t c = 0;
      for (uint32_t k = 0; k < nrep; ++k) c += s_h[k * stride + r];
      if (c) atomic_add_u64(hist + w0 + r, (uint64_t)c);
    }
    __syncthreads();
  }
  if (bad) (void)__hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Alphabets above kHDenseMax (single-tree build): a radix step keeps every count in LDS.
//  1. group count: per block (tile ranges as in the dense histogram) the symbols per window of
//     2^kHWinShift symbols, written window-major (gcnt[g * nblk + block]); the level-0 ones per tile
//     and the out-of-range flag on the way;
//  2. an exclusive scan of gcnt gives every (window, block) its slots;
//  3. group scatter: the blocks place their symbols in window order (LDS cursors);
//  4. window count: blocks over fixed ranges of the window-ordered symbols count each window piece
//     densely in LDS and add the nonzero counts to the histogram.
constexpr uint32_t kHWinShift = 15;          // 32768 symbols per window (128 KB of counters)
constexpr uint32_t kHMaxWin = 512;           // windows for WT_MAX_SIGMA = 2^24
constexpr uint64_t kHWinChunk = 1ull << 20;  // window-ordered symbols per block of the window count

template <typename E, typename PS, typename PH, typename PE>
__device__ __forceinline__ void hist_group_count_body(PS sym, uint64_t n, uint32_t sigma, uint32_t L, uint32_t aligned,
                                                      PH gcnt, PH tile_cnt0, PE err, uint64_t bid, uint64_t nblk) {
  using TL = Tile<E>;
  constexpr int EV = TL::EV, NCH = TL::NCH;
  __shared__ uint32_t s_g[kHMaxWin];
  const uint32_t tid = threadIdx.x, grp = tid / kBT, gt = tid % kBT, lane = tid & 63u;
  const uint32_t G = (sigma + (1u << kHWinShift) - 1) >> kHWinShift;
  for (uint32_t i = tid; i < G; i += kHT) s_g[i] = 0;
  __syncthreads();
  const uint64_t ntiles = (n + TL::T - 1) >> TL::TSHIFT;
  const uint64_t tb = ntiles * bid / nblk, te = ntiles * (bid + 1) / nblk;
  const uint64_t nit = (te - tb + kHG - 1) / kHG;
  const uint32_t lsh = L - 1;
  uint32_t bad = 0;
  for (uint64_t it = 0; it < nit; ++it) {
    const uint64_t t = tb + it * kHG + grp;
    if (t < te) {  // uniform over the group's waves
      const uint64_t t0 = t << TL::TSHIFT;
      const uint32_t cnt = (uint32_t)min<uint64_t>(TL::T, n - t0);
      uint32_t ones = 0;
#pragma unroll 1
      for (int k = 0; k < NCH; ++k) {
        const uint32_t q0 = (uint32_t)(k * kBT + gt) * EV;
        E v[EV];
        load16<E>(sym + t0, q0, cnt, aligned && (q0 + EV <= cnt), v);
#pragma unroll
        for (int e = 0; e < EV; ++e) {
          const uint32_t x = (uint32_t)v[e];
          if (q0 + e < cnt) {
            if (x < sigma) {
              atomicAdd(&s_g[x >> kHWinShift], 1u);
              ones += (x >> lsh) & 1u;
            } else {
              bad = 1;
            }
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) ones += __shfl_xor(ones, off, 64);
      if (lane == 0 && ones) atomic_add_u64(tile_cnt0 + t, (uint64_t)ones);
    }
  }
  __syncthreads();
  for (uint32_t g = tid; g < G; g += kHT) gcnt[(uint64_t)g * nblk + bid] = s_g[g];
  if (bid == 0 && tid == 0) gcnt[(uint64_t)G * nblk] = 0;  // so the scan's last entry is the total
  if (bad) (void)__hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// goff: the exclusive scan of gcnt. Symbols >= sigma are skipped (the build fails on them).
template <typename E, typename PS, typename PD>
__device__ __forceinline__ void hist_group_scatter_body(PS sym, uint64_t n, uint32_t sigma, uint32_t aligned,
                                                        const uint64_t* __restrict__ goff, PD dst, uint64_t bid,
                                                        uint64_t nblk) {
  using TL = Tile<E>;
  constexpr int EV = TL::EV, NCH = TL::NCH;
  __shared__ uint32_t s_cur[kHMaxWin];
  const uint32_t tid = threadIdx.x, grp = tid / kBT, gt = tid % kBT;
  const uint32_t G = (sigma + (1u << kHWinShift) - 1) >> kHWinShift;
  // slots of a block stay below n < 2^40; cursors count from the block's first slot per window
  __shared__ uint64_t s_base[kHMaxWin];
  for (uint32_t g = tid; g < G; g += kHT) {
    s_base[g] = goff[(uint64_t)g * nblk + bid];
    s_cur[g] = 0;
  }
  __syncthreads();
  const uint64_t ntiles = (n + TL::T - 1) >> TL::TSHIFT;
  const uint64_t tb = ntiles * bid / nblk, te = ntiles * (bid + 1) / nblk;
  const uint64_t nit = (te - tb + kHG - 1) / kHG;
  for (uint64_t it = 0; it < nit; ++it) {
    const uint64_t t = tb + it * kHG + grp;
    if (t >= te) continue;
    const uint64_t t0 = t << TL::TSHIFT;
    const uint32_t cnt = (uint32_t)min<uint64_t>(TL::T, n - t0);
#pragma unroll 1
    for (int k = 0; k < NCH; ++k) {
      const uint32_t q0 = (uint32_t)(k * kBT + gt) * EV;
      E v[EV];
      load16<E>(sym + t0, q0, cnt, aligned && (q0 + EV <= cnt), v);
#pragma unroll
      for (int e = 0; e < EV; ++e) {
        const uint32_t x = (uint32_t)v[e];
        if (q0 + e < cnt && x < sigma) {
          const uint32_t g = x >> kHWinShift;
          dst[s_base[g] + atomicAdd(&s_cur[g], 1u)] = (E)x;
        }
      }
    }
  }
}

// Window count over the window-ordered symbols src[0, total): block bid takes
// [bid * kHWinChunk, (bid + 1) * kHWinChunk) and counts each window piece in it densely.
template <typename E, typename PS, typename PH>
__device__ __forceinline__ void hist_window_count_body(PS src, const uint64_t* __restrict__ goff, uint64_t nblk1,
                                                       uint32_t sigma, PH hist, uint64_t bid) {
  __shared__ uint32_t s_h[1u << kHWinShift];
  const uint32_t tid = threadIdx.x;
  const uint32_t G = (sigma + (1u << kHWinShift) - 1) >> kHWinShift;
  const uint64_t total = goff[(uint64_t)G * nblk1];  // the scan's end entry: all valid symbols
  const uint64_t lo = bid * kHWinChunk, hi = min(lo + kHWinChunk, total);
  if (lo >= hi) return;  // whole block
  uint32_t g = (uint32_t)src[lo] >> kHWinShift;
  const uint32_t glast = (uint32_t)src[hi - 1] >> kHWinShift;
  for (; g <= glast; ++g) {
    const uint64_t a = max(lo, goff[(uint64_t)g * nblk1]);
    const uint64_t b = min(hi, g + 1 < G ? goff[(uint64_t)(g + 1) * nblk1] : total);
    const uint32_t w0 = g << kHWinShift;
    for (uint32_t i = tid; i < (1u << kHWinShift); i += kHT) s_h[i] = 0;
    __syncthreads();
    for (uint64_t j = a + tid; j < b; j += kHT) atomicAdd(&s_h[(uint32_t)src[j] - w0], 1u);
    __syncthreads();
    for (uint32_t r = tid; r < (1u << kHWinShift); r += kHT) {
      const uint32_t c = s_h[r];
      if (c) atomic_add_u64(hist + w0 + r, (uint64_t)c);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- node tables

// Heap entry h (level l = floor(lg(h+1)), code prefix p = h + 1 - 2^l): follow p from the root with
// the split rule of the reduced tree (left child = the largest power of two strictly below the
// width). A prefix that reaches a leaf before level l names no node at level l.
__device__ __forceinline__ void node_walk_body(uint32_t sigma, uint64_t nheap, const uint64_t* __restrict__ cum,
                                               NodeB* __restrict__ ntb, uint64_t* __restrict__ zeros, uint64_t h) {
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
__device__ __forceinline__ void node_final_body(uint64_t nheap, const uint64_t* __restrict__ zs,
                                                NodeB* __restrict__ ntb, NodeQ* __restrict__ ntq,
                                                LevelMeta* __restrict__ meta, uint64_t h) {
  // every lane of the wave takes part in the level-size reduction at the end
  const bool valid = h < nheap;
  const uint32_t l = valid ? 63u - (uint32_t)__clzll(h + 1) : 0xFFFFFFFFu;
  uint64_t endv = 0;
  if (valid) {
    const uint64_t base = (1ull << l) - 1;
    NodeB b = ntb[h];
    NodeQ q;
    if (b.start == kNoNode) {
      q.start = kNoNode;
      q.r0 = kNoNode;
      ntq[h] = q;
    } else {
      const uint64_t r0 = zs[h] - zs[base];
      const uint64_t mid = b.off0;
      q.start = b.start;
      q.r0 = r0;
      ntq[h] = q;
      b.off0 = b.start - r0;
      b.off1 = mid - b.start + r0;
      ntb[h] = b;
      endv = b.end;
    }
  }
  // level size = the largest node end of the level: one atomic per (wave, level) instead of per node
  const uint32_t lane = threadIdx.x & 63u;
  uint64_t pend = __ballot(valid);
  while (pend) {
    const int leader = __ffsll((unsigned long long)pend) - 1;
    const uint32_t ll = __shfl(l, leader, 64);
    const bool mine = valid && l == ll;
    uint64_t v = mine ? endv : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(v, off, 64);
      v = o > v ? o : v;
    }
    if (lane == (uint32_t)leader && v) atomicMax((unsigned long long*)&meta[ll].n, (unsigned long long)v);
    pend &= ~__ballot(mine);
  }
}

// ---------------------------------------------------------------- per-level tile prefix

// Sum of the ones of every chunk of kChunkTiles tiles of level l.
__device__ __forceinline__ void tile_reduce_body(const LevelMeta* __restrict__ meta, uint32_t l, uint32_t tshift,
                                                 const uint64_t* __restrict__ cnt, uint64_t* __restrict__ chunk,
                                                 uint64_t b) {
  __shared__ uint64_t s_w[kBT / 64];
  const uint64_t nl = meta[l].n;
  const uint64_t nt = (nl + (1ull << tshift) - 1) >> tshift;
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
__device__ __forceinline__ void tile_scan_body(LevelMeta* __restrict__ meta, uint32_t l, uint32_t tshift,
                                               const uint64_t* __restrict__ cnt, const uint64_t* __restrict__ chunk,
                                               uint64_t* __restrict__ pre, uint64_t* __restrict__ L1,
                                               uint16_t* __restrict__ L2, uint64_t b) {
  __shared__ uint64_t s_w[kBT / 64];
  const LevelMeta m = meta[l];
  const uint64_t nl = m.n;
  const uint64_t nt = (nl + (1ull << tshift) - 1) >> tshift;
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

// A non-empty node of a level, for finding nodes by position (narrow codes).
struct NodeS {
  uint64_t start;
  uint32_t pfx;  // code prefix (index in the level's node table)
  uint32_t pad;
};

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
  uint32_t matrix;      // wavelet matrix: the whole level is one node (ntb[0]: zeros then ones)
  // Narrow codes: once a level has written codes without their prefix bits, later levels find an
  // element's node by its position: the non-empty nodes of every level, in position order (ns, level l
  // at [ns_idx[2^l - 1], ns_idx[2^(l+1) - 1])), and the node holding each tile's first element.
  uint32_t pos_node;
  const NodeS* ns;
  const uint64_t* ns_idx;
  const uint32_t* tfirst;
  // Build error word (bit 1: an element fell outside its tile's staging slots, an internal error the
  // host reports), or NULL.
  uint32_t* err;
};

// The level pass's view of LevelArgs, with its pointers in the global address space.
struct LevelArgsG {
  const WT_GLOBAL char* in;
  WT_GLOBAL char* out;
  WT_GLOBAL uint64_t* bits;
  WT_GLOBAL uint64_t* L1;
  WT_GLOBAL uint16_t* L2;
  WT_GLOBAL uint64_t* smp;
  WT_GLOBAL LevelMeta* meta;
  const WT_GLOBAL uint64_t* pre;
  WT_GLOBAL uint64_t* cnt_next;
  const WT_GLOBAL NodeB* ntb;
  uint32_t l, L, sigma, pow2;
  uint32_t l2shift, sshift;
  uint32_t encode, in_vec, in_aligned, matrix;
  uint32_t pos_node;
  const WT_GLOBAL NodeS* ns;
  const WT_GLOBAL uint64_t* ns_idx;
  const WT_GLOBAL uint32_t* tfirst;
  WT_GLOBAL uint32_t* err;
};

__device__ __forceinline__ LevelArgsG to_global(const LevelArgs& a) {
  LevelArgsG g;
  g.in = (const WT_GLOBAL char*)a.in;
  g.out = (WT_GLOBAL char*)a.out;
  g.bits = (WT_GLOBAL uint64_t*)a.bits;
  g.L1 = (WT_GLOBAL uint64_t*)a.L1;
  g.L2 = (WT_GLOBAL uint16_t*)a.L2;
  g.smp = (WT_GLOBAL uint64_t*)a.smp;
  g.meta = (WT_GLOBAL LevelMeta*)a.meta;
  g.pre = (const WT_GLOBAL uint64_t*)a.pre;
  g.cnt_next = (WT_GLOBAL uint64_t*)a.cnt_next;
  g.ntb = (const WT_GLOBAL NodeB*)a.ntb;
  g.l = a.l;
  g.L = a.L;
  g.sigma = a.sigma;
  g.pow2 = a.pow2;
  g.l2shift = a.l2shift;
  g.sshift = a.sshift;
  g.encode = a.encode;
  g.in_vec = a.in_vec;
  g.in_aligned = a.in_aligned;
  g.matrix = a.matrix;
  g.pos_node = a.pos_node;
  g.ns = (const WT_GLOBAL NodeS*)a.ns;
  g.ns_idx = (const WT_GLOBAL uint64_t*)a.ns_idx;
  g.tfirst = (const WT_GLOBAL uint32_t*)a.tfirst;
  g.err = (WT_GLOBAL uint32_t*)a.err;
  return g;
}

// Adds, for the lanes in `cls`, their next-level ones (the bit `nbit`, or `cnt_lane` when nbit is
// unused) per destination tile to a running per-wave (tile, count) pair, flushing it to the global
// tile counter when the tile changes. Destinations increase with the processing order, so each tile
// is flushed about once per wave, and a tile counter sees few writers.
template <typename P>
__device__ __forceinline__ void count_next(uint64_t cls, uint64_t dt, uint32_t nbit, uint32_t lane,
                                           uint64_t& cur_tile, uint32_t& cur_c, P cnt, uint32_t cnt_lane) {
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
      if (cur_c && lane == 0) atomic_add_u64(cnt + cur_tile, cur_c);
      cur_tile = ldt;
      cur_c = c1;
    }
    cls &= ~same;
  }
}

// Select samples of one wave's words: every lane with c set holds a word w whose r-th set bit
// (r in [1, 64]) is sampled, at position pos0 + that bit, stored to *dst. The wave resolves those
// lanes one at a time: lane i tests bit i of the word, and a ballot gives the bit.
template <typename P>
__device__ __forceinline__ void wave_sample(bool c, uint64_t w, uint32_t r, uint64_t pos0, P dst, uint32_t lane) {
  uint64_t pend = __ballot(c);
  while (pend) {
    const int ld = __ffsll((unsigned long long)pend) - 1;
    const uint64_t wl = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(w >> 32), ld) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)w, ld);
    const uint32_t rl = (uint32_t)__builtin_amdgcn_readlane((int)r, ld);
    const bool hit = ((wl >> lane) & 1ull) && (uint32_t)__popcll(wl & ((1ull << lane) - 1ull)) + 1u == rl;
    const uint64_t hm = __ballot(hit);
    if (lane == (uint32_t)ld) *dst = pos0 + (uint64_t)(__ffsll((unsigned long long)hm) - 1);
    pend &= pend - 1;
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
// Per-tree build state of a batched (forest) build: the tree's parts and scratch, as the single-tree
// build keeps them, for device-side derivation of every phase's arguments.
struct TreeB {
  const void* sym;
  uint64_t n;
  uint32_t sigma, L, pow2, aligned;
  uint32_t l2shift, sshift, tshift, pad0;
  LevelMeta* meta;
  uint64_t* cum;
  NodeQ* nodes;
  uint64_t* bits;
  uint64_t* L1;
  uint16_t* L2;
  uint64_t* smp;
  uint64_t words_per_level, l1_per_level, l2_per_level, smp_per_level;
  void* seq[2];
  uint64_t* clear;  // [hist | tile counts | err], cleared at the start
  uint64_t clear_n;
  uint64_t* hist;
  uint64_t* tcnt;
  uint64_t* tpre;
  NodeB* ntb;
  uint64_t* z;
  uint64_t* zs;
  uint64_t* part;
  uint32_t* err;
  uint64_t ntiles, nchunks, cstride, nheap;
  // Carried code width of every level (2 bits per level l = 0 .. L: log2 of its element bytes; level 0
  // holds the symbols) and the levels whose nodes are found by position (bit l), with the tree's
  // non-empty nodes in position order for them (indexed through zs, as in the single-tree build).
  uint64_t wlog;
  uint32_t posmask, pad1;
  NodeS* ns;
};

__device__ __forceinline__ uint32_t forest_wlog(const TreeB& b, uint32_t l) {
  return (uint32_t)(b.wlog >> (2 * l)) & 3u;
}

// Blocks of a forest launch: block g = base + blockIdx.x of the map belongs to tree bmap[g] and is
// block g - boff[tree] of it (a launch may cover a range of the map's trees).
struct ForestGrid {
  const TreeB* tb;
  const uint32_t* bmap;
  const uint32_t* boff;
  uint32_t l;
  uint32_t base;
};

// Arguments of the level-l pass of a tree of a forest build (as the single-tree build sets them).
__device__ __forceinline__ LevelArgs forest_level_args(const TreeB& b, uint32_t l) {
  LevelArgs a;
  a.in = (l == 0 ? b.sym : b.seq[(l - 1) & 1]);
  a.out = (l + 1 < b.L) ? (b.seq[l & 1]) : nullptr;
  a.bits = (b.bits);
  a.L1 = (b.L1);
  a.L2 = (b.L2);
  a.smp = (b.smp);
  a.meta = (b.meta);
  a.pre = (b.tpre + (uint64_t)l * (b.ntiles + 1));
  a.cnt_next = (l + 1 < b.L) ? (b.tcnt + (uint64_t)(l + 1) * b.cstride) : nullptr;
  a.ntb = (b.ntb + ((1ull << l) - 1));
  a.l = l;
  a.L = b.L;
  a.sigma = b.sigma;
  a.pow2 = b.pow2;
  a.l2shift = b.l2shift;
  a.sshift = b.sshift;
  a.encode = (l == 0 && !b.pow2) ? 1u : 0u;
  a.in_vec = l == 0 ? 0u : 1u;
  a.in_aligned = l == 0 ? b.aligned : 1u;
  a.matrix = 0;
  a.pos_node = (b.posmask >> l) & 1u;
  a.ns = b.ns;
  a.ns_idx = b.zs;
  a.tfirst = nullptr;  // each tile finds its first node itself
  a.err = b.err;
  return a;
}

// Index of the last entry of ns[lo, hi) whose start is <= x, given ns[lo].start <= x and increasing
// starts: a 64-way search by one whole wave (three rounds of one load per lane for 2^17 entries).
template <typename P>
__device__ __forceinline__ uint64_t wave_find_start(P ns, uint64_t lo, uint64_t hi, uint64_t x, uint32_t lane) {
  while (hi - lo > 1) {
    const uint64_t step = (hi - lo + 63) / 64;
    const uint64_t i = lo + (uint64_t)lane * step;
    const bool le = i < hi && ns[i].start <= x;
    // the lanes with le are 0 .. c - 1 (lane 0 tests lo), so the answer is in [lo + (c-1) step, lo + c step)
    const uint32_t c = (uint32_t)__popcll(__ballot(le));
    const uint64_t nlo = lo + (uint64_t)(c - 1) * step;
    hi = min(hi, nlo + step);
    lo = nlo;
  }
  return lo;
}

// The body stays in the kernel (as a device function it needs far more registers).
// Waves per SIMD the level pass is compiled for (a register budget): six where the body fits in
// 80 registers without spilling, else five.
template <typename E, bool kForest, bool kPos = false>
constexpr int level_waves() {
  return !kPos && ((sizeof(E) == 1 && !kForest) || (sizeof(E) == 2 && kForest)) ? 6 : 5;
}

// E: element type of level l; EO: of level l + 1 (narrower when the codes need fewer bits below the
// level: the prefix bits are dropped and later levels find nodes by position).
// kPos: nodes by position (levels after the codes lost their prefix bits).
template <typename E, bool kForest, typename EO = E, bool kPos = false>
__global__ __launch_bounds__(kBT, (level_waves<E, kForest, kPos>())) void k_level(LevelArgs a_one, ForestGrid fg) {
  LevelArgsG a;
  uint64_t t;
  if constexpr (kForest) {
    const uint32_t g = blockIdx.x + fg.base;
    const uint32_t j = fg.bmap[g];
    t = g - fg.boff[j];
    a = to_global(forest_level_args(fg.tb[j], fg.l));
  } else {
    a = to_global(a_one);
    t = blockIdx.x;
  }
  using TL = Tile<E>;
  using TO = Tile<EO>;
  static_assert(sizeof(EO) <= sizeof(E), "codes only narrow");
  constexpr int T = TL::T, W = TL::W, EV = TL::EV, G = TL::G, NCH = TL::NCH;
  __shared__ __align__(16) EO s_stage[T + 16 / sizeof(EO) + 4];  // + slack for the 20-byte chunk reads
  __shared__ uint64_t s_words[W + 1];  // entry W: 0, so ranks are defined at x = T
  __shared__ uint32_t s_wpre[W + 1];   // entry W: ones of the tile
  __shared__ uint32_t s_w[kBT / 64];
  __shared__ Seg s_seg[kSegMax];
  __shared__ uint32_t s_cp[2 * kSegMax + 1];
  __shared__ uint32_t s_nseg;
  __shared__ uint64_t s_node[2];  // node of the tile's first and last element
  __shared__ uint64_t s_dst[2];   // single-node tile: destinations of its first zero and first one
  __shared__ uint32_t s_nc[4];    // single-node tile: next-level ones per (run, destination tile)
  __shared__ uint2 s_enc[32];     // level 0 of a reduced alphabet: (high code bits, shift) by h
  // nodes by position: bit q of s_nb is set where a node starts at tile position q > 0, s_nbp counts
  // the starts before each word, so the node of position q is the tile's node number (starts in
  // (0, q]); s_lpf holds the code prefixes of the first kSegMax nodes, s_i0 and s_i1 the entries of
  // the tile's first and last node in the level's position list
  __shared__ uint64_t s_nb[kPos ? W + 1 : 1];
  __shared__ uint32_t s_nbp[kPos ? W + 1 : 1];
  __shared__ uint32_t s_lpf[kSegMax];
  __shared__ uint64_t s_i0;
  __shared__ uint64_t s_i1;

  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t l = a.l, L = a.L;
  const LevelMeta m = ld_meta(a.meta + l);
  const uint64_t nl = m.n;
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

  // The reduced code of a symbol c depends on h, the highest bit where c and sigma differ: it is the
  // j1 = popc(sigma >> (h+1)) leading ones (the right steps taken before c's subtree), then c's low h
  // bits placed so that the code has its length len(h), left-aligned to L bits. One table entry per h.
  if (a.encode) {
    if (tid < 32) {
      const uint32_t h = tid, sg = a.sigma;
      const uint32_t j1 = h < 31 ? (uint32_t)__popc(sg >> (h + 1)) : 0u;
      const uint32_t len = j1 + ((sg & ((1u << h) - 1u)) == 0u ? 0u : 1u) + h;
      uint2 te;
      te.x = (len <= L && j1) ? ((1u << j1) - 1u) << (L - j1) : 0u;
      te.y = len <= L ? L - len : 0u;
      s_enc[h] = te;
    }
    __syncthreads();
  }

  // 1. load, encode (level 0 of a reduced alphabet), bit words
  const WT_GLOBAL E* in = pcast<const E>(a.in) + t0;
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
        const uint32_t h = 31u - (uint32_t)__clz(s ^ a.sigma);
        const uint2 te = s_enc[h];
        v[e] = (E)(te.x | ((s & ((1u << h) - 1u)) << te.y));
      }
    }
    __builtin_memcpy(&vx[k], v, 16);
  }
  uint32_t vmask[NCH];  // bit bsh of every element of vector k (0 beyond the tile)
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
    const uint32_t valid = q0 >= cnt ? 0u : (q0 + EV <= cnt ? (uint32_t)((1ull << EV) - 1) : (1u << (cnt - q0)) - 1u);
    const uint32_t mask = vec_bits<E>(vx[k], bsh) & valid;
    vmask[k] = mask;
    uint64_t word = (uint64_t)mask << ((tid % G) * EV);
#pragma unroll
    for (int off = 1; off < G; off <<= 1) word |= __shfl_xor(word, off, 64);
    if (tid % G == 0) s_words[k * (kBT / G) + tid / G] = word;
    if (q0 < cnt && q0 + EV > cnt - 1) {
      const uint32_t cx = elem128<E>(((uint64_t)vx[k].y << 32) | vx[k].x, ((uint64_t)vx[k].w << 32) | vx[k].z,
                                     cnt - 1 - q0);
      if (!kPos) s_node[1] = (l && !a.matrix) ? ((uint64_t)cx >> (L - l)) & ((1ull << l) - 1ull) : 0ull;
    }
    if (q0 == 0 && !kPos)
      s_node[0] = (l && !a.matrix) ? ((uint64_t)vec_elem<E>(vx[k], 0) >> (L - l)) & ((1ull << l) - 1ull) : 0ull;
  }
  if (tid < 4) s_nc[tid] = 0;
  if constexpr (kPos) {
    if (tid <= (uint32_t)W) s_nb[tid] = 0;
    if (tid < 128) {
      // the tile's nodes: entries i0 (the one holding t0, found by wave 0) .. i1 (the last starting
      // inside the tile, found by wave 1 at the same time)
      const uint64_t lo = a.ns_idx[(1ull << l) - 1], hi = a.ns_idx[(2ull << l) - 1];
      if (tid < 64) {
        const uint64_t i0 = a.tfirst ? lo + a.tfirst[t] : wave_find_start(a.ns, lo, hi, t0, lane);
        if (lane == 0) {
          const uint32_t p0 = a.ns[i0].pfx;
          s_i0 = i0;
          s_lpf[0] = p0;
          s_node[0] = p0;
        }
      } else {
        const uint64_t i1 = wave_find_start(a.ns, lo, hi, t0 + cnt - 1, lane);
        if (lane == 0) s_i1 = i1;
      }
    }
  }
  __syncthreads();
  bool single = false;  // a tile inside one node (the rule at shallow levels) takes the fast path
  if constexpr (kPos) {
    const uint32_t nn = (uint32_t)(s_i1 - s_i0 + 1);
    single = nn == 1;
    if (nn > 1) {
      // node starts inside the tile into the bitmap, and the first prefixes into the list
      const uint64_t i0 = s_i0;
      for (uint32_t j = 1 + tid; j < nn; j += kBT) {
        const uint32_t x = (uint32_t)(a.ns[i0 + j].start - t0);  // in [1, cnt)
        atomicOr((unsigned long long*)&s_nb[x >> 6], 1ull << (x & 63u));
        if (j < (uint32_t)kSegMax) s_lpf[j] = a.ns[i0 + j].pfx;
      }
      __syncthreads();
    }
  }
  // a tile inside one node: two runs, no segments
  if constexpr (!kPos) single = s_node[0] == s_node[1];
  if (single && !last && tid == 0) {
    const NodeB nb = ld_node(a.ntb + s_node[0]);
    s_dst[0] = nb.off0 + (t0 - G1);
    s_dst[1] = nb.off1 + G1;
  }

  // 2. tile-local rank1 at every word (and, for nodes by position, the node starts before every word:
  // both counts are at most T < 2^16, so one scan carries them in the two halves of a word)
  uint32_t tile_ones;
  {
    uint32_t pc = (tid < (uint32_t)W) ? popc64(s_words[tid]) : 0u;
    if constexpr (kPos) pc |= (tid < (uint32_t)W) ? popc64(s_nb[tid]) << 16 : 0u;
    const uint32_t ex = block_excl_scan_u32(pc, s_w, tile_ones);
    if constexpr (kPos) {
      if (tid < (uint32_t)W) s_nbp[tid] = ex >> 16;
      tile_ones &= 0xFFFFu;
    }
    if (tid < (uint32_t)W) s_wpre[tid] = ex & (kPos ? 0xFFFFu : 0xFFFFFFFFu);
    if (tid == 0) {
      s_wpre[W] = tile_ones;
      s_words[W] = 0;
    }
  }
  __syncthreads();

  // 3. bits and directory
  const uint64_t G0 = t0 - G1;  // zeros of the level before the tile
  if (tid < (uint32_t)W) {  // whole waves (W is a multiple of 64)
    const uint64_t word = s_words[tid];
    const uint64_t gw = ((uint64_t)t * W) + tid;
    a.bits[m.bits + gw] = word;
    const uint32_t q = tid * 64u;
    // a word holds at most one sampled one and one sampled zero (s >= 512 > 64)
    bool c1 = false, c0 = false;
    uint32_t r1 = 0, r0 = 0;
    uint64_t i1 = 0, i0 = 0, zw = 0;
    if (q < cnt) {
      const uint64_t ones_before = G1 + s_wpre[tid];
      const uint32_t l2w_shift = a.l2shift - 6;
      if ((gw & ((1ull << l2w_shift) - 1)) == 0) a.L2[m.l2 + (gw >> l2w_shift)] = (uint16_t)(ones_before - l1val);
      const uint32_t sh = a.sshift;
      const uint64_t k1 = (ones_before + popc64(word)) >> sh;
      c1 = k1 > (ones_before >> sh);
      r1 = (uint32_t)((k1 << sh) - ones_before);
      i1 = m.smp + k1 - 1;
      const uint32_t vb = min(64u, cnt - q);
      zw = ~word & (vb == 64u ? ~0ull : ((1ull << vb) - 1ull));
      const uint64_t zeros_before = t0 + q - ones_before;
      const uint64_t k0 = (zeros_before + popc64(zw)) >> sh;
      c0 = k0 > (zeros_before >> sh);
      r0 = (uint32_t)((k0 << sh) - zeros_before);
      i0 = m.smp + m.smp_cap - k0;
    }
    wave_sample(c1, word, r1, t0 + q, a.smp + i1, lane);
    wave_sample(c0, zw, r0, t0 + q, a.smp + i0, lane);
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
  // Nodes by position: the tile's node number of position q (node starts in (0, q]) identifies the
  // node inside the tile; its code prefix is looked up when a lane enters the node.
  auto knum = [&](uint32_t q) -> uint64_t {
    const uint32_t w = q >> 6;
    return s_nbp[w] + popc64(s_nb[w] & ((2ull << (q & 63u)) - 1ull));
  };
  auto kpfx = [&](uint64_t k) -> uint64_t {
    return k < (uint64_t)kSegMax ? (uint64_t)s_lpf[k] : (uint64_t)a.ns[s_i0 + k].pfx;
  };
  if (single) {
    // zeros fill slots [0, Z), ones [Z, cnt); each lane walks its vectors with running slots
    const uint32_t Z = cnt - tile_ones;
#pragma unroll
    for (int k = 0; k < NCH; ++k) {
      const uint32_t q0 = (uint32_t)(k * kBT + tid) * EV;
      if (q0 < cnt) {
        const uint32_t r1 = r1loc(s_words, s_wpre, q0);
        uint32_t p1 = Z + r1, p0 = q0 - r1;
        const uint32_t m = vmask[k];
        if (q0 + EV <= cnt) {
#pragma unroll
          for (int e = 0; e < EV; ++e) {
            const uint32_t b = (m >> e) & 1u;
            s_stage[b ? p1 : p0] = (EO)vec_elem<E>(vx[k], e);
            p1 += b;
            p0 += b ^ 1u;
          }
        } else {
          // ragged end of the last tile
          const uint64_t lo = ((uint64_t)vx[k].y << 32) | vx[k].x, hi = ((uint64_t)vx[k].w << 32) | vx[k].z;
          for (uint32_t e = 0; e < cnt - q0; ++e) {
            const uint32_t b = (m >> e) & 1u;
            s_stage[b ? p1 : p0] = (EO)elem128<E>(lo, hi, e);
            p1 += b;
            p0 += b ^ 1u;
          }
        }
      }
    }
    __syncthreads();
    // 4b. write-out of the two runs, one 16-byte destination chunk per lane; the next level's ones
    //     are counted per (run, destination tile): a run of at most T elements touches two tiles
    const uint64_t d0 = s_dst[0], d1 = s_dst[1];
    WT_GLOBAL char* outb = a.out;
    const uint32_t* st32 = reinterpret_cast<const uint32_t*>(s_stage);
    const uint32_t len0 = d0 < n_next ? (uint32_t)min<uint64_t>(Z, n_next - d0) : 0u;
    const uint32_t len1 = d1 < n_next ? (uint32_t)min<uint64_t>(cnt - Z, n_next - d1) : 0u;
    // Offsets relative to each run's first 16-byte destination chunk (32-bit): the run covers bytes
    // [a_r, e_r) from that chunk's base g_r; tb_r is the base's offset inside its destination tile.
    constexpr uint32_t w = (uint32_t)sizeof(EO);
    constexpr uint32_t kTileB = (uint32_t)TO::T * w;  // bytes of a destination tile
    const uint64_t g0 = (d0 * w) & ~15ull, g1 = (d1 * w) & ~15ull;
    const uint32_t a0 = (uint32_t)(d0 * w) & 15u, a1 = (uint32_t)(d1 * w) & 15u;
    const uint32_t e0 = a0 + len0 * w, e1 = a1 + len1 * w;
    const uint32_t C0 = len0 ? (e0 + 15u) >> 4 : 0u, C1 = len1 ? (e1 + 15u) >> 4 : 0u;
    const uint32_t tb0 = (uint32_t)g0 & (kTileB - 1u), tb1 = (uint32_t)g1 & (kTileB - 1u);
    uint32_t acc0 = 0, acc1 = 0;  // next-level ones of run 0 / run 1: first tile low 16 bits, second high
    for (uint32_t c = tid; c < C0 + C1; c += kBT) {
      const bool bb = c >= C0;
      const uint32_t rb = (bb ? c - C0 : c) << 4;  // chunk start, bytes from g_r
      const uint32_t ar = bb ? a1 : a0, er = bb ? e1 : e0;
      const uint32_t blo = max(rb, ar), bhi = min(rb + 16u, er);
      const uint32_t src = (bb ? Z * w : 0u) + blo - ar;  // LDS byte of blo
      WT_GLOBAL char* cp = outb + (bb ? g1 : g0) + rb;
      uint32_t nb = 0;
      if (blo == rb && bhi == rb + 16u) {
        const uint32_t dw = src >> 2, sh = src & 3u;
        const uint32_t x0 = st32[dw], x1 = st32[dw + 1], x2 = st32[dw + 2], x3 = st32[dw + 3], x4 = st32[dw + 4];
        uint4 y;
        y.x = __builtin_amdgcn_alignbyte(x1, x0, sh);
        y.y = __builtin_amdgcn_alignbyte(x2, x1, sh);
        y.z = __builtin_amdgcn_alignbyte(x3, x2, sh);
        y.w = __builtin_amdgcn_alignbyte(x4, x3, sh);
        st16(cp, y);
        nb = vec_count_bit<EO>(y, nbsh);  // next-level ones of the 16 / w elements
      } else {
        // run edge: element stores
        WT_GLOBAL EO* oe = pcast<EO>(cp);
        for (uint32_t x = blo; x < bhi; x += w) {
          const EO v = s_stage[(src + x - blo) / w];
          oe[(x - rb) / w] = v;
          nb += ((uint32_t)v >> nbsh) & 1u;
        }
      }
      // a run of at most T elements touches at most two destination tiles
      const uint32_t add = nb << (((bb ? tb1 : tb0) + rb) >= kTileB ? 16 : 0);
      acc0 += bb ? 0u : add;
      acc1 += bb ? add : 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc0 += __shfl_xor(acc0, off, 64);
      acc1 += __shfl_xor(acc1, off, 64);
    }
    if (lane == 0) {
      const uint32_t v[4] = {acc0 & 0xFFFFu, acc0 >> 16, acc1 & 0xFFFFu, acc1 >> 16};
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (v[r]) atomicAdd(&s_nc[r], v[r]);
    }
    __syncthreads();
    if (tid < 4) {
      const uint32_t c = s_nc[tid];
      const uint64_t d = (tid < 2) ? d0 : d1;
      if (c && d < n_next)
        atomic_add_u64(a.cnt_next + (d >> TO::TSHIFT) + (tid & 1u), c);
    }
    return;
  }
  bool bad = false;  // a staging slot fell outside the tile
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
        // node of the first and the last element (nodes by position: tile node numbers, and the
        // node starts at the vector's other elements, bits 1 .. nv-1 of sbits; EV divides 64)
        uint64_t Nf, Nl;
        uint32_t sbits = 0;
        if constexpr (kPos) {
          const uint32_t w = q0 >> 6;
          const uint64_t wb = s_nb[w];
          Nf = s_nbp[w] + popc64(wb & ((2ull << (q0 & 63u)) - 1ull));
          sbits = (uint32_t)(wb >> (q0 & 63u)) & ((2u << (nv - 1)) - 2u);
          Nl = Nf + (uint32_t)__popc(sbits);
        } else {
          const uint32_t cf = vec_elem<E>(vx[k], 0), cl = elem128<E>(lo, hi, nv - 1);
          Nf = l ? ((uint64_t)cf >> (L - l)) & pmask : 0ull;
          Nl = l ? ((uint64_t)cl >> (L - l)) & pmask : 0ull;
        }
        if (Nf == Nl) {
          // the whole vector lies in one node
          if (Nf != curN) enter_node(ld_node(a.ntb + (kPos ? kpfx(Nf) : Nf)), q0, t0, cnt, G0, G1, s_words, s_wpre, s_seg, &s_nseg, sa, zs, R1a), curN = Nf;
          // slot = R1a + rank0 or sa + zs - R1a + rank1 (tile-local ranks), as running slots
          uint32_t p1 = sa + zs - R1a + r1, p0 = R1a + q0 - r1;
          const uint32_t m = vmask[k];
          if (nv == (uint32_t)EV) {
#pragma unroll
            for (int e = 0; e < EV; ++e) {
              const uint32_t b = (m >> e) & 1u;
              bad = bad || (b ? p1 : p0) >= (uint32_t)T;
              s_stage[min(b ? p1 : p0, (uint32_t)T - 1u)] = (EO)vec_elem<E>(vx[k], e);
              p1 += b;
              p0 += b ^ 1u;
            }
          } else {
            for (uint32_t e = 0; e < nv; ++e) {
              const uint32_t b = (m >> e) & 1u;
              bad = bad || (b ? p1 : p0) >= (uint32_t)T;
              s_stage[min(b ? p1 : p0, (uint32_t)T - 1u)] = (EO)elem128<E>(lo, hi, e);
              p1 += b;
              p0 += b ^ 1u;
            }
          }
        } else {
          uint64_t Nk = Nf;  // nodes by position: the running node number
          for (uint32_t e = 0; e < nv; ++e) {
            const uint32_t code = elem128<E>(lo, hi, e);
            const uint32_t b = (code >> bsh) & 1u;
            const uint32_t q = q0 + e;
            if constexpr (kPos) Nk += (sbits >> e) & 1u;
            const uint64_t N = kPos ? Nk : l ? ((uint64_t)code >> (L - l)) & pmask : 0ull;
            if (N != curN) enter_node(ld_node(a.ntb + (kPos ? kpfx(N) : N)), q, t0, cnt, G0, G1, s_words, s_wpre, s_seg, &s_nseg, sa, zs, R1a), curN = N;
            const uint32_t slot = b ? sa + zs + (r1 - R1a) : sa + ((q - r1) - (sa - R1a));
            bad = bad || slot >= (uint32_t)T;
            s_stage[min(slot, (uint32_t)T - 1u)] = (EO)code;
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
  WT_GLOBAL char* outb = a.out;

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
        if (len) nch = (uint32_t)(((d + len - 1) * sizeof(EO) >> 4) - ((d * sizeof(EO)) >> 4) + 1);
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
        const uint64_t db = d * sizeof(EO), de = (d + len) * sizeof(EO);
        chunk = (db >> 4) + (c - s_cp[lo]);
        const uint64_t cb = chunk << 4;
        const uint64_t blo = max(db, cb), bhi = min(de, cb + 16);
        const uint32_t src = slot0 * (uint32_t)sizeof(EO) + (uint32_t)(blo - db);  // LDS byte of blo
        if (blo == cb && bhi == cb + 16) {
          const uint32_t dw = src >> 2, sh = src & 3u;
          const uint32_t x0 = st32[dw], x1 = st32[dw + 1], x2 = st32[dw + 2], x3 = st32[dw + 3],
                         x4 = st32[dw + 4];
          uint4 y;
          y.x = __builtin_amdgcn_alignbyte(x1, x0, sh);
          y.y = __builtin_amdgcn_alignbyte(x2, x1, sh);
          y.z = __builtin_amdgcn_alignbyte(x3, x2, sh);
          y.w = __builtin_amdgcn_alignbyte(x4, x3, sh);
          st16(outb + cb, y);
          nb1 = vec_count_bit<EO>(y, nbsh);
        } else {
          const uint32_t s0 = src / (uint32_t)sizeof(EO);
          WT_GLOBAL EO* oe = pcast<EO>(outb);
          const uint64_t e0 = blo / sizeof(EO), e1 = bhi / sizeof(EO);
          for (uint64_t e = e0; e < e1; ++e) {
            const EO v = s_stage[s0 + (uint32_t)(e - e0)];
            oe[e] = v;
            nb1 += ((uint32_t)v >> nbsh) & 1u;
          }
        }
      }
      const uint64_t dt = (chunk << 4) / ((uint64_t)TO::T * sizeof(EO));
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
        const uint64_t N = kPos ? knum(j) : l ? ((uint64_t)code >> (L - l)) & pmask : 0ull;
        if (N != curN) {
          const NodeB nb = ld_node(a.ntb + (kPos ? kpfx(N) : N));
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
          pcast<EO>(outb)[dest] = (EO)code;
          nbit = (code >> nbsh) & 1u;
        }
      }
      count_next(__ballot(cont), dest >> TO::TSHIFT, nbit, lane, cur_tile, cur_c, a.cnt_next, 0u);
    }
  }
  if (lane == 0 && cur_c) atomic_add_u64(a.cnt_next + cur_tile, cur_c);
  // a slot outside the tile (clamped above so LDS stays intact) is an internal error: reported, not hidden
  if (__ballot(bad) != 0 && lane == 0 && a.err)
    (void)__hip_atomic_fetch_or(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
}  // namespace wt
