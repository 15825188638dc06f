// Internal definitions shared by the build kernels, the query kernels and the C ABI.
// gfx950 (CDNA4): wave64, 160 KB LDS per CU, 128-byte L2 lines.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wt.h"

namespace wt {

constexpr uint32_t kL1Bits = 65536;  // L1 block (Section 4.1): u64 count per 65536 bits
constexpr uint32_t kL1Shift = 16;
constexpr uint64_t kNoNode = ~0ull;

// Per-level layout and counts, in device memory (written by the build kernels).
struct LevelMeta {
  uint64_t n;        // elements at this level (n_l)
  uint64_t ones;     // ones at this level
  uint64_t bits;     // word offset of the level in the bit pool
  uint64_t l1;       // entry offset in the L1 pool
  uint64_t l2;       // entry offset in the L2 pool
  uint64_t smp;      // entry offset in the sample pool
  uint64_t smp_cap;  // sample slots of this level: ones grow from the front, zeros from the back
  uint64_t pad;
};

// Node of the query table, indexed by code prefix (heap order: level l at [2^l - 1, 2^(l+1) - 1)).
struct NodeQ {
  uint64_t start;  // first position of the node in its level (= cumulative histogram at its first symbol)
  uint64_t r0;     // rank0 of the level at `start` (precomputed node-start rank)
};

// Node of the build table (same indexing).
struct NodeB {
  uint64_t start, end;  // [start, end) positions of the node in its level
  uint64_t off0, off1;  // level-(l+1) position of an element = off_b + rank_b(position)
};

// Presence word of an extracted alphabet: bit v mod 64 of word v / 64 is set when value v occurs;
// `pre` counts the values present in every earlier word (the code of the first value of this word).
struct AWord {
  uint64_t bits;
  uint32_t pre;
  uint32_t pad;
};

struct TreeDev {
  uint64_t* bits;
  uint64_t* L1;
  uint16_t* L2;
  uint64_t* smp;
  NodeQ* nodes;
  uint64_t* cum;  // sigma + 1
  LevelMeta* meta;
  uint64_t* wstart;  // wavelet matrix: first position of every symbol's run below the last level; tree: NULL
  // Huffman-shaped tree (NULL otherwise): per symbol len << 32 | left-aligned code; the symbol of
  // every rank; per depth d, F_d << 32 | I_d (the internal nodes of depth d are the prefixes [0, I_d),
  // the leaf with prefix p >= I_d is rank F_d + p - I_d)
  const uint64_t* hcode;
  const uint32_t* hsym;
  const uint64_t* hdepth;
};

// ---- small device helpers ----

__device__ __forceinline__ uint32_t popc64(uint64_t x) { return (uint32_t)__popcll(x); }

// Largest power of two strictly below x (x >= 2).
__host__ __device__ __forceinline__ uint64_t pow2_below(uint64_t x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return 1ull << (63 - __clzll(x - 1));
#else
  return 1ull << (63 - __builtin_clzll(x - 1));
#endif
}

// Bit position (0..63) of the r-th set bit of x, r in [1, popc(x)]: popcount bisection
// over halves of the word (Section 5.4, in-word select).
__device__ __forceinline__ uint32_t select_in_word(uint64_t x, uint32_t r) {
  uint32_t pos = 0;
  uint32_t c = __popc((uint32_t)x);
  if (r > c) { r -= c; x >>= 32; pos += 32; }
  c = __popc((uint32_t)x & 0xFFFFu);
  if (r > c) { r -= c; x >>= 16; pos += 16; }
  c = __popc((uint32_t)x & 0xFFu);
  if (r > c) { r -= c; x >>= 8; pos += 8; }
  c = __popc((uint32_t)x & 0xFu);
  if (r > c) { r -= c; x >>= 4; pos += 4; }
  c = __popc((uint32_t)x & 0x3u);
  if (r > c) { r -= c; x >>= 2; pos += 2; }
  c = (uint32_t)x & 1u;
  if (r > c) pos += 1;
  return pos;
}

// Reduced-tree code of symbol c < sigma (Section 5.1, Algorithm 3), left-aligned to L bits,
// and its length. For sigma = sum of powers 2^a1 > 2^a2 > ... > 2^ak the tree is a spine of
// k - 1 right steps whose left children are complete subtrees of sizes 2^a1, 2^a2, ...; the last
// right child is the complete subtree of size 2^ak. With h the highest bit where c and sigma
// differ, c lies in the subtree of size 2^h reached after popc(sigma >> (h+1)) right steps.
__host__ __device__ __forceinline__ uint32_t encode_sym(uint32_t c, uint32_t sigma, uint32_t L, uint32_t pow2,
                                                        uint32_t* len_out) {
  if (pow2) {
    *len_out = L;
    return c;
  }
#if defined(__HIP_DEVICE_COMPILE__)
  const uint32_t h = 31u - (uint32_t)__clz(c ^ sigma);
  const uint32_t j1 = (uint32_t)__popc(sigma >> (h + 1));
#else
  const uint32_t h = 31u - (uint32_t)__builtin_clz(c ^ sigma);
  const uint32_t j1 = (uint32_t)__builtin_popcount(sigma >> (h + 1));
#endif
  const uint32_t last = (sigma & ((1u << h) - 1u)) == 0u;  // h is the lowest set bit of sigma
  const uint32_t len = j1 + (last ? 0u : 1u) + h;
  const uint32_t code = (((1u << j1) - 1u) << (len - j1)) | (c & ((1u << h) - 1u));
  *len_out = len;
  return code << (L - len);
}

}  // namespace wt
