// Device parts of the queries shared by the plain and the learned query kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

constexpr int kQT = 256;

struct QArgs {
  TreeDev d;
  uint64_t n;
  uint32_t sigma, L, pow2, sshift;
};

// rank1 of the level at position i (0 <= i <= n_l) and the bit at i (meaningful for i < n_l).
// kMask: load only the 16-byte vectors of the L2 block up to the one holding word i / 64 (a lane's
// loads past it are masked off and cost no address cycles; faster for rank, not for access).
template <int L2S, bool kMask = false>
__device__ __forceinline__ uint64_t rank1_at(const TreeDev& d, const LevelMeta& m, uint64_t i, uint32_t& bit) {
  constexpr int L2W = (1 << L2S) / 64;
  const uint64_t j = i >> L2S;
  uint64_t r = d.L1[m.l1 + (i >> kL1Shift)] + d.L2[m.l2 + j];
  const uint64_t* blk = d.bits + m.bits + (j << (L2S - 6));
  const uint32_t wi = (uint32_t)(i >> 6) & (L2W - 1), bi = (uint32_t)i & 63u;
  uint64_t cur = 0;
  if constexpr (L2W <= 8) {
    uint64_t w[L2W];
#pragma unroll
    for (int k = 0; k < L2W / 2; ++k) {
      uint4 x = make_uint4(0u, 0u, 0u, 0u);
      if (!kMask || (uint32_t)(2 * k) <= wi) x = reinterpret_cast<const uint4*>(blk)[k];
      w[2 * k] = (uint64_t)x.x | ((uint64_t)x.y << 32);
      w[2 * k + 1] = (uint64_t)x.z | ((uint64_t)x.w << 32);
    }
#pragma unroll
    for (int k = 0; k < L2W; ++k) {
      r += ((uint32_t)k < wi) ? popc64(w[k]) : 0u;
      cur = ((uint32_t)k == wi) ? w[k] : cur;
    }
  } else {
    for (uint32_t k = 0; k < wi; ++k) r += popc64(blk[k]);
    cur = blk[wi];
  }
  r += popc64(cur & ((1ull << bi) - 1ull));
  bit = (uint32_t)(cur >> bi) & 1u;
  return r;
}

// Position of the k-th bit equal to b (1 <= k <= count of b) of the level (Algorithm 2).
// Offset of the kk-th bit equal to b (kk >= 1, present) inside the L2 block whose words start at
// wp: the word holding it is found by popcounts over 16-byte loads, then one in-word select after
// the scan (the select runs once for the whole wave). Blocks up to 512 bits are loaded at once (one
// memory round trip: the traversal is bound by its chain of dependent loads); larger ones are
// scanned a vector at a time, a lane leaving at the vector that holds its bit (also the form for
// kAll = false, which needs fewer registers).
template <int L2S, bool kAll = true>
__device__ __forceinline__ uint32_t block_select(const uint64_t* __restrict__ wp, uint32_t b, uint32_t kk) {
  constexpr int L2W = (1 << L2S) / 64;
  const uint4* vp = reinterpret_cast<const uint4*>(wp);  // the block is 64-byte aligned
  uint64_t sel = 0;
  uint32_t wsel = 0;
  if constexpr (kAll && L2W <= 8) {
    uint4 x[L2W / 2];
#pragma unroll
    for (int v = 0; v < L2W / 2; ++v) x[v] = vp[v];
    bool done = false;
#pragma unroll
    for (int v = 0; v < L2W / 2; ++v) {
      const uint64_t pair[2] = {((uint64_t)x[v].y << 32) | x[v].x, ((uint64_t)x[v].w << 32) | x[v].z};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint64_t word = b ? pair[h] : ~pair[h];
        const uint32_t pc = popc64(word);
        const bool hit = !done && kk <= pc;
        sel = hit ? word : sel;
        wsel = hit ? (uint32_t)(2 * v + h) : wsel;
        kk -= (!done && !hit) ? pc : 0u;
        done = done || hit;
      }
    }
  } else {
#pragma unroll 1
    for (int v = 0; v < L2W / 2; ++v) {
      const uint4 x = vp[v];
      const uint64_t pair[2] = {((uint64_t)x.y << 32) | x.x, ((uint64_t)x.w << 32) | x.z};
      bool done = false;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint64_t word = b ? pair[h] : ~pair[h];
        const uint32_t pc = popc64(word);
        sel = word;
        wsel = (uint32_t)(2 * v + h);
        if (kk <= pc) {
          done = true;
          break;
        }
        kk -= pc;
      }
      if (done) break;
    }
  }
  return 64u * wsel + select_in_word(sel, kk);
}

// kLine: resolve the L2 search on the first L2 counts in registers before the binary search, and
// load the found block's words at once (faster; the form without either needs fewer registers).
template <int L2S, bool kLine = true>
__device__ __forceinline__ uint64_t select_at(const TreeDev& d, const LevelMeta& m, uint32_t b, uint64_t k,
                                              uint32_t sshift) {
  constexpr uint64_t kPer = kL1Bits >> L2S;  // L2 blocks per L1 block
  const uint64_t nl = m.n;
  const uint64_t cntb = b ? m.ones : nl - m.ones;
  // samples bound the position: the (si s)-th and ((si+1) s)-th bit equal to b
  const uint64_t si = k >> sshift;
  uint64_t lo_pos = 0, hi_pos = nl;
  if (si) lo_pos = b ? d.smp[m.smp + si - 1] : d.smp[m.smp + m.smp_cap - si];
  if (((si + 1) << sshift) <= cntb) hi_pos = b ? d.smp[m.smp + si] : d.smp[m.smp + m.smp_cap - si - 1];
  const uint64_t nL1 = (nl + kL1Bits - 1) >> kL1Shift;
  const uint64_t* L1 = d.L1 + m.l1;
  const uint16_t* L2 = d.L2 + m.l2;
  // largest L1 block whose count of b before it is < k
  uint64_t blo = lo_pos >> kL1Shift, bhi = min(hi_pos >> kL1Shift, nL1 - 1);
  while (blo < bhi) {
    const uint64_t mid = (blo + bhi + 1) >> 1;
    const uint64_t cb = b ? L1[mid] : (mid << kL1Shift) - L1[mid];
    if (cb < k) blo = mid;
    else bhi = mid - 1;
  }
  const uint64_t blk = blo;
  k -= b ? L1[blk] : (blk << kL1Shift) - L1[blk];
  // largest L2 block of that L1 block whose count of b since the L1 start is < k; the samples
  // also bound the L2 range. The search starts on the aligned line of L2 counts holding jlo (64
  // entries, inside the L1 block), read at once: the counts are non-decreasing, so the blocks below
  // k form a prefix of the range and are counted in registers; only a range that leaves the line
  // continues with the binary search over the remaining entries.
  const uint64_t nL2 = (nl + (1ull << L2S) - 1) >> L2S;
  const uint64_t jb = blk * kPer;
  uint64_t jlo = max(jb, lo_pos >> L2S);
  uint64_t jhi = min(min(jb + kPer, nL2) - 1, hi_pos >> L2S);
  bool resolved = false;  // k already counted from the start of block jlo
  if constexpr (kLine) {
    // GN entries read at once (whole 16-byte vectors) from the vector holding jlo, moved down when
    // needed so the group stays inside the L1 block. Over an L1 block the count of b before each L2
    // block, y_e, never decreases, and it is below k at jlo (so at every entry from the group start
    // to jlo) and not below k past jhi (past the next sample): the blocks below k are a prefix of
    // the group, counted in registers. Only the level's last group can hold entries past its end,
    // which are masked; a prefix that fills the group continues with the binary search.
    constexpr uint32_t GN = L2S <= 9 ? 32u : 16u;
    static_assert(GN % 8 == 0 && GN <= kPer, "group inside an L1 block");
    const uint64_t gbase = min(jlo & ~7ull, jb + kPer - GN);
    const uint4* gp = reinterpret_cast<const uint4*>(L2 + gbase);
    const int32_t Ki = (int32_t)k;  // at most 2^16 (counted from the L1 block start)
    const int32_t sgn = b ? 1 : -1, step = b ? 0 : (1 << L2S);
    int32_t off = b ? 0 : (int32_t)((gbase - jb) << L2S);  // bits from the L1 start (b = 0)
    // entries past ehi count only inside the level (the last group of a level may hold padding)
    const uint32_t ehi = gbase + GN <= nL2 ? GN - 1 : (uint32_t)(jhi - gbase);
    uint32_t below = 0, seen = 0;
    int32_t ylast = 0;  // y of the last block below k
    // two vectors at a time: a lane stops at the first pair that ends the prefix or reaches jhi
#pragma unroll 1
    for (uint32_t v = 0; v < GN / 8; v += 2) {
      const uint4 xa = gp[v], xb = gp[v + 1];
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        const uint4 x = e < 8 ? xa : xb;
        const uint32_t ee = e & 7;
        const uint32_t dw = ee < 4 ? (ee < 2 ? x.x : x.y) : (ee < 6 ? x.z : x.w);
        const int32_t l2v = (int32_t)((dw >> ((ee & 1) * 16)) & 0xFFFFu);
        const int32_t y = off + sgn * l2v;
        const bool lt = v * 8 + e <= ehi && y < Ki;
        below += lt ? 1u : 0u;
        ylast = lt ? y : ylast;
        off += step;
      }
      seen += 16;
      if (below < seen || gbase + seen - 1 >= jhi) break;
    }
    const uint64_t last = gbase + below - 1;  // below >= 1
    if (last < gbase + seen - 1 || last >= jhi) {
      // resolved inside the group: y at that block is the count of b before it (from the L1 start)
      k -= (uint64_t)ylast;
      jhi = last;
      resolved = true;
    }
    jlo = last;
  }
  while (jlo < jhi) {
    const uint64_t mid = (jlo + jhi + 1) >> 1;
    const uint64_t cb = b ? (uint64_t)L2[mid] : ((mid - jb) << L2S) - L2[mid];
    if (cb < k) jlo = mid;
    else jhi = mid - 1;
  }
  if (!resolved) k -= b ? (uint64_t)L2[jlo] : ((jlo - jb) << L2S) - L2[jlo];
  return (jlo << L2S) + block_select<L2S, kLine>(d.bits + m.bits + (jlo << (L2S - 6)), b, (uint32_t)k);
}

// 64-bit value of the wave's first active lane.
__device__ __forceinline__ uint64_t first_lane_u64(uint64_t v) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
         (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
}

// Node-table entry `idx`. The lanes of a wave in a binned batch are mostly at the same node (always
// at the upper levels): then the entry is read through a wave-uniform address (scalar load).
__device__ __forceinline__ NodeQ node_at(const NodeQ* __restrict__ nodes, uint64_t idx) {
  const uint64_t i0 = first_lane_u64(idx);
  if (__ballot(idx != i0) == 0) return nodes[i0];
  return nodes[idx];
}

// Algorithm 5 (top-down): the bit of the element picks the child; its position in the child is its
// rank among the equal bits of the node. Stops once the node covers at most two symbols.
// Positions >= n give 0xFFFFFFFF.
template <int L2S>
__device__ __forceinline__ uint32_t access_one(const QArgs& a, const LevelMeta* meta, uint64_t i) {
  if (i >= a.n) return 0xFFFFFFFFu;
  uint32_t s = 0, e = a.sigma;
  uint64_t p = 0, x = i;
  NodeQ nd = node_at(a.d.nodes, 0);
  for (uint32_t l = 0; l < a.L; ++l) {
    const uint32_t width = e - s;
    const LevelMeta& m = meta[l];
    const uint64_t y = nd.start + x;
    if (width <= 2) {
      if (width == 2) s += (uint32_t)(a.d.bits[m.bits + (y >> 6)] >> (y & 63)) & 1u;
      break;
    }
    // the two children are adjacent entries of the next level: load both with this level's reads
    NodeQ c0 = nd, c1 = nd;
    if (l + 1 < a.L) {
      const uint64_t ci = (2ull << l) - 1 + 2 * p;
      c0 = a.d.nodes[ci];
      c1 = a.d.nodes[ci + 1];
    }
    uint32_t bit;
    const uint64_t r0 = y - rank1_at<L2S>(a.d, m, y, bit);
    const uint32_t half = (uint32_t)pow2_below(width);
    if (!bit) {
      x = r0 - nd.r0;
      e = s + half;
      p = 2 * p;
      nd = c0;
    } else {
      x = x - (r0 - nd.r0);
      s += half;
      p = 2 * p + 1;
      nd = c1;
    }
  }
  return s;
}

// Algorithm 6 (top-down along the symbol's path): the count of the symbol's side before the position.
// Positions > n give UINT64_MAX; symbols >= sigma give 0.
template <int L2S>
__device__ __forceinline__ uint64_t rank_one(const QArgs& a, const LevelMeta* meta, uint32_t c, uint64_t i) {
  if (i > a.n) return ~0ull;
  if (c >= a.sigma) return 0;
  uint32_t s = 0, e = a.sigma;
  uint64_t p = 0, x = i;
  NodeQ nd = node_at(a.d.nodes, 0);
  for (uint32_t l = 0; l < a.L; ++l) {
    if (e - s <= 1 || x == 0) break;
    const uint64_t y = nd.start + x;
    const uint32_t split = s + (uint32_t)pow2_below(e - s);
    const bool right = c >= split;
    // the symbol fixes the next node: load its entry with this level's reads
    NodeQ nx = nd;
    if (l + 1 < a.L) nx = a.d.nodes[(2ull << l) - 1 + 2 * p + (right ? 1 : 0)];
    uint32_t bit;
    const uint64_t r0 = y - rank1_at<L2S, true>(a.d, meta[l], y, bit);
    if (!right) {
      x = r0 - nd.r0;
      e = split;
      p = 2 * p;
    } else {
      x = x - (r0 - nd.r0);
      s = split;
      p = 2 * p + 1;
    }
    nd = nx;
  }
  return x;
}

// Algorithms 7 and 8 (bottom-up from the symbol's leaf): the k-th occurrence inside the current node
// is the (rank-at-node-start + k)-th bit equal to the node's side in the parent level.
// k = 0 gives UINT64_MAX; k > count(c) or c >= sigma gives n.
template <int L2S>
__device__ __forceinline__ uint64_t select_one(const QArgs& a, const LevelMeta* meta, uint32_t c, uint64_t k) {
  if (k == 0) return ~0ull;
  if (c >= a.sigma) return a.n;
  if (k > a.d.cum[c + 1] - a.d.cum[c]) return a.n;
  if (a.L == 0) return k - 1;
  uint32_t len;
  const uint32_t code = encode_sym(c, a.sigma, a.L, a.pow2, &len);
  uint64_t r = k;
  for (int l = (int)len - 1; l >= 0; --l) {
    const uint64_t p = l ? (uint64_t)(code >> (a.L - l)) : 0ull;
    const uint32_t b = (code >> (a.L - 1 - l)) & 1u;
    const NodeQ nd = node_at(a.d.nodes, (1ull << l) - 1 + p);
    const uint64_t target = b ? (nd.start - nd.r0) + r : nd.r0 + r;
    const uint64_t at = select_at<L2S>(a.d, meta[l], b, target, a.sshift);
    r = at - nd.start + 1;
  }
  return r - 1;
}

// ---- Huffman-shaped tree: the same levels and node table, over canonical prefix codes of different
// lengths (longer codes on the left). A code's bits pick the children; the traversal of an element
// ends where its prefix becomes a leaf: at depth d the internal nodes are the prefixes [0, I_d), and
// the leaf with prefix p >= I_d is the symbol of rank F_d + p - I_d (both per depth in hdepth).

// access: top-down until the prefix read so far is a leaf; where both children of the node are
// leaves the bit alone decides (no rank).
template <int L2S>
__device__ __forceinline__ uint32_t huff_access_one(const QArgs& a, const LevelMeta* meta, uint64_t i) {
  if (i >= a.n) return 0xFFFFFFFFu;
  if (a.L == 0) return a.d.hsym[0];
  uint64_t p = 0, x = i;
  NodeQ nd = node_at(a.d.nodes, 0);
  for (uint32_t l = 0; l < a.L; ++l) {
    const LevelMeta& m = meta[l];
    const uint64_t dep = a.d.hdepth[l + 1];
    const uint64_t I = (uint32_t)dep, F = dep >> 32;
    const uint64_t y = nd.start + x;
    uint32_t bit;
    if (2 * p >= I) {  // both children are leaves
      bit = (uint32_t)(a.d.bits[m.bits + (y >> 6)] >> (y & 63)) & 1u;
      p = 2 * p + bit;
      return a.d.hsym[F + p - I];
    }
    const uint64_t r0 = y - rank1_at<L2S>(a.d, m, y, bit);
    p = 2 * p + bit;
    if (p >= I) return a.d.hsym[F + p - I];
    x = bit ? x - (r0 - nd.r0) : r0 - nd.r0;
    nd = node_at(a.d.nodes, (2ull << l) - 1 + p);
  }
  return 0xFFFFFFFFu;  // not reached: every code ends by level L
}

// rank: top-down along the symbol's code (as rank_one, the code bits instead of the split rule).
template <int L2S>
__device__ __forceinline__ uint64_t huff_rank_one(const QArgs& a, const LevelMeta* meta, uint32_t c, uint64_t i) {
  if (i > a.n) return ~0ull;
  if (c >= a.sigma) return 0;
  const uint64_t hc = a.d.hcode[c];
  const uint32_t len = (uint32_t)(hc >> 32), code = (uint32_t)hc;
  if (len == 0) return a.d.cum[c + 1] > a.d.cum[c] ? i : 0;  // the lone symbol of the tree, or absent
  uint64_t p = 0, x = i;
  NodeQ nd = node_at(a.d.nodes, 0);
  for (uint32_t l = 0; l < len; ++l) {
    if (x == 0) break;
    const uint32_t b = (code >> (a.L - 1 - l)) & 1u;
    const uint64_t y = nd.start + x;
    NodeQ nx = nd;
    if (l + 1 < len) nx = a.d.nodes[(2ull << l) - 1 + 2 * p + b];
    uint32_t bit;
    const uint64_t r0 = y - rank1_at<L2S, true>(a.d, meta[l], y, bit);
    x = b ? x - (r0 - nd.r0) : r0 - nd.r0;
    p = 2 * p + b;
    nd = nx;
  }
  return x;
}

// select: bottom-up from the symbol's leaf (as select_one, the code and its length from the table).
template <int L2S>
__device__ __forceinline__ uint64_t huff_select_one(const QArgs& a, const LevelMeta* meta, uint32_t c, uint64_t k) {
  if (k == 0) return ~0ull;
  if (c >= a.sigma) return a.n;
  if (k > a.d.cum[c + 1] - a.d.cum[c]) return a.n;
  const uint64_t hc = a.d.hcode[c];
  const uint32_t len = (uint32_t)(hc >> 32), code = (uint32_t)hc;
  uint64_t r = k;
  for (int l = (int)len - 1; l >= 0; --l) {
    const uint64_t p = l ? (uint64_t)(code >> (a.L - l)) : 0ull;
    const uint32_t b = (code >> (a.L - 1 - l)) & 1u;
    const NodeQ nd = node_at(a.d.nodes, (1ull << l) - 1 + p);
    const uint64_t target = b ? (nd.start - nd.r0) + r : nd.r0 + r;
    const uint64_t at = select_at<L2S>(a.d, meta[l], b, target, a.sshift);
    r = at - nd.start + 1;
  }
  return r - 1;
}

// ---- wavelet matrix: every level holds all n elements; an element at position p of level l with bit b
// is at rank0_l(p) (b = 0) or zeros_l + rank1_l(p) (b = 1) in level l + 1, and its bit at level l is
// bit L-1-l of its symbol. One binary rank or select per level, no node table.

// access: the bits read top-down spell the symbol.
template <int L2S>
__device__ __forceinline__ uint32_t wm_access_one(const QArgs& a, const LevelMeta* meta, uint64_t i) {
  if (i >= a.n) return 0xFFFFFFFFu;
  uint32_t c = 0;
  uint64_t p = i;
  for (uint32_t l = 0; l < a.L; ++l) {
    const LevelMeta& m = meta[l];
    uint32_t bit;
    const uint64_t r1 = rank1_at<L2S>(a.d, m, p, bit);
    c = (c << 1) | bit;
    p = bit ? (m.n - m.ones) + r1 : p - r1;
  }
  return c;
}

// rank: follow position i down the symbol's bits; below the last level the occurrences of c before i
// end just before the followed position, and c's run starts at wstart[c].
template <int L2S>
__device__ __forceinline__ uint64_t wm_rank_one(const QArgs& a, const LevelMeta* meta, uint32_t c, uint64_t i) {
  if (i > a.n) return ~0ull;
  if (c >= a.sigma) return 0;
  const uint64_t base = a.d.wstart[c];
  uint64_t p = i;
  for (uint32_t l = 0; l < a.L; ++l) {
    const LevelMeta& m = meta[l];
    const uint32_t b = (c >> (a.L - 1 - l)) & 1u;
    uint32_t bit;
    const uint64_t r1 = rank1_at<L2S, true>(a.d, m, p, bit);
    p = b ? (m.n - m.ones) + r1 : p - r1;
  }
  return p - base;
}

// select: the k-th occurrence sits at wstart[c] + k - 1 below the last level; going up, a position p of
// level l + 1 is the (p + 1)-th zero of level l (b = 0) or its (p - zeros_l + 1)-th one (b = 1).
template <int L2S>
__device__ __forceinline__ uint64_t wm_select_one(const QArgs& a, const LevelMeta* meta, uint32_t c, uint64_t k) {
  if (k == 0) return ~0ull;
  if (c >= a.sigma) return a.n;
  if (k > a.d.cum[c + 1] - a.d.cum[c]) return a.n;
  if (a.L == 0) return k - 1;
  uint64_t p = a.d.wstart[c] + k - 1;
  for (int l = (int)a.L - 1; l >= 0; --l) {
    const LevelMeta& m = meta[l];
    const uint32_t b = (c >> (a.L - 1 - l)) & 1u;
    p = select_at<L2S>(a.d, m, b, b ? p - (m.n - m.ones) + 1 : p + 1, a.sshift);
  }
  return p;
}

// Logical block of a grid-stride query launch. Workgroups go to the kXcd dies (XCDs, each with its
// own L2) round-robin, so launch block g runs on die g mod kXcd; logical block x * G/kXcd + g/kXcd
// gives every die a contiguous 1/kXcd of each grid-wide window of the batch. With a binned batch the
// queries a die has in flight are then neighbours, and their lines are shared in that die's L2.
constexpr uint32_t kXcd = 8;
__device__ __forceinline__ uint64_t xcd_block() {
  const uint32_t g = gridDim.x, b = blockIdx.x;
  if (g % kXcd) return b;
  return (uint64_t)(b % kXcd) * (g / kXcd) + b / kXcd;
}

// Binning key of a query: access and rank, the position; select, the position of the wanted
// occurrence below the last level: in a tree, its rank in symbol order (cum[c] + k - 1), in a wavelet
// matrix wstart[c] + k - 1. Invalid queries key n.
__device__ __forceinline__ uint64_t sort_key(const QArgs& a, int kind, uint32_t c, uint64_t x) {
  if (kind != 2) return min(x, a.n);
  if (x == 0 || c >= a.sigma) return a.n;
  const uint64_t lo = a.d.cum[c], cnt = a.d.cum[c + 1] - lo;
  return x > cnt ? a.n : (a.d.wstart ? a.d.wstart[c] : lo) + x - 1;
}

// Threads per block of the access / rank / select traversal kernels: binned batches use kQB (the
// in-block reorder below works over the whole block), unbinned ones kQT (small batches spread over
// more CUs).
#ifndef WT_QB
#define WT_QB 1024
#endif
constexpr uint32_t kQB = WT_QB;
constexpr uint32_t qb_bits(uint32_t qb) { return qb == 1024 ? 10 : qb == 512 ? 9 : 8; }
static_assert((1u << qb_bits(kQB)) == kQB, "traversal block: 256, 512 or 1024 threads");

// A binned launch takes QB consecutive slots per block and round, which lie in one or two buckets.
// A counting sort in LDS by the next qb_bits(QB) key bits below the bucket gives each wave queries
// whose answers are close together, so the lanes of one load instruction share lines (not only the
// caches do); the larger the block, the narrower the key range of a wave.
template <uint32_t QB>
struct LocalOrder {
  uint32_t cnt[QB];  // one sub-bucket counter per thread
  uint32_t wsum[QB / 64];
  uint32_t id[QB];
  uint32_t sym[QB];
  uint64_t arg[QB];
};

// A query of a binned batch, written at its slot by the binning: its index in the batch and its
// arguments (so the traversal reads its slots in order instead of gathering through a permutation).
struct SQ {
  uint32_t id;
  uint32_t sym;
  uint64_t arg;
};

template <int KIND, uint32_t QB>
__device__ __forceinline__ bool local_order(const QArgs& a, const SQ* __restrict__ sq, uint64_t q, uint64_t j,
                                            uint32_t subshift, LocalOrder<QB>& L, uint32_t& jj, uint32_t& c,
                                            uint64_t& x) {
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t t = threadIdx.x;
  uint32_t id = kNone, cc = 0, sub = QB - 1;
  uint64_t xx = 0;
  if (j < q) {
    const SQ r = sq[j];
    id = r.id;
    xx = r.arg;
    cc = r.sym;
    sub = (uint32_t)(sort_key(a, KIND, cc, xx) >> subshift) & (QB - 1);
  }
  L.cnt[t] = 0;
  __syncthreads();
  const uint32_t r = atomicAdd(&L.cnt[sub], 1u);
  __syncthreads();
  const uint32_t v = L.cnt[t], lane = t & 63u;
  uint32_t inc = v;
#pragma unroll
  for (uint32_t off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) L.wsum[t >> 6] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (uint32_t w = 0; w < (t >> 6); ++w) pre += L.wsum[w];
  L.cnt[t] = pre + inc - v;
  __syncthreads();
  const uint32_t slot = L.cnt[sub] + r;
  L.id[slot] = id;
  L.sym[slot] = cc;
  L.arg[slot] = xx;
  __syncthreads();
  jj = L.id[t];
  c = L.sym[t];
  x = L.arg[t];
  return jj != kNone;
}

__device__ __forceinline__ void load_meta(const QArgs& a, LevelMeta* s_meta) {
  if (threadIdx.x < a.L) s_meta[threadIdx.x] = a.d.meta[threadIdx.x];
  __syncthreads();
}

inline QArgs make_args(const wt_tree* t) {
  QArgs a;
  a.d = t->dev;
  a.n = t->n;
  a.sigma = (uint32_t)t->sigma;
  a.L = t->L;
  a.pow2 = t->pow2;
  uint32_t sh = 0;
  while ((1u << sh) < t->srate) ++sh;
  a.sshift = sh;
  return a;
}

// Per-kernel timing of query calls (wt_query_profiling): HIP events recorded around every kernel of a
// call on its stream, kept per thread until wt_query_profile reads them.
void qprof_begin(const char* name, hipStream_t st);
void qprof_end(hipStream_t st);

// Locality binning of a query batch (wt_query.hip): on success with `binned`, sq holds the queries in
// bucket order (slot j runs query sq[j].id with the arguments stored beside it); the caller frees
// `block` (stream-ordered) after its traversal. With `pre` given (sort_batch_bytes(q) bytes of device
// memory), the buffers are carved from it, nothing is allocated and `block` stays NULL.
struct SortBufs {
  char* block = nullptr;
  uint32_t* cnt;
  SQ* sq;
  uint32_t subshift = 0;  // key bits below the ones that order queries inside a block
};
wt_status sort_batch(const wt_tree* t, const QArgs& a, int kind, const uint32_t* sym, const uint64_t* arg, uint64_t q,
                     hipStream_t st, SortBufs& sb, bool& binned, char* pre = nullptr);
size_t sort_batch_bytes(uint64_t q);

// One batch of queries of one kind (0 access: u32 answers; 1 rank, 2 select: u64 answers) on st, with
// pre = NULL (buffers allocated) or query_scratch_bytes(q) bytes of device scratch (wt_query.hip).
size_t query_scratch_bytes(uint64_t q);
wt_status query_run(const wt_tree* t, int kind, const uint32_t* d_sym, const uint64_t* d_arg, uint64_t q, void* d_out,
                    hipStream_t st, char* pre);

// Counting sort of q queries by bucket id (ids[j] < 32768; wt_query.hip). scratch: sort_ids_bytes(q)
// bytes; tot: 32768 entries, left holding the exclusive start of every bucket; perm: the slot order.
size_t sort_ids_bytes(uint64_t q);
void sort_ids_enqueue(const uint16_t* ids, uint64_t q, char* scratch, uint32_t* tot, uint32_t* perm, hipStream_t st);
constexpr uint32_t kSortIdBins = 32768;

// Blocks of a traversal launch: at most 2^20 threads (grid-stride over the batch), a multiple of kXcd.
inline uint32_t query_grid(uint64_t q, uint32_t qb) {
  return (uint32_t)round_up(std::min<uint64_t>(ceil_div(q, qb), 4096 * kQT / qb), kXcd);
}

// Launch of KERNEL<L2S, QB, WM> for the tree's |L2| (WM: the wavelet-matrix traversal).
#define WT_DISPATCH_L2_SH(bits, QB, SH, KERNEL, ...)                                                              \
  switch (bits) {                                                                                                 \
    case 256: hipLaunchKernelGGL((KERNEL<8, QB, SH>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break;          \
    case 512: hipLaunchKernelGGL((KERNEL<9, QB, SH>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break;          \
    case 1024: hipLaunchKernelGGL((KERNEL<10, QB, SH>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break;        \
    default: hipLaunchKernelGGL((KERNEL<11, QB, SH>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break;          \
  }

#define WT_DISPATCH_L2(bits, QB, KERNEL, ...)                                                          \
  switch (bits) {                                                                                     \
    case 256: hipLaunchKernelGGL((KERNEL<8, QB>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break;   \
    case 512: hipLaunchKernelGGL((KERNEL<9, QB>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break;   \
    case 1024: hipLaunchKernelGGL((KERNEL<10, QB>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL((KERNEL<11, QB>), dim3(grid), dim3(QB), 0, st, __VA_ARGS__); break;   \
  }

}  // namespace wt
