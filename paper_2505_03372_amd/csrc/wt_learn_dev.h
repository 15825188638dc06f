// Query side of the learned select index: the compiled (piecewise-linear) form of a trained network
// and the select that corrects its prediction exactly, shared by the learned select kernel and the
// mixed-query kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "wt_internal.h"
#include "wt_query_dev.h"

namespace wt {

constexpr int kH = 16;           // hidden units
constexpr int kNP = 3 * kH + 1;  // parameters: w1[16], b1[16], w2[16], b2

// L2 blocks the correction's group starts below the predicted block (rounded down to a vector).
#ifndef WT_LEARN_LEAD
#define WT_LEARN_LEAD 6
#endif
#ifndef WT_LEARN_LEAD_EPS
#define WT_LEARN_LEAD_EPS 0
#endif
// form of the sampled search taken by waves whose lanes are on different models
#ifndef WT_LEARN_MIXED_LINE
#define WT_LEARN_MIXED_LINE true
#endif
constexpr uint64_t kLearnLead = WT_LEARN_LEAD;

// Query form of a trained model. With one input, the network is linear between the points where a
// hidden unit switches on or off (u = -b1_k / w1_k), so on [0, 1] it is exactly a piecewise-linear
// function with at most 16 switch points: they are stored ascending (unused: 2, above every input)
// with one (slope, intercept) pair per piece. A query loads the header and the switch points (the
// first 128-byte line) and one piece, instead of the 49 parameters. 256 bytes.
struct LearnQ {
  uint64_t start;  // node range [start, start + len) in level l
  uint64_t len;
  uint64_t rank0;  // count of side-b bits of level l before `start`
  int32_t eps;     // error budget in L2 blocks (max error + 2); -1: no model
  uint32_t side;   // b
  float cntf;      // bits equal to b inside the node, as float (the input scale)
  uint32_t npieces;
  float lenf;      // len as float (the output scale)
  uint32_t pad0;
  float knot[kH];
  float2 piece[kH + 1];  // (slope, intercept) of v(u) on [knot[s-1], knot[s])
  uint64_t pad1;
};
static_assert(sizeof(LearnQ) == 256, "query model size");
static_assert(offsetof(LearnQ, knot) % 16 == 0 && offsetof(LearnQ, knot) + sizeof(float) * kH <= 128,
              "header and switch points share the first line");

// v(u) of a compiled model, clamped to [0, 1]: the piece is the number of switch points <= u.
// kUniform: Q is at a wave-uniform address; every piece is read with it (scalar loads, no second
// dependent read) and the lane's piece is picked in registers.
template <bool kUniform = false>
__device__ __forceinline__ float pla_eval(const LearnQ& Q, float u) {
  const float4* kp = reinterpret_cast<const float4*>(Q.knot);
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kH / 4; ++i) {
    const float4 x = kp[i];
    s += (uint32_t)(x.x <= u) + (uint32_t)(x.y <= u) + (uint32_t)(x.z <= u) + (uint32_t)(x.w <= u);
  }
  float2 pc;
  if constexpr (kUniform) {
    pc = Q.piece[0];
#pragma unroll
    for (uint32_t i = 1; i <= (uint32_t)kH; ++i) {
      const float2 y = Q.piece[i];
      pc.x = s == i ? y.x : pc.x;
      pc.y = s == i ? y.y : pc.y;
    }
  } else {
    pc = Q.piece[s];
  }
  return fminf(fmaxf(fmaf(pc.x, u, pc.y), 0.f), 1.f);
}

// Count of side-b bits of a level before position x (x a multiple of the L2 block, x <= n_l).
template <int L2S>
__device__ __forceinline__ uint64_t count_before(const TreeDev& d, const LevelMeta& m, uint32_t b, uint64_t x) {
  const uint64_t r1 = d.L1[m.l1 + (x >> kL1Shift)] + d.L2[m.l2 + (x >> L2S)];
  return b ? r1 : x - r1;
}

// Position of the j-th (1-based, node-local) side-b bit of the node of model Q at level m.
// GS: log2 of the L2 counts read at once around the prediction.
template <int L2S, int GS, bool kUniform = false>
__device__ __forceinline__ uint64_t select_learned_at(const TreeDev& d, const LevelMeta& m, const LearnQ& Q,
                                                      uint64_t j, uint32_t sshift) {
  const uint32_t b = Q.side;
  const uint64_t T = Q.rank0 + j;  // global target among the side-b bits of the level
  if (Q.eps < 0) return select_at<L2S, false>(d, m, b, T, sshift);
  const float v = pla_eval<kUniform>(Q, ((float)j - 0.5f) / Q.cntf);
  const uint64_t start = Q.start, end = Q.start + Q.len;
  const uint64_t guess = min(start + (uint64_t)(v * Q.lenf), end - 1);  // FP32: a few positions off at most
  const uint64_t Blo = start >> L2S, Bhi = (end - 1) >> L2S;
  const uint64_t B0 = guess >> L2S;
  const uint64_t budget = (uint64_t)Q.eps;
  // largest B in [Blo, Bhi] with count_before(B) < T; count_before(Blo) <= rank0 < T always.
  // First look at the group of GN L2 counts starting a little below B0 (whole 16-byte vectors; it may
  // cross into the next L1 block, whose vectors add the difference of the two L1 counts): the counts
  // never decrease, so the blocks below the target form a prefix of the group.
  constexpr uint32_t GN = 1u << GS;
  constexpr uint32_t kPerShift = kL1Shift - L2S;  // log2 of the L2 blocks per L1 block
  static_assert(GN <= (1u << kPerShift), "a group crosses at most one L1 boundary");
#if WT_LEARN_LEAD_EPS
  const uint64_t lead = min<uint64_t>((uint64_t)Q.eps, kLearnLead);
#else
  const uint64_t lead = kLearnLead;
#endif
  const uint64_t gbase = (B0 > lead ? B0 - lead : 0ull) & ~7ull;
  const uint64_t glo = max(gbase, Blo), ghi = min(gbase + GN - 1, Bhi);
  const uint64_t la = gbase >> kPerShift;
  const uint64_t l1v = d.L1[m.l1 + la];
  const uint64_t l1n = d.L1[m.l1 + ((gbase + GN - 1) >> kPerShift)];  // == l1v inside one block
  const uint4* gp = reinterpret_cast<const uint4*>(d.L2 + m.l2 + gbase);
  // below(e) <=> count_before(gbase + e) < T, in 32-bit arithmetic with saturation:
  // y_e = l2 (b = 1) or e 2^L2S - l2 (b = 0), plus the L1 step in the next block, below <=> y_e < D
  int64_t D;
  if (b) D = (int64_t)min<uint64_t>(T - min(T, l1v), 1ull << 20);
  else {
    const uint64_t base0 = (gbase << L2S) - l1v;  // zeros before the group
    D = T > base0 ? (int64_t)min<uint64_t>(T - base0, 1ull << 20) : -(int64_t)min<uint64_t>(base0 - T, 1ull << 20);
  }
  const int32_t Di = (int32_t)D;
  const int32_t sgn = b ? 1 : -1, step = b ? 0 : (1 << L2S);
  // entries from `cross` on lie in the next L1 block: there y adds the L1 step (at most one L1 block
  // of bits)
  const int32_t dl1 = sgn * (int32_t)(l1n - l1v);
  const uint32_t cross = (uint32_t)min<uint64_t>(((la + 1) << kPerShift) - gbase, GN);
  // Blocks before the node are below the target (count_before(Blo) <= rank0 < T) and blocks past the
  // node are not, so only padding past the level's end is masked.
  const uint64_t nL2 = (m.n + (1ull << L2S) - 1) >> L2S;
  const uint32_t ehi = gbase + GN <= nL2 ? GN - 1 : (uint32_t)(ghi - gbase);
  int32_t off = 0;
  uint32_t below = 0, seen = 0;
  int32_t ylast = 0;  // y of the last block below the target
  // two vectors at a time: a lane stops at the first pair that ends the prefix or reaches ghi
#pragma unroll 1
  for (uint32_t v = 0; v < GN / 8; v += 2) {
    const uint4 xa = gp[v], xb = gp[v + 1];
    const int32_t adja = 8 * v < cross ? 0 : dl1, adjb = 8 * v + 8 < cross ? 0 : dl1;
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint4 x = e < 8 ? xa : xb;
      const uint32_t ee = e & 7;
      const uint32_t dw = ee < 4 ? (ee < 2 ? x.x : x.y) : (ee < 6 ? x.z : x.w);
      const int32_t l2v = (int32_t)((dw >> ((ee & 1) * 16)) & 0xFFFFu);
      const int32_t y = off + sgn * l2v + (e < 8 ? adja : adjb);
      const bool lt = v * 8 + e <= ehi && y < Di;
      below += lt ? 1u : 0u;
      ylast = lt ? y : ylast;
      off += step;
    }
    seen += 16;
    if (below < seen || gbase + seen - 1 >= ghi) break;
  }
  // blocks gbase .. gbase + below - 1 are below the target; count from glo as the search expects
  below = below > (uint32_t)(glo - gbase) ? below - (uint32_t)(glo - gbase) : 0u;
  uint64_t lo = 0, hi = 0;  // invariant: count_before(lo) < T, and hi = Bhi + 1 or count_before(hi) >= T
  bool over = false;        // the prediction missed by more than the error budget
  uint32_t kk = 0;           // set when the group resolves the block: T - count_before(lo) = D - y(lo)
  if (below > 0 && (glo + below - 1 < ghi || ghi == Bhi)) {
    lo = glo + below - 1;
    hi = lo + 1;
    kk = (uint32_t)(Di - ylast);
  } else if (below == 0) {
    // target left of the group (glo > Blo here): gallop left from glo
    hi = glo;
    uint64_t step = 1;
    for (;;) {
      if (hi - Blo <= step) {
        lo = Blo;
        break;
      }
      const uint64_t nb = hi - step;
      if (count_before<L2S>(d, m, b, nb << L2S) < T) {
        lo = nb;
        break;
      }
      hi = nb;
      step <<= 1;
      if (glo - nb > budget) {
        over = true;
        break;
      }
    }
  } else {
    // every block of the group is below the target: gallop right from ghi
    lo = ghi;
    uint64_t step = 1;
    for (;;) {
      const uint64_t nb = lo + step;
      if (nb > Bhi) {
        hi = Bhi + 1;
        break;
      }
      if (count_before<L2S>(d, m, b, nb << L2S) >= T) {
        hi = nb;
        break;
      }
      lo = nb;
      step <<= 1;
      if (nb - ghi > budget) {
        over = true;
        break;
      }
    }
  }
  if (over) return select_at<L2S, false>(d, m, b, T, sshift);
  while (hi - lo > 1) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (count_before<L2S>(d, m, b, mid << L2S) < T) lo = mid;
    else hi = mid;
  }
  if (!kk) kk = (uint32_t)(T - count_before<L2S>(d, m, b, lo << L2S));
  return (lo << L2S) + block_select<L2S>(d.bits + m.bits + (lo << (L2S - 6)), b, kk);
}

// select_c(k) through the learned index (same results and sentinels as select_one).
template <int L2S, int GS>
__device__ __forceinline__ uint64_t select_learned_one(const QArgs& a, const LevelMeta* meta, const LearnQ* qm,
                                                       uint32_t c, uint64_t k) {
  if (k == 0) return ~0ull;
  if (c >= a.sigma) return a.n;
  if (k > a.d.cum[c + 1] - a.d.cum[c]) return a.n;
  if (a.L == 0) return k - 1;
  uint32_t len;
  const uint32_t code = encode_sym(c, a.sigma, a.L, a.pow2, &len);
  uint64_t r = k;
  for (int l = (int)len - 1; l >= 0; --l) {
    const uint64_t pc = (uint64_t)(code >> (a.L - 1 - l));  // child prefix at level l + 1
    const uint64_t mi = (1ull << (l + 1)) - 2 + pc;
    // In a binned batch the lanes of a wave mostly share the model: then it is read through a
    // wave-uniform address (scalar loads) instead of once per lane.
    const uint64_t m0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(mi >> 32)) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)mi);
    uint64_t at, start;
    if (__ballot(mi != m0) == 0) {
      const LearnQ& Q = qm[m0];
      at = select_learned_at<L2S, GS, true>(a.d, meta[l], Q, r, a.sshift);
      start = Q.start;
    } else {
      // Lanes on different models (small unbinned batches): each would read its own model through
      // two dependent vector loads, which costs more than the sampled search it replaces, so this
      // level takes the sampled search (the node entry gives the same target and start as the model).
      const uint64_t p = l ? (uint64_t)(code >> (a.L - l)) : 0ull;
      const uint32_t b = (code >> (a.L - 1 - l)) & 1u;
      const NodeQ nd = a.d.nodes[(1ull << l) - 1 + p];
      at = select_at<L2S, WT_LEARN_MIXED_LINE>(a.d, meta[l], b, b ? (nd.start - nd.r0) + r : nd.r0 + r, a.sshift);
      start = nd.start;
    }
    r = at - start + 1;
  }
  return r - 1;
}

// Group of L2 counts the learned correction reads at once around the prediction: 2^WT_LEARN_GS
// entries (one fewer power for 2048-bit blocks).
#ifndef WT_LEARN_GS
#define WT_LEARN_GS 5
#endif
template <int L2S>
constexpr int learn_gs() {
  return L2S <= 10 ? WT_LEARN_GS : WT_LEARN_GS - 1;
}

}  // namespace wt
