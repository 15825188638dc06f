// Rank and select support of a plain bit array (Section 4: the bit array, the L1/L2 rank directory of
// Section 4.1 and the select samples of Section 4.2), built from caller-supplied bits.
//
// A bit array is the level of a wavelet tree over the binary alphabet: a tree with sigma = 2 has one
// level whose bits are the sequence itself, its rank(1, i) is rank1(i), rank(0, i) = rank0(i),
// select(b, k) the position of the k-th bit b and access(i) the bit. So the bits are stored in the
// tree layout of one level (16384-bit tiles, 128-byte aligned, LSB-first 64-bit words), the directory
// and samples are those the level pass writes, and every query, export and learned-index call of a
// tree works on the result unchanged.
//
// Build: (1) per tile of 16384 bits, copy the words (bits past n cleared) and count the ones;
// (2) exclusive scan of the tile counts; (3) per tile, a block scan of the word popcounts gives the
// ones before every word: the L2 entries (ones since the enclosing L1 block's start, at every |L2|
// boundary), the L1 entry at every 65536-bit boundary, the select samples where the running count of
// ones or zeros crosses a multiple of s (s >= 512, so a word holds at most one crossing of each), and
// on the last tile the totals and the sentinel entries that make rank defined at i = n.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "wt_build_dev.h"
#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

constexpr uint32_t kBvTileWords = 256;  // 16384 bits: one word per thread of a 256-thread block
static_assert(kBvTileWords == (uint32_t)kBT, "one word per thread");

// Copies tile t (words past the array, and bits past n, cleared) and counts its ones.
__global__ __launch_bounds__(kBT) void k_bv_copy(const uint64_t* __restrict__ src, uint64_t n, uint64_t* __restrict__ dst,
                                                 uint64_t* __restrict__ tile_ones) {
  __shared__ uint64_t s_w[kBT / 64];
  const uint64_t t = blockIdx.x;
  const uint64_t gw = t * kBvTileWords + threadIdx.x;
  const uint64_t nwords = (n + 63) >> 6;
  uint64_t x = 0;
  if (gw < nwords) {
    x = src[gw];
    if (gw == nwords - 1 && (n & 63)) x &= (1ull << (n & 63)) - 1ull;
  }
  dst[gw] = x;
  uint64_t tot;
  block_excl_scan_u64((uint64_t)__popcll(x), s_w, tot);
  if (threadIdx.x == 0) tile_ones[t] = tot;
}

struct BvArgs {
  uint64_t* bits;
  uint64_t* L1;
  uint16_t* L2;
  uint64_t* smp;
  LevelMeta* meta;
  uint64_t* cum;
  NodeQ* nodes;
  const uint64_t* pre;  // ones before every tile
  uint64_t n, smp_cap;
  uint32_t l2w_shift;   // log2 of the words per L2 block
  uint32_t sshift;      // log2 s
};

__global__ __launch_bounds__(kBT) void k_bv_dir(BvArgs a, uint64_t ntiles) {
  __shared__ uint64_t s_w[kBT / 64];
  const uint64_t t = blockIdx.x;
  const uint64_t gw = t * kBvTileWords + threadIdx.x;
  const uint64_t x = a.bits[gw];
  uint64_t tile_tot;
  const uint64_t G1 = a.pre[t];
  const uint64_t p = G1 + block_excl_scan_u64((uint64_t)__popcll(x), s_w, tile_tot);  // ones before word gw
  const uint64_t b0 = gw << 6;                                                           // first bit of the word
  if (b0 < a.n) {
    // L2: ones since the enclosing L1 block's start (tiles hold 16384 bits: 4 tiles per L1 block)
    if ((gw & ((1ull << a.l2w_shift) - 1)) == 0) {
      const uint64_t l1v = a.pre[(b0 >> kL1Shift) << 2];
      a.L2[gw >> a.l2w_shift] = (uint16_t)(p - l1v);
    }
    const uint32_t valid = (uint32_t)min<uint64_t>(64, a.n - b0);
    const uint32_t c1 = (uint32_t)__popcll(x), c0 = valid - c1;
    // the (m s)-th one lies in this word when m s is in (p, p + c1]
    const uint64_t m1 = (p + c1) >> a.sshift;
    if (c1 && m1 > (p >> a.sshift)) a.smp[m1 - 1] = b0 + select_in_word(x, (uint32_t)((m1 << a.sshift) - p));
    const uint64_t z = b0 - p;  // zeros before the word
    const uint64_t m0 = (z + c0) >> a.sshift;
    if (c0 && m0 > (z >> a.sshift)) {
      const uint64_t zw = ~x & (valid == 64 ? ~0ull : ((1ull << valid) - 1ull));
      a.smp[a.smp_cap - m0] = b0 + select_in_word(zw, (uint32_t)((m0 << a.sshift) - z));
    }
  }
  if (threadIdx.x == 0) {
    const uint64_t t0 = t * kBvTileWords * 64;  // first bit of the tile
    if ((t0 & (kL1Bits - 1)) == 0) a.L1[t0 >> kL1Shift] = G1;
    if (t == ntiles - 1) {
      // totals, sentinels (rank defined at i = n), the node entry and cumulative histogram of sigma = 2
      const uint64_t total = G1 + tile_tot;
      const uint64_t n = a.n;
      LevelMeta m = *a.meta;
      m.n = n;
      m.ones = total;
      *a.meta = m;
      a.L1[(n + kL1Bits - 1) >> kL1Shift] = total;
      const uint32_t l2s = a.l2w_shift + 6;
      const uint64_t j = (n + (1ull << l2s) - 1) >> l2s;
      const uint64_t blk = (j << l2s) >> kL1Shift;
      const uint64_t lv = ((blk << kL1Shift) >= n) ? total : a.pre[blk << 2];
      a.L2[j] = (uint16_t)(total - lv);
      a.cum[0] = 0;
      a.cum[1] = n - total;
      a.cum[2] = n;
      NodeQ root;
      root.start = 0;
      root.r0 = 0;
      a.nodes[0] = root;
    }
  }
}

// The empty array: its sentinel entries, totals, node entry and histogram.
__global__ void k_bv_empty(BvArgs a) {
  if (threadIdx.x) return;
  LevelMeta m = *a.meta;
  m.n = 0;
  m.ones = 0;
  *a.meta = m;
  a.L1[0] = 0;
  a.L2[0] = 0;
  a.cum[0] = a.cum[1] = a.cum[2] = 0;
  NodeQ root;
  root.start = 0;
  root.r0 = 0;
  a.nodes[0] = root;
}

__global__ void k_bv_meta(LevelMeta m, LevelMeta* __restrict__ meta) {
  if (threadIdx.x == 0) *meta = m;
}

// tile ones, their scan, scan partials, and the sigma = 2 histogram and node entry that k_bv_dir also
// writes (not used for a level of a larger tree)
size_t bv_directory_scratch_bytes(uint64_t n) {
  const uint64_t ntiles = ceil_div(std::max<uint64_t>(n, 1), (uint64_t)kBvTileWords * 64);
  return (2 * (ntiles + 1) + ceil_div(ntiles + 1, kScanChunk) + 1 + 8) * 8;
}

hipError_t bv_directory(uint64_t* bits, uint64_t* L1, uint16_t* L2, uint64_t* smp, LevelMeta* meta, uint64_t n,
                        uint64_t smp_cap, uint32_t l2_bits, uint32_t srate, char* scratch, hipStream_t st) {
  const uint64_t ntiles = ceil_div(n, (uint64_t)kBvTileWords * 64);
  uint64_t* tile_ones = (uint64_t*)scratch;
  uint64_t* pre = tile_ones + ntiles + 1;
  uint64_t* part = pre + ntiles + 1;
  uint64_t* dummy = part + ceil_div(ntiles + 1, kScanChunk) + 1;
  uint32_t l2w_shift = 0, sshift = 0;
  while ((64u << l2w_shift) < l2_bits) ++l2w_shift;
  while ((1u << sshift) < srate) ++sshift;
  BvArgs a{bits, L1, L2, smp, meta, dummy, (NodeQ*)(dummy + 3), pre, n, smp_cap, l2w_shift, sshift};
  if (ntiles == 0) {
    hipLaunchKernelGGL(k_bv_empty, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
  }
  // in place: clears the bits past n and counts the ones of every tile
  hipLaunchKernelGGL(k_bv_copy, dim3((uint32_t)ntiles), dim3(kBT), 0, st, (const uint64_t*)bits, n, bits, tile_ones);
  hipError_t he = exclusive_scan_u64(tile_ones, ntiles, pre, part, st);
  if (he != hipSuccess) return he;
  hipLaunchKernelGGL(k_bv_dir, dim3((uint32_t)ntiles), dim3(kBT), 0, st, a, ntiles);
  return hipGetLastError();
}

}  // namespace wt

using namespace wt;

extern "C" wt_status wt_bv_build(const uint64_t* d_words, uint64_t n_bits, const wt_build_opts* opts, wt_stream_t stream,
                                 wt_tree** out) {
  clear_error();
  if (!out) return fail(WT_ERR_ARG, "wt_bv_build: out is NULL");
  *out = nullptr;
  if (n_bits && !d_words) return fail(WT_ERR_ARG, "wt_bv_build: d_words is NULL");
  if (n_bits >= (1ull << 40)) return fail(WT_ERR_ARG, "wt_bv_build: n_bits too large");
  const wt_status orc = check_build_opts(opts);
  if (orc != WT_OK) return orc;
  const uint32_t l2_bits = opts && opts->l2_bits ? opts->l2_bits : 512;
  const uint32_t srate = opts && opts->sample_rate ? opts->sample_rate : 4096;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  WT_HIP(hipGetDevice(&dev));
  // one level of a binary-alphabet tree; a tile of a 1-byte level holds 16384 elements = 256 words
  const TreePlan P = plan_tree(n_bits, 1, 2, 1, l2_bits, srate);
  wt_tree* t = new wt_tree();
  t->n = n_bits;
  t->sigma = 2;
  t->L = 1;
  t->w = 1;
  t->l2_bits = l2_bits;
  t->srate = srate;
  t->pow2 = 1;
  t->device = dev;
  t->block_bytes = P.total;
  t->block = dev_alloc(P.total, st);
  if (!t->block) {
    delete t;
    return fail(WT_ERR_OOM, "wt_bv_build: allocation of %zu bytes failed", P.total);
  }
  char* base = (char*)t->block;
  t->dev.meta = (LevelMeta*)(base + P.off_meta);
  t->dev.cum = (uint64_t*)(base + P.off_cum);
  t->dev.nodes = (NodeQ*)(base + P.off_nodes);
  t->dev.bits = (uint64_t*)(base + P.off_bits);
  t->dev.L1 = (uint64_t*)(base + P.off_l1);
  t->dev.L2 = (uint16_t*)(base + P.off_l2);
  t->dev.smp = (uint64_t*)(base + P.off_smp);
  t->bytes_bits = P.words_per_level * 8;
  t->bytes_l1 = P.l1_per_level * 8;
  t->bytes_l2 = P.l2_per_level * 2;
  t->bytes_smp = P.smp_per_level * 8;
  t->bytes_nodes = sizeof(NodeQ);
  t->bytes_cum = 3 * 8;
  LevelMeta m{};
  m.bits = 0;
  m.l1 = 0;
  m.l2 = 0;
  m.smp = 0;
  m.smp_cap = P.smp_per_level;
  const uint64_t ntiles = ceil_div(n_bits, (uint64_t)kBvTileWords * 64);
  uint64_t* scratch = (uint64_t*)dev_alloc((2 * (ntiles + 1) + ceil_div(ntiles + 1, 4096) + 1) * 8, st);
  if (!scratch) {
    dev_free(t->block, st);
    delete t;
    return fail(WT_ERR_OOM, "wt_bv_build: scratch allocation failed");
  }
  uint64_t* tile_ones = scratch;
  uint64_t* pre = scratch + ntiles + 1;
  uint64_t* part = pre + ntiles + 1;
  uint32_t l2w_shift = 0, sshift = 0;
  while ((64u << l2w_shift) < l2_bits) ++l2w_shift;
  while ((1u << sshift) < srate) ++sshift;
  BvArgs a{t->dev.bits, t->dev.L1, t->dev.L2, t->dev.smp, t->dev.meta, t->dev.cum, t->dev.nodes, pre,
           n_bits, P.smp_per_level, l2w_shift, sshift};
  hipError_t he;
  hipLaunchKernelGGL(k_bv_meta, dim3(1), dim3(64), 0, st, m, t->dev.meta);
  if (ntiles == 0) {
    hipLaunchKernelGGL(k_bv_empty, dim3(1), dim3(64), 0, st, a);
    he = hipGetLastError();
  } else {
    hipLaunchKernelGGL(k_bv_copy, dim3((uint32_t)ntiles), dim3(kBT), 0, st, d_words, n_bits, t->dev.bits, tile_ones);
    he = exclusive_scan_u64(tile_ones, ntiles, pre, part, st);
    if (he == hipSuccess) {
      hipLaunchKernelGGL(k_bv_dir, dim3((uint32_t)ntiles), dim3(kBT), 0, st, a, ntiles);
      he = hipGetLastError();
    }
  }
  LevelMeta hm{};
  if (he == hipSuccess) he = hipMemcpyAsync(&hm, t->dev.meta, sizeof(LevelMeta), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  dev_free(scratch, st);
  if (he != hipSuccess) {
    dev_free(t->block, st);
    delete t;
    return fail(WT_ERR_HIP, "wt_bv_build: %s", hipGetErrorString(he));
  }
  t->hmeta[0] = hm;
  *out = t;
  return WT_OK;
}
