// Build of the level-wise tree from host memory in chunks: the chunked construction the thesis's
// Conclusion names as its next step (the copy to the device hidden behind the building, and no need
// for the whole sequence on the device).
//
// The level-wise order keeps sequence order inside a node (Section 5.1: each level is the sequence
// stably sorted by the code bits above it), so the elements of node N at level l are the elements of
// N in chunk 0, then those in chunk 1, and so on. A chunk's own tree holds, at level l, the segment
// of every node N as one run of bits; in the tree of the whole sequence that run starts at the node's
// start plus the elements of N in the earlier chunks. Node starts come from the histogram alone
// (Section 5), so the counts of the whole sequence must be known before a segment is placed:
//   one pass   per chunk: copy, the chunk's tree (the device build), its counts added up; then the
//              node tables and level sizes of the whole tree, and every chunk's segments placed;
//   two passes per chunk: copy, counts added up; node tables; then per chunk: copy, the chunk's tree,
//              its segments placed at once (the device holds a few chunks only);
// placement: or-ed in as bit runs, one wave per 4096 bits of a segment, 64 per lane, bit-unaligned on
// both sides, the node's running count advanced; then per level the rank directory and select samples
// from the bits (Sections 4.1, 4.2). The next chunk's copy is in flight while a chunk is processed (two
// device slots; pageable arrays go through two page-locked staging buffers filled by host threads).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <thread>
#include <vector>

#include "wt_build_dev.h"
#include "wt_host.h"
#include "wt_internal.h"

namespace wt {
namespace {

constexpr uint64_t kDefaultBuildChunk = 1ull << 27;
constexpr uint64_t kPieceBits = 4096;  // bits of a node segment one wave places at a time

// Per heap entry p of one level: the node's segment [src, src + len) in the chunk's level, its
// destination in the tree's level (the node's start plus its elements in earlier chunks) and its
// number of pieces; the running count `done` advances by len. pieces[np] = 0 closes the scan.
__global__ __launch_bounds__(kBT) void k_place_plan(const NodeB* __restrict__ ntb_c, const NodeB* __restrict__ ntb_g,
                                                    uint64_t np, uint64_t* __restrict__ done, uint64_t* __restrict__ src,
                                                    uint64_t* __restrict__ len, uint64_t* __restrict__ dst,
                                                    uint64_t* __restrict__ pieces) {
  const uint64_t p = (uint64_t)blockIdx.x * kBT + threadIdx.x;
  if (p > np) return;
  if (p == np) {
    pieces[np] = 0;
    return;
  }
  const NodeB c = ntb_c[p];
  uint64_t s = 0, ln = 0, d = 0;
  if (c.start != kNoNode) {
    s = c.start;
    ln = c.end - c.start;
    d = ntb_g[p].start + done[p];
    done[p] += ln;
  }
  src[p] = s;
  len[p] = ln;
  dst[p] = d;
  pieces[p] = (ln + kPieceBits - 1) / kPieceBits;
}

// One wave per piece (grid-stride over the poff[np] pieces): lane j moves bits [64 j, 64 j + 64) of
// the piece from the chunk's level to the tree's level. Segments are disjoint and the tree's levels
// start cleared, so or-ing composes them exactly.
__global__ __launch_bounds__(kBT) void k_place(const uint64_t* __restrict__ sbits, uint64_t* __restrict__ dbits,
                                               const uint64_t* __restrict__ poff, uint64_t np,
                                               const uint64_t* __restrict__ src, const uint64_t* __restrict__ len,
                                               const uint64_t* __restrict__ dst) {
  const uint64_t total = poff[np];
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t nwaves = ((uint64_t)gridDim.x * kBT) >> 6;
  for (uint64_t i = ((uint64_t)blockIdx.x * kBT + threadIdx.x) >> 6; i < total; i += nwaves) {
    // the node of piece i: the last p with poff[p] <= i (it has at least one piece)
    uint64_t lo = 0, hi = np;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (poff[mid] <= i) lo = mid;
      else hi = mid;
    }
    const uint64_t off = (i - poff[lo]) * kPieceBits + 64ull * lane;
    const uint64_t ln = len[lo];
    if (off >= ln) continue;
    const uint32_t cnt = (uint32_t)min<uint64_t>(64, ln - off);
    const uint64_t a = src[lo] + off;
    const uint32_t sh = (uint32_t)(a & 63);
    uint64_t x = sbits[a >> 6] >> sh;
    if (sh && sh + cnt > 64) x |= sbits[(a >> 6) + 1] << (64 - sh);
    if (cnt < 64) x &= (1ull << cnt) - 1ull;
    const uint64_t d = dst[lo] + off;
    const uint32_t dsh = (uint32_t)(d & 63);
    atomicOr((unsigned long long*)&dbits[d >> 6], (unsigned long long)(x << dsh));
    if (dsh && dsh + cnt > 64) atomicOr((unsigned long long*)&dbits[(d >> 6) + 1], (unsigned long long)(x >> (64 - dsh)));
  }
}

// Everything of one call that must be released on every exit.
struct HostBuild {
  hipStream_t cs = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
  char* stage[2] = {nullptr, nullptr};
  void* work = nullptr;
  void* pool = nullptr;  // one pass: every chunk's build node table
  hipStream_t st = nullptr;
  wt_tree* t = nullptr;  // the tree until it is handed out
  std::vector<wt_tree*> cts;  // one pass: the chunks' trees until they are placed
  ~HostBuild() {
    if (cs) (void)hipStreamSynchronize(cs);
    if (st) (void)hipStreamSynchronize(st);
    for (wt_tree* ct : cts) {
      if (!ct) continue;
      dev_free(ct->block, st);
      delete ct;
    }
    if (pool) dev_free(pool, st);
    for (int k = 0; k < 2; ++k) {
      if (copied[k]) (void)hipEventDestroy(copied[k]);
      if (freed[k]) (void)hipEventDestroy(freed[k]);
      if (stage[k]) (void)hipHostFree(stage[k]);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (work) dev_free(work, st);
    if (t) {
      if (t->block) dev_free(t->block, st);
      delete t;
    }
    if (st) (void)hipStreamSynchronize(st);
  }
};

}  // namespace
}  // namespace wt

using namespace wt;

extern "C" wt_status wt_build_host(const void* h_sym, uint64_t n, uint32_t sym_bytes, uint64_t sigma,
                                   const wt_build_opts* opts, uint64_t chunk, wt_build_host_stats* stats,
                                   wt_stream_t stream, wt_tree** out) {
  clear_error();
  const auto t_start = std::chrono::steady_clock::now();
  auto ms_since = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - a).count();
  };
  if (!out) return fail(WT_ERR_ARG, "wt_build_host: out is NULL");
  *out = nullptr;
  if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4)
    return fail(WT_ERR_ARG, "wt_build_host: sym_bytes must be 1, 2 or 4 (got %u)", sym_bytes);
  if (n && !h_sym) return fail(WT_ERR_ARG, "wt_build_host: h_sym is NULL");
  if (sigma == 0) return fail(WT_ERR_ARG, "wt_build_host: sigma must be >= 1 (no alphabet extraction here)");
  if (sigma > WT_MAX_SIGMA) return fail(WT_ERR_ARG, "wt_build_host: sigma %llu exceeds %llu",
                                        (unsigned long long)sigma, (unsigned long long)WT_MAX_SIGMA);
  if (sym_bytes < 4 && sigma > (1ull << (8 * sym_bytes)))
    return fail(WT_ERR_ARG, "wt_build_host: sigma %llu does not fit %u-byte symbols", (unsigned long long)sigma,
                sym_bytes);
  if (n >= (1ull << 40)) return fail(WT_ERR_ARG, "wt_build_host: n too large");
  const wt_status orc = check_build_opts(opts);
  if (orc != WT_OK) return orc;
  const uint32_t flags = opts ? opts->flags : 0u;
  if (flags & (WT_BUILD_MATRIX | WT_BUILD_HUFFMAN))
    return fail(WT_ERR_ARG, "wt_build_host: builds the level-wise tree only (no WT_BUILD_MATRIX / WT_BUILD_HUFFMAN)");
  if (chunk == 0) chunk = kDefaultBuildChunk;
  if (chunk < (1ull << 16)) return fail(WT_ERR_ARG, "wt_build_host: chunk must be at least 2^16 symbols");
  const uint32_t l2_bits = opts && opts->l2_bits ? opts->l2_bits : 512;
  const uint32_t srate = opts && opts->sample_rate ? opts->sample_rate : 4096;
  hipStream_t st = (hipStream_t)stream;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n == 0) return build_tree(nullptr, 0, sym_bytes, sigma, opts, stream, out);
  chunk = std::min<uint64_t>(chunk, n);

  int dev = 0;
  WT_HIP(hipGetDevice(&dev));
  uint32_t L = 0;
  while ((1ull << L) < sigma) ++L;
  const TreePlan P = plan_tree(n, sym_bytes, sigma, L, l2_bits, srate);
  const uint64_t nch = ceil_div(n, chunk);
  const bool pinned = is_pinned(h_sym);

  HostBuild H;
  H.st = st;
  H.t = new wt_tree();
  wt_tree* t = H.t;
  t->n = n;
  t->sigma = sigma;
  t->L = L;
  t->w = sym_bytes;
  t->l2_bits = l2_bits;
  t->srate = srate;
  t->pow2 = (sigma & (sigma - 1)) == 0;
  t->device = dev;
  t->block_bytes = P.total;
  t->block = dev_alloc(P.total, st);
  if (!t->block) return fail(WT_ERR_OOM, "wt_build_host: tree allocation of %zu bytes failed", P.total);
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

  // working set: two chunk slots, counts, node tables, per-level placement arrays, scratch
  const uint64_t nheap = P.nheap;
  const uint64_t nlev = L ? (1ull << (L - 1)) + 1 : 1;  // heap entries of the widest level, + 1
  size_t so = 0;
  auto take = [&](size_t bytes) {
    const size_t o = so;
    so = round_up(so + bytes, 256);
    return o;
  };
  const size_t o_in0 = take(chunk * sym_bytes), o_in1 = take(chunk * sym_bytes);
  const size_t o_hist = take((sigma + 1) * 8), o_err = take(64);
  const size_t o_hs = take(hist_add_scratch_bytes(chunk, sym_bytes, sigma));
  const size_t o_ntbg = take(std::max<uint64_t>(nheap, 1) * sizeof(NodeB));
  const size_t o_ntbc = take(std::max<uint64_t>(nheap, 1) * sizeof(NodeB));
  const size_t o_z = take((nheap + 1) * 8), o_zs = take((nheap + 1) * 8), o_done = take((nheap + 1) * 8);
  const size_t o_src = take(nlev * 8), o_len = take(nlev * 8), o_dst = take(nlev * 8);
  const size_t o_pc = take(nlev * 8), o_poff = take(nlev * 8);
  const size_t o_part = take((ceil_div(std::max<uint64_t>(std::max<uint64_t>(sigma, nheap), nlev) + 1, kScanChunk) + 1) * 8);
  const size_t o_dir = take(bv_directory_scratch_bytes(n));
  H.work = dev_alloc(so, st);
  if (!H.work) return fail(WT_ERR_OOM, "wt_build_host: working memory of %zu bytes failed", so);
  char* wb = (char*)H.work;
  char* in[2] = {wb + o_in0, wb + o_in1};
  uint64_t* hist = (uint64_t*)(wb + o_hist);
  uint32_t* err = (uint32_t*)(wb + o_err);
  NodeB* ntb_g = (NodeB*)(wb + o_ntbg);
  NodeB* ntb_c = (NodeB*)(wb + o_ntbc);
  uint64_t* z = (uint64_t*)(wb + o_z);
  uint64_t* zs = (uint64_t*)(wb + o_zs);
  uint64_t* done = (uint64_t*)(wb + o_done);
  uint64_t* psrc = (uint64_t*)(wb + o_src);
  uint64_t* plen = (uint64_t*)(wb + o_len);
  uint64_t* pdst = (uint64_t*)(wb + o_dst);
  uint64_t* pcs = (uint64_t*)(wb + o_pc);
  uint64_t* poff = (uint64_t*)(wb + o_poff);
  uint64_t* part = (uint64_t*)(wb + o_part);

  WT_HIP(hipStreamCreateWithFlags(&H.cs, hipStreamNonBlocking));
  for (int k = 0; k < 2; ++k) {
    WT_HIP(hipEventCreateWithFlags(&H.copied[k], hipEventDisableTiming));
    WT_HIP(hipEventCreateWithFlags(&H.freed[k], hipEventDisableTiming));
    if (!pinned && hipHostMalloc((void**)&H.stage[k], chunk * sym_bytes, 0) != hipSuccess) {
      (void)hipGetLastError();
      return fail(WT_ERR_OOM, "wt_build_host: page-locked staging of %llu bytes failed",
                  (unsigned long long)(chunk * sym_bytes));
    }
  }

  const char* hs = (const char*)h_sym;
  auto csize = [&](uint64_t c) { return std::min<uint64_t>(chunk, n - c * chunk); };
  // Copy of chunk c into device slot k, after that slot's previous chunk was processed (freed[k]).
  // Pageable: the staging buffer k is refilled once its previous copy has left it (copied[k]).
  auto upload = [&](uint64_t c, int k) -> hipError_t {
    const size_t bytes = csize(c) * sym_bytes;
    const char* src = hs + c * chunk * sym_bytes;
    hipError_t e = hipStreamWaitEvent(H.cs, H.freed[k], 0);
    if (e != hipSuccess) return e;
    if (!pinned) {
      e = hipEventSynchronize(H.copied[k]);
      if (e != hipSuccess) return e;
      par_copy(H.stage[k], src, bytes);
      src = H.stage[k];
    }
    e = hipMemcpyAsync(in[k], src, bytes, hipMemcpyHostToDevice, H.cs);
    if (e != hipSuccess) return e;
    return hipEventRecord(H.copied[k], H.cs);
  };

  // One pass keeps every chunk's tree (and its build node table) until the counts are complete: chosen
  // when that fits in what the device has free, with room for one chunk build's scratch.
  wt_build_opts copts{};
  copts.l2_bits = l2_bits;
  copts.sample_rate = srate;
  copts.flags = flags & (WT_BUILD_WIDE | WT_BUILD_NARROW);
  const size_t pool_bytes = (size_t)nch * std::max<uint64_t>(nheap, 1) * sizeof(NodeB);
  size_t keep_bytes = pool_bytes;
  for (uint64_t c = 0; c < nch; ++c) keep_bytes += plan_tree(csize(c), sym_bytes, sigma, L, l2_bits, srate).total;
  bool one_pass = !(flags & WT_BUILD_HOST_TWO_PASS) && L > 0;
  if (one_pass) {
    size_t fr = 0, tot = 0;
    WT_HIP(hipMemGetInfo(&fr, &tot));
    const size_t build_scratch = (size_t)chunk * sym_bytes * 4 + (size_t)nheap * 96 + (64u << 20);
    one_pass = keep_bytes + build_scratch < fr;
  }
  if (one_pass) {
    H.pool = dev_alloc(pool_bytes, st);
    if (!H.pool) one_pass = false;
  }
  NodeB* pool = (NodeB*)H.pool;

  // Places every node segment of the chunk tree ct (build node table ntb_c) into the tree's levels.
  uint64_t chunk_tree_bytes = 0;
  auto place = [&](const wt_tree* ct, const NodeB* ntb_c) -> hipError_t {
    hipError_t he = hipSuccess;
    for (uint32_t l = 0; l < L && he == hipSuccess; ++l) {
      const uint64_t ncl = ct->hmeta[l].n;
      if (ncl == 0) continue;
      const uint64_t np = 1ull << l, hb = np - 1;
      hipLaunchKernelGGL(k_place_plan, dim3((uint32_t)ceil_div(np + 1, kBT)), dim3(kBT), 0, st, ntb_c + hb,
                         (const NodeB*)(ntb_g + hb), np, done + hb, psrc, plen, pdst, pcs);
      he = hipGetLastError();
      if (he == hipSuccess) he = exclusive_scan_u64(pcs, np + 1, poff, part, st);
      if (he == hipSuccess) {
        const uint64_t waves = std::min<uint64_t>(ceil_div(ncl, kPieceBits) + np, 1ull << 16);
        hipLaunchKernelGGL(k_place, dim3((uint32_t)ceil_div(waves, kBT / 64)), dim3(kBT), 0, st,
                           (const uint64_t*)(ct->dev.bits + ct->hmeta[l].bits), t->dev.bits + t->hmeta[l].bits,
                           (const uint64_t*)poff, np, (const uint64_t*)psrc, (const uint64_t*)plen,
                           (const uint64_t*)pdst);
        he = hipGetLastError();
      }
    }
    return he;
  };

  // ---- first pass: counts (and, in one pass, the chunks' trees)
  WT_HIP(fill_u64(hist, sigma + 1, 0ull, st));
  WT_HIP(fill_u64((uint64_t*)err, 8, 0ull, st));
  WT_HIP(fill_u64(done, nheap + 1, 0ull, st));
  WT_HIP(fill_u64(t->dev.bits, (uint64_t)L * P.words_per_level, 0ull, st));
  WT_HIP(init_levels(P, t->dev.meta, t->hmeta, st));
  for (int k = 0; k < 2; ++k) WT_HIP(hipEventRecord(H.freed[k], st));  // the slots are free after the fills
  WT_HIP(upload(0, 0));
  for (uint64_t c = 0; c < nch; ++c) {
    const int k = (int)(c & 1);
    if (c + 1 < nch) WT_HIP(upload(c + 1, k ^ 1));
    WT_HIP(hipStreamWaitEvent(st, H.copied[k], 0));
    WT_HIP(hist_add(in[k], csize(c), sym_bytes, sigma, hist, err, wb + o_hs, st));
    if (one_pass) {
      wt_tree* ct = nullptr;
      const wt_status brc = build_tree(in[k], csize(c), sym_bytes, sigma, &copts, st, &ct, pool + c * nheap);
      if (brc != WT_OK) return brc;
      H.cts.push_back(ct);
      chunk_tree_bytes += ct->block_bytes;
    }
    WT_HIP(hipEventRecord(H.freed[k], st));
  }
  uint32_t bad = 0;
  WT_HIP(hipMemcpyAsync(&bad, err, 4, hipMemcpyDeviceToHost, st));
  WT_HIP(hipStreamSynchronize(st));
  if (bad) return fail(WT_ERR_SYMBOL_RANGE, "wt_build_host: a symbol is >= sigma (%llu)", (unsigned long long)sigma);
  WT_HIP(exclusive_scan_u64(hist, sigma + 1, t->dev.cum, part, st));
  WT_HIP(node_tables((uint32_t)sigma, nheap, t->dev.cum, ntb_g, z, zs, part, t->dev.nodes, t->dev.meta, st));
  std::vector<LevelMeta> rb(WT_MAX_LEVELS);
  WT_HIP(hipMemcpyAsync(rb.data(), t->dev.meta, sizeof(LevelMeta) * WT_MAX_LEVELS, hipMemcpyDeviceToHost, st));
  WT_HIP(hipStreamSynchronize(st));
  const float ms_counts = ms_since(t_start);

  // ---- placement (one pass: the kept trees; two passes: a second pass over the chunks)
  const auto t_build = std::chrono::steady_clock::now();
  if (one_pass) {
    for (uint64_t c = 0; c < nch; ++c) {
      const hipError_t he = place(H.cts[c], pool + c * nheap);
      if (he != hipSuccess) return fail(WT_ERR_HIP, "wt_build_host: placement: %s", hipGetErrorString(he));
      dev_free(H.cts[c]->block, st);
      delete H.cts[c];
      H.cts[c] = nullptr;
    }
    chunk_tree_bytes += pool_bytes;
  } else if (L > 0) {
    WT_HIP(upload(0, 0));
    for (uint64_t c = 0; c < nch; ++c) {
      const int k = (int)(c & 1);
      if (c + 1 < nch) WT_HIP(upload(c + 1, k ^ 1));
      WT_HIP(hipStreamWaitEvent(st, H.copied[k], 0));
      wt_tree* ct = nullptr;
      const wt_status brc = build_tree(in[k], csize(c), sym_bytes, sigma, &copts, st, &ct, ntb_c);
      if (brc != WT_OK) return brc;
      WT_HIP(hipEventRecord(H.freed[k], st));
      chunk_tree_bytes = std::max<uint64_t>(chunk_tree_bytes, ct->block_bytes);
      const hipError_t he = place(ct, ntb_c);
      dev_free(ct->block, st);
      delete ct;
      if (he != hipSuccess) return fail(WT_ERR_HIP, "wt_build_host: placement: %s", hipGetErrorString(he));
    }
  }
  // ---- rank directory and select samples of every level
  for (uint32_t l = 0; l < L; ++l) {
    const LevelMeta& m = t->hmeta[l];
    WT_HIP(bv_directory(t->dev.bits + m.bits, t->dev.L1 + m.l1, t->dev.L2 + m.l2, t->dev.smp + m.smp, t->dev.meta + l,
                        rb[l].n, m.smp_cap, l2_bits, srate, wb + o_dir, st));
  }
  WT_HIP(hipMemcpyAsync(rb.data(), t->dev.meta, sizeof(LevelMeta) * WT_MAX_LEVELS, hipMemcpyDeviceToHost, st));
  WT_HIP(hipStreamSynchronize(st));
  for (uint32_t l = 0; l < L; ++l) t->hmeta[l] = rb[l];
  if (stats) {
    stats->chunks = (uint32_t)nch;
    stats->pinned = pinned ? 1u : 0u;
    stats->passes = one_pass ? 1u : 2u;
    stats->ms_counts = ms_counts;
    stats->ms_build = ms_since(t_build);
    stats->ms_total = ms_since(t_start);
    stats->work_bytes = so + chunk_tree_bytes;
  }
  *out = t;
  H.t = nullptr;
  return WT_OK;
}
