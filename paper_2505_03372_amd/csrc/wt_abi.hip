// C ABI plumbing: errors, allocator hook, tree lifetime, info, canonical export, profile.
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wt_host.h"
#include "wt_internal.h"

namespace wt {

static thread_local char g_err[512] = "";

wt_status fail(wt_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

void clear_error() { g_err[0] = 0; }

static wt_alloc_fn g_alloc = nullptr;
static wt_free_fn g_free = nullptr;
static void* g_ctx = nullptr;

void* dev_alloc(size_t bytes, hipStream_t s) {
  if (bytes == 0) bytes = 256;
  if (g_alloc) return g_alloc(bytes, (wt_stream_t)s, g_ctx);
  static bool pool_set = false;
  if (!pool_set) {
    // keep freed blocks in the stream-ordered pool so repeated builds do not return memory to the OS
    int dev = 0;
    hipMemPool_t pool;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = ~0ull;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    pool_set = true;
  }
  void* p = nullptr;
  if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void* p, hipStream_t s) {
  if (!p) return;
  if (g_free) {
    g_free(p, (wt_stream_t)s, g_ctx);
    return;
  }
  (void)hipFreeAsync(p, s);
}

}  // namespace wt

uint64_t wt::next_tree_uid() {
  static std::atomic<uint64_t> next{1};
  return next.fetch_add(1);
}

using namespace wt;

extern "C" const char* wt_last_error(void) { return g_err; }

extern "C" const char* wt_version(void) { return "wt-mi355x 0.1 (gfx950)"; }

extern "C" wt_status wt_set_allocator(wt_alloc_fn alloc_fn, wt_free_fn free_fn, void* ctx) {
  clear_error();
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(WT_ERR_ARG, "wt_set_allocator: give both functions or neither");
  g_alloc = alloc_fn;
  g_free = free_fn;
  g_ctx = ctx;
  return WT_OK;
}

extern "C" wt_status wt_free(wt_tree* t) {
  clear_error();
  if (!t) return WT_OK;
  if (t->borrowed) return fail(WT_ERR_STATE, "wt_free: the tree belongs to a forest (use wt_forest_free)");
  WT_HIP(hipDeviceSynchronize());
  if (t->learn) dev_free(t->learn, nullptr);
  if (t->alpha_block) dev_free(t->alpha_block, nullptr);
  if (t->alpha) dev_free((void*)t->alpha, nullptr);
  dev_free(t->block, nullptr);
  WT_HIP(hipDeviceSynchronize());
  delete t;
  return WT_OK;
}

extern "C" wt_status wt_info(const wt_tree* t, wt_info_t* out) {
  clear_error();
  if (!t || !out) return fail(WT_ERR_ARG, "wt_info: NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->n = t->n;
  out->sigma = t->sigma;
  out->levels = t->L;
  out->sym_bytes = t->w;
  out->l2_bits = t->l2_bits;
  out->sample_rate = t->srate;
  for (uint32_t l = 0; l < t->L; ++l) {
    out->level_n[l] = t->hmeta[l].n;
    out->level_ones[l] = t->hmeta[l].ones;
  }
  out->bytes_bits = t->bytes_bits;
  out->bytes_l1 = t->bytes_l1;
  out->bytes_l2 = t->bytes_l2;
  out->bytes_samples = t->bytes_smp;
  out->bytes_nodes = t->bytes_nodes + t->bytes_cum;
  out->bytes_total = t->block_bytes;
  out->alphabet_extracted = t->amap ? 1u : 0u;
  out->matrix = t->matrix;
  out->huffman = t->huff;
  out->max_symbol = t->amap ? t->max_symbol : (t->sigma ? t->sigma - 1 : 0);
  return WT_OK;
}

extern "C" wt_status wt_export(const wt_tree* t, int level, int part, void* h_dst, size_t cap, size_t* needed) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_export: tree is NULL");
  if (part == WT_PART_ALPHABET) {
    const size_t bytes = (size_t)t->sigma * 4;
    if (needed) *needed = bytes;
    if (!h_dst) return WT_OK;
    if (cap < bytes) return fail(WT_ERR_ARG, "wt_export: capacity %zu < %zu bytes", cap, bytes);
    if (t->alpha) {
      WT_HIP(hipDeviceSynchronize());
      WT_HIP(hipMemcpy(h_dst, t->alpha, bytes, hipMemcpyDeviceToHost));
    } else {
      for (uint64_t c = 0; c < t->sigma; ++c) ((uint32_t*)h_dst)[c] = (uint32_t)c;
    }
    return WT_OK;
  }
  if (part == WT_PART_WM_STARTS) {
    if (!t->matrix) return fail(WT_ERR_ARG, "wt_export: WT_PART_WM_STARTS needs a wavelet matrix");
    const size_t bytes = (size_t)t->sigma * 8;
    if (needed) *needed = bytes;
    if (!h_dst) return WT_OK;
    if (cap < bytes) return fail(WT_ERR_ARG, "wt_export: capacity %zu < %zu bytes", cap, bytes);
    WT_HIP(hipDeviceSynchronize());
    WT_HIP(hipMemcpy(h_dst, t->dev.wstart, bytes, hipMemcpyDeviceToHost));
    return WT_OK;
  }
  if (part == WT_PART_HUFF_CODES) {
    if (!t->huff) return fail(WT_ERR_ARG, "wt_export: WT_PART_HUFF_CODES needs a Huffman-shaped tree");
    const size_t bytes = (size_t)t->sigma * 8;
    if (needed) *needed = bytes;
    if (!h_dst) return WT_OK;
    if (cap < bytes) return fail(WT_ERR_ARG, "wt_export: capacity %zu < %zu bytes", cap, bytes);
    WT_HIP(hipDeviceSynchronize());
    uint64_t* o = (uint64_t*)h_dst;
    WT_HIP(hipMemcpy(o, t->dev.hcode, bytes, hipMemcpyDeviceToHost));
    // stored left-aligned to L bits; exported right-aligned
    for (uint64_t c = 0; c < t->sigma; ++c) {
      const uint32_t len = (uint32_t)(o[c] >> 32);
      o[c] = len ? ((uint64_t)len << 32) | ((uint32_t)o[c] >> (t->L - len)) : 0ull;
    }
    return WT_OK;
  }
  if (t->matrix && (part == WT_PART_NODE_START || part == WT_PART_NODE_R0))
    return fail(WT_ERR_ARG, "wt_export: a wavelet matrix has no node table");
  if (part != WT_PART_CUM_HIST && (level < 0 || (uint32_t)level >= t->L))
    return fail(WT_ERR_ARG, "wt_export: level %d out of range [0, %u)", level, t->L);
  const LevelMeta m = part == WT_PART_CUM_HIST ? LevelMeta{} : t->hmeta[level];
  const uint64_t nl = m.n;
  const uint64_t s = t->srate;
  size_t bytes = 0;
  const void* src = nullptr;
  bool reverse_samples = false;
  switch (part) {
    case WT_PART_BITS:
      bytes = ceil_div(nl, 64) * 8;
      src = t->dev.bits + m.bits;
      break;
    case WT_PART_L1:
      bytes = (ceil_div(nl, kL1Bits) + 1) * 8;
      src = t->dev.L1 + m.l1;
      break;
    case WT_PART_L2:
      bytes = (ceil_div(nl, t->l2_bits) + 1) * 2;
      src = t->dev.L2 + m.l2;
      break;
    case WT_PART_SAMPLES1:
      bytes = (m.ones / s) * 8;
      src = t->dev.smp + m.smp;
      break;
    case WT_PART_SAMPLES0:
      bytes = ((nl - m.ones) / s) * 8;
      src = t->dev.smp + m.smp + m.smp_cap - (nl - m.ones) / s;
      reverse_samples = true;
      break;
    case WT_PART_NODE_START:
    case WT_PART_NODE_R0:
      bytes = (1ull << level) * 8;
      src = t->dev.nodes + ((1ull << level) - 1);
      break;
    case WT_PART_CUM_HIST:
      bytes = (t->sigma + 1) * 8;
      src = t->dev.cum;
      break;
    default:
      return fail(WT_ERR_ARG, "wt_export: unknown part %d", part);
  }
  if (needed) *needed = bytes;
  if (!h_dst) return WT_OK;
  if (cap < bytes) return fail(WT_ERR_ARG, "wt_export: capacity %zu < %zu bytes", cap, bytes);
  if (bytes == 0) return WT_OK;
  WT_HIP(hipDeviceSynchronize());
  if (part == WT_PART_NODE_START || part == WT_PART_NODE_R0) {
    std::vector<NodeQ> tmp((size_t)1 << level);
    WT_HIP(hipMemcpy(tmp.data(), src, tmp.size() * sizeof(NodeQ), hipMemcpyDeviceToHost));
    uint64_t* d = (uint64_t*)h_dst;
    for (size_t i = 0; i < tmp.size(); ++i) d[i] = part == WT_PART_NODE_START ? tmp[i].start : tmp[i].r0;
    return WT_OK;
  }
  WT_HIP(hipMemcpy(h_dst, src, bytes, hipMemcpyDeviceToHost));
  if (reverse_samples) std::reverse((uint64_t*)h_dst, (uint64_t*)h_dst + bytes / 8);
  return WT_OK;
}

extern "C" wt_status wt_build_profile(const wt_tree* t, wt_prof_entry* out, uint32_t cap, uint32_t* count) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_build_profile: tree is NULL");
  if (count) *count = (uint32_t)t->prof.size();
  if (out) {
    const uint32_t k = std::min<uint32_t>(cap, (uint32_t)t->prof.size());
    for (uint32_t i = 0; i < k; ++i) out[i] = t->prof[i];
  }
  return WT_OK;
}
