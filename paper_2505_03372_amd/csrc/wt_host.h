// Host-side tree object and helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "wt_internal.h"

namespace wt {
// A number no other tree object of the process has had (keys of cached per-tree state).
uint64_t next_tree_uid();
}  // namespace wt

struct wt_tree {
  uint64_t uid = wt::next_tree_uid();
  uint64_t n = 0, sigma = 0;
  uint32_t L = 0, w = 0, l2_bits = 512, srate = 4096, pow2 = 1;
  uint32_t matrix = 0;  // 1: wavelet matrix (no node table; dev.wstart holds the symbols' bottom starts)
  uint32_t huff = 0;    // 1: Huffman-shaped tree (dev.hcode / hsym / hdepth hold its code tables)
  int device = 0;
  void* block = nullptr;  // one allocation holding every device part of the tree
  bool borrowed = false;  // the parts live in a forest's allocation (freed with the forest)
  size_t block_bytes = 0;
  wt::TreeDev dev{};
  wt::LevelMeta hmeta[WT_MAX_LEVELS]{};
  size_t bytes_bits = 0, bytes_l1 = 0, bytes_l2 = 0, bytes_smp = 0, bytes_nodes = 0, bytes_cum = 0;
  std::vector<wt_prof_entry> prof;
  void* learn = nullptr;  // learned select models (device), one per child node
  uint32_t nmodels = 0;
  uint32_t learn_version = 0;  // incremented by every training of the learned index
  wt_learned_info_t linfo{};
  // Alphabet extracted by the build (sigma = 0 given): the tree is built over the codes [0, sigma) of
  // the distinct values; amap maps a value to its code, alpha a code to its value.
  void* alpha_block = nullptr;
  const wt::AWord* amap = nullptr;
  uint64_t amap_words = 0;  // values [0, 64 amap_words) are covered
  const uint32_t* alpha = nullptr;
  uint64_t max_symbol = 0;
};

namespace wt {

wt_status fail(wt_status s, const char* fmt, ...);

// Validation of the build options (|L2| and s), shared by both build paths (wt_build.hip).
wt_status check_build_opts(const wt_build_opts* opts);
// Build of a declared alphabet (wt_build.hip); wt_build itself also handles sigma = 0.
// ntb_out: when given (2^L - 1 entries of device memory), receives the build node table (node
// [start, end) per code prefix, heap order) of a level-wise tree.
wt_status build_tree(const void* d_sym, uint64_t n, uint32_t sym_bytes, uint64_t sigma, const wt_build_opts* opts,
                     wt_stream_t stream, wt_tree** out, NodeB* ntb_out = nullptr);
// Extracted alphabets (wt_alpha.hip): query symbols as codes (*mapped = d_sym when the tree has a
// declared alphabet; otherwise a q-entry buffer, returned in *scratch for the caller to free after the
// traversal; with `buf` given, that q-entry buffer is used and nothing is allocated) and access answers
// back to values.
wt_status alpha_map_syms(const wt_tree* t, const uint32_t* d_sym, uint64_t q, hipStream_t st, const uint32_t** mapped,
                         void** scratch, uint32_t* buf = nullptr);
wt_status alpha_unmap_access(const wt_tree* t, uint32_t* d_out, uint64_t q, hipStream_t st);
// out[i] = sum of in[0, i) (wt_build.hip); part: ceil(n / 4096) + 1 entries of scratch.
hipError_t exclusive_scan_u64(const uint64_t* in, uint64_t n, uint64_t* out, uint64_t* part, hipStream_t st);
void clear_error();
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// Checks a HIP call; on failure records the message and returns WT_ERR_HIP from the caller.
#define WT_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return ::wt::fail(WT_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t round_up(uint64_t a, uint64_t b) { return ceil_div(a, b) * b; }

// Byte sizes of the tree parts for n elements (every level gets the capacity of level 0).
struct TreePlan {
  uint64_t n, sigma;
  uint32_t L, w, l2_bits, srate, tile;
  uint64_t words_per_level;  // bit words per level (padded to whole tiles + one L2 block, 128 B aligned)
  uint64_t l1_per_level, l2_per_level, smp_per_level;
  uint64_t nheap;  // node table entries: 2^L - 1
  size_t off_meta, off_cum, off_nodes, off_bits, off_l1, off_l2, off_smp, off_wstart, off_huff, total;
};

// Bytes of one training record of the learned index (the query forms follow the records).
size_t learn_model_bytes();

// matrix: the parts of a wavelet matrix (no node table; sigma bottom starts instead).
// huff: room for the code tables of a Huffman-shaped tree (huff_table_bytes(sigma) bytes at off_huff).
TreePlan plan_tree(uint64_t n, uint32_t w, uint64_t sigma, uint32_t L, uint32_t l2_bits, uint32_t srate,
                   bool matrix = false, bool huff = false);
// Code tables of a Huffman-shaped tree: hcode (sigma u64), hsym (sigma u32), hdepth (WT_MAX_LEVELS + 1 u64).
inline size_t huff_hsym_off(uint64_t sigma) { return ((sigma * 8 + 255) / 256) * 256; }
inline size_t huff_hdepth_off(uint64_t sigma) { return huff_hsym_off(sigma) + ((sigma * 4 + 255) / 256) * 256; }
inline size_t huff_table_bytes(uint64_t sigma) { return huff_hdepth_off(sigma) + (WT_MAX_LEVELS + 1) * 8; }

// Host memory: page-locked (hipHostMalloc or registered with HIP), and a memcpy split over a few
// threads (a single thread does not reach the host's memory bandwidth). wt_hostq.hip.
bool is_pinned(const void* p);
void par_copy(void* dst, const void* src, size_t bytes);

// Build steps shared by the device build and the build from host memory (wt_build.hip, wt_bv.hip).
// hist[c] += count of c in d_sym[0, n), *err set when a symbol is >= sigma; scratch of
// hist_add_scratch_bytes(n, w, sigma) bytes.
size_t hist_add_scratch_bytes(uint64_t n, uint32_t w, uint64_t sigma);
hipError_t hist_add(const void* d_sym, uint64_t n, uint32_t w, uint64_t sigma, uint64_t* hist, uint32_t* err,
                    char* scratch, hipStream_t st);
// Level metadata (offsets of every level's parts, counts cleared) on the device and the host.
hipError_t init_levels(const TreePlan& P, LevelMeta* d_meta, LevelMeta* h_meta, hipStream_t st);
hipError_t fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st);
// Node tables of a level-wise tree from the cumulative histogram: build entries, query entries, and
// the level sizes (meta[l].n). z, zs: nheap + 1 entries; part: scan partials.
hipError_t node_tables(uint32_t sigma, uint64_t nheap, const uint64_t* cum, NodeB* ntb, uint64_t* z, uint64_t* zs,
                       uint64_t* part, NodeQ* nodes, LevelMeta* meta, hipStream_t st);
// Rank directory and select samples of one level from its bits (bits past n cleared); sets meta->n and
// meta->ones. scratch: bv_directory_scratch_bytes(n) bytes.
size_t bv_directory_scratch_bytes(uint64_t n);
hipError_t bv_directory(uint64_t* bits, uint64_t* L1, uint16_t* L2, uint64_t* smp, LevelMeta* meta, uint64_t n,
                        uint64_t smp_cap, uint32_t l2_bits, uint32_t srate, char* scratch, hipStream_t st);

// Bytes of the level sequence one level-kernel block handles; a tile holds kTileBytes / w elements.
constexpr uint32_t kTileBytes = 16384;
inline uint32_t tile_elems(uint32_t w) { return kTileBytes / w; }

}  // namespace wt
