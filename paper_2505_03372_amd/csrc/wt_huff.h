// Huffman-shaped tree: host-side code construction and the device steps of its build (wt_huff.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "wt_internal.h"

namespace wt {

// Codes of a Huffman-shaped tree for one histogram.
struct HuffCode {
  uint32_t L = 0;                // longest code (levels of the tree); 0 for at most one occurring symbol
  uint64_t m = 0;                // occurring symbols
  std::vector<uint64_t> hcode;   // per symbol: len << 32 | code left-aligned to L bits (0: no code)
  std::vector<uint32_t> sym;     // symbol of every rank (canonical order)
  std::vector<uint32_t> code_r;  // left-aligned code of every rank (ascending)
  std::vector<uint64_t> cumr;    // occurrences of the ranks before r (m + 1 entries)
  std::vector<uint64_t> depth;   // d = 0 .. L: F_d << 32 | I_d (ranks from F_d have length <= d;
                                 // the internal nodes of depth d are the prefixes [0, I_d))
};

// Longest code allowed for m occurring symbols: ceil(lg m) + 8, at most WT_MAX_LEVELS.
uint32_t huff_limit(uint64_t m);

// Optimal codes of at most huff_limit(m) bits for the counts hist[0, sigma) (package-merge; ties:
// lighter, then smaller symbol first; a symbol before a package of equal weight), canonical with the
// longer codes on the left.
void huff_code(const uint64_t* hist, uint64_t sigma, HuffCode& hc);

// d_out[i] = left-aligned code of d_sym[i] (wc bytes per element), cnt0[t] = ones of code bit L - 1 in
// tile t (tiles of kTileBytes / wc elements). L >= 1.
hipError_t huff_encode(const void* d_sym, uint32_t w, uint64_t n, uint32_t sigma, const uint64_t* d_hcode,
                       uint32_t L, void* d_out, uint32_t wc, uint64_t* cnt0, hipStream_t st);

// Build node table entries (heap order) and left-child sizes from the codes in rank order.
hipError_t huff_node_walk(uint32_t L, uint64_t m, uint64_t nheap, const uint32_t* d_code_r, const uint64_t* d_cumr,
                          NodeB* ntb, uint64_t* zeros, hipStream_t st);

}  // namespace wt
