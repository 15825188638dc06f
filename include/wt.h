/*
 * wt.h — C ABI of the MI355X (gfx950) level-wise wavelet tree.
 *
 * The operations follow the thesis "GPU Implementation of the Wavelet Tree"
 * (M. Franzreb Salgado, 2025):
 *   access(i), rank_c(i), select_c(k) ............ Introduction (query definitions)
 *   tree shape, reduced codes, level construction . Section 5.1 (Construction, Algorithms 3 and 4)
 *   bit arrays, L1/L2 rank directory .............. Section 4, Section 4.1 (Algorithm 1)
 *   select samples ................................ Section 4.2 (Algorithm 2)
 *   precomputed node-start ranks .................. Sections 5.2-5.4
 *   query traversals .............................. Section 5.2 (Algorithm 5), 5.3 (Algorithm 6),
 *                                                   5.4 (Algorithms 7 and 8)
 *
 * Conventions (all calls):
 *  - Positions are 0-based, k is 1-based, rank has an exclusive upper bound
 *    (rank_c(i) counts c in S[0, i), i in [0, n]).
 *  - Pointers named d_* are device pointers (HBM) owned by the caller; they must stay
 *    valid until the work enqueued on `stream` completes. Pointers named h_* are host.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream). Query calls
 *    enqueue one kernel and return without synchronising.
 *  - A tree is owned by the library, immutable after wt_build returns, and may be
 *    queried concurrently from several streams. Its memory comes from the allocator
 *    installed with wt_set_allocator (default: hipMallocAsync / hipFreeAsync).
 *  - Calls never throw; they return a wt_status and, on failure, set a thread-local
 *    message readable with wt_last_error().
 */
#ifndef WT_H
#define WT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wt_tree wt_tree;
typedef void* wt_stream_t; /* hipStream_t */

typedef enum {
  WT_OK = 0,
  WT_ERR_ARG = 1,          /* invalid argument (null pointer, unsupported width or alphabet, ...) */
  WT_ERR_SYMBOL_RANGE = 2, /* a symbol >= sigma was found during the build; no tree is created */
  WT_ERR_OOM = 3,          /* the allocator returned NULL */
  WT_ERR_HIP = 4,          /* a HIP runtime call failed */
  WT_ERR_STATE = 5         /* call not valid in the current state (e.g. no GPU) */
} wt_status;

/* Build options. Zero-initialised fields take the defaults. */
typedef struct {
  uint32_t l2_bits;     /* L2 block size |L2| in bits (Section 4.1): 256, 512 (default), 1024, 2048 */
  uint32_t sample_rate; /* select sample interval s (Section 4.2): power of two in [512, 2^20]; default 4096 */
  uint32_t flags;       /* WT_BUILD_PROFILE: time every build kernel with HIP events (wt_build_profile);
                           WT_BUILD_MATRIX: build the wavelet matrix instead of the level-wise tree;
                           WT_BUILD_WIDE / WT_BUILD_NARROW: carried code width (below);
                           WT_BUILD_HUFFMAN: Huffman-shaped tree */
  uint32_t reserved;
} wt_build_opts;

#define WT_BUILD_PROFILE 1u
/* Wavelet matrix (the layout the thesis's Conclusion names as further work; the structure of Claude,
   Navarro and Ordonez): L = ceil(lg sigma) levels of n bits each, symbols as plain L-bit numbers (no
   reduced codes). Level 0 holds S; level l + 1 holds level l stably partitioned by its bit: every zero
   of the whole level before every one (no nodes), so an element at position p of level l with bit b is
   at rank0_l(p), or at zeros_l + rank1_l(p), in level l + 1. Bit l of an element is bit L-1-l of its
   symbol. Queries need one binary rank (access, rank) or select (select) per level and no node table;
   rank and select also read start[c], the first position of symbol c's run in the order below the
   last level. The same calls (access, rank, select and their sentinels, alphabet extraction, info,
   export of bits / L1 / L2 / samples / WT_PART_WM_STARTS, wt_select_noalloc, wt_free) work on it; the
   learned index, forests and the node-table parts do not (WT_ERR_ARG). */
#define WT_BUILD_MATRIX 2u
/* Carried code width. Narrowing: the level sequence narrows (4 -> 2 -> 1 bytes per element) as soon
   as the code bits the remaining levels need fit, and the levels after the code's prefix bits are
   dropped find each element's node by its position (a node list built from the node table). It saves
   bytes per level but costs launches and node-list passes per build (measured: slower up to 2^24
   symbols, faster from 2^26 on, for 2-byte symbols over 2^16 and 4-byte ones over 2^20), so by
   default it is used from WT_NARROW_MIN_N symbols on. WT_BUILD_WIDE keeps full-width codes at every
   level, WT_BUILD_NARROW narrows at any size (WIDE wins if both are given). The tree is the same
   either way. */
#define WT_BUILD_WIDE 4u
#define WT_BUILD_NARROW 32u
#define WT_NARROW_MIN_N (1ull << 25)
/* Huffman-shaped tree (the Huffman variant the thesis's Conclusion names as a next step; the
   Huffman-shaped wavelet tree of Navarro's survey, which Section 2 cites): the same level-wise layout,
   rank directory, select samples and queries, but the codes are an optimal prefix code for the
   symbol counts of d_sym, so a symbol's elements take as many levels as its code has bits and the
   levels hold sum_c count(c) len(c) bits in all (the zero-order entropy plus less than one bit per
   symbol) instead of n ceil(lg sigma).
   * Lengths: optimal among the prefix codes of the symbols that occur with no code longer than
     min(WT_MAX_LEVELS, ceil(lg m) + 8) bits (m = number of distinct symbols), by package-merge
     (Larmore and Hirschberg): the list of the deepest length is the occurring symbols ordered by
     (count, symbol); every shorter list merges them with the consecutive pairs of the next deeper
     list (an odd last item dropped), by weight, a symbol before a pair of equal weight; the first
     2m - 2 items of the length-1 list are taken, and every pair taken takes its two items one length
     deeper; a symbol's length is the number of lists in which it is taken. A lone symbol gets no code
     (a tree of no level); symbols that do not occur get none either (rank 0, select n).
   * Codes (canonical): the occurring symbols ordered by (length descending, symbol ascending) take
     consecutive left-aligned code values from 0 (each adds 2^(L - length), L = the longest length),
     so at every level the nodes of the longer codes come first and a node starts at the count of
     the symbols ordered before it.
   The code lengths are computed on the host from the histogram (one extra pass over d_sym and one
   copy of sigma counts to the host); WT_PART_HUFF_CODES exports the codes. Not combinable with
   WT_BUILD_MATRIX; forests and the learned index refuse Huffman-shaped trees (WT_ERR_ARG). */
#define WT_BUILD_HUFFMAN 8u

/* Largest declared alphabet: the node tables are indexed by code prefix (2^L entries). */
#define WT_MAX_SIGMA (1ull << 24)
#define WT_MAX_LEVELS 24

typedef void* (*wt_alloc_fn)(size_t bytes, wt_stream_t stream, void* ctx);
typedef void (*wt_free_fn)(void* ptr, wt_stream_t stream, void* ctx);

/* Install the device allocator used for tree memory and build scratch (NULL, NULL restores
   the default). Returned pointers must be 256-byte aligned device memory. */
wt_status wt_set_allocator(wt_alloc_fn alloc_fn, wt_free_fn free_fn, void* ctx);

/*
 * Build the level-wise wavelet tree of d_sym[0, n) (Section 5.1, Algorithm 4).
 *   d_sym     device array of n symbols of sym_bytes bytes each (1, 2 or 4), little-endian.
 *   sigma     declared alphabet size, 1 <= sigma <= min(2^(8 sym_bytes), WT_MAX_SIGMA); every
 *             symbol must lie in [0, sigma). Absent symbols are allowed. Alphabets that are not
 *             powers of two use the thesis's reduced codes (Algorithm 3).
 *             sigma = 0: extract the alphabet (Section 5.1's minimal alphabet; Section 6.3.1 builds
 *             with the alphabet extracted and passed): the distinct values of d_sym, in increasing
 *             order, become the codes 0 .. d-1 and the tree is built over them with sigma = d (at most
 *             WT_MAX_SIGMA distinct values; an empty sequence gets sigma = 1 and no symbol). The tree
 *             keeps the map both ways: every query call takes and returns the caller's values (a value
 *             that does not occur is absent: rank 0, select n), wt_info reports sigma = d and
 *             alphabet_extracted = 1, and WT_PART_ALPHABET exports the values. The extraction reads
 *             d_sym three times more (largest value for 4-byte symbols, presence, rewrite as codes)
 *             and needs a presence map of (largest value + 1) / 4 bytes, kept with the tree.
 *   opts      may be NULL (defaults).
 *   out       receives the tree on WT_OK, NULL otherwise.
 * The call enqueues the build on `stream` and waits for it to finish (it must read back the
 * level sizes and the symbol-range flag). d_sym is not retained.
 * Errors: WT_ERR_ARG (bad arguments, more than WT_MAX_SIGMA distinct values), WT_ERR_SYMBOL_RANGE
 * (a symbol >= sigma), WT_ERR_OOM, WT_ERR_HIP, WT_ERR_STATE (internal error: a level pass found an
 * element whose staging slot lies outside its tile; the write is kept inside the tile and the tree is
 * refused, since the tables it would hold are inconsistent).
 */
wt_status wt_build(const void* d_sym, uint64_t n, uint32_t sym_bytes, uint64_t sigma, const wt_build_opts* opts,
                   wt_stream_t stream, wt_tree** out);

/*
 * Build from host memory in chunks (the chunked construction the thesis's Conclusion names as its next
 * step: the copy to the device overlaps the building, and the device never holds the whole sequence, so
 * sequences larger than what a device-resident build can take are built without unified memory).
 * The result is the tree wt_build makes from a device copy of the same symbols: every part identical.
 *   h_sym     host array (page-locked or pageable) of n symbols of sym_bytes bytes (1, 2 or 4).
 *   sigma     declared alphabet, 1 <= sigma <= WT_MAX_SIGMA (sigma = 0 is not supported here).
 *   opts      as wt_build (l2_bits, sample_rate, WT_BUILD_WIDE / WT_BUILD_NARROW for the chunks' trees, and
 *             WT_BUILD_HOST_TWO_PASS below);
 *             WT_BUILD_MATRIX and WT_BUILD_HUFFMAN are refused.
 *   chunk     symbols per chunk (0: 2^27), at least 2^16.
 *   stats     may be NULL.
 * Every chunk is copied to the device while the previous one is processed, and gets its own tree (the
 * device build). The level-wise order keeps sequence order inside a node, so a node's elements at a
 * level are its segments in the chunks' trees one after the other: each segment is copied, as a bit
 * run, to the node's start (known from the whole sequence's histogram) plus the node's elements in the
 * earlier chunks. Then the rank directory and select samples of every level are made from its bits.
 *   One pass (default, when device memory allows): the chunks' trees (about the tree's size in all) are
 *   kept until the last chunk has added its counts, then placed.
 *   Two passes (WT_BUILD_HOST_TWO_PASS, or when the chunks' trees would not fit): a first pass over
 *   h_sym adds up the counts; the second builds each chunk's tree and places it at once, so the device
 *   holds the tree, its node tables and a working set of a few chunks only, at the price of copying
 *   h_sym twice.
 * Pageable arrays are staged through two page-locked buffers of chunk sym_bytes bytes, filled by host
 * threads. The call waits for the build. Errors: those of wt_build.
 */
#define WT_BUILD_HOST_TWO_PASS 16u

typedef struct {
  uint32_t chunks;     /* chunks per pass */
  uint32_t pinned;     /* 1: h_sym was page-locked (no staging) */
  uint32_t passes;     /* 1 or 2 (see above) */
  float ms_counts;     /* until the counts of the whole sequence are known (the first pass), host clock */
  float ms_build;      /* the rest: placement (and the second pass) and the directories, host clock */
  float ms_total;      /* the whole call */
  uint64_t work_bytes; /* device memory beside the tree, largest */
} wt_build_host_stats;

wt_status wt_build_host(const void* h_sym, uint64_t n, uint32_t sym_bytes, uint64_t sigma, const wt_build_opts* opts,
                        uint64_t chunk, wt_build_host_stats* stats, wt_stream_t stream, wt_tree** out);

/* Release a tree (waits for the device to be idle first). NULL is accepted. */
wt_status wt_free(wt_tree* t);

/*
 * Batched access (Section 5.2, Algorithm 5): d_out[j] = S[d_pos[j]] for j in [0, q).
 * Positions >= n give 0xFFFFFFFF. One kernel on `stream`; q = 0 is a no-op.
 */
wt_status wt_access(const wt_tree* t, const uint64_t* d_pos, uint64_t q, uint32_t* d_out, wt_stream_t stream);

/*
 * Batched rank (Section 5.3, Algorithm 6): d_out[j] = number of d_sym[j] in S[0, d_pos[j]).
 * Positions > n give UINT64_MAX; symbols >= sigma give 0.
 */
wt_status wt_rank(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_pos, uint64_t q, uint64_t* d_out,
                  wt_stream_t stream);

/*
 * Batched select (Section 5.4, Algorithms 7 and 8 with the binary select of Algorithm 2):
 * d_out[j] = 0-based position of the d_k[j]-th occurrence of d_sym[j].
 * k = 0 gives UINT64_MAX; k > count(c) or c >= sigma gives n.
 */
wt_status wt_select(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_k, uint64_t q, uint64_t* d_out,
                    wt_stream_t stream);

/*
 * wt_select without allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same arguments, answers and
 * sentinels as wt_select, and the same kernels. The binning buffers (and, for a tree built with
 * sigma = 0, the symbols mapped to codes) live in a statically sized device array of the library,
 * about 20.6 MiB, that every GPU the library runs on holds until the process ends; the call makes no
 * allocation and no hipFree. At most 2^20 queries per call (WT_ERR_ARG above that; use wt_select).
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (two streams, or two
 * threads) race and must be serialised by the caller (one stream, or an event between them).
 * The first call on a device looks up the array's device address (hipGetSymbolAddress).
 */
wt_status wt_select_noalloc(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_k, uint64_t q,
                            uint64_t* d_out, wt_stream_t stream);

/* Sizes and per-level counts of a built tree. */
typedef struct {
  uint64_t n, sigma;
  uint32_t levels, sym_bytes, l2_bits, sample_rate;
  uint64_t level_n[WT_MAX_LEVELS];    /* elements per level (n_l) */
  uint64_t level_ones[WT_MAX_LEVELS]; /* ones per level */
  uint64_t bytes_bits, bytes_l1, bytes_l2, bytes_samples, bytes_nodes, bytes_total; /* allocated */
  uint32_t alphabet_extracted; /* 1: built with sigma = 0 (queries map values to codes and back) */
  uint32_t matrix;             /* 1: a wavelet matrix (WT_BUILD_MATRIX); level_n[l] = n at every level */
  uint64_t max_symbol;         /* largest symbol value of the alphabet */
  uint32_t huffman;            /* 1: a Huffman-shaped tree (WT_BUILD_HUFFMAN) */
  uint32_t reserved1;
} wt_info_t;

wt_status wt_info(const wt_tree* t, wt_info_t* out);

/* Parts of a tree in canonical form (independent of the physical layout):
 *   WT_PART_BITS       u64[ceil(n_l/64)]      level bits, LSB-first, zero padding
 *   WT_PART_L1         u64[ceil(n_l/65536)+1] ones before each 65536-bit block; last = total
 *   WT_PART_L2         u16[ceil(n_l/|L2|)+1]  ones from the enclosing L1 block start to each |L2| block
 *   WT_PART_SAMPLES1   u64[floor(ones/s)]     position of the (k s)-th one, k = 1, 2, ...
 *   WT_PART_SAMPLES0   u64[floor(zeros/s)]    position of the (k s)-th zero
 *   WT_PART_NODE_START u64[2^l]               start of the node with code prefix p (UINT64_MAX: no node)
 *   WT_PART_NODE_R0    u64[2^l]               rank0 of the level at that start (UINT64_MAX: no node)
 *   WT_PART_CUM_HIST   u64[sigma+1]           exclusive prefix sums of the histogram (level ignored)
 *   WT_PART_ALPHABET   u32[sigma]             symbol value of every code (level ignored): the sorted
 *                                             distinct values of an extracted alphabet, else 0 .. sigma-1
 *   WT_PART_WM_STARTS  u64[sigma]             wavelet matrix only (level ignored): first position of every
 *                                             code's run in the order below the last level (the elements
 *                                             sorted stably by their codes read bit-reversed)
 *   WT_PART_HUFF_CODES u64[sigma]             Huffman-shaped tree only (level ignored): len(c) << 32 |
 *                                             code(c), the code right-aligned (0: c has no code)
 * A wavelet matrix has no node parts (WT_PART_NODE_START / WT_PART_NODE_R0 give WT_ERR_ARG).
 */
enum {
  WT_PART_BITS = 0,
  WT_PART_L1 = 1,
  WT_PART_L2 = 2,
  WT_PART_SAMPLES1 = 3,
  WT_PART_SAMPLES0 = 4,
  WT_PART_NODE_START = 5,
  WT_PART_NODE_R0 = 6,
  WT_PART_CUM_HIST = 7,
  WT_PART_ALPHABET = 8,
  WT_PART_WM_STARTS = 9,
  WT_PART_HUFF_CODES = 10
};

/* Copy one part to host memory h_dst of cap bytes; *needed receives the byte size of the part
   (h_dst may be NULL to query it). Synchronous. WT_ERR_ARG if cap is too small. */
wt_status wt_export(const wt_tree* t, int level, int part, void* h_dst, size_t cap, size_t* needed);

/* Per-kernel durations of the last build of a tree made with WT_BUILD_PROFILE. */
typedef struct {
  char kernel[32]; /* "hist", "scan", "nodes", "tile_scan", "level", ... */
  int32_t level;   /* tree level, or -1 */
  float ms;        /* duration between HIP events recorded around the launch on the build stream */
} wt_prof_entry;

/* Copies up to cap entries; *count receives the number available. */
wt_status wt_build_profile(const wt_tree* t, wt_prof_entry* out, uint32_t cap, uint32_t* count);

/* Per-kernel timing of the query calls of this thread (off by default): while on, every query call
   records HIP events around each of its kernels on its stream. wt_query_profile waits for them, copies
   up to cap entries ({"sort_count" | "sort_scan" | "sort_scatter" | "access" | "rank" | "select" |
   "select_learned", -1, ms} in call order; the sort entries belong to the binning of batches of at
   least 2^16 queries) and clears the list; *count receives the number recorded. */
wt_status wt_query_profiling(int on);
wt_status wt_query_profile(wt_prof_entry* out, uint32_t cap, uint32_t* count);

/* ---- rank and select support of a plain bit array (Section 4, Algorithms 1 and 2) ----
 *
 * wt_bv_build copies the bits d_words[0, ceil(n_bits / 64)) (bit j at bit j mod 64 of word j / 64,
 * LSB-first; bits past n_bits are ignored) into library memory and builds their rank directory
 * (L1 per 65536 bits, L2 per |L2| bits; Section 4.1) and select samples (every s-th one and zero;
 * Section 4.2), with |L2| and s from opts (NULL: 512 and 4096). A bit array is the one level of a
 * wavelet tree over the binary alphabet, so the result is an ordinary tree with sigma = 2 and one
 * level: wt_access(i) gives bit i, wt_rank with symbol b gives rank_b(i) (b in {0, 1}), wt_select
 * with symbol b gives the 0-based position of the k-th bit b, with the sentinels of those calls;
 * wt_export, wt_info, wt_learn_select / wt_select_learned and wt_free work on it as on any tree.
 * Enqueued on `stream`, waits for completion; d_words is not retained.
 * Errors: WT_ERR_ARG (NULL pointers, n_bits >= 2^40, bad options), WT_ERR_OOM, WT_ERR_HIP.
 */
wt_status wt_bv_build(const uint64_t* d_words, uint64_t n_bits, const wt_build_opts* opts, wt_stream_t stream,
                      wt_tree** out);

/* ---- learned select index (an extension of Section 5.4; not in the thesis) ----
 *
 * For every child node of the tree (a node's zeros side or ones side at some level) a small FP32
 * network u -> 1 -> 16 -> 1 (ReLU) -> v maps the node-local occurrence rank of a bit (u in [0, 1],
 * normalised by the child's size) to its position inside the node (v in [0, 1]). It is trained on
 * the GPU, by full-batch Adam on the build's own rank directory (the node-local rank at the start of
 * every |L2| block inside the node, subsampled), with the library's own forward and backward kernels.
 * A learned select then predicts the L2 block of each level's target, corrects the prediction
 * exactly by galloping over the L2 counts within a budget derived from the model's measured error,
 * and falls back to the plain sampled binary search (Algorithm 2) when the budget is exhausted.
 * Answers are identical to wt_select.
 */
typedef struct {
  uint32_t epochs;     /* Adam steps (full batch); 0 = 500 */
  uint32_t max_points; /* training points per model, <= 2048; 0 = 2048 */
  float lr;            /* initial learning rate (linear decay to lr/10); 0 = 3e-3 */
  uint32_t flags;      /* reserved */
} wt_learn_opts;

typedef struct {
  uint32_t models;             /* child nodes with a trained model */
  uint32_t params_per_model;   /* 49 */
  double mean_err_blocks;      /* mean |predicted - true| L2 block over every L2 boundary of every node */
  double max_err_blocks;
  double mean_err_init_blocks; /* same for the untrained starting point (the linear map v = u) */
  double max_err_init_blocks;
  double final_loss_mean;      /* mean over models of the final training loss */
  float train_ms;              /* duration of the training kernels (HIP events) */
  uint32_t reserved;
} wt_learned_info_t;

/* Trains (or retrains) the models of a tree; enqueued on `stream`, waits for completion. */
wt_status wt_learn_select(wt_tree* t, const wt_learn_opts* opts, wt_stream_t stream);

/* Batched select through the learned index (same arguments and results as wt_select). On every
   level, a wavefront whose queries share the level's model predicts the L2 block with it and corrects
   the prediction exactly; a wavefront whose queries are on different models (small unbinned batches)
   takes the sampled binary search of wt_select for that level, as does a prediction that misses by
   more than the model's error budget. WT_ERR_STATE if wt_learn_select has not been called on the tree. */
wt_status wt_select_learned(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_k, uint64_t q,
                            uint64_t* d_out, wt_stream_t stream);

wt_status wt_learned_info(const wt_tree* t, wt_learned_info_t* out);

/* One model of the learned index, read back for inspection. Slots are numbered by child node: the
   child on side b of node (level l, code prefix p) has slot 2^(l+1) - 2 + 2p + b, for 2^(L+1) - 2
   slots in all (L = levels); slots of empty children or of leaves carry eps = -1 and no model.
   For queries the trained network is compiled into its exact piecewise-linear form on [0, 1]:
   v(u) = slope[s] u + intercept[s], where s is the number of knots <= u (the knots are the inputs
   where a hidden unit switches, inside (0, 1), ascending; unused knots are 2). Synchronous.
   WT_ERR_STATE before wt_learn_select, WT_ERR_ARG for a slot out of range. */
typedef struct {
  int32_t level;    /* level l of the parent node (the child's bits are those of level l) */
  uint32_t side;    /* b */
  int32_t eps;      /* correction budget in L2 blocks; -1: no model */
  uint32_t points;  /* training points */
  uint64_t start, len; /* node range in level l */
  uint64_t count;   /* bits equal to b inside the node */
  uint64_t rank0;   /* bits equal to b in level l before start */
  float params[49]; /* w1[16], b1[16], w2[16], b2 */
  uint32_t pieces;  /* number of linear pieces (knots inside (0, 1) plus one) */
  float knots[16];
  float slope[17], intercept[17];
  float err_mean, err_max, err_init_mean, err_init_max; /* in L2 blocks, over every L2 boundary */
  float loss;       /* final training loss */
} wt_learned_model_t;

wt_status wt_learned_model(const wt_tree* t, uint32_t slot, wt_learned_model_t* out);

/* One evaluation of the training objective on the device, with the same device code the training
   kernel uses: d_out[0] = mean squared error of the network d_params (49 floats: w1[16], b1[16],
   w2[16], b2) over the P points (d_u[i], d_v[i]); d_out[1 + j] = its derivative by parameter j.
   For gradient checks against a reference. */
wt_status wt_mlp_loss_grad(const float* d_params, const float* d_u, const float* d_v, uint32_t P, float* d_out,
                           wt_stream_t stream);

/* ---- batched forest build (an extension; the thesis builds one tree at a time) ----
 *
 * Many independent sequences of uneven length and alphabet are built into a forest of wavelet trees
 * by one launch of a captured HIP graph. Every construction phase of Section 5.1 (histogram,
 * cumulative histogram, node tables, and per level the tile prefix and the level pass) runs as one
 * kernel over the blocks of every tree that has work in it; the blocks of a launch are mapped to
 * trees by a table uploaded once, so small trees cost a few blocks instead of a launch sequence each.
 * Each tree is identical to the tree wt_build makes from the same sequence and options.
 */
typedef struct wt_forest wt_forest;

typedef struct {
  const void* d_sym;    /* device symbols of the sequence (sym_bytes each; see wt_build_forest) */
  uint64_t n;           /* length (0 allowed) */
  uint64_t sigma;       /* declared alphabet size, as for wt_build */
  uint32_t l2_bits;     /* 0: chosen by the tuning table of the options, else the default 512 */
  uint32_t sample_rate; /* 0: chosen by the tuning table of the options, else the default 4096 */
} wt_seq_desc;

/* Tuning table: per shape bucket (floor(log2 n) / 2, floor(log2 sigma) / 4), the |L2| and s the
   autotuner picked (0 = not tuned: defaults). Written by wt_autotune. */
#define WT_TUNE_NB 21
#define WT_TUNE_SB 7
typedef struct {
  uint32_t l2_bits[WT_TUNE_NB][WT_TUNE_SB];
  uint32_t sample_rate[WT_TUNE_NB][WT_TUNE_SB];
} wt_tune_table;

typedef struct {
  uint64_t max_probe_n;      /* symbols of the probe sequence of a bucket (a prefix); 0 = 2^22 */
  uint32_t queries;          /* queries per kind and probe; 0 = 2^16 */
  uint32_t reserved;
  double queries_per_symbol; /* expected queries per symbol weighing query time against build time; 0 = 1/64 */
  double space_cap;          /* largest (L2 + L1 + samples) / bits allowed; 0 = 0.10 */
} wt_tune_opts;

typedef struct {
  uint32_t buckets, probes;  /* buckets tuned, builds probed */
  float total_ms;
  uint32_t reserved;
  float cost_ns_per_symbol[WT_TUNE_NB][WT_TUNE_SB]; /* winning cost of every tuned bucket */
} wt_tune_report;

/*
 * Autotuner of |L2| in {256, 512, 1024} and s in {1024, 4096, 16384} (the two parameters Sections 4.1
 * and 4.2 leave open) per shape bucket of the given sequences. For every bucket with a sequence of
 * length >= 1 and sigma >= 2, its longest sequence (a prefix of at most max_probe_n symbols) is built
 * with every pair whose directory and samples fit the space cap, and a batch of each query kind is
 * timed (HIP events) on it; the pair with the least build time per symbol plus queries_per_symbol
 * times the mean query time wins. Buckets without a sequence stay 0 (defaults). Synchronous; the
 * answers of trees built with any pair are the same. report may be NULL.
 */
wt_status wt_autotune(const wt_seq_desc* h_descs, uint32_t count, uint32_t sym_bytes, const wt_tune_opts* opts,
                      wt_stream_t stream, wt_tune_table* out, wt_tune_report* report);

typedef struct {
  const wt_tune_table* tune; /* may be NULL */
  uint32_t flags;            /* WT_BUILD_WIDE: every level carries full-width codes. Default: each tree's
                                carried codes narrow as its levels consume bits (the single-tree rule of
                                WT_BUILD_NARROW, for every tree whatever its length); the trees are the same. */
  uint32_t reserved;
} wt_forest_opts;

typedef struct {
  uint32_t trees, levels_max;
  uint64_t symbols;          /* total length */
  uint64_t bytes_trees;      /* device bytes of every tree's parts (one allocation) */
  uint64_t bytes_scratch;    /* build scratch (freed when wt_build_forest returns) */
  uint32_t graph_kernels;    /* kernel nodes of the captured build graph */
  uint32_t reserved;
  float plan_ms;             /* host planning and the upload of the block tables */
  float capture_ms;          /* graph capture and instantiation */
  float graph_ms;            /* the graph launch (HIP events around it on the stream) */
  float total_ms;            /* the whole call, host clock */
} wt_forest_info_t;

/*
 * Build a forest (one tree per descriptor). All sequences use sym_bytes-byte symbols (1, 2 or 4).
 * Same argument rules and errors as wt_build for every tree; WT_ERR_SYMBOL_RANGE names the first
 * offending tree in wt_last_error. Enqueued on `stream` (a private stream when NULL) and waited for.
 */
wt_status wt_build_forest(const wt_seq_desc* h_descs, uint32_t count, uint32_t sym_bytes, const wt_forest_opts* opts,
                          wt_stream_t stream, wt_forest** out);

/* Borrowed handle of tree j (valid until wt_forest_free): usable with every query, info, export and
   learned-index call; wt_free refuses it (WT_ERR_STATE). */
wt_status wt_forest_tree(const wt_forest* f, uint32_t j, wt_tree** out);

wt_status wt_forest_info(const wt_forest* f, wt_forest_info_t* out);

/* Release a forest and its trees (waits for the device to be idle first). NULL is accepted. */
wt_status wt_forest_free(wt_forest* f);

/*
 * Mixed batched queries over the trees of a forest: query j asks tree d_tree[j] for
 *   d_op[j] = WT_OP_ACCESS: access(d_arg[j])            (d_sym ignored; 0xFFFFFFFF if out of range)
 *             WT_OP_RANK:   rank_{d_sym[j]}(d_arg[j])
 *             WT_OP_SELECT: select_{d_sym[j]}(d_arg[j])
 *             WT_OP_SELECT_LEARNED: accepted and answered as WT_OP_SELECT (the learned index is
 *                           not used inside mixed batches; wt_select_learned uses it)
 * with the results and sentinels of wt_access / wt_rank / wt_select, widened to 64 bits in d_out[j].
 * An unknown tree or op gives UINT64_MAX. Batches above 16384 queries are grouped by (op, |L2| of the
 * tree) on the device so that each wavefront runs one traversal, and from 2^16 queries also by
 * place (tree and position in it) so that a wavefront's traversals share lines; d_out is in the
 * order of the queries. d_sym may be NULL when every op is an access. At most 2^32 - 1 queries per call.
 */
enum { WT_OP_ACCESS = 0, WT_OP_RANK = 1, WT_OP_SELECT = 2, WT_OP_SELECT_LEARNED = 3 };

wt_status wt_query_mixed(const wt_forest* f, const uint32_t* d_tree, const uint8_t* d_op, const uint32_t* d_sym,
                         const uint64_t* d_arg, uint64_t q, uint64_t* d_out, wt_stream_t stream);

/* ---- queries from host memory (Section 5.2.1; Sections 6.3.2-6.3.4) ----
 *
 * wt_query_host answers q queries whose arguments and answers live in host memory: op is
 * WT_OP_ACCESS (h_arg = positions, h_out = u32 answers, h_sym unused), WT_OP_RANK (h_sym, h_arg =
 * positions, u64 answers) or WT_OP_SELECT (h_sym, h_arg = k, u64 answers), with the answers and
 * sentinels of wt_access / wt_rank / wt_select. The batch is cut into chunks of opts->chunk queries
 * (0: 2^22; at most 2^28); each chunk is copied to the device, answered and copied back, and a chunk's
 * copies overlap the kernels of its neighbours, with at most two chunks (their arguments and answers) on
 * the device at a time and one chunk's kernels running at a time.
 *  - Page-locked host arrays (hipHostMalloc, torch pin_memory): with more than one chunk the whole
 *    pipeline is one HIP graph (copy nodes plus each chunk's kernels), instantiated on the first call and
 *    kept, with its chunk buffers, for calls with the same tree, op, arrays, q and chunk (one such graph
 *    per process; wt_query_host_release drops it). WT_HOST_NO_GRAPH enqueues the chunks on streams instead.
 *  - Pageable host arrays: every chunk goes through two page-locked staging slots that the host fills
 *    and empties with its own threads while the device works (no host memory is pinned in place); the
 *    staging buffers are kept for later calls until wt_query_host_release.
 * The call waits for the answers (they are in h_out when it returns). Work starts after what is queued
 * on `stream`. Concurrent calls are safe (serialised on the shared graph and staging). The tree must stay
 * alive during the call. stats may be NULL.
 * Errors: WT_ERR_ARG (NULL arrays, unknown op, chunk too large), WT_ERR_OOM, WT_ERR_HIP.
 */
typedef struct {
  uint64_t chunk;   /* queries per chunk; 0 = 2^22 */
  uint32_t flags;   /* WT_HOST_NO_GRAPH */
  uint32_t reserved;
} wt_host_opts;

#define WT_HOST_NO_GRAPH 1u

typedef struct {
  uint32_t chunks;  /* chunks the batch was cut into */
  uint32_t pinned;  /* 1: the arrays were page-locked (no staging) */
  uint32_t graph;   /* 1: answered by the captured graph */
  uint32_t reserved;
  float ms;         /* wall time of the call (host clock), copies included */
  uint32_t reserved2;
} wt_host_stats;

wt_status wt_query_host(const wt_tree* t, int op, const uint32_t* h_sym, const uint64_t* h_arg, uint64_t q,
                        void* h_out, const wt_host_opts* opts, wt_host_stats* stats, wt_stream_t stream);

/* Drops the cached graph (and its device chunk buffers) and the page-locked staging of wt_query_host. */
wt_status wt_query_host_release(void);

/* ---- serving (an extension): continuous batching over a resident forest ----
 *
 * A server keeps a forest resident and replays a trace of query batches (requests) on its own clock:
 * a request becomes visible at its arrival time and is admitted in arrival order as soon as one of
 * the server's slots (a stream each) is free and the request's device buffers fit in what the memory
 * budget has left (the budget is carved once from device memory at creation). An admitted request
 * copies its queries to the device, runs wt_query_mixed's kernels and copies the answers back, all on
 * its slot's stream, so requests that arrive while others are on the GPU overlap with them.
 * Small requests are coalesced: when a slot frees up, the oldest waiting request and the waiting
 * requests after it, in arrival order, are admitted together while their total stays within
 * coalesce_q queries; they are copied side by side into one device batch, answered by one run of the
 * mixed kernels and copied back each to its own answer array, and complete together; such a batch
 * goes through page-locked staging buffers of its slot (one copy up, one copy down).
 * Latency = completion (observed by the server) - arrival. A request's answers do not depend on what
 * else is in flight. A request larger than the whole budget is rejected (status WT_ERR_OOM).
 */
typedef struct wt_server wt_server;

typedef struct {
  uint32_t slots;          /* batches in flight at once (a stream each); 0 = 8, at most 64 */
  uint32_t coalesce_q;     /* largest total of a coalesced batch of requests; 0 = 16384, 1 = no coalescing */
  uint64_t mem_budget;     /* device bytes for in-flight requests; 0 = 4 GiB */
  double sim_ns_per_query; /* > 0: no GPU; a request occupies its slot for q * this many ns (scheduler tests) */
} wt_server_opts;

typedef struct {
  const uint32_t* h_tree;  /* host arrays of q entries (page-locked memory gives asynchronous copies) */
  const uint8_t* h_op;     /* ops as in wt_query_mixed */
  const uint32_t* h_sym;   /* may be NULL when every op is an access */
  const uint64_t* h_arg;
  uint64_t* h_out;         /* answers as in wt_query_mixed */
  uint64_t q;
  double arrival_s;        /* arrival on the server clock (seconds from the start of wt_server_run) */
} wt_request;

typedef struct {
  double arrival_s, admit_s, done_s;
  uint32_t slot;           /* slot that ran it (UINT32_MAX: rejected) */
  wt_status status;        /* WT_OK, or WT_ERR_OOM when larger than the budget */
} wt_completion;

typedef struct {
  uint32_t requests, rejected, peak_in_flight; /* peak_in_flight counts requests */
  uint32_t batches;        /* device batches run (one per admitted group of coalesced requests) */
  uint64_t queries;        /* answered */
  uint64_t peak_bytes;     /* most device bytes held by admitted requests at once */
  double makespan_s;       /* first arrival to last completion */
  double qps;              /* answered queries / makespan */
  double lat_p50_s, lat_p99_s, lat_mean_s, lat_max_s;
} wt_serve_stats;

/* f may be NULL only with sim_ns_per_query > 0. */
wt_status wt_server_create(const wt_forest* f, const wt_server_opts* opts, wt_server** out);

/* Replays `count` requests sorted by arrival; returns when all are answered or rejected. comps[i]
   describes reqs[i]; stats may be NULL. */
wt_status wt_server_run(wt_server* s, const wt_request* reqs, uint32_t count, wt_completion* comps,
                        wt_serve_stats* stats);

wt_status wt_server_destroy(wt_server* s);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* wt_last_error(void);

/* Library version string. */
const char* wt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WT_H */
