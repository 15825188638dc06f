/*
 * Plain CPU oracle for the level-wise wavelet tree — TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load or
 * call this library. It shares no code with the HIP path: the two meet only in the
 * seeded input generators of workloads/.
 *
 * Everything follows the definitions of the thesis "GPU Implementation of the
 * Wavelet Tree" (M. Franzreb Salgado, 2025) written out directly, without blocking,
 * fusion or reordering:
 *
 *  - queries (Introduction): access(i) = S[i] for i in [0, n);
 *    rank_c(i) = #{ j < i : S[j] = c } for i in [0, n] (exclusive bound, SDSL
 *    convention of Section 4); select_c(k) = 0-based position of the k-th c, k >= 1.
 *  - codes (Section 5.1, reduced tree): the node covering symbols [s, e) with
 *    e - s >= 2 splits into [s, s + P) and [s + P, e), P the largest power of two
 *    strictly below e - s; the left child appends bit 0, the right child bit 1.
 *    Codes are stored left-aligned to L = ceil(lg sigma) bits.
 *  - levels (Section 5.1, Construction): level l holds the sequence stably sorted
 *    by the top l code bits, restricted to the elements whose code is longer than
 *    l; its bit for an element is code bit l counted from the MSB.
 *  - bit arrays (Section 4): bit j sits at bit (j mod 64) of 64-bit word j / 64
 *    (least significant bit first); padding bits are zero.
 *  - rank directory (Section 4.1): L1[b] = ones in [0, min(65536 b, n_l)) for
 *    b = 0 .. ceil(n_l / 65536) (the last entry is the total); L2[j] = ones in
 *    [65536 floor(|L2| j / 65536), min(|L2| j, n_l)) for j = 0 .. ceil(n_l / |L2|).
 *  - select samples (Section 4.2): the positions of every s-th one and of every
 *    s-th zero: samples1[k - 1] = position of the (k s)-th one, k >= 1.
 *  - node starts (Section 5, extended level-wise tree): the node with code prefix
 *    p at level l starts at the number of level-l elements with a smaller prefix;
 *    its precomputed rank is rank0 of level l at that start.
 *
 *  - Huffman-shaped tree (Conclusion, named as a further variant; the Huffman-shaped
 *    wavelet tree of Navarro's survey): the same levels, but the codes are an optimal
 *    prefix code for the symbol frequencies of S with no code longer than a limit
 *    (package-merge). Canonical form: the occurring symbols ordered by (code length
 *    descending, symbol ascending) receive consecutive left-aligned code values, so at
 *    every depth the internal nodes are the leftmost prefixes and a node's elements are
 *    preceded in its level by exactly the elements of the symbols ordered before it.
 *
 * Query answers outside the domains of the definitions are sentinels:
 *   access(i >= n) = 0xFFFFFFFF; rank(c, i > n) = UINT64_MAX; rank(c >= sigma, i) = 0;
 *   select(c, 0) = UINT64_MAX; select(c, k > count(c)) = n; select(c >= sigma, k) = n.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sym_at(const void* S, int w, uint64_t i) {
  if (w == 1) return ((const uint8_t*)S)[i];
  if (w == 2) return ((const uint16_t*)S)[i];
  if (w == 4) return ((const uint32_t*)S)[i];
  return ((const uint64_t*)S)[i];
}

/* L = ceil(lg sigma): the smallest L with 2^L >= sigma (sigma >= 1). */
int oracle_num_levels(uint64_t sigma) {
  int L = 0;
  while ((1ull << L) < sigma) ++L;
  return L;
}

/* Largest power of two strictly below x (x >= 2). */
static uint64_t pow2_below(uint64_t x) {
  uint64_t p = 1;
  while (p * 2 < x) p *= 2;
  return p;
}

static void codes_rec(uint64_t s, uint64_t e, uint64_t prefix, int depth, int L, uint64_t* code, uint32_t* len) {
  if (e - s == 1) {
    code[s] = L ? (prefix << (L - depth)) : 0;
    len[s] = (uint32_t)depth;
    return;
  }
  uint64_t P = pow2_below(e - s);
  codes_rec(s, s + P, prefix << 1, depth + 1, L, code, len);
  codes_rec(s + P, e, (prefix << 1) | 1, depth + 1, L, code, len);
}

/* Reduced-tree codes of all symbols in [0, sigma), left-aligned to L bits. */
void oracle_codes(uint64_t sigma, uint64_t* code, uint32_t* len) {
  if (sigma == 0) return;
  codes_rec(0, sigma, 0, 0, oracle_num_levels(sigma), code, len);
}

/* hist[c] = number of occurrences of c in S; returns 1 if some symbol is >= sigma. */
int oracle_hist(const void* S, uint64_t n, int w, uint64_t sigma, uint64_t* hist) {
  memset(hist, 0, sigma * sizeof(uint64_t));
  int bad = 0;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t c = sym_at(S, w, i);
    if (c >= sigma) bad = 1; else hist[c]++;
  }
  return bad;
}

/*
 * Level bits of every level for the given codes (left-aligned to L bits) and code
 * lengths. bits is L rows of `stride` words each (zero padded); level_n[l] receives
 * n_l. The sequence of level l is obtained from S by a stable counting sort on the
 * key code >> (L - l) (the top l code bits); elements whose code length is <= l are
 * left out. Returns -1 if a symbol is >= sigma.
 */
int oracle_level_bits_codes(const void* S, uint64_t n, int w, uint64_t sigma, int L, const uint64_t* code,
                            const uint32_t* len, uint64_t stride, uint64_t* bits, uint64_t* level_n) {
  if (L == 0) return 0;
  uint64_t* order = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  for (uint64_t i = 0; i < n; ++i)
    if (sym_at(S, w, i) >= sigma) { free(order); return -1; }
  memset(bits, 0, (size_t)L * stride * sizeof(uint64_t));
  for (int l = 0; l < L; ++l) {
    /* stable counting sort of positions by the top-l code bits */
    uint64_t nkeys = 1ull << l;
    uint64_t* start = (uint64_t*)calloc(nkeys + 1, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t key = l ? code[sym_at(S, w, i)] >> (L - l) : 0;
      start[key + 1]++;
    }
    for (uint64_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t key = l ? code[sym_at(S, w, i)] >> (L - l) : 0;
      order[start[key]++] = i;
    }
    free(start);
    /* keep the elements whose code continues below level l */
    uint64_t* row = bits + (size_t)l * stride;
    uint64_t m = 0;
    for (uint64_t r = 0; r < n; ++r) {
      uint64_t c = sym_at(S, w, order[r]);
      if (len[c] <= (uint32_t)l) continue;
      uint64_t b = (code[c] >> (L - 1 - l)) & 1;
      if (b) row[m / 64] |= 1ull << (m % 64);
      ++m;
    }
    level_n[l] = m;
  }
  free(order);
  return 0;
}

/* The levels of the reduced tree (codes of oracle_codes, L = ceil(lg sigma)). */
int oracle_level_bits(const void* S, uint64_t n, int w, uint64_t sigma, uint64_t stride,
                      uint64_t* bits, uint64_t* level_n) {
  int L = oracle_num_levels(sigma);
  if (L == 0) return 0;
  uint64_t* code = (uint64_t*)malloc(sigma * sizeof(uint64_t));
  uint32_t* len = (uint32_t*)malloc(sigma * sizeof(uint32_t));
  oracle_codes(sigma, code, len);
  int rc = oracle_level_bits_codes(S, n, w, sigma, L, code, len, stride, bits, level_n);
  free(code); free(len);
  return rc;
}

static int bit_at(const uint64_t* row, uint64_t j) { return (int)((row[j / 64] >> (j % 64)) & 1); }

/* Rank directory of one level from its definition; L1 has ceil(nl/65536)+1
   entries, L2 has ceil(nl/l2)+1 entries. */
void oracle_directory(const uint64_t* row, uint64_t nl, uint64_t l2, uint64_t* L1, uint16_t* L2) {
  uint64_t nL1 = (nl + 65535) / 65536 + 1, nL2 = (nl + l2 - 1) / l2 + 1;
  /* ones_before[x] for x in [0, nl] */
  uint64_t* ones_before = (uint64_t*)malloc((nl + 1) * sizeof(uint64_t));
  ones_before[0] = 0;
  for (uint64_t x = 0; x < nl; ++x) ones_before[x + 1] = ones_before[x] + (uint64_t)bit_at(row, x);
  for (uint64_t b = 0; b < nL1; ++b) {
    uint64_t x = 65536 * b;
    L1[b] = ones_before[x < nl ? x : nl];
  }
  for (uint64_t j = 0; j < nL2; ++j) {
    uint64_t x = l2 * j;
    uint64_t blk = 65536 * (x / 65536);
    uint64_t hi = x < nl ? x : nl, lo = blk < nl ? blk : nl;
    L2[j] = (uint16_t)(ones_before[hi] - ones_before[lo]);
  }
  free(ones_before);
}

/* Select samples of one level. s1 receives floor(ones/s) entries, s0 floor(zeros/s). */
void oracle_samples(const uint64_t* row, uint64_t nl, uint64_t s, uint64_t* s1, uint64_t* n1, uint64_t* s0,
                    uint64_t* n0) {
  uint64_t ones = 0, zeros = 0;
  *n1 = 0; *n0 = 0;
  for (uint64_t x = 0; x < nl; ++x) {
    if (bit_at(row, x)) {
      ++ones;
      if (ones % s == 0) s1[(*n1)++] = x;
    } else {
      ++zeros;
      if (zeros % s == 0) s0[(*n0)++] = x;
    }
  }
}

/*
 * Node starts and precomputed ranks at level l for every code prefix p in [0, 2^l), for the given
 * codes (left-aligned to L bits) and lengths.
 * A prefix names a node when some symbol whose code is longer than l carries it;
 * otherwise both outputs are UINT64_MAX.
 */
void oracle_nodes_codes(const void* S, uint64_t n, int w, uint64_t sigma, int L, const uint64_t* code,
                        const uint32_t* len, int l, const uint64_t* row, uint64_t* start, uint64_t* r0) {
  uint64_t np = 1ull << l;
  char* exists = (char*)calloc(np, 1);
  uint64_t* count = (uint64_t*)calloc(np, sizeof(uint64_t));
  for (uint64_t c = 0; c < sigma; ++c)
    if (len[c] > (uint32_t)l) exists[l ? code[c] >> (L - l) : 0] = 1;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t c = sym_at(S, w, i);
    if (len[c] > (uint32_t)l) count[l ? code[c] >> (L - l) : 0]++;
  }
  uint64_t nl = 0;
  for (uint64_t p = 0; p < np; ++p) nl += count[p];
  /* zeros_before[x] = zeros of the level in [0, x) */
  uint64_t* zeros_before = (uint64_t*)malloc((nl + 1) * sizeof(uint64_t));
  zeros_before[0] = 0;
  for (uint64_t x = 0; x < nl; ++x) zeros_before[x + 1] = zeros_before[x] + (uint64_t)(1 - bit_at(row, x));
  uint64_t before = 0;
  for (uint64_t p = 0; p < np; ++p) {
    if (exists[p]) {
      start[p] = before;
      r0[p] = zeros_before[before];
    } else {
      start[p] = UINT64_MAX;
      r0[p] = UINT64_MAX;
    }
    before += count[p];
  }
  free(zeros_before); free(exists); free(count);
}

/* Node starts of the reduced tree (codes of oracle_codes). */
void oracle_nodes(const void* S, uint64_t n, int w, uint64_t sigma, int l, const uint64_t* row,
                  uint64_t* start, uint64_t* r0) {
  int L = oracle_num_levels(sigma);
  uint64_t* code = (uint64_t*)malloc(sigma * sizeof(uint64_t));
  uint32_t* len = (uint32_t*)malloc(sigma * sizeof(uint32_t));
  oracle_codes(sigma, code, len);
  oracle_nodes_codes(S, n, w, sigma, L, code, len, l, row, start, r0);
  free(code); free(len);
}

/*
 * Huffman-shaped tree: code lengths. For the symbols that occur (hist[c] > 0), lengths of an
 * optimal prefix code (least sum of hist[c] * len[c]) among those with no length above `limit`,
 * by the package-merge method of Larmore and Hirschberg: the list of depth `limit` is the
 * occurring symbols ordered by (count, symbol); the list of depth d < limit merges those symbols
 * with the packages of the list of depth d + 1 (its items paired in order, first with second,
 * third with fourth, ..., an odd last item dropped; a package weighs the sum of its pair), by
 * weight, a symbol before a package of equal weight. The first 2m - 2 items of the depth-1 list
 * are taken (m occurring symbols), and the packages taken at depth d take their two items at
 * depth d + 1; a symbol's length is the number of depths at which it is taken. Symbols that do not
 * occur get length 0, and so does a lone occurring symbol (a tree of no level). Returns the
 * largest length, or -1 if 2^limit < m.
 */
typedef struct {
  uint64_t weight;
  uint64_t sym;
} HLeaf;

static int hleaf_cmp(const void* a, const void* b) {
  const HLeaf* x = (const HLeaf*)a;
  const HLeaf* y = (const HLeaf*)b;
  if (x->weight != y->weight) return x->weight < y->weight ? -1 : 1;
  return x->sym < y->sym ? -1 : (x->sym > y->sym);
}

int oracle_huffman_lengths(const uint64_t* hist, uint64_t sigma, int limit, uint32_t* len) {
  memset(len, 0, sigma * sizeof(uint32_t));
  uint64_t m = 0;
  for (uint64_t c = 0; c < sigma; ++c) m += hist[c] > 0;
  if (m <= 1) return 0;
  if (limit < 1 || (limit < 63 && (1ull << limit) < m)) return -1;
  HLeaf* leaf = (HLeaf*)malloc(m * sizeof(HLeaf));
  uint64_t j = 0;
  for (uint64_t c = 0; c < sigma; ++c)
    if (hist[c] > 0) { leaf[j].weight = hist[c]; leaf[j].sym = c; ++j; }
  qsort(leaf, m, sizeof(HLeaf), hleaf_cmp);
  /* is_leaf[d][x]: item x of the list of depth d (1..limit) is a symbol (1) or a package (0) */
  uint64_t cap = 2 * m;
  char* is_leaf = (char*)calloc((size_t)(limit + 1) * cap, 1);
  uint64_t* items = (uint64_t*)calloc((size_t)(limit + 1), sizeof(uint64_t));
  uint64_t* wprev = (uint64_t*)malloc(cap * sizeof(uint64_t));
  uint64_t* wcur = (uint64_t*)malloc(cap * sizeof(uint64_t));
  uint64_t nprev = 0;
  for (int d = limit; d >= 1; --d) {
    char* fl = is_leaf + (size_t)d * cap;
    uint64_t npk = d == limit ? 0 : nprev / 2, a = 0, k = 0, x = 0;
    while (a < m || k < npk) {
      uint64_t pw = k < npk ? wprev[2 * k] + wprev[2 * k + 1] : 0;
      if (a < m && (k >= npk || leaf[a].weight <= pw)) {
        wcur[x] = leaf[a].weight;
        fl[x] = 1;
        ++a;
      } else {
        wcur[x] = pw;
        fl[x] = 0;
        ++k;
      }
      ++x;
    }
    items[d] = x;
    nprev = x;
    uint64_t* tmp = wprev; wprev = wcur; wcur = tmp;
  }
  uint64_t take = 2 * m - 2;
  int maxlen = 0;
  for (int d = 1; d <= limit && take > 0; ++d) {
    const char* fl = is_leaf + (size_t)d * cap;
    uint64_t leaves = 0;
    for (uint64_t x = 0; x < take && x < items[d]; ++x) leaves += (uint64_t)fl[x];
    for (uint64_t a = 0; a < leaves; ++a) {
      len[leaf[a].sym] += 1;
      if ((int)len[leaf[a].sym] > maxlen) maxlen = (int)len[leaf[a].sym];
    }
    take = 2 * (take - leaves);
  }
  free(leaf); free(is_leaf); free(items); free(wprev); free(wcur);
  return maxlen;
}

/*
 * Huffman-shaped tree: canonical codes for the lengths len[] (0 = no code). The symbols with a
 * code, ordered by (length descending, symbol ascending), get ranks 0, 1, ... and left-aligned
 * code values (L = the largest length) V_0 = 0, V_{r+1} = V_r + 2^(L - len_r); rank[c] =
 * UINT32_MAX for a symbol without a code. Returns L.
 */
int oracle_huffman_codes(const uint32_t* len, uint64_t sigma, uint64_t* code, uint32_t* rank) {
  int L = 0;
  for (uint64_t c = 0; c < sigma; ++c) if ((int)len[c] > L) L = (int)len[c];
  uint64_t v = 0;
  uint32_t r = 0;
  for (uint64_t c = 0; c < sigma; ++c) { code[c] = 0; rank[c] = UINT32_MAX; }
  for (int ell = L; ell >= 1; --ell)
    for (uint64_t c = 0; c < sigma; ++c)
      if ((int)len[c] == ell) {
        code[c] = v;
        rank[c] = r++;
        v += 1ull << (L - ell);
      }
  return L;
}

/*
 * Wavelet matrix (named in the thesis's Conclusion as a further layout; the structure of Claude,
 * Navarro and Ordonez): every level holds all n elements. Symbols are plain L-bit binary numbers
 * (L = ceil(lg sigma)). Level l holds S stably sorted by the key rev_l(c >> (L - l)), the top l bits
 * of the symbol read in reverse order (the least significant of them first), which is what l stable
 * zeros-then-ones partitions by the bits L-1, L-2, ... leave behind; its bit for an element is bit
 * L-1-l of the symbol. zeros[l] receives the zeros of level l. Returns -1 if a symbol is >= sigma.
 */
static uint64_t rev_bits(uint64_t x, int l) {
  uint64_t r = 0;
  for (int i = 0; i < l; ++i) r |= ((x >> i) & 1) << (l - 1 - i);
  return r;
}

int oracle_wm_level_bits(const void* S, uint64_t n, int w, uint64_t sigma, uint64_t stride, uint64_t* bits,
                         uint64_t* zeros) {
  int L = oracle_num_levels(sigma);
  if (L == 0) return 0;
  for (uint64_t i = 0; i < n; ++i)
    if (sym_at(S, w, i) >= sigma) return -1;
  uint64_t* order = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  memset(bits, 0, (size_t)L * stride * sizeof(uint64_t));
  for (int l = 0; l < L; ++l) {
    /* stable counting sort of positions by the reversed top-l bits */
    uint64_t nkeys = 1ull << l;
    uint64_t* start = (uint64_t*)calloc(nkeys + 1, sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) start[rev_bits(sym_at(S, w, i) >> (L - l), l) + 1]++;
    for (uint64_t k = 0; k < nkeys; ++k) start[k + 1] += start[k];
    for (uint64_t i = 0; i < n; ++i) order[start[rev_bits(sym_at(S, w, i) >> (L - l), l)]++] = i;
    free(start);
    uint64_t* row = bits + (size_t)l * stride;
    uint64_t z = 0;
    for (uint64_t r = 0; r < n; ++r) {
      uint64_t b = (sym_at(S, w, order[r]) >> (L - 1 - l)) & 1;
      if (b) row[r / 64] |= 1ull << (r % 64);
      else ++z;
    }
    zeros[l] = z;
  }
  free(order);
  return 0;
}

/* Start of every symbol's run in the order below the last wavelet-matrix level (S stably sorted by
   rev_L(c)): starts[c] = number of elements whose reversed symbol is smaller than rev_L(c), i.e. the
   exclusive prefix sums of the counts taken in increasing order of the reversed symbols (a sort of
   the symbols by their reversed codes gives that order). */
typedef struct { uint64_t key, c; } rkey;

static int rkey_cmp(const void* a, const void* b) {
  const rkey* x = (const rkey*)a;
  const rkey* y = (const rkey*)b;
  return x->key < y->key ? -1 : (x->key > y->key);
}

void oracle_wm_starts(const void* S, uint64_t n, int w, uint64_t sigma, uint64_t* starts) {
  int L = oracle_num_levels(sigma);
  uint64_t* cnt = (uint64_t*)calloc(sigma ? sigma : 1, sizeof(uint64_t));
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t x = sym_at(S, w, i);
    if (x < sigma) cnt[x]++;
  }
  rkey* order = (rkey*)malloc((sigma ? sigma : 1) * sizeof(rkey));
  for (uint64_t c = 0; c < sigma; ++c) { order[c].key = rev_bits(c, L); order[c].c = c; }
  qsort(order, sigma, sizeof(rkey), rkey_cmp);
  uint64_t before = 0;
  for (uint64_t r = 0; r < sigma; ++r) {
    starts[order[r].c] = before;
    before += cnt[order[r].c];
  }
  free(order);
  free(cnt);
}

/* Minimal alphabet (Section 5.1: the symbols are the distinct values of the sequence, numbered in
   increasing order): the distinct values of S, ascending, in values[] (capacity n); returns their number. */
static int u64_cmp(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y);
}

uint64_t oracle_alphabet(const void* S, uint64_t n, int w, uint64_t* values) {
  for (uint64_t i = 0; i < n; ++i) values[i] = sym_at(S, w, i);
  qsort(values, n, sizeof(uint64_t), u64_cmp);
  uint64_t d = 0;
  for (uint64_t i = 0; i < n; ++i)
    if (d == 0 || values[i] != values[d - 1]) values[d++] = values[i];
  return d;
}

/* ---- query answers from the raw sequence (sweep over S) ---- */

void oracle_access(const void* S, uint64_t n, int w, const uint64_t* pos, uint64_t q, uint32_t* out) {
  for (uint64_t j = 0; j < q; ++j) out[j] = pos[j] < n ? (uint32_t)sym_at(S, w, pos[j]) : 0xFFFFFFFFu;
}

typedef struct { uint64_t key1, key2, idx; } qent;

static int qent_cmp(const void* a, const void* b) {
  const qent* x = (const qent*)a;
  const qent* y = (const qent*)b;
  if (x->key1 != y->key1) return x->key1 < y->key1 ? -1 : 1;
  if (x->key2 != y->key2) return x->key2 < y->key2 ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* rank answers: queries sorted by position, one sweep of S with running counts. */
void oracle_rank(const void* S, uint64_t n, int w, uint64_t sigma, const uint32_t* c, const uint64_t* i,
                 uint64_t q, uint64_t* out) {
  qent* e = (qent*)malloc((q ? q : 1) * sizeof(qent));
  uint64_t m = 0;
  for (uint64_t j = 0; j < q; ++j) {
    if (i[j] > n) { out[j] = UINT64_MAX; continue; }
    if (c[j] >= sigma) { out[j] = 0; continue; }
    e[m].key1 = i[j]; e[m].key2 = c[j]; e[m].idx = j; ++m;
  }
  qsort(e, m, sizeof(qent), qent_cmp);
  uint64_t* cnt = (uint64_t*)calloc(sigma ? sigma : 1, sizeof(uint64_t));
  uint64_t r = 0;
  for (uint64_t p = 0; p <= n; ++p) {
    while (r < m && e[r].key1 == p) { out[e[r].idx] = cnt[e[r].key2]; ++r; }
    if (p < n) { uint64_t s = sym_at(S, w, p); if (s < sigma) cnt[s]++; }
  }
  free(cnt); free(e);
}

/* select answers: queries grouped by symbol and sorted by k; one sweep of S. */
void oracle_select(const void* S, uint64_t n, int w, uint64_t sigma, const uint32_t* c, const uint64_t* k,
                   uint64_t q, uint64_t* out) {
  qent* e = (qent*)malloc((q ? q : 1) * sizeof(qent));
  uint64_t m = 0;
  for (uint64_t j = 0; j < q; ++j) {
    if (k[j] == 0) { out[j] = UINT64_MAX; continue; }
    if (c[j] >= sigma) { out[j] = n; continue; }
    out[j] = n; /* stays n when k exceeds the count of c */
    e[m].key1 = c[j]; e[m].key2 = k[j]; e[m].idx = j; ++m;
  }
  qsort(e, m, sizeof(qent), qent_cmp);
  uint64_t* head = (uint64_t*)malloc((sigma ? sigma : 1) * sizeof(uint64_t));
  uint64_t* endq = (uint64_t*)malloc((sigma ? sigma : 1) * sizeof(uint64_t));
  uint64_t* cnt = (uint64_t*)calloc(sigma ? sigma : 1, sizeof(uint64_t));
  for (uint64_t s = 0; s < sigma; ++s) { head[s] = 0; endq[s] = 0; }
  for (uint64_t r = 0; r < m;) {
    uint64_t s = e[r].key1, r2 = r;
    while (r2 < m && e[r2].key1 == s) ++r2;
    head[s] = r; endq[s] = r2; r = r2;
  }
  for (uint64_t p = 0; p < n; ++p) {
    uint64_t s = sym_at(S, w, p);
    if (s >= sigma) continue;
    cnt[s]++;
    while (head[s] < endq[s] && e[head[s]].key2 == cnt[s]) { out[e[head[s]].idx] = p; head[s]++; }
  }
  free(head); free(endq); free(cnt); free(e);
}

/* ---- learned select predictor: 1 -> 16 -> 1 ReLU network, FP64 reference ----
 * Parameters theta[49]: w1[16], b1[16], w2[16], b2.
 *   h_k = w1_k u + b1_k,  a_k = max(h_k, 0),  y = sum_k w2_k a_k + b2.
 * Loss over P points: L = (1/P) sum_i (y_i - v_i)^2. The ReLU derivative at 0 is taken as 0.
 */
#define MLP_H 16

double oracle_mlp_forward(const double* th, double u) {
  double y = th[48];
  for (int k = 0; k < MLP_H; ++k) {
    double h = th[k] * u + th[16 + k];
    if (h > 0) y += th[32 + k] * h;
  }
  return y;
}

/* Loss and its gradient with respect to the 49 parameters (grad may be NULL). */
double oracle_mlp_loss_grad(const double* th, const double* u, const double* v, int P, double* grad) {
  double loss = 0;
  if (grad) memset(grad, 0, 49 * sizeof(double));
  for (int i = 0; i < P; ++i) {
    double y = oracle_mlp_forward(th, u[i]);
    double r = y - v[i];
    loss += r * r;
    if (!grad) continue;
    double g = 2.0 * r / P;
    grad[48] += g;
    for (int k = 0; k < MLP_H; ++k) {
      double h = th[k] * u[i] + th[16 + k];
      if (h > 0) {
        grad[32 + k] += g * h;
        grad[k] += g * th[32 + k] * u[i];
        grad[16 + k] += g * th[32 + k];
      }
    }
  }
  return loss / P;
}
