/*
 * All-core form of the CPU oracle (OpenMP) — TEST INFRASTRUCTURE ONLY.
 *
 * Same status as wt_oracle.c: only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
 * leg may load it; it shares no code with the HIP path.
 *
 * The answers are those of the definitions in the thesis's Introduction (access, exclusive rank,
 * 1-based select) and the tree parts of Sections 4 and 5.1, exactly as wt_oracle.c computes them.
 * Only the work is spread over host threads, in the plainest way that keeps every step checkable:
 *
 *  queries (sweep form): S is cut into T contiguous chunks (T = 4 x threads). Every chunk counts
 *  its symbols (C[t][c]); an exclusive prefix over the chunks gives P[t][c], the occurrences of c
 *  before chunk t, and total[c] = count(c).
 *   - rank(c, i), i < n: the query goes to chunk t = i / chunk length; the chunk's queries are
 *     sorted by i and answered by one sweep of the chunk with running counts that start at
 *     P[t][.]. rank(c, n) = total[c].
 *   - select(c, k), 1 <= k <= total[c]: the chunk is the t with P[t][c] < k <= P[t][c] + C[t][c];
 *     k' = k - P[t][c]; the chunk's queries are sorted by (c, k') and answered by one sweep that
 *     counts each symbol's occurrences inside the chunk.
 *   Sentinels as in wt_oracle.c: access(i >= n) = 0xFFFFFFFF; rank(c, i > n) = UINT64_MAX;
 *   rank(c >= sigma, i) = 0; select(c, 0) = UINT64_MAX; select(c, k > count) = select(c >= sigma) = n.
 *
 *  tree parts: the levels are independent of each other (level l is S stably sorted by the top l
 *  code bits), so each level is computed by one thread, with the functions of wt_oracle.c.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from wt_oracle.c */
int oracle_num_levels(uint64_t sigma);
void oracle_codes(uint64_t sigma, uint64_t* code, uint32_t* len);
void oracle_directory(const uint64_t* row, uint64_t nl, uint64_t l2, uint64_t* L1, uint16_t* L2);
void oracle_samples(const uint64_t* row, uint64_t nl, uint64_t s, uint64_t* s1, uint64_t* n1, uint64_t* s0,
                    uint64_t* n0);

static uint64_t psym(const void* S, int w, uint64_t i) {
  if (w == 1) return ((const uint8_t*)S)[i];
  if (w == 2) return ((const uint16_t*)S)[i];
  if (w == 4) return ((const uint32_t*)S)[i];
  return ((const uint64_t*)S)[i];
}

int oracle_par_threads(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

void oracle_par_access(const void* S, uint64_t n, int w, const uint64_t* pos, uint64_t q, uint32_t* out,
                       int nthreads) {
  const int nt = oracle_par_threads(nthreads);
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t j = 0; j < (int64_t)q; ++j) out[j] = pos[j] < n ? (uint32_t)psym(S, w, pos[j]) : 0xFFFFFFFFu;
}

/* Chunk counts C[t][c] (T x sigma) and their exclusive prefix P over t; total[c]. */
typedef struct {
  uint64_t T, cl;  /* chunks, chunk length */
  uint64_t* C;
  uint64_t* P;
  uint64_t* total;
} chunks_t;

static void chunk_counts(const void* S, uint64_t n, int w, uint64_t sigma, int nt, chunks_t* ch) {
  ch->T = 4 * (uint64_t)nt;
  ch->cl = (n + ch->T - 1) / ch->T;
  if (ch->cl == 0) ch->cl = 1;
  ch->C = (uint64_t*)calloc(ch->T * sigma, sizeof(uint64_t));
  ch->P = (uint64_t*)calloc(ch->T * sigma, sizeof(uint64_t));
  ch->total = (uint64_t*)calloc(sigma, sizeof(uint64_t));
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
  for (int64_t t = 0; t < (int64_t)ch->T; ++t) {
    uint64_t a = (uint64_t)t * ch->cl, b = a + ch->cl;
    if (b > n) b = n;
    uint64_t* row = ch->C + (uint64_t)t * sigma;
    for (uint64_t i = a; i < b; ++i) {
      uint64_t c = psym(S, w, i);
      if (c < sigma) row[c]++;
    }
  }
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t c = 0; c < (int64_t)sigma; ++c) {
    uint64_t run = 0;
    for (uint64_t t = 0; t < ch->T; ++t) {
      ch->P[t * sigma + c] = run;
      run += ch->C[t * sigma + c];
    }
    ch->total[c] = run;
  }
}

static void chunks_free(chunks_t* ch) {
  free(ch->C);
  free(ch->P);
  free(ch->total);
}

typedef struct { uint64_t key1, key2, idx; } pq_t;

static int pq_cmp(const void* a, const void* b) {
  const pq_t* x = (const pq_t*)a;
  const pq_t* y = (const pq_t*)b;
  if (x->key1 != y->key1) return x->key1 < y->key1 ? -1 : 1;
  if (x->key2 != y->key2) return x->key2 < y->key2 ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Queries grouped by chunk: a counting sort of (chunk, entry) pairs. */
static void bucket(const uint64_t* chunk_of, const pq_t* e, uint64_t m, uint64_t T, uint64_t** start_out,
                   pq_t** sorted_out) {
  uint64_t* start = (uint64_t*)calloc(T + 1, sizeof(uint64_t));
  pq_t* s = (pq_t*)malloc((m ? m : 1) * sizeof(pq_t));
  for (uint64_t r = 0; r < m; ++r) start[chunk_of[r] + 1]++;
  for (uint64_t t = 0; t < T; ++t) start[t + 1] += start[t];
  uint64_t* cur = (uint64_t*)malloc((T + 1) * sizeof(uint64_t));
  memcpy(cur, start, (T + 1) * sizeof(uint64_t));
  for (uint64_t r = 0; r < m; ++r) s[cur[chunk_of[r]]++] = e[r];
  free(cur);
  *start_out = start;
  *sorted_out = s;
}

void oracle_par_rank(const void* S, uint64_t n, int w, uint64_t sigma, const uint32_t* c, const uint64_t* i,
                     uint64_t q, uint64_t* out, int nthreads) {
  const int nt = oracle_par_threads(nthreads);
  chunks_t ch;
  chunk_counts(S, n, w, sigma ? sigma : 1, nt, &ch);
  pq_t* e = (pq_t*)malloc((q ? q : 1) * sizeof(pq_t));
  uint64_t* tof = (uint64_t*)malloc((q ? q : 1) * sizeof(uint64_t));
  uint64_t m = 0;
  for (uint64_t j = 0; j < q; ++j) {
    if (i[j] > n) { out[j] = UINT64_MAX; continue; }
    if (c[j] >= sigma) { out[j] = 0; continue; }
    if (i[j] == n) { out[j] = ch.total[c[j]]; continue; }
    e[m].key1 = i[j]; e[m].key2 = c[j]; e[m].idx = j;
    tof[m] = i[j] / ch.cl;
    ++m;
  }
  uint64_t* start;
  pq_t* s;
  bucket(tof, e, m, ch.T, &start, &s);
#pragma omp parallel num_threads(nt)
  {
    uint64_t* cnt = (uint64_t*)malloc(sigma * sizeof(uint64_t));
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < (int64_t)ch.T; ++t) {
      uint64_t lo = start[t], hi = start[t + 1];
      if (lo == hi) continue;
      qsort(s + lo, hi - lo, sizeof(pq_t), pq_cmp);
      memcpy(cnt, ch.P + (uint64_t)t * sigma, sigma * sizeof(uint64_t));
      uint64_t p = (uint64_t)t * ch.cl, r = lo;
      for (; r < hi; ++p) {
        while (r < hi && s[r].key1 == p) { out[s[r].idx] = cnt[s[r].key2]; ++r; }
        if (p < n) {
          uint64_t x = psym(S, w, p);
          if (x < sigma) cnt[x]++;
        }
      }
    }
    free(cnt);
  }
  free(start); free(s); free(tof); free(e);
  chunks_free(&ch);
}

void oracle_par_select(const void* S, uint64_t n, int w, uint64_t sigma, const uint32_t* c, const uint64_t* k,
                       uint64_t q, uint64_t* out, int nthreads) {
  const int nt = oracle_par_threads(nthreads);
  chunks_t ch;
  chunk_counts(S, n, w, sigma ? sigma : 1, nt, &ch);
  pq_t* e = (pq_t*)malloc((q ? q : 1) * sizeof(pq_t));
  uint64_t* tof = (uint64_t*)malloc((q ? q : 1) * sizeof(uint64_t));
  uint64_t m = 0;
  for (uint64_t j = 0; j < q; ++j) {
    if (k[j] == 0) { out[j] = UINT64_MAX; continue; }
    if (c[j] >= sigma || k[j] > ch.total[c[j]]) { out[j] = n; continue; }
    /* largest chunk t with P[t][c] < k: the k-th occurrence lies in it */
    uint64_t lo = 0, hi = ch.T - 1;
    while (lo < hi) {
      uint64_t mid = (lo + hi + 1) / 2;
      if (ch.P[mid * sigma + c[j]] < k[j]) lo = mid;
      else hi = mid - 1;
    }
    e[m].key1 = c[j]; e[m].key2 = k[j] - ch.P[lo * sigma + c[j]]; e[m].idx = j;
    tof[m] = lo;
    ++m;
  }
  uint64_t* start;
  pq_t* s;
  bucket(tof, e, m, ch.T, &start, &s);
#pragma omp parallel num_threads(nt)
  {
    uint64_t* cnt = (uint64_t*)calloc(sigma, sizeof(uint64_t));
    uint64_t* head = (uint64_t*)malloc(sigma * sizeof(uint64_t));
    uint64_t* endq = (uint64_t*)malloc(sigma * sizeof(uint64_t));
    uint64_t* mark = (uint64_t*)calloc(sigma, sizeof(uint64_t)); /* t + 1 when asked in chunk t */
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < (int64_t)ch.T; ++t) {
      uint64_t lo = start[t], hi = start[t + 1];
      if (lo == hi) continue;
      qsort(s + lo, hi - lo, sizeof(pq_t), pq_cmp);
      /* the symbols asked in this chunk: their pending queries [head, endq), sorted by k' */
      for (uint64_t r = lo; r < hi;) {
        uint64_t x = s[r].key1, r2 = r;
        while (r2 < hi && s[r2].key1 == x) ++r2;
        head[x] = r; endq[x] = r2; cnt[x] = 0; mark[x] = (uint64_t)t + 1;
        r = r2;
      }
      uint64_t a = (uint64_t)t * ch.cl, b = a + ch.cl;
      if (b > n) b = n;
      for (uint64_t p = a; p < b; ++p) {
        uint64_t x = psym(S, w, p);
        if (x >= sigma || mark[x] != (uint64_t)t + 1) continue;
        cnt[x]++;
        while (head[x] < endq[x] && s[head[x]].key2 == cnt[x]) { out[s[head[x]].idx] = p; head[x]++; }
      }
    }
    free(mark);
    free(cnt); free(head); free(endq);
  }
  free(start); free(s); free(tof); free(e);
  chunks_free(&ch);
}

/*
 * Every tree part of every level, one level per thread: the level's bits by a stable counting sort
 * on the top-l code bits (the definition of wt_oracle.c's oracle_level_bits), then its directory and
 * samples with oracle_directory / oracle_samples. bits: L rows of `stride` words; L1: L rows of
 * l1_stride; L2: L rows of l2_stride; s1/s0: L rows of s_stride; n1/n0/level_n: L entries.
 * Returns -1 if a symbol is >= sigma.
 */
int oracle_par_tree(const void* S, uint64_t n, int w, uint64_t sigma, uint64_t l2, uint64_t srate, uint64_t stride,
                    uint64_t* bits, uint64_t* level_n, uint64_t l1_stride, uint64_t* L1, uint64_t l2_stride,
                    uint16_t* L2, uint64_t s_stride, uint64_t* s1, uint64_t* n1, uint64_t* s0, uint64_t* n0,
                    int nthreads) {
  const int nt = oracle_par_threads(nthreads);
  const int L = oracle_num_levels(sigma);
  if (L == 0) return 0;
  uint64_t* code = (uint64_t*)malloc(sigma * sizeof(uint64_t));
  uint32_t* len = (uint32_t*)malloc(sigma * sizeof(uint32_t));
  oracle_codes(sigma, code, len);
  int bad = 0;
#pragma omp parallel for num_threads(nt) reduction(| : bad)
  for (int64_t i = 0; i < (int64_t)n; ++i)
    if (psym(S, w, (uint64_t)i) >= sigma) bad = 1;
  if (bad) { free(code); free(len); return -1; }
  memset(bits, 0, (size_t)L * stride * sizeof(uint64_t));
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
  for (int l = 0; l < L; ++l) {
    uint64_t nkeys = 1ull << l;
    uint64_t* start = (uint64_t*)calloc(nkeys + 1, sizeof(uint64_t));
    uint64_t* order = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) start[(l ? code[psym(S, w, i)] >> (L - l) : 0) + 1]++;
    for (uint64_t x = 0; x < nkeys; ++x) start[x + 1] += start[x];
    for (uint64_t i = 0; i < n; ++i) order[start[l ? code[psym(S, w, i)] >> (L - l) : 0]++] = i;
    uint64_t* row = bits + (size_t)l * stride;
    uint64_t m = 0;
    for (uint64_t r = 0; r < n; ++r) {
      uint64_t c = psym(S, w, order[r]);
      if (len[c] <= (uint32_t)l) continue;
      if ((code[c] >> (L - 1 - l)) & 1) row[m / 64] |= 1ull << (m % 64);
      ++m;
    }
    level_n[l] = m;
    free(order);
    free(start);
    oracle_directory(row, m, l2, L1 + (size_t)l * l1_stride, L2 + (size_t)l * l2_stride);
    oracle_samples(row, m, srate, s1 + (size_t)l * s_stride, n1 + l, s0 + (size_t)l * s_stride, n0 + l);
  }
  free(code);
  free(len);
  return 0;
}
