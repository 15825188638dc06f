/*
 * Seeded synthetic input generators for the wavelet-tree workloads.
 *
 * This module is shared by the CPU oracle tests and the GPU path and therefore
 * holds none of the wavelet-tree arithmetic: only counter-based random streams,
 * value distributions (uniform, Zipf, log-uniform) and permutations.
 *
 * Random stream: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used counter-based:
 *     out(seed, j) = mix64(seed + (j + 1) * 0x9E3779B97F4A7C15).
 * Element j of every generated array uses out(seed, j), so results do not depend
 * on the number of threads.
 *   uniform integer in [0, m): (out * m) >> 64 on 128-bit products (Lemire 2019);
 *   uniform double in [0, 1): (out >> 11) * 2^-53;
 *   Zipf(s) over ranks 1..K: inverse CDF over the running sums of r^-s;
 *   permutation: Fisher-Yates driven by the stream.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN64 0x9E3779B97F4A7C15ull

uint64_t gen_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t rng_at(uint64_t seed, uint64_t j) {
  return gen_mix64(seed + (j + 1) * GOLDEN64);
}

static inline uint64_t below(uint64_t r, uint64_t m) {
  return (uint64_t)(((unsigned __int128)r * (unsigned __int128)m) >> 64);
}

static inline double unit01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }

static inline void put(void* out, int w, uint64_t j, uint64_t v) {
  if (w == 1) ((uint8_t*)out)[j] = (uint8_t)v;
  else if (w == 2) ((uint16_t*)out)[j] = (uint16_t)v;
  else if (w == 4) ((uint32_t*)out)[j] = (uint32_t)v;
  else ((uint64_t*)out)[j] = v;
}

static inline uint64_t get(const void* in, int w, uint64_t j) {
  if (w == 1) return ((const uint8_t*)in)[j];
  if (w == 2) return ((const uint16_t*)in)[j];
  if (w == 4) return ((const uint32_t*)in)[j];
  return ((const uint64_t*)in)[j];
}

/* Sub-seed for a named stream (tag) of a base seed. */
uint64_t gen_subseed(uint64_t base, uint64_t tag) { return gen_mix64(base ^ (tag * GOLDEN64)); }

/* Raw stream values out(seed, j) for j in [a, b). */
void gen_raw(uint64_t seed, uint64_t a, uint64_t b, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = (int64_t)a; j < (int64_t)b; ++j) out[j - a] = rng_at(seed, (uint64_t)j);
}

/* out[j] = uniform integer in [lo, lo + m) for j in [a, b); width w bytes. */
void gen_fill_uniform(uint64_t seed, uint64_t a, uint64_t b, uint64_t lo, uint64_t m, int w, void* out) {
#pragma omp parallel for schedule(static)
  for (int64_t j = (int64_t)a; j < (int64_t)b; ++j)
    put(out, w, (uint64_t)j, lo + below(rng_at(seed, (uint64_t)j), m));
}

/* Fisher-Yates permutation of [0, K). */
void gen_permutation(uint64_t seed, uint64_t K, uint32_t* perm) {
  for (uint64_t i = 0; i < K; ++i) perm[i] = (uint32_t)i;
  for (uint64_t i = K; i > 1; --i) {
    uint64_t j = below(rng_at(seed, K - i), i);
    uint32_t t = perm[i - 1];
    perm[i - 1] = perm[j];
    perm[j] = t;
  }
}

/* Unnormalised Zipf CDF: cdf[r-1] = sum_{i=1..r} i^-s. */
void gen_zipf_cdf(uint64_t K, double s, double* cdf) {
  double acc = 0.0;
  for (uint64_t r = 1; r <= K; ++r) {
    acc += pow((double)r, -s);
    cdf[r - 1] = acc;
  }
}

/* out[j] = perm[r - 1] where r ~ Zipf over K ranks drawn from out(seed, j), j in [a, b). */
void gen_fill_zipf(uint64_t seed, uint64_t a, uint64_t b, const double* cdf, uint64_t K,
                   const uint32_t* perm, int w, void* out) {
  const double total = cdf[K - 1];
#pragma omp parallel for schedule(static)
  for (int64_t j = (int64_t)a; j < (int64_t)b; ++j) {
    double target = unit01(rng_at(seed, (uint64_t)j)) * total;
    uint64_t lo = 0, hi = K - 1; /* first index with cdf > target */
    while (lo < hi) {
      uint64_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > target) hi = mid; else lo = mid + 1;
    }
    put(out, w, (uint64_t)j, perm ? perm[lo] : lo);
  }
}

/* out[j] = floor(2^(lg lo + u (lg hi - lg lo))) clamped to [lo, hi], j in [a, b). */
void gen_fill_loguniform(uint64_t seed, uint64_t a, uint64_t b, uint64_t lo, uint64_t hi, uint64_t* out) {
  const double l0 = log2((double)lo), l1 = log2((double)hi);
  for (uint64_t j = a; j < b; ++j) {
    double v = floor(exp2(l0 + unit01(rng_at(seed, j)) * (l1 - l0)));
    uint64_t x = (uint64_t)v;
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    out[j - a] = x;
  }
}

/* out_c[j] = S[uniform(n)] as u32 ("a symbol drawn from S"), j in [0, q). */
void gen_draw_from_seq(uint64_t seed, const void* S, uint64_t n, int w, uint64_t q, uint32_t* out_c) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)q; ++j) out_c[j] = (uint32_t)get(S, w, below(rng_at(seed, (uint64_t)j), n));
}

/* out_k[j] = 1 + uniform(counts[c[j]]) (0 when the count is 0), j in [0, q). */
void gen_draw_rank_in_count(uint64_t seed, const uint32_t* c, const uint64_t* counts, uint64_t q, uint64_t* out_k) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < (int64_t)q; ++j) {
    uint64_t m = counts[c[j]];
    out_k[j] = m ? 1 + below(rng_at(seed, (uint64_t)j), m) : 0;
  }
}

/* Words of a bit array (bit j at bit j mod 64 of word j / 64): bit j is one when the uniform double of
   out(seed, j) is below p_lo for j < split and below p_hi from split on; bits past n_bits are zero. */
void gen_bits(uint64_t seed, uint64_t n_bits, uint64_t split, double p_lo, double p_hi, uint64_t* words) {
  const int64_t nw = (int64_t)((n_bits + 63) / 64);
#pragma omp parallel for schedule(static)
  for (int64_t w = 0; w < nw; ++w) {
    uint64_t x = 0;
    for (uint64_t b = 0; b < 64; ++b) {
      const uint64_t j = 64 * (uint64_t)w + b;
      if (j >= n_bits) break;
      const double p = j < split ? p_lo : p_hi;
      if (unit01(rng_at(seed, j)) < p) x |= 1ull << b;
    }
    words[w] = x;
  }
}
