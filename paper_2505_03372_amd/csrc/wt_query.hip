// Batched access / rank / select on gfx950: one lane per query, persistent grid-stride loop.
//
// Large batches are first binned by where their answers lie (access and rank by position, select by
// the rank of the wanted occurrence in symbol order, cum[c] + k - 1): a counting pass into 2^16
// buckets, a scan and a scatter put the queries in bucket order, the traversal reads them in that
// order and writes every answer to its query's index. Queries that are close in the key touch the
// same lines of bits, L2 counts and samples at every level (each traversal keeps the order inside a
// node), so the cache lines a wave fetches are shared instead of fetched once per query.
//
// Per level a query needs the node entry (start position and precomputed rank0, indexed by code
// prefix), then one binary rank (Section 4.1, Algorithm 1: L1 + L2 + popcount of the words of one
// L2 block, read as 16-byte vectors) or one binary select (Section 4.2, Algorithm 2: samples ->
// binary search over L1 -> binary search over L2 -> word scan -> in-word select).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "wt_host.h"
#include "wt_internal.h"
#include "wt_query_dev.h"

namespace wt {

// One traversal of the tree's shape SH: 0 level-wise tree, 1 wavelet matrix, 2 Huffman-shaped tree.
template <int L2S, int SH>
__device__ __forceinline__ uint32_t access_sh(const QArgs& a, const LevelMeta* m, uint64_t x) {
  if constexpr (SH == 1) return wm_access_one<L2S>(a, m, x);
  else if constexpr (SH == 2) return huff_access_one<L2S>(a, m, x);
  else return access_one<L2S>(a, m, x);
}

template <int L2S, int SH>
__device__ __forceinline__ uint64_t rank_sh(const QArgs& a, const LevelMeta* m, uint32_t c, uint64_t x) {
  if constexpr (SH == 1) return wm_rank_one<L2S>(a, m, c, x);
  else if constexpr (SH == 2) return huff_rank_one<L2S>(a, m, c, x);
  else return rank_one<L2S>(a, m, c, x);
}

template <int L2S, int SH>
__device__ __forceinline__ uint64_t select_sh(const QArgs& a, const LevelMeta* m, uint32_t c, uint64_t k) {
  if constexpr (SH == 1) return wm_select_one<L2S>(a, m, c, k);
  else if constexpr (SH == 2) return huff_select_one<L2S>(a, m, c, k);
  else return select_one<L2S>(a, m, c, k);
}

// sq: NULL, or the queries in binned order: slot j runs query sq[j].id with the arguments stored in sq[j] (its
// answer written at that index).
template <int L2S, uint32_t QB, int SH = 0>
__global__ __launch_bounds__(QB, 8) void k_access(QArgs a, const uint64_t* __restrict__ pos, uint64_t q,
                                                uint32_t* __restrict__ out, const SQ* __restrict__ sq,
                                                uint32_t subshift) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  __shared__ LocalOrder<QB> s_ord;
  load_meta(a, s_meta);
  if (sq) {
    for (uint64_t j0 = xcd_block() * QB; j0 < q; j0 += (uint64_t)gridDim.x * QB) {
      uint32_t jj, c;
      uint64_t x;
      if (local_order<0, QB>(a, sq, q, j0 + threadIdx.x, subshift, s_ord, jj, c, x))
        out[jj] = access_sh<L2S, SH>(a, s_meta, x);
    }
    return;
  }
  for (uint64_t j = xcd_block() * QB + threadIdx.x; j < q; j += (uint64_t)gridDim.x * QB)
    out[j] = access_sh<L2S, SH>(a, s_meta, pos[j]);
}

template <int L2S, uint32_t QB, int SH = 0>
__global__ __launch_bounds__(QB, 8) void k_rank(QArgs a, const uint32_t* __restrict__ sym,
                                              const uint64_t* __restrict__ pos, uint64_t q,
                                              uint64_t* __restrict__ out, const SQ* __restrict__ sq,
                                              uint32_t subshift) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  __shared__ LocalOrder<QB> s_ord;
  load_meta(a, s_meta);
  if (sq) {
    for (uint64_t j0 = xcd_block() * QB; j0 < q; j0 += (uint64_t)gridDim.x * QB) {
      uint32_t jj, c;
      uint64_t x;
      if (local_order<1, QB>(a, sq, q, j0 + threadIdx.x, subshift, s_ord, jj, c, x))
        out[jj] = rank_sh<L2S, SH>(a, s_meta, c, x);
    }
    return;
  }
  for (uint64_t j = xcd_block() * QB + threadIdx.x; j < q; j += (uint64_t)gridDim.x * QB)
    out[j] = rank_sh<L2S, SH>(a, s_meta, sym[j], pos[j]);
}

template <int L2S, uint32_t QB, int SH = 0>
__global__ __launch_bounds__(QB, 8) void k_select(QArgs a, const uint32_t* __restrict__ sym,
                                                const uint64_t* __restrict__ kin, uint64_t q,
                                                uint64_t* __restrict__ out, const SQ* __restrict__ sq,
                                                uint32_t subshift) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  __shared__ LocalOrder<QB> s_ord;
  load_meta(a, s_meta);
  if (sq) {
    for (uint64_t j0 = xcd_block() * QB; j0 < q; j0 += (uint64_t)gridDim.x * QB) {
      uint32_t jj, c;
      uint64_t x;
      if (local_order<2, QB>(a, sq, q, j0 + threadIdx.x, subshift, s_ord, jj, c, x))
        out[jj] = select_sh<L2S, SH>(a, s_meta, c, x);
    }
    return;
  }
  for (uint64_t j = xcd_block() * QB + threadIdx.x; j < q; j += (uint64_t)gridDim.x * QB)
    out[j] = select_sh<L2S, SH>(a, s_meta, sym[j], kin[j]);
}

// ---------------------------------------------------------------- per-kernel timing

namespace {
struct QProfRec {
  char name[32];
  hipEvent_t a, b;
};
thread_local bool t_qprof_on = false;
thread_local std::vector<QProfRec> t_qprof;
}  // namespace

void qprof_begin(const char* name, hipStream_t st) {
  if (!t_qprof_on) return;
  QProfRec r{};
  std::strncpy(r.name, name, sizeof(r.name) - 1);
  if (hipEventCreate(&r.a) != hipSuccess) return;
  if (hipEventCreate(&r.b) != hipSuccess) {
    (void)hipEventDestroy(r.a);
    return;
  }
  (void)hipEventRecord(r.a, st);
  t_qprof.push_back(r);
}

void qprof_end(hipStream_t st) {
  if (!t_qprof_on || t_qprof.empty()) return;
  (void)hipEventRecord(t_qprof.back().b, st);
}

// ---------------------------------------------------------------- locality binning

// Counting sort of the queries by bucket = key >> shift (kBins buckets), block-local: every block
// counts its chunk in an LDS histogram (128 KB: one 1024-thread block per CU), a pass gives every
// (bucket, block) its offset, and the scatter places the chunk with LDS cursors (all atomics in LDS).
// The buckets are fine enough that the 64 queries of a wave fall within a few lines of every array.
// kBins is the largest bucket count (the LDS arrays); a batch uses nb = 2^nbl <= kBins buckets. Access
// batches take 2^14 (measured on 2^26 queries over 2^30 symbols: the scatter's 2^15 buckets cost more
// than the finer order saves the traversal, 6.1 against 6.7 ms); rank and select take 2^15.
constexpr uint32_t kBinsLog = 15;
constexpr uint32_t kBins = 1u << kBinsLog;
constexpr uint32_t kAccessBinsLog = 14;
static_assert((1u << kAccessBinsLog) >= 1024, "bucket count: at least one per thread of the scan block");
constexpr uint32_t kBinT = 1024;                // threads of the counting and scatter blocks
constexpr uint32_t kBinChunk = kBinT * 256;     // queries per block
constexpr uint64_t kSortMinQ = 1ull << 16;

// Each thread takes kBinU queries of its chunk per round (kBinT apart, so every load is coalesced)
// and issues all their loads before it uses any: with one 1024-thread block per CU, a round of one
// query per thread would leave the passes waiting on one load chain at a time.
constexpr uint32_t kBinU = 8;
constexpr uint32_t kBinNone = 0xFFFFFFFFu;  // slot past the batch

template <int KIND>
__device__ __forceinline__ void bin_round(const QArgs& a, const uint32_t* __restrict__ sym,
                                          const uint64_t* __restrict__ arg, uint64_t q, uint32_t shift, uint32_t nb,
                                          uint64_t j0, uint32_t (&bin)[kBinU], uint64_t (&x)[kBinU],
                                          uint32_t (&c)[kBinU]) {
#pragma unroll
  for (uint32_t u = 0; u < kBinU; ++u) {
    const uint64_t j = j0 + (uint64_t)u * kBinT;
    x[u] = j < q ? arg[j] : 0;
    c[u] = (KIND && j < q) ? sym[j] : 0u;
  }
#pragma unroll
  for (uint32_t u = 0; u < kBinU; ++u) {
    const uint64_t j = j0 + (uint64_t)u * kBinT;
    bin[u] = j < q ? (uint32_t)min<uint64_t>(sort_key(a, KIND, c[u], x[u]) >> shift, nb - 1) : kBinNone;
  }
}

template <int KIND>
__global__ __launch_bounds__(kBinT) void k_bin_count(QArgs a, const uint32_t* __restrict__ sym,
                                                   const uint64_t* __restrict__ arg, uint64_t q, uint32_t shift,
                                                   uint32_t nb, uint32_t* __restrict__ bhist) {
  __shared__ uint32_t h[kBins];
  for (uint32_t b = threadIdx.x; b < nb; b += kBinT) h[b] = 0;
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kBinChunk;
  for (uint32_t i = threadIdx.x; i < kBinChunk; i += kBinT * kBinU) {
    uint32_t bin[kBinU], c[kBinU];
    uint64_t x[kBinU];
    bin_round<KIND>(a, sym, arg, q, shift, nb, c0 + i, bin, x, c);
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u)
      if (bin[u] != kBinNone) atomicAdd(&h[bin[u]], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += kBinT) bhist[(uint64_t)blockIdx.x * nb + b] = h[b];
}

// Per bucket: exclusive prefix over the blocks (in place) and the bucket total. The column is read
// 16 entries at a time (loads issued together) before they are rewritten.
__global__ __launch_bounds__(kQT) void k_bin_offsets(uint32_t* __restrict__ bhist, uint32_t nblk, uint32_t nb,
                                                     uint32_t* __restrict__ tot) {
  constexpr uint32_t R = 16;
  const uint32_t b = blockIdx.x * kQT + threadIdx.x;
  if (b >= nb) return;
  uint32_t run = 0;
  for (uint32_t k0 = 0; k0 < nblk; k0 += R) {
    uint32_t v[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) v[r] = k0 + r < nblk ? bhist[(uint64_t)(k0 + r) * nb + b] : 0u;
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
      if (k0 + r < nblk) bhist[(uint64_t)(k0 + r) * nb + b] = run;
      run += v[r];
    }
  }
  tot[b] = run;
}

// In place exclusive scan of the nb bucket totals (one block of 1024 threads, nb / 1024 per thread).
__global__ __launch_bounds__(1024) void k_bin_scan(uint32_t* __restrict__ tot, uint32_t nb) {
  __shared__ uint32_t s_w[16];
  constexpr uint32_t kPer = kBins / 1024;
  const uint32_t per = nb / 1024;
  uint32_t v[kPer], sum = 0;
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    v[i] = i < per ? tot[threadIdx.x * per + i] : 0u;
    sum += v[i];
  }
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  uint32_t inc = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if ((int)lane >= off) inc += y;
  }
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (uint32_t w = 0; w < wv; ++w) pre += s_w[w];
  uint32_t run = pre + inc - sum;
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    if (i < per) tot[threadIdx.x * per + i] = run;
    run += v[i];
  }
}

// Every query is written at its slot with its arguments (SQ).
template <int KIND>
__global__ __launch_bounds__(kBinT) void k_bin_scatter(QArgs a, const uint32_t* __restrict__ sym,
                                                     const uint64_t* __restrict__ arg, uint64_t q, uint32_t shift,
                                                     uint32_t nb, const uint32_t* __restrict__ bhist,
                                                     const uint32_t* __restrict__ base, SQ* __restrict__ sq) {
  __shared__ uint32_t cur[kBins];
  for (uint32_t b = threadIdx.x; b < nb; b += kBinT) cur[b] = base[b] + bhist[(uint64_t)blockIdx.x * nb + b];
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kBinChunk;
  for (uint32_t i = threadIdx.x; i < kBinChunk; i += kBinT * kBinU) {
    uint32_t bin[kBinU], c[kBinU];
    uint64_t x[kBinU];
    bin_round<KIND>(a, sym, arg, q, shift, nb, c0 + i, bin, x, c);
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u)
      if (bin[u] != kBinNone) {
        SQ r;
        r.id = (uint32_t)(c0 + i + u * kBinT);
        r.sym = c[u];
        r.arg = x[u];
        sq[atomicAdd(&cur[bin[u]], 1u)] = r;
      }
  }
}

// Large batches place their queries in two passes instead of the scatter above. Its stores go one
// query to a line (a block's few queries of a bucket arrive at different times), so it runs at the
// rate of random line writes and every 16-byte record costs a 32-byte write. The two passes store
// whole runs instead: the first puts every block's chunk into kCoarse coarse buckets (kCoarse
// consecutive groups of buckets), a round of kRound queries at a time, staged in LDS in coarse order;
// the second gives each coarse bucket one block, which places its queries into the buckets the same
// way. Both read and write every record once more than the scatter, all of it in runs. Measured on
// 2^26 queries over 2^30 symbols: 1.7 -> 1.05 ms for 2^15 buckets (rank, select), 1.18 -> 0.92 ms
// for 2^14 (access).
constexpr uint32_t kCoarseLog = 8;
constexpr uint32_t kCoarse = 1u << kCoarseLog;
constexpr uint32_t kRound = kBinT * kBinU;          // queries per round of a block
constexpr uint64_t kTwoPassMinQ = 1ull << 24;       // batches from this size on (a block per CU at least)
static_assert((kBins >> kCoarseLog) <= 256 && (1u << kAccessBinsLog) >= kCoarse, "bucket groups");

// Wave 0: exclusive offsets of cnt[0, n) (n <= 256) into off, the cursors' old values into base, cur
// advanced by the counts, and the total into *tot.
__device__ __forceinline__ void round_offsets(const uint32_t* cnt, uint32_t n, uint32_t* off, uint32_t* base,
                                              uint32_t* cur, uint32_t* tot, uint32_t lane) {
  uint32_t v[4], s = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    v[k] = i < n ? cnt[i] : 0u;
    s += v[k];
  }
  uint32_t inc = s;
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  uint32_t ex = inc - s;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t i = 4 * lane + k;
    if (i < n) {
      off[i] = ex;
      base[i] = cur[i];
      cur[i] += v[k];
    }
    ex += v[k];
  }
  if (lane == 63) *tot = inc;
}

// First pass: the block's chunk into tmp by coarse bucket. bhist holds every (block, bucket) offset
// over the blocks before it, start every bucket's first slot.
template <int KIND>
__global__ __launch_bounds__(kBinT) void k_bin_coarse(QArgs a, const uint32_t* __restrict__ sym,
                                                    const uint64_t* __restrict__ arg, uint64_t q, uint32_t shift,
                                                    uint32_t nb, const uint32_t* __restrict__ bhist,
                                                    const uint32_t* __restrict__ start, SQ* __restrict__ tmp) {
  __shared__ SQ s_rec[kRound];
  __shared__ uint8_t s_grp[kRound];
  __shared__ uint32_t s_cur[kCoarse], s_cnt[kCoarse], s_off[kCoarse], s_base[kCoarse];
  __shared__ uint32_t s_nr;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t fb = nb >> kCoarseLog;  // buckets per coarse bucket
  uint32_t fbl = 0;
  while ((1u << fbl) < fb) ++fbl;
  {
    // the block's first slot in each coarse bucket: its start plus the queries of earlier blocks
    // (four threads per coarse bucket, a quarter of its buckets each)
    const uint32_t g = tid >> 2, part = tid & 3u, per = fb / 4;
    const uint32_t* h = bhist + (uint64_t)blockIdx.x * nb + (uint64_t)g * fb + part * per;
    uint32_t sum = 0;
    for (uint32_t f = 0; f < per; ++f) sum += h[f];
    sum += __shfl_xor(sum, 1, 64);
    sum += __shfl_xor(sum, 2, 64);
    if (part == 0) s_cur[g] = start[(uint64_t)g * fb] + sum;
  }
  const uint64_t c0 = (uint64_t)blockIdx.x * kBinChunk;
  for (uint32_t i = tid; i < kBinChunk; i += kRound) {
    uint32_t bin[kBinU], c[kBinU], r[kBinU];
    uint64_t x[kBinU];
    bin_round<KIND>(a, sym, arg, q, shift, nb, c0 + i, bin, x, c);
    if (tid < kCoarse) s_cnt[tid] = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u) r[u] = bin[u] != kBinNone ? atomicAdd(&s_cnt[bin[u] >> fbl], 1u) : 0u;
    __syncthreads();
    if (tid < 64) round_offsets(s_cnt, kCoarse, s_off, s_base, s_cur, &s_nr, lane);
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u)
      if (bin[u] != kBinNone) {
        const uint32_t g = bin[u] >> fbl, sl = s_off[g] + r[u];
        SQ rec;
        rec.id = (uint32_t)(c0 + i + u * kBinT);
        rec.sym = c[u];
        rec.arg = x[u];
        s_rec[sl] = rec;
        s_grp[sl] = (uint8_t)g;
      }
    __syncthreads();
    const uint32_t nr = s_nr;
    for (uint32_t k = tid; k < nr; k += kBinT) {
      const uint32_t g = s_grp[k];
      tmp[s_base[g] + (k - s_off[g])] = s_rec[k];
    }
    __syncthreads();
  }
}

// Second pass: coarse bucket g is placed by kFineParts blocks; part p takes the records that the
// first pass's blocks [b0, b1) wrote (a contiguous slice of the bucket), whose first slot in every
// bucket follows from the same per-(block, bucket) offsets. Rounds of kRound2 records keep the LDS at
// two blocks per CU.
constexpr uint32_t kFineParts = 4;
constexpr uint32_t kRound2 = kBinT * 4;
template <int KIND>
__global__ __launch_bounds__(kBinT) void k_bin_fine(QArgs a, uint64_t q, uint32_t shift, uint32_t nb, uint32_t nblk,
                                                  const uint32_t* __restrict__ bhist,
                                                  const uint32_t* __restrict__ start, const SQ* __restrict__ tmp,
                                                  SQ* __restrict__ sq) {
  constexpr uint32_t U = kRound2 / kBinT;
  __shared__ SQ s_rec[kRound2];
  __shared__ uint8_t s_grp[kRound2];
  __shared__ uint32_t s_cur[kCoarse], s_cnt[kCoarse], s_off[kCoarse], s_base[kCoarse];
  __shared__ uint32_t s_nr, s_lo, s_len;
  const uint32_t tid = threadIdx.x, lane = tid & 63u;
  const uint32_t fb = nb >> kCoarseLog, g = blockIdx.x / kFineParts, p = blockIdx.x % kFineParts;
  const uint32_t b0 = (uint32_t)((uint64_t)p * nblk / kFineParts), b1 = (uint32_t)((uint64_t)(p + 1) * nblk / kFineParts);
  if (b0 == b1) return;
  // per bucket of the group: the part's first slot, and the part's records before it (s_cnt)
  if (tid < fb) {
    const uint32_t bin = g * fb + tid;
    const uint32_t o0 = bhist[(uint64_t)b0 * nb + bin];
    const uint32_t o1 = b1 < nblk ? bhist[(uint64_t)b1 * nb + bin]
                                  : (uint32_t)((bin + 1 < nb ? (uint64_t)start[bin + 1] : q) - start[bin]);
    s_cur[tid] = start[bin] + o0;
    s_cnt[tid] = o0;
    s_off[tid] = o1 - o0;
  }
  __syncthreads();
  if (tid < 64) {
    uint32_t before = 0, len = 0;
    for (uint32_t f = lane; f < fb; f += 64) {
      before += s_cnt[f];
      len += s_off[f];
    }
#pragma unroll
    for (uint32_t d = 32; d > 0; d >>= 1) {
      before += __shfl_xor(before, d, 64);
      len += __shfl_xor(len, d, 64);
    }
    if (lane == 0) {
      s_lo = start[g * fb] + before;
      s_len = len;
    }
  }
  __syncthreads();
  const uint64_t lo = s_lo, hi = lo + s_len;
  for (uint64_t r0 = lo; r0 < hi; r0 += kRound2) {
    SQ rec[U];
    uint32_t f[U], r[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint64_t j = r0 + tid + (uint64_t)u * kBinT;
      if (j < hi) rec[u] = tmp[j];
    }
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint64_t j = r0 + tid + (uint64_t)u * kBinT;
      f[u] = j < hi ? (uint32_t)min<uint64_t>(sort_key(a, KIND, rec[u].sym, rec[u].arg) >> shift, nb - 1) & (fb - 1)
                    : kBinNone;
    }
    if (tid < kCoarse) s_cnt[tid] = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) r[u] = f[u] != kBinNone ? atomicAdd(&s_cnt[f[u]], 1u) : 0u;
    __syncthreads();
    if (tid < 64) round_offsets(s_cnt, fb, s_off, s_base, s_cur, &s_nr, lane);
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < U; ++u)
      if (f[u] != kBinNone) {
        const uint32_t sl = s_off[f[u]] + r[u];
        s_rec[sl] = rec[u];
        s_grp[sl] = (uint8_t)f[u];
      }
    __syncthreads();
    const uint32_t nr = s_nr;
    for (uint32_t k = tid; k < nr; k += kBinT) {
      const uint32_t b = s_grp[k];
      sq[s_base[b] + (k - s_off[b])] = s_rec[k];
    }
    __syncthreads();
  }
}

// Counting sort by precomputed bucket ids (< kBins), same passes as above: bhist, then the bucket
// offsets, then the slot order.
__global__ __launch_bounds__(kBinT) void k_bin_count_ids(const uint16_t* __restrict__ ids, uint64_t q,
                                                         uint32_t* __restrict__ bhist) {
  __shared__ uint32_t h[kBins];
  for (uint32_t b = threadIdx.x; b < kBins; b += kBinT) h[b] = 0;
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kBinChunk;
  for (uint32_t i = threadIdx.x; i < kBinChunk; i += kBinT * kBinU) {
    uint32_t id[kBinU];
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u) {
      const uint64_t j = c0 + i + u * kBinT;
      id[u] = j < q ? (uint32_t)ids[j] : kBinNone;
    }
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u)
      if (id[u] != kBinNone) atomicAdd(&h[id[u]], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < kBins; b += kBinT) bhist[(uint64_t)blockIdx.x * kBins + b] = h[b];
}

__global__ __launch_bounds__(kBinT) void k_bin_scatter_ids(const uint16_t* __restrict__ ids, uint64_t q,
                                                           const uint32_t* __restrict__ bhist,
                                                           const uint32_t* __restrict__ base,
                                                           uint32_t* __restrict__ perm) {
  __shared__ uint32_t cur[kBins];
  for (uint32_t b = threadIdx.x; b < kBins; b += kBinT) cur[b] = base[b] + bhist[(uint64_t)blockIdx.x * kBins + b];
  __syncthreads();
  const uint64_t c0 = (uint64_t)blockIdx.x * kBinChunk;
  for (uint32_t i = threadIdx.x; i < kBinChunk; i += kBinT * kBinU) {
    uint32_t id[kBinU];
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u) {
      const uint64_t j = c0 + i + u * kBinT;
      id[u] = j < q ? (uint32_t)ids[j] : kBinNone;
    }
#pragma unroll
    for (uint32_t u = 0; u < kBinU; ++u)
      if (id[u] != kBinNone) perm[atomicAdd(&cur[id[u]], 1u)] = (uint32_t)(c0 + i + u * kBinT);
  }
}

size_t sort_ids_bytes(uint64_t q) {
  const uint32_t nblk = (uint32_t)ceil_div(q, kBinChunk);
  return round_up((size_t)nblk * kBins * 4, 256) + round_up(4 * kBins, 256);
}

void sort_ids_enqueue(const uint16_t* ids, uint64_t q, char* scratch, uint32_t* tot, uint32_t* perm, hipStream_t st) {
  const uint32_t nblk = (uint32_t)ceil_div(q, kBinChunk);
  uint32_t* bhist = (uint32_t*)scratch;
  hipLaunchKernelGGL(k_bin_count_ids, dim3(nblk), dim3(kBinT), 0, st, ids, q, bhist);
  hipLaunchKernelGGL(k_bin_offsets, dim3(kBins / kQT), dim3(kQT), 0, st, bhist, nblk, kBins, tot);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, tot, kBins);
  hipLaunchKernelGGL(k_bin_scatter_ids, dim3(nblk), dim3(kBinT), 0, st, ids, q, (const uint32_t*)bhist,
                     (const uint32_t*)tot, perm);
}

// Bins the batch on st (kind 0 access, 1 rank, 2 select); binned = false when the batch is too small
// to pay (or too large for 32-bit slots).
// Bytes of the binning buffers of a batch of q queries: per-block bucket histograms, bucket totals, slots.
size_t sort_batch_bytes(uint64_t q) {
  const uint32_t nblk = (uint32_t)ceil_div(q, kBinChunk);
  return round_up((size_t)nblk * kBins * 4, 256) + round_up(4 * kBins, 256) + round_up(sizeof(SQ) * q, 256);
}

wt_status sort_batch(const wt_tree* t, const QArgs& a, int kind, const uint32_t* sym, const uint64_t* arg,
                     uint64_t q, hipStream_t st, SortBufs& sb, bool& binned, char* pre) {
  binned = false;
  if (q < kSortMinQ || q >= (1ull << 32)) return WT_OK;
  const uint32_t nblk = (uint32_t)ceil_div(q, kBinChunk);
  const size_t o_t = round_up((size_t)nblk * kBins * 4, 256), o_p = o_t + round_up(4 * kBins, 256);
  char* blk = pre;
  const uint32_t nbl = kind == 0 ? kAccessBinsLog : kBinsLog, nb = 1u << nbl;
  const bool two = !pre && q >= kTwoPassMinQ;  // two passes need a second record array
  SQ* tmp = nullptr;
  if (!blk) {
    const size_t bytes = sort_batch_bytes(q), all = bytes + (two ? round_up(sizeof(SQ) * q, 256) : 0);
    sb.block = (char*)dev_alloc(all, st);
    if (!sb.block) return fail(WT_ERR_OOM, "query binning: scratch allocation of %zu bytes failed", all);
    blk = sb.block;
    if (two) tmp = (SQ*)(blk + bytes);
  }
  uint32_t* bhist = (uint32_t*)blk;
  uint32_t* tot = (uint32_t*)(blk + o_t);
  sb.cnt = tot;
  sb.sq = (SQ*)(blk + o_p);
  uint32_t bits = 0;
  while ((1ull << bits) < a.n + 1) ++bits;
  const uint32_t shift = bits > nbl ? bits - nbl : 0;
  sb.subshift = shift > qb_bits(kQB) ? shift - qb_bits(kQB) : 0;
  if (!pre) qprof_begin("sort_count", st);
  if (kind == 0) hipLaunchKernelGGL(k_bin_count<0>, dim3(nblk), dim3(kBinT), 0, st, a, sym, arg, q, shift, nb, bhist);
  else if (kind == 1)
    hipLaunchKernelGGL(k_bin_count<1>, dim3(nblk), dim3(kBinT), 0, st, a, sym, arg, q, shift, nb, bhist);
  else hipLaunchKernelGGL(k_bin_count<2>, dim3(nblk), dim3(kBinT), 0, st, a, sym, arg, q, shift, nb, bhist);
  if (!pre) qprof_end(st);
  if (!pre) qprof_begin("sort_scan", st);
  hipLaunchKernelGGL(k_bin_offsets, dim3(nb / kQT), dim3(kQT), 0, st, bhist, nblk, nb, tot);
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, tot, nb);
  if (!pre) qprof_end(st);
  if (!pre) qprof_begin("sort_scatter", st);
  if (two) {
#define WT_TWO(K)                                                                                          \
  do {                                                                                                     \
    hipLaunchKernelGGL(k_bin_coarse<K>, dim3(nblk), dim3(kBinT), 0, st, a, sym, arg, q, shift, nb,          \
                       (const uint32_t*)bhist, (const uint32_t*)tot, tmp);                                  \
    hipLaunchKernelGGL(k_bin_fine<K>, dim3(kCoarse * kFineParts), dim3(kBinT), 0, st, a, q, shift, nb, nblk,   \
                       (const uint32_t*)bhist, (const uint32_t*)tot, (const SQ*)tmp, sb.sq);                \
  } while (0)
    if (kind == 0) WT_TWO(0);
    else if (kind == 1) WT_TWO(1);
    else WT_TWO(2);
#undef WT_TWO
  } else if (kind == 0)
    hipLaunchKernelGGL(k_bin_scatter<0>, dim3(nblk), dim3(kBinT), 0, st, a, sym, arg, q, shift, nb,
                       (const uint32_t*)bhist, (const uint32_t*)tot, sb.sq);
  else if (kind == 1)
    hipLaunchKernelGGL(k_bin_scatter<1>, dim3(nblk), dim3(kBinT), 0, st, a, sym, arg, q, shift, nb,
                       (const uint32_t*)bhist, (const uint32_t*)tot, sb.sq);
  else
    hipLaunchKernelGGL(k_bin_scatter<2>, dim3(nblk), dim3(kBinT), 0, st, a, sym, arg, q, shift, nb,
                       (const uint32_t*)bhist, (const uint32_t*)tot, sb.sq);
  if (!pre) qprof_end(st);
  WT_HIP(hipGetLastError());
  binned = true;
  (void)t;
  return WT_OK;
}

}  // namespace wt

namespace wt {

// Bytes of the preallocated scratch of query_run for q queries: the binning buffers, then the symbols
// mapped to codes (trees with an extracted alphabet).
size_t query_scratch_bytes(uint64_t q) { return round_up(sort_batch_bytes(q), 256) + round_up(4 * q, 256); }

// One batch of queries of one kind (0 access, 1 rank, 2 select) on st: symbols mapped to codes (extracted
// alphabets), binning of large batches, the traversal kernel of the tree or matrix, access answers mapped
// back to values. pre: NULL (buffers allocated and freed stream-ordered) or query_scratch_bytes(q) bytes
// of device memory (nothing allocated, no profiling events).
wt_status query_run(const wt_tree* t, int kind, const uint32_t* d_sym, const uint64_t* d_arg, uint64_t q, void* d_out,
                    hipStream_t st, char* pre) {
  const QArgs a = make_args(t);
  const uint32_t* sym = d_sym;
  void* mapped = nullptr;
  if (kind != 0) {
    const wt_status rc = alpha_map_syms(t, d_sym, q, st, &sym, &mapped,
                                        pre ? (uint32_t*)(pre + round_up(sort_batch_bytes(q), 256)) : nullptr);
    if (rc != WT_OK) return rc;
  }
  SortBufs sb;
  bool binned;
  const wt_status rc = sort_batch(t, a, kind, sym, d_arg, q, st, sb, binned, pre);
  if (rc != WT_OK) {
    if (mapped) dev_free(mapped, st);
    return rc;
  }
  static const char* const kName[3] = {"access", "rank", "select"};
  if (!pre) qprof_begin(kName[kind], st);
  const SQ* sq = binned ? (const SQ*)sb.sq : nullptr;
  const uint32_t sub = binned ? sb.subshift : 0u;
  const uint32_t grid = query_grid(q, binned ? kQB : kQT);
  uint32_t* o32 = (uint32_t*)d_out;
  uint64_t* o64 = (uint64_t*)d_out;
#define WT_RUN_SH(QB, SH)                                                                               \
  do {                                                                                                  \
    if (kind == 0) { WT_DISPATCH_L2_SH(t->l2_bits, QB, SH, k_access, a, d_arg, q, o32, sq, sub); }        \
    else if (kind == 1) { WT_DISPATCH_L2_SH(t->l2_bits, QB, SH, k_rank, a, sym, d_arg, q, o64, sq, sub); } \
    else { WT_DISPATCH_L2_SH(t->l2_bits, QB, SH, k_select, a, sym, d_arg, q, o64, sq, sub); }             \
  } while (0)
#define WT_DISPATCH_SH0(QB)                                                                    \
  do {                                                                                         \
    if (kind == 0) { WT_DISPATCH_L2(t->l2_bits, QB, k_access, a, d_arg, q, o32, sq, sub); }      \
    else if (kind == 1) { WT_DISPATCH_L2(t->l2_bits, QB, k_rank, a, sym, d_arg, q, o64, sq, sub); } \
    else { WT_DISPATCH_L2(t->l2_bits, QB, k_select, a, sym, d_arg, q, o64, sq, sub); }           \
  } while (0)
#define WT_RUN(QB)                       \
  do {                                   \
    if (t->matrix) WT_RUN_SH(QB, 1);     \
    else if (t->huff) WT_RUN_SH(QB, 2);  \
    else WT_DISPATCH_SH0(QB);            \
  } while (0)
  if (binned) WT_RUN(kQB);
  else WT_RUN(kQT);
#undef WT_RUN
#undef WT_RUN_SH
#undef WT_DISPATCH_SH0
  if (!pre) qprof_end(st);
  if (sb.block) dev_free(sb.block, st);
  if (mapped) dev_free(mapped, st);
  WT_HIP(hipGetLastError());
  return kind == 0 ? alpha_unmap_access(t, o32, q, st) : WT_OK;
}

}  // namespace wt

using namespace wt;

extern "C" wt_status wt_access(const wt_tree* t, const uint64_t* d_pos, uint64_t q, uint32_t* d_out,
                               wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_access: tree is NULL");
  if (q == 0) return WT_OK;
  if (!d_pos || !d_out) return fail(WT_ERR_ARG, "wt_access: NULL buffer");
  return query_run(t, 0, nullptr, d_pos, q, d_out, (hipStream_t)stream, nullptr);
}

extern "C" wt_status wt_rank(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_pos, uint64_t q,
                             uint64_t* d_out, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_rank: tree is NULL");
  if (q == 0) return WT_OK;
  if (!d_sym || !d_pos || !d_out) return fail(WT_ERR_ARG, "wt_rank: NULL buffer");
  return query_run(t, 1, d_sym, d_pos, q, d_out, (hipStream_t)stream, nullptr);
}

extern "C" wt_status wt_select(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_k, uint64_t q,
                               uint64_t* d_out, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_select: tree is NULL");
  if (q == 0) return WT_OK;
  if (!d_sym || !d_k || !d_out) return fail(WT_ERR_ARG, "wt_select: NULL buffer");
  return query_run(t, 2, d_sym, d_k, q, d_out, (hipStream_t)stream, nullptr);
}

// ---------------------------------------------------------------- select without allocation

namespace wt {
namespace {
// Largest batch of wt_select_noalloc and the bytes of its scratch (query_scratch_bytes of such a batch).
constexpr uint64_t kNoAllocMaxQ = 1ull << 20;
constexpr size_t kNoAllocBytes = ((kNoAllocMaxQ + kBinChunk - 1) / kBinChunk) * kBins * 4 + 4 * kBins +
                                 sizeof(SQ) * kNoAllocMaxQ + 4 * kNoAllocMaxQ;
static_assert(((kNoAllocMaxQ + kBinChunk - 1) / kBinChunk) * kBins * 4 % 256 == 0 && (4 * kBins) % 256 == 0 &&
                  (sizeof(SQ) * kNoAllocMaxQ) % 256 == 0 && (4 * kNoAllocMaxQ) % 256 == 0,
              "the parts of the scratch are whole 256-byte units, as query_scratch_bytes rounds them");
}  // namespace
}  // namespace wt

// Device memory of wt_select_noalloc (each GPU holds its own copy while the library is loaded). Host
// code never passes this name to a kernel: it takes the device address from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[wt::kNoAllocBytes];

namespace wt {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array, looked up once per device.
wt_status noalloc_scratch(char** out) {
  int dev = 0;
  WT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(WT_ERR_STATE, "wt_select_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    WT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(WT_ERR_HIP, "wt_select_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return WT_OK;
}
}  // namespace
}  // namespace wt

extern "C" wt_status wt_select_noalloc(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_k, uint64_t q,
                                       uint64_t* d_out, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_select_noalloc: tree is NULL");
  if (q > kNoAllocMaxQ)
    return fail(WT_ERR_ARG, "wt_select_noalloc: %llu queries exceed the limit of %llu (use wt_select)",
                (unsigned long long)q, (unsigned long long)kNoAllocMaxQ);
  if (q == 0) return WT_OK;
  if (!d_sym || !d_k || !d_out) return fail(WT_ERR_ARG, "wt_select_noalloc: NULL buffer");
  char* buf = nullptr;
  const wt_status rc = noalloc_scratch(&buf);
  if (rc != WT_OK) return rc;
  return query_run(t, 2, d_sym, d_k, q, d_out, (hipStream_t)stream, buf);
}

extern "C" wt_status wt_query_profiling(int on) {
  clear_error();
  t_qprof_on = on != 0;
  return WT_OK;
}

extern "C" wt_status wt_query_profile(wt_prof_entry* out, uint32_t cap, uint32_t* count) {
  clear_error();
  if (count) *count = (uint32_t)t_qprof.size();
  uint32_t i = 0;
  wt_status rc = WT_OK;
  for (QProfRec& r : t_qprof) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = WT_ERR_HIP;
    if (out && i < cap) {
      std::memset(&out[i], 0, sizeof(out[i]));
      std::memcpy(out[i].kernel, r.name, sizeof(out[i].kernel));
      out[i].level = -1;
      out[i].ms = ms;
    }
    ++i;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  t_qprof.clear();
  if (rc != WT_OK) return fail(rc, "wt_query_profile: event query failed");
  return WT_OK;
}
