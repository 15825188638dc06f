// Learned select index: per child node an FP32 network u -> 1x16 ReLU -> v predicting where the
// node-local occurrence of rank u (normalised) lies inside the node (v normalised), trained on the
// GPU by full-batch Adam on the rank directory of the built tree, then used by a select that
// corrects the prediction exactly (galloping over the L2 counts) and falls back to the sampled
// binary search of Section 4.2 (Algorithm 2) when the correction exceeds the model's error budget.
//
// Child node of node (level l, code prefix p) on side b: heap index h = 2^(l+1) - 1 + 2p + b,
// model slot h - 1 (slots for levels 1..L).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "wt_host.h"
#include "wt_internal.h"
#include "wt_query_dev.h"

namespace wt {

constexpr int kH = 16;           // hidden units
constexpr int kNP = 3 * kH + 1;  // parameters: w1[16], b1[16], w2[16], b2
constexpr int kPMax = 2048;      // training points per model
constexpr int kLT = 256;         // threads of the training block

struct LearnModel {  // 320 bytes; the fields a query reads sit in the first 240
  float p[kNP];
  int32_t eps;     // error budget in L2 blocks (max error + 2); -1: no model
  uint32_t side;   // b
  float pad0;
  uint64_t start;  // node range [start, start + len) in level l
  uint64_t len;
  uint64_t cnt;    // bits equal to the side b inside the node (size of the child)
  uint64_t rank0;  // count of side-b bits of level l before `start`
  uint32_t npts;   // training points
  uint32_t level;
  float err_mean, err_init_mean, err_max, err_init_max;  // in L2 blocks, over every L2 boundary
  float loss;
  float pad1[13];
};
static_assert(sizeof(LearnModel) == 320, "model size");

__device__ __forceinline__ float mlp_eval(const float* __restrict__ p, float u) {
  float y = p[3 * kH];
#pragma unroll
  for (int k = 0; k < kH; ++k) y += p[2 * kH + k] * fmaxf(fmaf(p[k], u, p[kH + k]), 0.f);
  return y;
}

// Adds the contribution of one point (u, v) to the loss and the gradient (scale = 2 / P).
__device__ __forceinline__ void mlp_point(const float* __restrict__ p, float u, float v, float scale, float* g,
                                          float& loss) {
  float h[kH];
  float y = p[3 * kH];
#pragma unroll
  for (int k = 0; k < kH; ++k) {
    h[k] = fmaf(p[k], u, p[kH + k]);
    y += p[2 * kH + k] * fmaxf(h[k], 0.f);
  }
  const float r = y - v;
  loss += r * r;
  const float gy = scale * r;
  g[3 * kH] += gy;
#pragma unroll
  for (int k = 0; k < kH; ++k) {
    const bool on = h[k] > 0.f;
    g[2 * kH + k] += on ? gy * h[k] : 0.f;
    const float gh = on ? gy * p[2 * kH + k] : 0.f;
    g[k] += gh * u;
    g[kH + k] += gh;
  }
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Loss and gradient over P points held by the block, reduced in a fixed order (deterministic).
// Every thread passes its points; the result lands in s_red[0] (loss) and s_red[1..49].
__device__ void block_loss_grad(const float* __restrict__ p, const float* u, const float* v, int nmine, float scale,
                                float* s_wred /* [4][50] */, float* s_red /* [50] */) {
  float g[kNP];
#pragma unroll
  for (int j = 0; j < kNP; ++j) g[j] = 0.f;
  float loss = 0.f;
  for (int i = 0; i < nmine; ++i) mlp_point(p, u[i], v[i], scale, g, loss);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  loss = wave_sum(loss);
  if (lane == 0) s_wred[wv * 64] = loss;
#pragma unroll
  for (int j = 0; j < kNP; ++j) {
    const float s = wave_sum(g[j]);
    if (lane == 0) s_wred[wv * 64 + 1 + j] = s;
  }
  __syncthreads();
  if (threadIdx.x < kNP + 1) {
    float s = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += s_wred[w * 64 + threadIdx.x];
    s_red[threadIdx.x] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- setup and training data

// Node range, side counts and the starting parameters (the identity v = u on [0, 1]) of every model.
__global__ void k_learn_setup(uint32_t sigma, uint32_t L, const uint64_t* __restrict__ cum,
                              const NodeQ* __restrict__ nodes, LearnModel* __restrict__ models, uint64_t nmodels) {
  const uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nmodels) return;
  const uint64_t hc = slot + 1;
  const uint32_t lc = 63u - (uint32_t)__clzll(hc + 1);  // child level
  const uint64_t pc = hc + 1 - (1ull << lc);
  const uint32_t l = lc - 1, b = (uint32_t)(pc & 1);
  const uint64_t p = pc >> 1;
  LearnModel M;
  for (int k = 0; k < kNP; ++k) M.p[k] = 0.f;
  for (int k = 0; k < kH; ++k) {
    M.p[k] = 1.f;
    M.p[kH + k] = -(float)k / (float)kH;
  }
  M.p[2 * kH] = 1.f;
  M.pad0 = 0.f;
  M.level = l;
  M.side = b;
  M.eps = -1;
  M.npts = 0;
  M.start = M.len = M.cnt = M.rank0 = 0;
  M.err_mean = M.err_init_mean = M.err_max = M.err_init_max = 0.f;
  M.loss = 0.f;
  for (int k = 0; k < 13; ++k) M.pad1[k] = 0.f;
  // symbol range of node (l, p) by the split rule of the reduced tree
  uint64_t s = 0, e = sigma;
  bool exists = true;
  for (int i = (int)l - 1; i >= 0; --i) {
    if (e - s <= 1) {
      exists = false;
      break;
    }
    const uint64_t half = pow2_below(e - s);
    if ((p >> i) & 1) s += half;
    else e = s + half;
  }
  if (exists && e - s >= 2) {
    const uint64_t mid = s + pow2_below(e - s);
    const NodeQ nd = nodes[(1ull << l) - 1 + p];
    M.start = cum[s];
    M.len = cum[e] - cum[s];
    M.cnt = b ? cum[e] - cum[mid] : cum[mid] - cum[s];
    M.rank0 = b ? nd.start - nd.r0 : nd.r0;
    if (M.cnt > 0) M.eps = 0;  // a model exists; the budget is set after training
  }
  models[slot] = M;
}

// Count of side-b bits of a level before position x (x a multiple of the L2 block, x <= n_l).
template <int L2S>
__device__ __forceinline__ uint64_t count_before(const TreeDev& d, const LevelMeta& m, uint32_t b, uint64_t x) {
  const uint64_t r1 = d.L1[m.l1 + (x >> kL1Shift)] + d.L2[m.l2 + (x >> L2S)];
  return b ? r1 : x - r1;
}

// Training points of one model: the node-local side-b rank at every L2 boundary inside the node
// (evenly subsampled to at most kPMax - 2) plus the two ends (0, 0) and (1, 1).
template <int L2S>
__global__ __launch_bounds__(kLT) void k_learn_data(TreeDev d, LearnModel* __restrict__ models,
                                                    float2* __restrict__ pts, uint32_t pmax) {
  const uint64_t slot = blockIdx.x;
  LearnModel& M = models[slot];
  if (M.eps < 0) return;
  const LevelMeta m = d.meta[M.level];
  const uint64_t start = M.start, len = M.len, cnt = M.cnt;
  const uint64_t blo = (start + (1ull << L2S) - 1) >> L2S;  // first boundary strictly inside
  const uint64_t bhi = (start + len - 1) >> L2S;            // last boundary below the end
  const uint64_t nb = bhi >= blo ? bhi - blo + 1 : 0;
  const uint32_t take = (uint32_t)min<uint64_t>(nb, (uint64_t)pmax - 2);
  float2* P = pts + slot * pmax;
  for (uint32_t i = threadIdx.x; i < take; i += blockDim.x) {
    const uint64_t B = take == nb ? blo + i : blo + (uint64_t)((double)i * (double)(nb - 1) / (double)(take - 1));
    const uint64_t x = B << L2S;
    const uint64_t r = count_before<L2S>(d, m, M.side, x) - M.rank0;
    P[1 + i] = make_float2((float)((double)r / (double)cnt), (float)((double)(x - start) / (double)len));
  }
  if (threadIdx.x == 0) {
    P[0] = make_float2(0.f, 0.f);
    P[take + 1] = make_float2(1.f, 1.f);
    M.npts = take + 2;
  }
}

// Full-batch Adam, one block per model.
__global__ __launch_bounds__(kLT) void k_learn_train(LearnModel* __restrict__ models, const float2* __restrict__ pts,
                                                     uint32_t pmax, uint32_t epochs, float lr) {
  __shared__ float s_p[kNP + 3];
  __shared__ float s_wred[4 * 64];
  __shared__ float s_red[kNP + 1];
  const uint64_t slot = blockIdx.x;
  LearnModel& M = models[slot];
  if (M.eps < 0) return;
  const uint32_t np = M.npts;
  constexpr int kPer = kPMax / kLT;
  float u[kPer], v[kPer];
  int nmine = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const uint32_t j = threadIdx.x + (uint32_t)i * kLT;
    u[i] = 0.f;
    v[i] = 0.f;
    if (j < np) {
      const float2 q = pts[slot * pmax + j];
      u[i] = q.x;
      v[i] = q.y;
      nmine = i + 1;
    }
  }
  if (threadIdx.x < kNP) s_p[threadIdx.x] = M.p[threadIdx.x];
  float am = 0.f, av = 0.f;  // Adam moments of parameter threadIdx.x
  float b1t = 1.f, b2t = 1.f;
  const float scale = 2.f / (float)np;
  __syncthreads();
  float loss = 0.f;
  for (uint32_t t = 1; t <= epochs; ++t) {
    float pr[kNP];
#pragma unroll
    for (int j = 0; j < kNP; ++j) pr[j] = s_p[j];
    block_loss_grad(pr, u, v, nmine, scale, s_wred, s_red);
    loss = s_red[0] / (float)np;
    if (threadIdx.x < kNP) {
      const float g = s_red[1 + threadIdx.x];
      b1t *= 0.9f;
      b2t *= 0.999f;
      am = 0.9f * am + 0.1f * g;
      av = 0.999f * av + 0.001f * g * g;
      const float mh = am / (1.f - b1t), vh = av / (1.f - b2t);
      const float rate = lr * (1.f - 0.9f * (float)t / (float)epochs);
      s_p[threadIdx.x] = s_p[threadIdx.x] - rate * mh / (sqrtf(vh) + 1e-8f);
    }
    __syncthreads();
  }
  if (threadIdx.x < kNP) M.p[threadIdx.x] = s_p[threadIdx.x];
  if (threadIdx.x == 0) M.loss = loss;
}

// Prediction error in L2 blocks at every L2 boundary inside the node, for the trained model and for
// the starting point; sets the correction budget eps = ceil(max error) + 2.
template <int L2S>
__global__ __launch_bounds__(kLT) void k_learn_eval(TreeDev d, LearnModel* __restrict__ models) {
  __shared__ float s_r[4][4];
  const uint64_t slot = blockIdx.x;
  LearnModel& M = models[slot];
  if (M.eps < 0) return;
  const LevelMeta m = d.meta[M.level];
  float p[kNP];
#pragma unroll
  for (int j = 0; j < kNP; ++j) p[j] = M.p[j];
  const uint64_t start = M.start, len = M.len, cnt = M.cnt;
  const uint64_t blo = (start + (1ull << L2S) - 1) >> L2S, bhi = (start + len - 1) >> L2S;
  const double bl = (double)(1u << L2S);
  float smax = 0.f, ssum = 0.f, imax = 0.f, isum = 0.f;
  for (uint64_t B = blo + threadIdx.x; B <= bhi && bhi >= blo; B += blockDim.x) {
    const uint64_t x = B << L2S;
    const double u = (double)(count_before<L2S>(d, m, M.side, x) - M.rank0) / (double)cnt;
    const double tv = (double)(x - start);
    const float e = (float)(fabs((double)mlp_eval(p, (float)u) * (double)len - tv) / bl);
    const float ei = (float)(fabs(u * (double)len - tv) / bl);
    smax = fmaxf(smax, e);
    ssum += e;
    imax = fmaxf(imax, ei);
    isum += ei;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    smax = fmaxf(smax, __shfl_xor(smax, off, 64));
    imax = fmaxf(imax, __shfl_xor(imax, off, 64));
    ssum += __shfl_xor(ssum, off, 64);
    isum += __shfl_xor(isum, off, 64);
  }
  if (lane == 0) {
    s_r[wv][0] = smax;
    s_r[wv][1] = ssum;
    s_r[wv][2] = imax;
    s_r[wv][3] = isum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float a = 0.f, bsum = 0.f, c = 0.f, dsum = 0.f;
    for (int w = 0; w < 4; ++w) {
      a = fmaxf(a, s_r[w][0]);
      bsum += s_r[w][1];
      c = fmaxf(c, s_r[w][2]);
      dsum += s_r[w][3];
    }
    const float nb = bhi >= blo ? (float)(bhi - blo + 1) : 1.f;
    M.err_max = a;
    M.err_mean = bsum / nb;
    M.err_init_max = c;
    M.err_init_mean = dsum / nb;
    M.eps = (int32_t)ceilf(a) + 2;
  }
}

// ---------------------------------------------------------------- learned select

// Position of the j-th (1-based, node-local) side-b bit of the node of model M at level m.
template <int L2S>
__device__ __forceinline__ uint64_t select_learned_at(const TreeDev& d, const LevelMeta& m, const LearnModel& M,
                                                      uint32_t b, uint64_t j, uint32_t sshift) {
  const uint64_t T = M.rank0 + j;  // global target among the side-b bits of the level
  if (M.eps < 0) return select_at<L2S>(d, m, b, T, sshift);
  float p[kNP];
  {
    const float4* mp = reinterpret_cast<const float4*>(M.p);
#pragma unroll
    for (int k = 0; k < kNP / 4; ++k) {
      const float4 x = mp[k];
      p[4 * k] = x.x;
      p[4 * k + 1] = x.y;
      p[4 * k + 2] = x.z;
      p[4 * k + 3] = x.w;
    }
    p[kNP - 1] = M.p[kNP - 1];
  }
  const float u = ((float)j - 0.5f) / (float)M.cnt;
  const float v = fminf(fmaxf(mlp_eval(p, u), 0.f), 1.f);
  const uint64_t start = M.start, end = M.start + M.len;
  uint64_t guess = start + (uint64_t)((double)v * (double)M.len);
  guess = min(guess, end - 1);
  const uint64_t Blo = start >> L2S, Bhi = (end - 1) >> L2S;
  const uint64_t B0 = guess >> L2S;
  const uint64_t budget = (uint64_t)M.eps;
  // largest B in [Blo, Bhi] with count_before(B) < T; count_before(Blo) <= rank0 < T always.
  // First look at the aligned group of L2 counts holding B0 (one 128-byte line, inside one L1
  // block): the counts are non-decreasing, so the blocks below the target form a prefix of it.
  constexpr int GS = L2S <= 10 ? 6 : 5;
  constexpr uint32_t GN = 1u << GS;
  const uint64_t gbase = B0 & ~(uint64_t)(GN - 1);
  const uint64_t glo = max(gbase, Blo), ghi = min(gbase + GN - 1, Bhi);
  const uint64_t l1v = d.L1[m.l1 + ((gbase << L2S) >> kL1Shift)];
  const uint4* gp = reinterpret_cast<const uint4*>(d.L2 + m.l2 + gbase);
  uint4 g[GN / 8];
#pragma unroll
  for (uint32_t i = 0; i < GN / 8; ++i) g[i] = gp[i];
  // below(e) <=> count_before(gbase + e) < T, in 32-bit arithmetic with saturation
  int64_t D;
  if (b) D = (int64_t)min<uint64_t>(T - min(T, l1v), 1ull << 20);  // l2 < D
  else {
    const uint64_t base0 = (gbase << L2S) - l1v;  // zeros before the group
    D = T > base0 ? (int64_t)min<uint64_t>(T - base0, 1ull << 20) : -(int64_t)min<uint64_t>(base0 - T, 1ull << 20);
  }
  const int32_t Di = (int32_t)D;
  const uint32_t elo = (uint32_t)(glo - gbase), ehi = (uint32_t)(ghi - gbase);
  uint32_t below = 0;
#pragma unroll
  for (uint32_t e = 0; e < GN; ++e) {
    const uint32_t dw = (e & 7) < 4 ? ((e & 7) < 2 ? g[e >> 3].x : g[e >> 3].y) : ((e & 7) < 6 ? g[e >> 3].z : g[e >> 3].w);
    const int32_t l2v = (int32_t)((dw >> ((e & 1) * 16)) & 0xFFFFu);
    const bool lt = b ? (l2v < Di) : ((int32_t)(e << L2S) - l2v < Di);
    below += (lt && e >= elo && e <= ehi) ? 1u : 0u;
  }
  uint64_t lo, hi;  // invariant: count_before(lo) < T, and hi = Bhi + 1 or count_before(hi) >= T
  if (below > 0 && (glo + below - 1 < ghi || ghi == Bhi)) {
    lo = glo + below - 1;
    hi = lo + 1;
  } else if (below == 0) {
    // target left of the group (glo > Blo here): gallop left from glo
    hi = glo;
    uint64_t step = 1;
    for (;;) {
      if (hi - Blo <= step) {
        lo = Blo;
        break;
      }
      const uint64_t nb = hi - step;
      if (count_before<L2S>(d, m, b, nb << L2S) < T) {
        lo = nb;
        break;
      }
      hi = nb;
      step <<= 1;
      if (glo - nb > budget) return select_at<L2S>(d, m, b, T, sshift);
    }
  } else {
    // every block of the group is below the target: gallop right from ghi
    lo = ghi;
    uint64_t step = 1;
    for (;;) {
      const uint64_t nb = lo + step;
      if (nb > Bhi) {
        hi = Bhi + 1;
        break;
      }
      if (count_before<L2S>(d, m, b, nb << L2S) >= T) {
        hi = nb;
        break;
      }
      lo = nb;
      step <<= 1;
      if (nb - ghi > budget) return select_at<L2S>(d, m, b, T, sshift);
    }
  }
  while (hi - lo > 1) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (count_before<L2S>(d, m, b, mid << L2S) < T) lo = mid;
    else hi = mid;
  }
  // word scan inside the block, then the in-word select
  constexpr int L2W = (1 << L2S) / 64;
  uint32_t kk = (uint32_t)(T - count_before<L2S>(d, m, b, lo << L2S));
  const uint64_t* wp = d.bits + m.bits + (lo << (L2S - 6));
#pragma unroll
  for (int w = 0; w < L2W; ++w) {
    uint64_t word = wp[w];
    if (!b) word = ~word;
    const uint32_t pc = popc64(word);
    if (kk <= pc) return (lo << L2S) + 64u * (uint32_t)w + select_in_word(word, kk);
    kk -= pc;
  }
  return select_at<L2S>(d, m, b, T, sshift);  // not reached for valid targets
}

template <int L2S>
__global__ __launch_bounds__(kQT) void k_select_learned(QArgs a, const LearnModel* __restrict__ models,
                                                        const uint32_t* __restrict__ sym,
                                                        const uint64_t* __restrict__ kin, uint64_t q,
                                                        uint64_t* __restrict__ out) {
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  load_meta(a, s_meta);
  for (uint64_t j = (uint64_t)blockIdx.x * kQT + threadIdx.x; j < q; j += (uint64_t)gridDim.x * kQT) {
    const uint32_t c = sym[j];
    const uint64_t k = kin[j];
    uint64_t res;
    if (k == 0) {
      res = ~0ull;
    } else if (c >= a.sigma) {
      res = a.n;
    } else if (k > a.d.cum[c + 1] - a.d.cum[c]) {
      res = a.n;
    } else if (a.L == 0) {
      res = k - 1;
    } else {
      uint32_t len;
      const uint32_t code = encode_sym(c, a.sigma, a.L, a.pow2, &len);
      uint64_t r = k;
      for (int l = (int)len - 1; l >= 0; --l) {
        const uint64_t pc = (uint64_t)(code >> (a.L - 1 - l));  // child prefix at level l + 1
        const LearnModel& M = models[(1ull << (l + 1)) - 2 + pc];
        const uint64_t at = select_learned_at<L2S>(a.d, s_meta[l], M, M.side, r, a.sshift);
        r = at - M.start + 1;
      }
      res = r - 1;
    }
    out[j] = res;
  }
}

// One evaluation of the training objective (same device code as k_learn_train).
__global__ __launch_bounds__(kLT) void k_mlp_loss_grad(const float* __restrict__ params, const float* __restrict__ u,
                                                       const float* __restrict__ v, uint32_t P,
                                                       float* __restrict__ out) {
  __shared__ float s_wred[4 * 64];
  __shared__ float s_red[kNP + 1];
  float p[kNP];
#pragma unroll
  for (int j = 0; j < kNP; ++j) p[j] = params[j];
  constexpr int kPer = kPMax / kLT;
  float uu[kPer], vv[kPer];
  int nmine = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const uint32_t jj = threadIdx.x + (uint32_t)i * kLT;
    uu[i] = jj < P ? u[jj] : 0.f;
    vv[i] = jj < P ? v[jj] : 0.f;
    if (jj < P) nmine = i + 1;
  }
  block_loss_grad(p, uu, vv, nmine, 2.f / (float)P, s_wred, s_red);
  if (threadIdx.x == 0) out[0] = s_red[0] / (float)P;
  if (threadIdx.x < kNP) out[1 + threadIdx.x] = s_red[1 + threadIdx.x];
}

}  // namespace wt

using namespace wt;

extern "C" wt_status wt_learn_select(wt_tree* t, const wt_learn_opts* opts, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_learn_select: tree is NULL");
  uint32_t epochs = 500, pmax = kPMax;
  float lr = 3e-3f;
  if (opts) {
    if (opts->epochs) epochs = opts->epochs;
    if (opts->max_points) pmax = opts->max_points;
    if (opts->lr > 0.f) lr = opts->lr;
  }
  if (pmax < 4 || pmax > (uint32_t)kPMax) return fail(WT_ERR_ARG, "wt_learn_select: max_points must be in [4, 2048]");
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nmodels = t->L ? (1ull << (t->L + 1)) - 2 : 0;
  if (t->learn) {
    dev_free(t->learn, st);
    t->learn = nullptr;
  }
  t->nmodels = (uint32_t)nmodels;
  std::memset(&t->linfo, 0, sizeof(t->linfo));
  t->linfo.params_per_model = kNP;
  if (nmodels == 0) {
    t->learn = dev_alloc(256, st);
    if (!t->learn) return fail(WT_ERR_OOM, "wt_learn_select: allocation failed");
    return WT_OK;
  }
  const size_t mbytes = nmodels * sizeof(LearnModel);
  t->learn = dev_alloc(mbytes, st);
  if (!t->learn) return fail(WT_ERR_OOM, "wt_learn_select: model allocation failed");
  float2* pts = (float2*)dev_alloc(nmodels * pmax * sizeof(float2), st);
  if (!pts) return fail(WT_ERR_OOM, "wt_learn_select: training data allocation failed");
  LearnModel* models = (LearnModel*)t->learn;
  hipEvent_t e0, e1;
  WT_HIP(hipEventCreate(&e0));
  WT_HIP(hipEventCreate(&e1));
  const uint32_t grid = (uint32_t)ceil_div(nmodels, 256);
  hipLaunchKernelGGL(k_learn_setup, dim3(grid), dim3(256), 0, st, (uint32_t)t->sigma, t->L,
                     (const uint64_t*)t->dev.cum, (const NodeQ*)t->dev.nodes, models, nmodels);
  WT_HIP(hipEventRecord(e0, st));
  switch (t->l2_bits) {
    case 256: hipLaunchKernelGGL(k_learn_data<8>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models, pts, pmax); break;
    case 512: hipLaunchKernelGGL(k_learn_data<9>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models, pts, pmax); break;
    case 1024: hipLaunchKernelGGL(k_learn_data<10>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models, pts, pmax); break;
    default: hipLaunchKernelGGL(k_learn_data<11>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models, pts, pmax); break;
  }
  hipLaunchKernelGGL(k_learn_train, dim3((uint32_t)nmodels), dim3(kLT), 0, st, models, (const float2*)pts, pmax,
                     epochs, lr);
  WT_HIP(hipEventRecord(e1, st));
  switch (t->l2_bits) {
    case 256: hipLaunchKernelGGL(k_learn_eval<8>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models); break;
    case 512: hipLaunchKernelGGL(k_learn_eval<9>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models); break;
    case 1024: hipLaunchKernelGGL(k_learn_eval<10>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models); break;
    default: hipLaunchKernelGGL(k_learn_eval<11>, dim3((uint32_t)nmodels), dim3(kLT), 0, st, t->dev, models); break;
  }
  WT_HIP(hipGetLastError());
  std::vector<LearnModel> hm(nmodels);
  WT_HIP(hipMemcpyAsync(hm.data(), models, mbytes, hipMemcpyDeviceToHost, st));
  WT_HIP(hipStreamSynchronize(st));
  dev_free(pts, st);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // statistics weighted by the number of L2 boundaries of each node
  double wsum = 0, es = 0, eis = 0, emax = 0, eimax = 0, ls = 0;
  uint32_t nm = 0;
  for (const auto& M : hm) {
    if (M.eps < 0) continue;
    ++nm;
    const double w = std::max<double>(1.0, (double)M.len / (double)t->l2_bits);
    wsum += w;
    es += w * M.err_mean;
    eis += w * M.err_init_mean;
    emax = std::max<double>(emax, M.err_max);
    eimax = std::max<double>(eimax, M.err_init_max);
    ls += M.loss;
  }
  t->linfo.models = nm;
  t->linfo.mean_err_blocks = wsum > 0 ? es / wsum : 0;
  t->linfo.mean_err_init_blocks = wsum > 0 ? eis / wsum : 0;
  t->linfo.max_err_blocks = emax;
  t->linfo.max_err_init_blocks = eimax;
  t->linfo.final_loss_mean = nm ? ls / nm : 0;
  t->linfo.train_ms = ms;
  return WT_OK;
}

extern "C" wt_status wt_select_learned(const wt_tree* t, const uint32_t* d_sym, const uint64_t* d_k, uint64_t q,
                                       uint64_t* d_out, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_select_learned: tree is NULL");
  if (!t->learn) return fail(WT_ERR_STATE, "wt_select_learned: call wt_learn_select first");
  if (q == 0) return WT_OK;
  if (!d_sym || !d_k || !d_out) return fail(WT_ERR_ARG, "wt_select_learned: NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  const QArgs a = make_args(t);
  const uint32_t grid = query_grid(q);
  const LearnModel* models = (const LearnModel*)t->learn;
  WT_DISPATCH_L2(t->l2_bits, k_select_learned, a, models, d_sym, d_k, q, d_out);
  WT_HIP(hipGetLastError());
  return WT_OK;
}

extern "C" wt_status wt_learned_info(const wt_tree* t, wt_learned_info_t* out) {
  clear_error();
  if (!t || !out) return fail(WT_ERR_ARG, "wt_learned_info: NULL argument");
  if (!t->learn) return fail(WT_ERR_STATE, "wt_learned_info: no learned index");
  *out = t->linfo;
  return WT_OK;
}

extern "C" wt_status wt_mlp_loss_grad(const float* d_params, const float* d_u, const float* d_v, uint32_t P,
                                      float* d_out, wt_stream_t stream) {
  clear_error();
  if (!d_params || !d_u || !d_v || !d_out) return fail(WT_ERR_ARG, "wt_mlp_loss_grad: NULL buffer");
  if (P == 0 || P > (uint32_t)kPMax) return fail(WT_ERR_ARG, "wt_mlp_loss_grad: P must be in [1, 2048]");
  hipLaunchKernelGGL(k_mlp_loss_grad, dim3(1), dim3(kLT), 0, (hipStream_t)stream, d_params, d_u, d_v, P, d_out);
  WT_HIP(hipGetLastError());
  return WT_OK;
}
