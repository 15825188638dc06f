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
#include <cstddef>
#include <cstring>
#include <vector>

#include "wt_host.h"
#include "wt_internal.h"
#include "wt_learn_dev.h"
#include "wt_query_dev.h"

namespace wt {

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

// Adds the contribution of one point (u, v) to the loss and the gradient (scale = 2 / P); a point with
// scale = wl = 0 adds nothing (a thread's unused point slots), so every slot is computed without a
// branch and the slots' independent chains overlap. The output sum is taken as four partial sums.
__device__ __forceinline__ void mlp_point(const float* __restrict__ p, float u, float v, float scale, float wl,
                                          float* g, float& loss) {
  float h[kH];
  float ys[4] = {p[3 * kH], 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < kH; ++k) {
    h[k] = fmaf(p[k], u, p[kH + k]);
    ys[k & 3] = fmaf(p[2 * kH + k], fmaxf(h[k], 0.f), ys[k & 3]);
  }
  const float y = (ys[0] + ys[1]) + (ys[2] + ys[3]);
  const float r = y - v;
  loss += wl * (r * r);
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
#pragma unroll
  for (int i = 0; i < kPMax / kLT; ++i) {
    const bool use = i < nmine;
    mlp_point(p, u[i], v[i], use ? scale : 0.f, use ? 1.f : 0.f, g, loss);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // Wave reduce-scatter of the 64 slots [loss, g, 0...]: at each halving step a lane keeps one half
  // of its current slots and adds the partner's copy of that half; lane l ends with the wave total
  // of slot l (63 exchanges instead of 6 per value).
  static_assert(kNP + 1 <= 64, "one slot per lane");
  float x[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) x[j] = j == 0 ? loss : (j <= kNP ? g[j - 1] : 0.f);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int i = 0; i < o; ++i) {
      const float send = up ? x[i] : x[i + o];
      const float keep = up ? x[i + o] : x[i];
      x[i] = keep + __shfl_xor(send, o, 64);
    }
  }
  if (lane <= kNP) s_wred[wv * 64 + lane] = x[0];
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

// Piecewise-linear form of every trained network (one thread per model), computed in FP64: the
// switch points inside (0, 1), sorted, and on each piece the sum of the active units' slopes and
// intercepts (a unit is active on a piece when it is positive at the piece's midpoint).
__global__ void k_learn_compile(const LearnModel* __restrict__ models, LearnQ* __restrict__ qm, uint64_t nmodels) {
  const uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nmodels) return;
  const LearnModel& M = models[slot];
  LearnQ Q;
  Q.start = M.start;
  Q.len = M.len;
  Q.rank0 = M.rank0;
  Q.eps = M.eps < 0 ? -1 : 0;
  Q.side = M.side;
  Q.cntf = (float)M.cnt;
  Q.lenf = (float)M.len;
  Q.pad0 = 0;
  Q.pad1 = 0;
  double t[kH];
  uint32_t m = 0;
  for (int k = 0; k < kH; ++k) {
    const double w = M.p[k], c = M.p[kH + k];
    if (w != 0.0) {
      const double x = -c / w;
      if (x > 0.0 && x < 1.0) t[m++] = x;
    }
  }
  for (uint32_t i = 1; i < m; ++i) {  // insertion sort (at most 16)
    const double x = t[i];
    uint32_t k = i;
    for (; k > 0 && t[k - 1] > x; --k) t[k] = t[k - 1];
    t[k] = x;
  }
  for (uint32_t s = 0; s <= m; ++s) {
    const double lo = s ? t[s - 1] : 0.0, hi = s < m ? t[s] : 1.0;
    const double mid = 0.5 * (lo + hi);
    double A = 0.0, C = M.p[3 * kH];
    for (int k = 0; k < kH; ++k) {
      const double w = M.p[k], c = M.p[kH + k], o = M.p[2 * kH + k];
      if (w * mid + c > 0.0) {
        A += o * w;
        C += o * c;
      }
    }
    Q.piece[s] = make_float2((float)A, (float)C);
  }
  for (uint32_t s = m + 1; s <= (uint32_t)kH; ++s) Q.piece[s] = Q.piece[m];
  for (uint32_t s = 0; s < (uint32_t)kH; ++s) Q.knot[s] = s < m ? (float)t[s] : 2.f;
  Q.npieces = m + 1;
  qm[slot] = Q;
}

// Prediction error in L2 blocks at every L2 boundary inside the node, for the compiled trained model
// (the evaluation queries use) and for the starting point; sets the correction budget
// eps = ceil(max error) + 2.
constexpr uint32_t kEvalChunks = 64;  // blocks per model in the error evaluation

template <int L2S>
__global__ __launch_bounds__(kLT) void k_learn_eval(TreeDev d, const LearnModel* __restrict__ models,
                                                    const LearnQ* __restrict__ qm, float4* __restrict__ part) {
  __shared__ float s_r[4][4];
  const uint64_t slot = blockIdx.x;
  const uint32_t ch = blockIdx.y;
  const LearnModel& M = models[slot];
  if (M.eps < 0) return;
  const LevelMeta m = d.meta[M.level];
  const LearnQ& Q = qm[slot];
  const uint64_t start = M.start, len = M.len, cnt = M.cnt;
  const uint64_t blo = (start + (1ull << L2S) - 1) >> L2S, bhi = (start + len - 1) >> L2S;
  const double bl = (double)(1u << L2S);
  float smax = 0.f, ssum = 0.f, imax = 0.f, isum = 0.f;
  for (uint64_t B = blo + (uint64_t)ch * kLT + threadIdx.x; B <= bhi && bhi >= blo; B += (uint64_t)kLT * kEvalChunks) {
    const uint64_t x = B << L2S;
    const double u = (double)(count_before<L2S>(d, m, M.side, x) - M.rank0) / (double)cnt;
    const double tv = (double)(x - start);
    const float e = (float)(fabs((double)pla_eval(Q, (float)u) * (double)len - tv) / bl);
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
    part[slot * kEvalChunks + ch] = make_float4(a, bsum, c, dsum);
  }
}

// Per model, the chunks' partial results in a fixed order: error statistics and the budget
// eps = ceil(max error) + 2.
template <int L2S>
__global__ void k_learn_finish(LearnModel* __restrict__ models, LearnQ* __restrict__ qm,
                               const float4* __restrict__ part, uint64_t nmodels) {
  const uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nmodels) return;
  LearnModel& M = models[slot];
  if (M.eps < 0) return;
  float a = 0.f, bsum = 0.f, c = 0.f, dsum = 0.f;
  for (uint32_t ch = 0; ch < kEvalChunks; ++ch) {
    const float4 v = part[slot * kEvalChunks + ch];
    a = fmaxf(a, v.x);
    bsum += v.y;
    c = fmaxf(c, v.z);
    dsum += v.w;
  }
  const uint64_t blo = (M.start + (1ull << L2S) - 1) >> L2S, bhi = (M.start + M.len - 1) >> L2S;
  const float nb = bhi >= blo ? (float)(bhi - blo + 1) : 1.f;
  M.err_max = a;
  M.err_mean = bsum / nb;
  M.err_init_max = c;
  M.err_init_mean = dsum / nb;
  M.eps = (int32_t)ceilf(a) + 2;
  qm[slot].eps = M.eps;
}

// ---------------------------------------------------------------- learned select


template <int L2S, uint32_t QB>
__global__ __launch_bounds__(QB, 8) void k_select_learned(QArgs a, const LearnQ* __restrict__ qm,
                                                        const uint32_t* __restrict__ sym,
                                                        const uint64_t* __restrict__ kin, uint64_t q,
                                                        uint64_t* __restrict__ out,
                                                        const SQ* __restrict__ sq, uint32_t subshift) {
  constexpr int GS = learn_gs<L2S>();
  __shared__ LevelMeta s_meta[WT_MAX_LEVELS];
  __shared__ LocalOrder<QB> s_ord;
  load_meta(a, s_meta);
  if (sq) {
    for (uint64_t j0 = xcd_block() * QB; j0 < q; j0 += (uint64_t)gridDim.x * QB) {
      uint32_t jj, c;
      uint64_t x;
      if (local_order<2, QB>(a, sq, q, j0 + threadIdx.x, subshift, s_ord, jj, c, x))
        out[jj] = select_learned_one<L2S, GS>(a, s_meta, qm, c, x);
    }
    return;
  }
  for (uint64_t j = xcd_block() * QB + threadIdx.x; j < q; j += (uint64_t)gridDim.x * QB)
    out[j] = select_learned_one<L2S, GS>(a, s_meta, qm, sym[j], kin[j]);
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

namespace wt {
size_t learn_model_bytes() { return sizeof(LearnModel); }
}  // namespace wt

extern "C" wt_status wt_learn_select(wt_tree* t, const wt_learn_opts* opts, wt_stream_t stream) {
  clear_error();
  if (!t) return fail(WT_ERR_ARG, "wt_learn_select: tree is NULL");
  if (t->matrix) return fail(WT_ERR_ARG, "wt_learn_select: the learned index needs the tree's node table (not a wavelet matrix)");
  if (t->huff) return fail(WT_ERR_ARG, "wt_learn_select: the learned index is built for balanced and reduced trees, not Huffman-shaped ones");
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
  ++t->learn_version;
  std::memset(&t->linfo, 0, sizeof(t->linfo));
  t->linfo.params_per_model = kNP;
  if (nmodels == 0) {
    t->learn = dev_alloc(256, st);
    if (!t->learn) return fail(WT_ERR_OOM, "wt_learn_select: allocation failed");
    return WT_OK;
  }
  const size_t mbytes = nmodels * sizeof(LearnModel);
  t->learn = dev_alloc(mbytes + nmodels * sizeof(LearnQ), st);  // training records, then query forms
  if (!t->learn) return fail(WT_ERR_OOM, "wt_learn_select: model allocation failed");
  // training points (stride pmax per model), reused for the evaluation's partial results
  const size_t pts_per_model = std::max<size_t>(pmax, kEvalChunks * sizeof(float4) / sizeof(float2));
  float2* pts = (float2*)dev_alloc(nmodels * pts_per_model * sizeof(float2), st);
  if (!pts) return fail(WT_ERR_OOM, "wt_learn_select: training data allocation failed");
  LearnModel* models = (LearnModel*)t->learn;
  LearnQ* qm = (LearnQ*)((char*)t->learn + mbytes);
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
  hipLaunchKernelGGL(k_learn_compile, dim3(grid), dim3(256), 0, st, (const LearnModel*)models, qm, nmodels);
  WT_HIP(hipEventRecord(e1, st));
  // error evaluation: partial results of kEvalChunks blocks per model in the (no longer needed)
  // training-point buffer, then one thread per model combines them
  float4* part = reinterpret_cast<float4*>(pts);
  const dim3 eg((uint32_t)nmodels, kEvalChunks);
#define WT_EVAL(S)                                                                                        \
  hipLaunchKernelGGL(k_learn_eval<S>, eg, dim3(kLT), 0, st, t->dev, (const LearnModel*)models,           \
                     (const LearnQ*)qm, part);                                                           \
  hipLaunchKernelGGL(k_learn_finish<S>, dim3(grid), dim3(256), 0, st, models, qm, (const float4*)part, nmodels)
  switch (t->l2_bits) {
    case 256: WT_EVAL(8); break;
    case 512: WT_EVAL(9); break;
    case 1024: WT_EVAL(10); break;
    default: WT_EVAL(11); break;
  }
#undef WT_EVAL
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
  const LearnQ* qm = (const LearnQ*)((const char*)t->learn + (size_t)t->nmodels * sizeof(LearnModel));
  SortBufs sb;
  bool binned;
  const uint32_t* sym = d_sym;
  void* mapped = nullptr;
  wt_status rc = alpha_map_syms(t, d_sym, q, st, &sym, &mapped);
  if (rc != WT_OK) return rc;
  rc = sort_batch(t, a, 2, sym, d_k, q, st, sb, binned);
  if (rc != WT_OK) {
    if (mapped) dev_free(mapped, st);
    return rc;
  }
  qprof_begin("select_learned", st);
  if (binned) {
    const uint32_t grid = query_grid(q, kQB);
    WT_DISPATCH_L2(t->l2_bits, kQB, k_select_learned, a, qm, sym, d_k, q, d_out, (const SQ*)sb.sq, sb.subshift);
    dev_free(sb.block, st);
  } else {
    const uint32_t grid = query_grid(q, kQT);
    WT_DISPATCH_L2(t->l2_bits, kQT, k_select_learned, a, qm, sym, d_k, q, d_out, (const SQ*)nullptr, 0u);
  }
  qprof_end(st);
  if (mapped) dev_free(mapped, st);
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

extern "C" wt_status wt_learned_model(const wt_tree* t, uint32_t slot, wt_learned_model_t* out) {
  clear_error();
  if (!t || !out) return fail(WT_ERR_ARG, "wt_learned_model: NULL argument");
  if (!t->learn) return fail(WT_ERR_STATE, "wt_learned_model: no learned index");
  if (slot >= t->nmodels) return fail(WT_ERR_ARG, "wt_learned_model: slot %u >= %u", slot, t->nmodels);
  LearnModel M;
  LearnQ Q;
  WT_HIP(hipDeviceSynchronize());
  WT_HIP(hipMemcpy(&M, (const LearnModel*)t->learn + slot, sizeof(M), hipMemcpyDeviceToHost));
  WT_HIP(hipMemcpy(&Q, (const char*)t->learn + (size_t)t->nmodels * sizeof(LearnModel) + (size_t)slot * sizeof(LearnQ),
                   sizeof(Q), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  out->level = (int32_t)M.level;
  out->side = M.side;
  out->eps = Q.eps;
  out->points = M.npts;
  out->start = M.start;
  out->len = M.len;
  out->count = M.cnt;
  out->rank0 = M.rank0;
  for (int k = 0; k < kNP; ++k) out->params[k] = M.p[k];
  out->pieces = Q.npieces;
  for (int k = 0; k < kH; ++k) out->knots[k] = Q.knot[k];
  for (int k = 0; k <= kH; ++k) {
    out->slope[k] = Q.piece[k].x;
    out->intercept[k] = Q.piece[k].y;
  }
  out->err_mean = M.err_mean;
  out->err_max = M.err_max;
  out->err_init_mean = M.err_init_mean;
  out->err_init_max = M.err_init_max;
  out->loss = M.loss;
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
