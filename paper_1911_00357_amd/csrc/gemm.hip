// Host launchers of the MFMA GEMM core (see gemm.h): tile-shape choice,
// split-K and the ordered split-K reduction.
#include "gemm.h"
#include "kernels.h"

__global__ void __launch_bounds__(256) splitk_reduce_kernel(const float* __restrict__ part, int splits,
                                                            int M, int N, Epi e) {
  const size_t MN = (size_t)M * N;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < MN; i += (size_t)gridDim.x * 256) {
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += part[(size_t)z * MN + i];
    const int m = (int)(i / N), n = (int)(i - (size_t)m * N);
    v *= e.alpha;
    float* cp = e.C + (size_t)m * e.ldc + n;
    if (e.accumulate) v += *cp;
    if (e.bias) v += e.bias[n];
    if (e.relu) v = fmaxf(v, 0.f);
    *cp = v;
  }
}

namespace {

constexpr int BK = 32;

enum Tile { T128x128, T128x64, T64x128, T64x64, T128x32, T32x128 };

struct TileDim {
  int bm, bn;
};
TileDim dim_of(Tile t) {
  switch (t) {
    case T128x128: return {128, 128};
    case T128x64: return {128, 64};
    case T64x128: return {64, 128};
    case T64x64: return {64, 64};
    case T128x32: return {128, 32};
    default: return {32, 128};
  }
}

Tile choose(long M, long N, int prec) {
  const bool f32 = prec == 0;  // float32 tiles stay within 64 KB of LDS
  if (N <= 32) return T128x32;
  if (M <= 32) return T32x128;
  if (M <= 64) return N >= 128 ? T64x128 : T64x64;
  if (N <= 64) return T128x64;
  if (M * N <= 256L * 128 * 128) return T64x64;  // small problems: more workgroups
  return f32 ? T128x64 : T128x128;
}

// Workgroups wanted before splitting K: a few per CU (256 CUs).
int splits_for(long tiles, long K) {
  if (tiles >= 512) return 1;
  long want = (1024 + tiles - 1) / tiles;
  // >= 4 K tiles per split; >= 2 for very few output tiles (latency-bound launches)
  const long kmax = std::max<long>(1, K / ((tiles < 64 ? 2 : 4) * BK));
  return (int)std::max<long>(1, std::min<long>({want, kmax, 256}));
}

template <class Prob, typename TC, int BM, int BN, int WGM, int WGN, bool SPLIT>
int launch(const Prob& p, Epi e, int splits, float* partial, hipStream_t s, bool defer) {
  const int tiles_m = cdiv(p.M, BM), tiles_n = cdiv(p.N, BN);
  int kps = cdiv(cdiv(p.K, splits), BK) * BK;
  if (kps <= 0) kps = BK;
  splits = std::max(1, cdiv(p.K, kps));
  Epi ek = e;
  ek.partial = splits > 1 ? partial : nullptr;
  hipLaunchKernelGGL((gemm_kernel<Prob, TC, BM, BN, WGM, WGN, SPLIT>), dim3(tiles_m * tiles_n, splits),
                     dim3(256), 0, s, p, ek, tiles_n, kps);
  if (splits > 1 && !defer) {
    const size_t MN = (size_t)p.M * p.N;
    const int nb = (int)std::min<size_t>(2048, (MN + 255) / 256);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(nb), dim3(256), 0, s, partial, splits, p.M, p.N, e);
  }
  return splits;
}

// Returns the K split used; with defer and a split > 1 the partial tiles are
// left in `partial` ([splits][M][N]) for the caller to sum.
template <class Prob, typename TC, bool SPLIT>
int run(const Prob& p, Epi e, size_t partial_bytes, float* partial, hipStream_t s, int prec, bool defer = false) {
  if (p.M <= 0 || p.N <= 0) return 1;
  const Tile t = choose(p.M, p.N, prec);
  const TileDim d = dim_of(t);
  const long tiles = (long)cdiv(p.M, d.bm) * cdiv(p.N, d.bn);
  int splits = p.K > 0 ? splits_for(tiles, p.K) : 1;
  const long cap = (long)(partial_bytes / (sizeof(float) * (size_t)p.M * p.N));
  if (splits > cap) splits = (int)std::max<long>(1, cap);
  switch (t) {
    case T128x128: return launch<Prob, TC, 128, 128, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T128x64: return launch<Prob, TC, 128, 64, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T64x128: return launch<Prob, TC, 64, 128, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T64x64: return launch<Prob, TC, 64, 64, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T128x32: return launch<Prob, TC, 128, 32, 4, 1, SPLIT>(p, e, splits, partial, s, defer);
    default: return launch<Prob, TC, 32, 128, 1, 4, SPLIT>(p, e, splits, partial, s, defer);
  }
}

// bfloat16 with the gradient operand split (backward products) or not.
template <class Prob>
void run_prec(const Prob& p, Epi e, int prec, bool split_a, size_t pb, float* partial, hipStream_t s) {
  if (prec == 0) run<Prob, float, false>(p, e, pb, partial, s, 0);
  else if (split_a) run<Prob, bf16_t, true>(p, e, pb, partial, s, 1);
  else run<Prob, bf16_t, false>(p, e, pb, partial, s, 1);
}

}  // namespace

int gemm_max_splits_for(long M, long N, long K, int prec) {
  const TileDim d = dim_of(choose(M, N, prec));
  return splits_for((long)cdiv(M, d.bm) * cdiv(N, d.bn), K);
}

int gemm_conv_fwd(int prec, const ConvGeo& g, const float* x, const void* w, Epi e, size_t pb,
                  float* partial, hipStream_t s, bool defer) {
  const int M = g.B * g.Ho * g.Wo, N = g.Co, K = g.KH * g.KW * g.C;
  const FastDiv dC = fast_div(g.C), dKW = fast_div(g.KW), dHoWo = fast_div(g.Ho * g.Wo), dWo = fast_div(g.Wo);
  if (prec == 1) {
    ConvFwdProb<bf16_t> p{g, dC, dKW, dHoWo, dWo, x, (const bf16_t*)w, M, N, K};
    return run<ConvFwdProb<bf16_t>, bf16_t, false>(p, e, pb, partial, s, 1, defer);
  }
  ConvFwdProb<float> p{g, dC, dKW, dHoWo, dWo, x, (const float*)w, M, N, K};
  return run<ConvFwdProb<float>, float, false>(p, e, pb, partial, s, 0, defer);
}

void gemm_conv_dgrad(int prec, const ConvGeo& g, const float* dy, const void* w, Epi e, size_t pb,
                     float* partial, hipStream_t s) {
  const int M = g.B * g.H * g.W, N = g.C, K = g.KH * g.KW * g.Co;
  const FastDiv dCo = fast_div(g.Co), dKW = fast_div(g.KW), dHW = fast_div(g.H * g.W), dW = fast_div(g.W);
  if (prec == 1) {
    ConvDgradProb<bf16_t> p{g, dCo, dKW, dHW, dW, dy, (const bf16_t*)w, M, N, K};
    run_prec(p, e, 1, true, pb, partial, s);
  } else {
    ConvDgradProb<float> p{g, dCo, dKW, dHW, dW, dy, (const float*)w, M, N, K};
    run_prec(p, e, 0, false, pb, partial, s);
  }
}

void gemm_conv_wgrad(int prec, const ConvGeo& g, const float* x, const float* dy, Epi e, size_t pb,
                     float* partial, hipStream_t s) {
  ConvWgradProb p{g, fast_div(g.C), fast_div(g.KW), fast_div(g.Ho * g.Wo), fast_div(g.Wo), x, dy, g.Co,
                  g.KH * g.KW * g.C, g.B * g.Ho * g.Wo};
  run_prec(p, e, prec, true, pb, partial, s);
}

template <typename TB, bool TA, bool TBt>
static void dense_t(int prec, bool split_a, const float* a, int lda, const TB* b, int ldb, int M, int N,
                    int K, Epi e, size_t pb, float* partial, hipStream_t s) {
  DenseProb<float, TB, TA, TBt> p{a, b, lda, ldb, M, N, K};
  run_prec(p, e, prec, split_a, pb, partial, s);
}

void gemm_dense(int prec, bool ta, bool tb, const float* a, int lda, const void* b, bool b_lp, int ldb,
                int M, int N, int K, Epi e, bool split_a, size_t pb, float* partial, hipStream_t s) {
#define DENSE_CASE(TBTYPE, TA_, TB_) \
  dense_t<TBTYPE, TA_, TB_>(prec, split_a, a, lda, (const TBTYPE*)b, ldb, M, N, K, e, pb, partial, s)
  if (b_lp) {
    if (!ta && !tb) DENSE_CASE(bf16_t, false, false);
    else if (!ta && tb) DENSE_CASE(bf16_t, false, true);
    else if (ta && !tb) DENSE_CASE(bf16_t, true, false);
    else DENSE_CASE(bf16_t, true, true);
  } else {
    if (!ta && !tb) DENSE_CASE(float, false, false);
    else if (!ta && tb) DENSE_CASE(float, false, true);
    else if (ta && !tb) DENSE_CASE(float, true, false);
    else DENSE_CASE(float, true, true);
  }
#undef DENSE_CASE
}
