// Host launchers of the MFMA GEMM core (see gemm.h).
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

template <typename TC>
struct Tile;
template <>
struct Tile<float> {
  static constexpr int BM = 64, BN = 64, BK = 32;
};
template <>
struct Tile<bf16_t> {
  static constexpr int BM = 64, BN = 64, BK = 64;
};

template <class Prob, typename TC>
void run(const Prob& p, Epi e, int splits, float* partial, hipStream_t s) {
  constexpr int BM = Tile<TC>::BM, BN = Tile<TC>::BN, BK = Tile<TC>::BK;
  if (p.M <= 0 || p.N <= 0) return;
  const int tiles_m = cdiv(p.M, BM), tiles_n = cdiv(p.N, BN);
  if (splits < 1) splits = 1;
  int kps = cdiv(cdiv(p.K, splits), BK) * BK;
  if (kps <= 0) kps = BK;
  splits = cdiv(p.K, kps);
  if (splits < 1) splits = 1;
  Epi ek = e;
  if (splits > 1) ek.partial = partial;
  else ek.partial = nullptr;
  hipLaunchKernelGGL((gemm_kernel<Prob, TC, BM, BN, BK>), dim3(tiles_m * tiles_n, splits), dim3(256),
                     0, s, p, ek, tiles_n, kps);
  if (splits > 1) {
    const size_t MN = (size_t)p.M * p.N;
    const int nb = (int)std::min<size_t>(2048, (MN + 255) / 256);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(nb), dim3(256), 0, s, partial, splits, p.M, p.N, e);
  }
}

}  // namespace

int gemm_max_splits_for(long M, long N, long K, int prec) {
  // enough workgroups to cover the chip (256 CUs) a few times, each split
  // keeping at least a few K tiles
  const int BM = 64, BN = 64, BK = prec == 1 ? 64 : 32;
  const long tiles = (long)cdiv(M, BM) * cdiv(N, BN);
  long want = (1024 + tiles - 1) / tiles;
  const long kmax = std::max<long>(1, K / (4 * BK));
  if (want > kmax) want = kmax;
  if (want > 512) want = 512;
  return (int)std::max<long>(1, want);
}

void gemm_conv_fwd(int prec, const ConvGeo& g, const float* x, const void* w, Epi e, int splits,
                   float* partial, hipStream_t s) {
  const int M = g.B * g.Ho * g.Wo, N = g.Co, K = g.KH * g.KW * g.C;
  if (prec == 1) {
    ConvFwdProb<bf16_t> p{g, x, (const bf16_t*)w, M, N, K};
    run<ConvFwdProb<bf16_t>, bf16_t>(p, e, splits, partial, s);
  } else {
    ConvFwdProb<float> p{g, x, (const float*)w, M, N, K};
    run<ConvFwdProb<float>, float>(p, e, splits, partial, s);
  }
}

void gemm_conv_dgrad(int prec, const ConvGeo& g, const float* dy, const void* w, Epi e, int splits,
                     float* partial, hipStream_t s) {
  const int M = g.B * g.H * g.W, N = g.C, K = g.KH * g.KW * g.Co;
  if (prec == 1) {
    ConvDgradProb<bf16_t> p{g, dy, (const bf16_t*)w, M, N, K};
    run<ConvDgradProb<bf16_t>, bf16_t>(p, e, splits, partial, s);
  } else {
    ConvDgradProb<float> p{g, dy, (const float*)w, M, N, K};
    run<ConvDgradProb<float>, float>(p, e, splits, partial, s);
  }
}

void gemm_conv_wgrad(int prec, const ConvGeo& g, const float* x, const float* dy, Epi e, int splits,
                     float* partial, hipStream_t s) {
  ConvWgradProb p{g, x, dy, g.Co, g.KH * g.KW * g.C, g.B * g.Ho * g.Wo};
  if (prec == 1) run<ConvWgradProb, bf16_t>(p, e, splits, partial, s);
  else run<ConvWgradProb, float>(p, e, splits, partial, s);
}

template <typename TB, bool TA, bool TBt>
static void dense_t(int prec, const float* a, int lda, const TB* b, int ldb, int M, int N, int K,
                    Epi e, int splits, float* partial, hipStream_t s) {
  DenseProb<float, TB, TA, TBt> p{a, b, lda, ldb, M, N, K};
  if (prec == 1) run<DenseProb<float, TB, TA, TBt>, bf16_t>(p, e, splits, partial, s);
  else run<DenseProb<float, TB, TA, TBt>, float>(p, e, splits, partial, s);
}

void gemm_dense(int prec, bool ta, bool tb, const float* a, int lda, const void* b, bool b_lp,
                int ldb, int M, int N, int K, Epi e, int splits, float* partial, hipStream_t s) {
#define DENSE_CASE(TBTYPE, TA_, TB_) \
  dense_t<TBTYPE, TA_, TB_>(prec, a, lda, (const TBTYPE*)b, ldb, M, N, K, e, splits, partial, s)
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
