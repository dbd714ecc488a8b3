// Host launchers of the MFMA GEMM core (see gemm.h): tile-shape choice,
// split-K and the ordered split-K reduction.
#include "gemm.h"
#include "kernels.h"

// out = epilogue(sum_z part[z]): a block owns 64 outputs; wavefront w sums the
// splits z = w (mod 4) with 8 loads in flight, then the 4 partial sums are
// added in a fixed order (deterministic).
__global__ void __launch_bounds__(256) splitk_reduce_kernel(const float* __restrict__ part, int splits,
                                                            int M, int N, Epi e) {
  __shared__ float red[4][64];
  const size_t MN = (size_t)M * N;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const size_t i = (size_t)blockIdx.x * 64 + lane;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (i < MN) {
    int z = w;
    for (; z + 28 < splits; z += 32) {
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += part[(size_t)(z + 4 * q) * MN + i];
    }
    for (; z < splits; z += 4) acc[0] += part[(size_t)z * MN + i];
  }
  red[w][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (w == 0 && i < MN) {
    float v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    const int m = (int)(i / N), n = (int)(i - (size_t)m * N);
    v *= e.alpha;
    float* cp = e.C + crow(e, m) * e.ldc + n;
    if (e.accumulate) v += *cp;
    if (e.bias) v += e.bias[n];
    if (e.relu) v = fmaxf(v, 0.f);
    *cp = v;
  }
}

thread_local GemmTimer* g_gemm_timer = nullptr;
thread_local GemmTune* g_gemm_tune = nullptr;

namespace {

constexpr int BK = 32;

GemmTimer* active_timer(hipStream_t s) {
  GemmTimer* t = g_gemm_timer;
  if (!t || t->n >= t->cap) return nullptr;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  return t;
}

enum Tile { T128x128, T128x64, T64x128, T64x64, T128x32, T32x128 };
static_assert((int)T32x128 + 1 == kGemmTiles, "tile table range");

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
  GemmTimer* tm = active_timer(s);
  if (tm) hipEventRecord(tm->start[tm->n], s);
  hipLaunchKernelGGL((gemm_kernel<Prob, TC, BM, BN, WGM, WGN, SPLIT>), dim3(tiles_m * tiles_n, splits),
                     dim3(256), 0, s, p, ek, tiles_n, kps);
  if (tm) {
    hipEventRecord(tm->end[tm->n], s);
    ++tm->n;
    tm->flops += 2.0 * p.M * p.N * p.K;
    tm->wbytes += (double)p.N * p.K * WeightBytes<Prob>::v;
  }
  if (splits > 1 && !defer) {
    const size_t MN = (size_t)p.M * p.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((MN + 63) / 64)), dim3(256), 0, s, partial, splits,
                       p.M, p.N, e);
  }
  return splits;
}

template <class Prob, typename TC, bool SPLIT>
int launch_tile(Tile t, const Prob& p, Epi e, int splits, float* partial, hipStream_t s, bool defer) {
  switch (t) {
    case T128x128: return launch<Prob, TC, 128, 128, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T128x64: return launch<Prob, TC, 128, 64, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T64x128: return launch<Prob, TC, 64, 128, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T64x64: return launch<Prob, TC, 64, 64, 2, 2, SPLIT>(p, e, splits, partial, s, defer);
    case T128x32: return launch<Prob, TC, 128, 32, 4, 1, SPLIT>(p, e, splits, partial, s, defer);
    default: return launch<Prob, TC, 32, 128, 1, 4, SPLIT>(p, e, splits, partial, s, defer);
  }
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
}

// Times every (tile, split) candidate of one problem on stream s (output
// redirected to scratch, so accumulating epilogues are not disturbed; 2
// launches, or the better of two runs of 16 when those take under 0.2 ms) and
// returns the fastest; falls back to `dflt` when timing is not possible.
template <class Prob, typename TC, bool SPLIT>
std::pair<int, int> tune(const Prob& p, const Epi& e, long cap, float* partial, hipStream_t s,
                         std::pair<int, int> dflt, int min_split) {
  // rows of C written: up to the row of m = M-1 (the row map is monotone in m)
  size_t rows = (size_t)p.M;
  if (e.rq > 0) {
    const int m = p.M - 1, b = m / e.rq, q = m - b * e.rq, h = q / e.rwq, w = q - h * e.rwq;
    rows = (size_t)b * e.rs1 + (size_t)h * e.rs2 + (size_t)w * e.rs3 + e.r0 + 1;
  }
  float* scratch = nullptr;
  if (hipMalloc(&scratch, rows * (size_t)e.ldc * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    return dflt;
  }
  Epi et = e;
  et.C = scratch;
  et.accumulate = 0;
  hipEvent_t a = nullptr, b = nullptr;
  std::pair<int, int> best = dflt;
  float best_ms = 1e30f;
  if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
    const long kmax = std::max<long>(1, (long)cdiv(p.K, BK));
    for (int ti = 0; ti < kGemmTiles; ++ti) {
      const TileDim d = dim_of((Tile)ti);
      const long tiles = (long)cdiv(p.M, d.bm) * cdiv(p.N, d.bn);
      const int s0 = p.K > 0 ? splits_for(tiles, p.K) : 1;
      int cand[6] = {1, s0 / 2, s0, 2 * s0, 4 * s0, 8 * s0};
      int last = -1;
      for (int z : cand) {
        z = (int)std::min<long>({(long)std::max(z, min_split), cap, kmax, 256L});
        if (z < 1 || z == last) continue;
        last = z;
        launch_tile<Prob, TC, SPLIT>((Tile)ti, p, et, z, partial, s, false);
        hipEventRecord(a, s);
        for (int r = 0; r < 2; ++r) launch_tile<Prob, TC, SPLIT>((Tile)ti, p, et, z, partial, s, false);
        hipEventRecord(b, s);
        float ms = 0.f;
        if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) continue;
        if (ms < 0.2f) {  // short launches: the better of two runs of 16 (per 2 launches)
          float best16 = 1e30f;
          for (int rep = 0; rep < 2; ++rep) {
            hipEventRecord(a, s);
            for (int r = 0; r < 16; ++r) launch_tile<Prob, TC, SPLIT>((Tile)ti, p, et, z, partial, s, false);
            hipEventRecord(b, s);
            float m16 = 0.f;
            if (hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&m16, a, b) == hipSuccess)
              best16 = std::min(best16, m16);
          }
          if (best16 >= 1e30f) continue;
          ms = best16 / 8.f;
        }
        if (ms < best_ms) {
          best_ms = ms;
          best = {ti, z};
        }
      }
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(s);
  (void)hipFree(scratch);
  (void)hipGetLastError();
  return best;
}

// Returns the K split used; with defer and a split > 1 the partial tiles are
// left in `partial` ([splits][M][N]) for the caller to sum.
template <class Prob, typename TC, bool SPLIT>
int run(const Prob& p, Epi e, size_t partial_bytes, float* partial, hipStream_t s, int prec, bool defer = false) {
  if (p.M <= 0 || p.N <= 0) return 1;
  Tile t = choose(p.M, p.N, prec);
  const TileDim d = dim_of(t);
  const long tiles = (long)cdiv(p.M, d.bm) * cdiv(p.N, d.bn);
  int splits = p.K > 0 ? splits_for(tiles, p.K) : 1;
  const long cap = (long)(partial_bytes / (sizeof(float) * (size_t)p.M * p.N));
  if (splits > cap) splits = (int)std::max<long>(1, cap);
  // An act-step product (Epi::act, its partials summed by a GroupNorm) is split into
  // at least min(4, K/64) parts: in the act graph each product reads its
  // weights past a cold L2 right after its producer, where more workgroups
  // fetching a share each pay more than back-to-back timing shows (measured
  // on the whole act loop; the learner's products are better left as tuned).
  const bool act = e.act && defer;
  const int min_split = act ? (int)std::max<long>(1, std::min<long>({4L, (long)p.K / 64, cap})) : 1;
  splits = std::max(splits, min_split);
  GemmTune* tu = g_gemm_tune;
  if (tu) {
    // a deferred product (its partial tiles summed by the consumer) is tuned
    // on its own key, timed with the ordered reduction as the consumer's
    // stand-in; an act-step product on another
    const std::array<long long, 5> key{Prob::kKind, p.M, p.N, p.K,
                                       2 * prec + (int)SPLIT + 4 * (int)defer + 8 * (int)act};
    auto it = tu->best.find(key);
    if (it == tu->best.end() && tu->tuning && !capturing(s))
      it = tu->best
               .emplace(key, tune<Prob, TC, SPLIT>(p, e, std::max<long>(1, cap), partial, s, {(int)t, splits},
                                                   min_split))
               .first;
    if (it != tu->best.end()) {
      t = (Tile)it->second.first;
      splits = (int)std::max<long>(min_split, std::min<long>(it->second.second, std::max<long>(1, cap)));
    }
  }
  return launch_tile<Prob, TC, SPLIT>(t, p, e, splits, partial, s, defer);
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

// wt[ci][tap][co] = w[co][tap][ci]
template <typename T>
__global__ void __launch_bounds__(256) conv_w_transpose_kernel(const T* __restrict__ w, int Co, int KK, int C,
                                                                T* __restrict__ wt) {
  __shared__ T tile[32][33];
  const int c0 = blockIdx.x * 32, o0 = blockIdx.y * 32, tap = blockIdx.z;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8)
    if (o0 + y < Co && c0 + tx < C) tile[y][tx] = w[((size_t)(o0 + y) * KK + tap) * C + c0 + tx];
  __syncthreads();
  for (int y = ty; y < 32; y += 8)
    if (c0 + y < C && o0 + tx < Co) wt[((size_t)(c0 + y) * KK + tap) * Co + o0 + tx] = tile[tx][y];
}

// C rows of one parity class set to zero (a class no tap reaches, e.g. the
// odd pixels of a 1x1 stride-2 convolution).
__global__ void __launch_bounds__(256) zero_rows_kernel(Epi e, int M, int N) {
  const size_t MN = (size_t)M * N;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < MN; i += (size_t)gridDim.x * 256) {
    const int m = (int)(i / N), n = (int)(i - (size_t)m * N);
    e.C[crow(e, m) * e.ldc + n] = 0.f;
  }
}

void gemm_conv_dgrad(int prec, const ConvGeo& g, const float* dy, const void* w, void* wt, Epi e, size_t pb,
                     float* partial, hipStream_t s) {
  const int KK = g.KH * g.KW;
  const dim3 tg(cdiv(g.C, 32), cdiv(g.Co, 32), KK);
  if (prec == 1)
    hipLaunchKernelGGL(conv_w_transpose_kernel<bf16_t>, tg, dim3(256), 0, s, (const bf16_t*)w, g.Co, KK, g.C,
                       (bf16_t*)wt);
  else
    hipLaunchKernelGGL(conv_w_transpose_kernel<float>, tg, dim3(256), 0, s, (const float*)w, g.Co, KK, g.C,
                       (float*)wt);
  const int step = g.stride == 2 ? 2 : 1;
  for (int rh = 0; rh < step; ++rh)
    for (int rw = 0; rw < step; ++rw) {
      // taps with (pixel + pad - k) divisible by the stride
      const int kh0 = (rh + g.pad) % step, kw0 = (rw + g.pad) % step;
      const int nkh = kh0 < g.KH ? (g.KH - kh0 + step - 1) / step : 0;
      const int nkw = kw0 < g.KW ? (g.KW - kw0 + step - 1) / step : 0;
      const int Hq = (g.H - rh + step - 1) / step, Wq = (g.W - rw + step - 1) / step;
      const int M = g.B * Hq * Wq, N = g.C, K = nkh * nkw * g.Co;
      Epi ec = e;
      if (step == 2) {
        ec.rq = Hq * Wq;
        ec.rwq = Wq;
        ec.rs1 = g.H * g.W;
        ec.rs2 = 2 * g.W;
        ec.rs3 = 2;
        ec.r0 = rh * g.W + rw;
      }
      if (M <= 0) continue;
      if (K <= 0) {
        if (!e.accumulate)
          hipLaunchKernelGGL(zero_rows_kernel, dim3((unsigned)std::min<size_t>(4096, ((size_t)M * N + 255) / 256)),
                             dim3(256), 0, s, ec, M, N);
        continue;
      }
      const FastDiv dCo = fast_div(g.Co), dNkw = fast_div(nkw), dHqWq = fast_div(Hq * Wq), dWq = fast_div(Wq);
      if (prec == 1) {
        ConvDgradProb<bf16_t> p{g, dCo, dNkw, dHqWq, dWq, dy, (const bf16_t*)wt, M, N, K,
                                step, rh, rw, kh0, kw0, nkw, Wq};
        run_prec(p, ec, 1, true, pb, partial, s);
      } else {
        ConvDgradProb<float> p{g, dCo, dNkw, dHqWq, dWq, dy, (const float*)wt, M, N, K,
                               step, rh, rw, kh0, kw0, nkw, Wq};
        run_prec(p, ec, 0, false, pb, partial, s);
      }
    }
}

void gemm_conv_wgrad(int prec, const ConvGeo& g, const float* x, const float* dy, Epi e, size_t pb,
                     float* partial, hipStream_t s) {
  const int M = g.Co, N = g.KH * g.KW * g.C, K = g.B * g.Ho * g.Wo;
  // channel-vector chunks pay for their transposed LDS writes only where the
  // scalar gather is worst: fewer than 8 input channels per tap (the stem)
  if (g.Co % 8 == 0 && g.C % 8 != 0 && g.C % 4 == 0 && (((uintptr_t)x | (uintptr_t)dy) & 15) == 0) {
    ConvWgradRTProb p{g, fast_div(g.Ho * g.Wo), fast_div(g.Wo), x, dy, M, N, K};
    run_prec(p, e, prec, true, pb, partial, s);
    return;
  }
  ConvWgradProb p{g, fast_div(g.C), fast_div(g.KW), fast_div(g.Ho * g.Wo), fast_div(g.Wo), x, dy, M, N, K};
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
