// LDS-tiled MFMA GEMM core and its operand loaders (convolution forward,
// data gradient, weight gradient as implicit GEMMs; plain dense products).
//
// C[m][n] = alpha * sum_k A(m, k) B(n, k)  (+ bias[n]) (ReLU) (+= C)
//
// A workgroup of 256 threads (4 wavefronts in a 2x2 grid) owns a BM x BN
// tile.  Each K step stages an A tile [BM][BK] and a B tile [BN][BK] in LDS
// (k contiguous, converted to the MFMA operand type), while the next tile's
// global loads are already in flight in registers.  Every lane reads 16
// bytes of k per 16-row fragment: one v_mfma_f32_16x16x32_bf16 (bfloat16) or
// four v_mfma_f32_16x16x4_f32 (float32) per fragment pair.  A and B use the
// same lane -> k assignment, so the order of k inside a step is irrelevant.
// Accumulation is float32; a split over K writes partial tiles that a second
// kernel sums in a fixed order (no float atomics: results are deterministic).
#pragma once
#include "common.h"
#include "kernels.h"

// ----------------------------------------------------------------- operands
// Loaders return 8 consecutive values along their contiguous axis:
//   KCONTIG: A(m, k..k+7) / B(n, k..k+7);  otherwise A(m..m+7, k) / B(n..n+7, k).
// Out-of-range entries are 0.

template <typename T>
DEV void load8(const T* p, float v[8]);
template <>
DEV void load8<float>(const float* p, float v[8]) {
  const float4 a = *(const float4*)p, b = *(const float4*)(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
template <>
DEV void load8<bf16_t>(const bf16_t* p, float v[8]) {
  const uint4 a = *(const uint4*)p;
  const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __uint_as_float(w[i] << 16);
    v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}

DEV bool aligned16(const void* p) { return (((uintptr_t)p) & 15) == 0; }

// Forward: A(m = (b,ho,wo), k = (kh,kw,ci)) = x[b][ho*s-p+kh][wo*s-p+kw][ci];
//          B(n = co, k) = w[co][k].
template <typename TW>
struct ConvFwdProb {
  static constexpr bool A_KCONTIG = true, B_KCONTIG = true;
  ConvGeo g;
  const float* x;
  const TW* w;
  int M, N, K;
  DEV void a8(int m, int k, float v[8]) const {
    if (m >= M) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0.f;
      return;
    }
    const int hw = g.Ho * g.Wo;
    const int b = m / hw, r = m - b * hw;
    const int ho = r / g.Wo, wo = r - ho * g.Wo;
    const int h0 = ho * g.stride - g.pad, w0 = wo * g.stride - g.pad;
    if ((g.C & 7) == 0 && k + 8 <= K) {
      const int tap = k / g.C, ci = k - tap * g.C;
      const int kh = tap / g.KW, kw = tap - kh * g.KW;
      const int hi = h0 + kh, wi = w0 + kw;
      if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W) {
        load8(x + (((size_t)b * g.H + hi) * g.W + wi) * g.C + ci, v);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.f;
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k + e;
      float val = 0.f;
      if (kk < K) {
        const int tap = kk / g.C, ci = kk - tap * g.C;
        const int kh = tap / g.KW, kw = tap - kh * g.KW;
        const int hi = h0 + kh, wi = w0 + kw;
        if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W)
          val = x[(((size_t)b * g.H + hi) * g.W + wi) * g.C + ci];
      }
      v[e] = val;
    }
  }
  DEV void b8(int n, int k, float v[8]) const {
    const TW* p = w + (size_t)n * K + k;
    if (n < N && k + 8 <= K && aligned16(p)) {
      load8(p, v);
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (n < N && k + e < K) ? ldf(p + e) : 0.f;
  }
};

// Data gradient: A(m = (b,hi,wi), k = (kh,kw,co)) = dy[b][(hi+p-kh)/s][(wi+p-kw)/s][co]
// when the division is exact and in range; B(n = ci, k) = w[co][kh][kw][ci]
// (contiguous along n).
template <typename TW>
struct ConvDgradProb {
  static constexpr bool A_KCONTIG = true, B_KCONTIG = false;
  ConvGeo g;
  const float* dy;
  const TW* w;
  int M, N, K;  // M = B*H*W, N = C, K = KH*KW*Co
  DEV void a8(int m, int k, float v[8]) const {
    if (m >= M) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0.f;
      return;
    }
    const int hw = g.H * g.W;
    const int b = m / hw, r = m - b * hw;
    const int hi = r / g.W, wi = r - hi * g.W;
    if ((g.Co & 7) == 0 && k + 8 <= K) {
      const int tap = k / g.Co, co = k - tap * g.Co;
      const int kh = tap / g.KW, kw = tap - kh * g.KW;
      const int th = hi + g.pad - kh, tw = wi + g.pad - kw;
      bool ok = th >= 0 && tw >= 0;
      int ho = 0, wo = 0;
      if (ok) {
        ho = th / g.stride;
        wo = tw / g.stride;
        ok = ho * g.stride == th && wo * g.stride == tw && ho < g.Ho && wo < g.Wo;
      }
      if (ok) {
        load8(dy + (((size_t)b * g.Ho + ho) * g.Wo + wo) * g.Co + co, v);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.f;
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k + e;
      float val = 0.f;
      if (kk < K) {
        const int tap = kk / g.Co, co = kk - tap * g.Co;
        const int kh = tap / g.KW, kw = tap - kh * g.KW;
        const int th = hi + g.pad - kh, tw = wi + g.pad - kw;
        if (th >= 0 && tw >= 0) {
          const int ho = th / g.stride, wo = tw / g.stride;
          if (ho * g.stride == th && wo * g.stride == tw && ho < g.Ho && wo < g.Wo)
            val = dy[(((size_t)b * g.Ho + ho) * g.Wo + wo) * g.Co + co];
        }
      }
      v[e] = val;
    }
  }
  DEV void b8(int n, int k, float v[8]) const {  // B(n..n+7, k)
    if (k >= K) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0.f;
      return;
    }
    const int tap = k / g.Co, co = k - tap * g.Co;
    const TW* p = w + ((size_t)co * g.KH * g.KW + tap) * g.C + n;
    if (n + 8 <= N && aligned16(p)) {
      load8(p, v);
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (n + e < N) ? ldf(p + e) : 0.f;
  }
};

// Weight gradient: C(m = co, n = (kh,kw,ci)) = sum_r dy[r][co] * im2col(x)[r][n],
// r = (b,ho,wo) runs over the reduction.  A(m..m+7, r) reads dy along co;
// B(n..n+7, r) reads the input along ci.
struct ConvWgradProb {
  static constexpr bool A_KCONTIG = false, B_KCONTIG = false;
  ConvGeo g;
  const float* x;
  const float* dy;
  int M, N, K;  // M = Co, N = KH*KW*C, K = B*Ho*Wo
  DEV void a8(int m, int r, float v[8]) const {
    const float* p = dy + (size_t)r * g.Co + m;
    if (r < K && m + 8 <= M && aligned16(p)) {
      load8(p, v);
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (r < K && m + e < M) ? p[e] : 0.f;
  }
  DEV void b8(int n, int r, float v[8]) const {
    if (r >= K) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = 0.f;
      return;
    }
    const int hw = g.Ho * g.Wo;
    const int b = r / hw, q = r - b * hw;
    const int ho = q / g.Wo, wo = q - ho * g.Wo;
    const int h0 = ho * g.stride - g.pad, w0 = wo * g.stride - g.pad;
    if ((g.C & 7) == 0 && n + 8 <= N) {
      const int tap = n / g.C, ci = n - tap * g.C;
      const int kh = tap / g.KW, kw = tap - kh * g.KW;
      const int hi = h0 + kh, wi = w0 + kw;
      if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W) {
        load8(x + (((size_t)b * g.H + hi) * g.W + wi) * g.C + ci, v);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = 0.f;
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int nn = n + e;
      float val = 0.f;
      if (nn < N) {
        const int tap = nn / g.C, ci = nn - tap * g.C;
        const int kh = tap / g.KW, kw = tap - kh * g.KW;
        const int hi = h0 + kh, wi = w0 + kw;
        if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W)
          val = x[(((size_t)b * g.H + hi) * g.W + wi) * g.C + ci];
      }
      v[e] = val;
    }
  }
};

// Dense: A(m, k) = a[m*lda + k] (or a[k*lda + m] when TA), B(n, k) = b[n*ldb + k]
// (or b[k*ldb + n] when TB).  Optional per-row scale of A (episode masks).
template <typename TAe, typename TBe, bool TA, bool TB>
struct DenseProb {
  static constexpr bool A_KCONTIG = !TA, B_KCONTIG = !TB;
  const TAe* a;
  const TBe* b;
  int lda, ldb;
  int M, N, K;
  DEV void a8(int m, int k, float v[8]) const {
    if (!TA) {
      const TAe* p = a + (size_t)m * lda + k;
      if (m < M && k + 8 <= K && aligned16(p)) {
        load8(p, v);
        return;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (m < M && k + e < K) ? ldf(p + e) : 0.f;
    } else {
      const TAe* p = a + (size_t)k * lda + m;
      if (k < K && m + 8 <= M && aligned16(p)) {
        load8(p, v);
        return;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k < K && m + e < M) ? ldf(p + e) : 0.f;
    }
  }
  DEV void b8(int n, int k, float v[8]) const {
    if (!TB) {
      const TBe* p = b + (size_t)n * ldb + k;
      if (n < N && k + 8 <= K && aligned16(p)) {
        load8(p, v);
        return;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (n < N && k + e < K) ? ldf(p + e) : 0.f;
    } else {
      const TBe* p = b + (size_t)k * ldb + n;
      if (k < K && n + 8 <= N && aligned16(p)) {
        load8(p, v);
        return;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k < K && n + e < N) ? ldf(p + e) : 0.f;
    }
  }
};

// ------------------------------------------------------------------ kernel
template <typename TC>
struct MmaT;
template <>
struct MmaT<float> {
  static constexpr int KS = 16;  // k per step: 4 lane groups x 4 floats
};
template <>
struct MmaT<bf16_t> {
  static constexpr int KS = 32;  // 4 lane groups x 8 bfloat16
};

DEV void to_lds(float* d, float v) { *d = v; }
DEV void to_lds(bf16_t* d, float v) { *d = f2bf(v); }

template <typename TC>
DEV v4f mma_step(const TC* a, const TC* b, v4f acc);
template <>
DEV v4f mma_step<float>(const float* a, const float* b, v4f acc) {
  const float4 x = *(const float4*)a, y = *(const float4*)b;
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.y, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, y.z, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, y.w, acc, 0, 0, 0);
  return acc;
}
template <>
DEV v4f mma_step<bf16_t>(const bf16_t* a, const bf16_t* b, v4f acc) {
  const v8bf x = *(const v8bf*)a, y = *(const v8bf*)b;
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc, 0, 0, 0);
}

template <class Prob, typename TC, int BM, int BN, int BK>
__global__ void __launch_bounds__(256) gemm_kernel(Prob p, Epi e, int tiles_n, int k_per_split) {
  constexpr int PAD = 16 / sizeof(TC);
  constexpr int LDK = BK + PAD;
  constexpr int KS = MmaT<TC>::KS;
  constexpr int WM = BM / 2, WN = BN / 2;  // wave tile
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int QA = BM * BK / 8 / 256, QB = BN * BK / 8 / 256;
  static_assert(QA >= 1 && QB >= 1, "tile too small for 256 threads");
  __shared__ __attribute__((aligned(16))) TC As[BM * LDK];
  __shared__ __attribute__((aligned(16))) TC Bs[BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = blockIdx.y * k_per_split;
  const int kend = min(p.K, kbeg + k_per_split);
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;

  v4f acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  float ra[QA][8], rb[QB][8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int c = tid + 256 * q;
      if (Prob::A_KCONTIG) {
        const int r = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        const int k = k0 + kc;
        if (k < kend) p.a8(m0 + r, k, ra[q]);
        else
#pragma unroll
          for (int x = 0; x < 8; ++x) ra[q][x] = 0.f;
        // entries past kend inside the chunk belong to the next split
        if (k + 8 > kend && k < kend)
#pragma unroll
          for (int x = 0; x < 8; ++x)
            if (k + x >= kend) ra[q][x] = 0.f;
      } else {
        const int kk = c / (BM / 8), mc = (c % (BM / 8)) * 8;
        if (k0 + kk < kend) p.a8(m0 + mc, k0 + kk, ra[q]);
        else
#pragma unroll
          for (int x = 0; x < 8; ++x) ra[q][x] = 0.f;
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int c = tid + 256 * q;
      if (Prob::B_KCONTIG) {
        const int r = c / (BK / 8), kc = (c % (BK / 8)) * 8;
        const int k = k0 + kc;
        if (k < kend) p.b8(n0 + r, k, rb[q]);
        else
#pragma unroll
          for (int x = 0; x < 8; ++x) rb[q][x] = 0.f;
        if (k + 8 > kend && k < kend)
#pragma unroll
          for (int x = 0; x < 8; ++x)
            if (k + x >= kend) rb[q][x] = 0.f;
      } else {
        const int kk = c / (BN / 8), nc = (c % (BN / 8)) * 8;
        if (k0 + kk < kend) p.b8(n0 + nc, k0 + kk, rb[q]);
        else
#pragma unroll
          for (int x = 0; x < 8; ++x) rb[q][x] = 0.f;
      }
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int c = tid + 256 * q;
      if (Prob::A_KCONTIG) {
        const int r = c / (BK / 8), kc = (c % (BK / 8)) * 8;
#pragma unroll
        for (int x = 0; x < 8; ++x) to_lds(&As[r * LDK + kc + x], ra[q][x]);
      } else {
        const int kk = c / (BM / 8), mc = (c % (BM / 8)) * 8;
#pragma unroll
        for (int x = 0; x < 8; ++x) to_lds(&As[(mc + x) * LDK + kk], ra[q][x]);
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int c = tid + 256 * q;
      if (Prob::B_KCONTIG) {
        const int r = c / (BK / 8), kc = (c % (BK / 8)) * 8;
#pragma unroll
        for (int x = 0; x < 8; ++x) to_lds(&Bs[r * LDK + kc + x], rb[q][x]);
      } else {
        const int kk = c / (BN / 8), nc = (c % (BN / 8)) * 8;
#pragma unroll
        for (int x = 0; x < 8; ++x) to_lds(&Bs[(nc + x) * LDK + kk], rb[q][x]);
      }
    }
  };

  if (kbeg < kend) {
    gload(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      __syncthreads();
      sstore();
      __syncthreads();
      if (k0 + BK < kend) gload(k0 + BK);
      const int kofs = (lane >> 4) * (KS / 4);
#pragma unroll
      for (int ks = 0; ks < BK; ks += KS) {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const TC* ap = &As[(wm0 + i * 16 + (lane & 15)) * LDK + ks + kofs];
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const TC* bp = &Bs[(wn0 + j * 16 + (lane & 15)) * LDK + ks + kofs];
            acc[i][j] = mma_step<TC>(ap, bp, acc[i][j]);
          }
        }
      }
    }
  }

  // epilogue: lane holds rows 4*(lane/16)+r, column lane%16 of each fragment
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn0 + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm0 + i * 16 + (lane >> 4) * 4 + r;
        if (m < p.M && n < p.N) {
          float v = acc[i][j][r];
          if (e.partial) {
            e.partial[((size_t)blockIdx.y * p.M + m) * p.N + n] = v;
          } else {
            v *= e.alpha;
            float* cp = e.C + (size_t)m * e.ldc + n;
            if (e.accumulate) v += *cp;
            if (e.bias) v += e.bias[n];
            if (e.relu) v = fmaxf(v, 0.f);
            *cp = v;
          }
        }
      }
    }
}

// Sum of split-K partials in split order, then the epilogue.
__global__ void __launch_bounds__(256) splitk_reduce_kernel(const float* __restrict__ part, int splits,
                                                            int M, int N, Epi e);
