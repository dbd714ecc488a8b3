// LDS-tiled MFMA GEMM core and its operand loaders (convolution forward,
// data gradient, weight gradient as implicit GEMMs; plain dense products).
//
// C[m][n] = alpha * sum_k A(m, k) B(n, k)  (+= C) (+ bias[n]) (ReLU)
//
// A workgroup of 256 threads (4 wavefronts) owns a BM x BN tile.  Operands
// are staged through double-buffered LDS as [rows][k] (k contiguous), one
// barrier per K tile; the next tile's global loads are in flight while the
// current tile feeds the matrix cores.  Every operand "chunk" is 8
// consecutive k of one row: for operands contiguous along k it is one or two
// vector loads, for operands contiguous along rows (transposed reads) the
// lanes of a wavefront walk the rows so each of the 8 scalar loads is
// coalesced; either way the chunk lands in LDS with one 16-byte write.
// Operands read as 8-row vectors at one k (RT: the stem's weight gradient)
// are staged two k at a time and stored as 8 row pairs (put8t2).
//
// bfloat16: v_mfma_f32_32x32x16_bf16 on 32x32 fragments.  float32: four
// v_mfma_f32_16x16x4_f32 per 16-k step on 16x16 fragments.  A and B use the
// same lane -> k assignment, so the order of k inside a step is irrelevant.
// SPLIT (bfloat16 only): A is carried as hi + lo bfloat16 parts (two MFMAs),
// giving the gradient operand of backward products a 16-bit mantissa.
// Accumulation is float32; a split over K writes partial tiles that a second
// kernel sums in a fixed order (no float atomics: results are deterministic).
#pragma once
#include "common.h"
#include "kernels.h"

typedef float v16f __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------- loads
DEV void zero8(float v[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = 0.f;
}

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

// ------------------------------------------------------------ problems
// Each problem exposes, for A (rows m) and B (rows n): a per-row state built
// once per thread (rowA / rowB) and a chunk loader (a8 / b8) returning the 8
// values at k .. k+7 (k a multiple of 8; entries past K are 0).

// Forward: A(m = (b,ho,wo), k = (kh,kw,ci)) = x[b][ho*s-p+kh][wo*s-p+kw][ci]; B(n = co, k) = w[co][k].
template <typename TW>
struct ConvFwdProb {
  static constexpr int kKind = 1;
  ConvGeo g;
  FastDiv dC, dKW, dHoWo, dWo;
  const float* x;
  const TW* w;
  int M, N, K;
  struct RA {
    int off, h0, w0, ok;
  };
  struct RB {
    const TW* p;
    int ok;
  };
  DEV RA rowA(int m) const {
    RA r{0, 0, 0, m < M};
    if (r.ok) {
      const int b = dHoWo.div(m), q = m - b * g.Ho * g.Wo;
      const int ho = dWo.div(q), wo = q - ho * g.Wo;
      r.off = b * g.H * g.W * g.C;
      r.h0 = ho * g.stride - g.pad;
      r.w0 = wo * g.stride - g.pad;
    }
    return r;
  }
  DEV RB rowB(int n) const { return RB{w + (size_t)n * K, n < N}; }
  DEV void a8(const RA& r, int k, float v[8]) const {
    if (!r.ok) return zero8(v);
    if ((g.C & 7) == 0) {
      if (k >= K) return zero8(v);
      const int tap = dC.div(k), ci = k - tap * g.C;
      const int kh = dKW.div(tap), kw = tap - kh * g.KW;
      const int hi = r.h0 + kh, wi = r.w0 + kw;
      if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W)
        return load8(x + r.off + ((size_t)hi * g.W + wi) * g.C + ci, v);
      return zero8(v);
    }
    if ((g.C & 3) == 0) {
      // two 4-channel quads (one or two taps), each one float4 load
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kk = k + 4 * h;
        float* o = v + 4 * h;
        o[0] = o[1] = o[2] = o[3] = 0.f;
        if (kk >= K) continue;
        const int tap = dC.div(kk), ci = kk - tap * g.C;
        const int kh = dKW.div(tap), kw = tap - kh * g.KW;
        const int hi = r.h0 + kh, wi = r.w0 + kw;
        if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W) {
          const float4 t = *(const float4*)(x + r.off + ((size_t)hi * g.W + wi) * g.C + ci);
          o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
        }
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k + e;
      float val = 0.f;
      if (kk < K) {
        const int tap = dC.div(kk), ci = kk - tap * g.C;
        const int kh = dKW.div(tap), kw = tap - kh * g.KW;
        const int hi = r.h0 + kh, wi = r.w0 + kw;
        if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W)
          val = x[r.off + ((size_t)hi * g.W + wi) * g.C + ci];
      }
      v[e] = val;
    }
  }
  DEV void b8(const RB& r, int k, float v[8]) const {
    if (!r.ok) return zero8(v);
    if (k + 8 <= K && aligned16(r.p + k)) return load8(r.p + k, v);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (k + e < K) ? ldf(r.p + k + e) : 0.f;
  }
};

// Data gradient over one class of input pixels: rows m = (b, hq, wq) are
// the pixels hi = step*hq + rh, wi = step*wq + rw (step 1: every pixel;
// step 2: one of the four parity classes of a stride-2 convolution), and k =
// (tap t of the class, co) with kh = kh0 + step*(t / nkw), kw = kw0 +
// step*(t % nkw), the only taps for which (hi + pad - kh) / stride is exact.
// A(m, k) = dy[b][(hi+pad-kh)/s][(wi+pad-kw)/s][co] (0 outside the output);
// B(n = ci, k) = wt[ci][kh*KW + kw][co] (weights reordered so B rows are
// contiguous along k).
template <typename TW>
struct ConvDgradProb {
  static constexpr int kKind = 2;
  ConvGeo g;
  FastDiv dCo, dNkw, dHqWq, dWq;
  const float* dy;
  const TW* wt;
  int M, N, K;  // M = B*Hq*Wq, N = C, K = nkh*nkw*Co
  int step, rh, rw, kh0, kw0, nkw, Wq;
  struct RA {
    int off, th, tw, ok;
  };
  struct RB {
    const TW* p;
    int ok;
  };
  DEV RA rowA(int m) const {
    RA r{0, 0, 0, m < M};
    if (r.ok) {
      const int b = dHqWq.div(m), q = m - b * (M / g.B);
      const int hq = dWq.div(q), wq = q - hq * Wq;
      r.off = b * g.Ho * g.Wo * g.Co;
      r.th = step * hq + rh + g.pad;
      r.tw = step * wq + rw + g.pad;
    }
    return r;
  }
  DEV RB rowB(int n) const { return RB{wt + (size_t)n * g.KH * g.KW * g.Co, n < N}; }
  // tap t -> (kh, kw) and the source output pixel; false outside the output
  DEV bool src(const RA& r, int t, int& tap, int& pix) const {
    const int ih = dNkw.div(t), iw = t - ih * nkw;
    const int kh = kh0 + step * ih, kw = kw0 + step * iw;
    tap = kh * g.KW + kw;
    const int th = r.th - kh, tw = r.tw - kw;
    if (th < 0 || tw < 0) return false;
    const int ho = g.stride == 2 ? th >> 1 : th, wo = g.stride == 2 ? tw >> 1 : tw;
    if (ho >= g.Ho || wo >= g.Wo) return false;
    pix = ho * g.Wo + wo;
    return true;
  }
  DEV void a8(const RA& r, int k, float v[8]) const {
    if (!r.ok || k >= K) return zero8(v);
    if ((g.Co & 7) == 0) {
      const int t = dCo.div(k), co = k - t * g.Co;
      int tap, pix;
      if (src(r, t, tap, pix)) return load8(dy + r.off + (size_t)pix * g.Co + co, v);
      return zero8(v);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k + e;
      float val = 0.f;
      if (kk < K) {
        const int t = dCo.div(kk), co = kk - t * g.Co;
        int tap, pix;
        if (src(r, t, tap, pix)) val = dy[r.off + (size_t)pix * g.Co + co];
      }
      v[e] = val;
    }
  }
  DEV void b8(const RB& r, int k, float v[8]) const {
    if (!r.ok || k >= K) return zero8(v);
    if ((g.Co & 7) == 0) {
      const int t = dCo.div(k), co = k - t * g.Co;
      const int ih = dNkw.div(t), iw = t - ih * nkw;
      const int tap = (kh0 + step * ih) * g.KW + kw0 + step * iw;
      const TW* p = r.p + (size_t)tap * g.Co + co;
      if (aligned16(p)) return load8(p, v);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = ldf(p + e);
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k + e;
      float val = 0.f;
      if (kk < K) {
        const int t = dCo.div(kk), co = kk - t * g.Co;
        const int ih = dNkw.div(t), iw = t - ih * nkw;
        val = ldf(r.p + (size_t)((kh0 + step * ih) * g.KW + kw0 + step * iw) * g.Co + co);
      }
      v[e] = val;
    }
  }
};

// Weight gradient: C(m = co, n = (kh,kw,ci)) = sum_r dy[r][co] * im2col(x)[r][n],
// r = (b,ho,wo) is the reduction.  Both operands are contiguous along their
// rows: lanes walk co (A) or n (B); 8 consecutive r per chunk.
struct ConvWgradProb {
  static constexpr int kKind = 3;
  ConvGeo g;
  FastDiv dC, dKW, dHoWo, dWo;
  const float* x;
  const float* dy;
  int M, N, K;  // M = Co, N = KH*KW*C, K = B*Ho*Wo
  struct RA {
    int co, ok;
  };
  struct RB {
    int kh, kw, ci, ok;
  };
  DEV RA rowA(int m) const { return RA{m, m < M}; }
  DEV RB rowB(int n) const {
    RB r{0, 0, 0, n < N};
    if (r.ok) {
      const int tap = dC.div(n);
      r.ci = n - tap * g.C;
      r.kh = dKW.div(tap);
      r.kw = tap - r.kh * g.KW;
    }
    return r;
  }
  DEV void a8(const RA& r, int k, float v[8]) const {
    if (!r.ok) return zero8(v);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (k + e < K) ? dy[(size_t)(k + e) * g.Co + r.co] : 0.f;
  }
  DEV void b8(const RB& r, int k, float v[8]) const {
    if (!r.ok || k >= K) return zero8(v);
    const int hw = g.Ho * g.Wo;
    int b = dHoWo.div(k);
    const int q = k - b * hw;
    int ho = dWo.div(q), wo = q - ho * g.Wo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float val = 0.f;
      if (k + e < K) {
        const int hi = ho * g.stride - g.pad + r.kh, wi = wo * g.stride - g.pad + r.kw;
        if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W)
          val = x[(((size_t)b * g.H + hi) * g.W + wi) * g.C + r.ci];
      }
      v[e] = val;
      if (++wo == g.Wo) {
        wo = 0;
        if (++ho == g.Ho) {
          ho = 0;
          ++b;
        }
      }
    }
  }
};

// Weight gradient with channel-vector chunks: a chunk is the 8 consecutive
// rows m..m+7 (output channels co for A, (kh,kw,ci) for B) at one reduction
// index r = (b,ho,wo), read as two float4 along the NHWC channel axis and
// written transposed into the k-contiguous LDS rows.  Needs Co % 8 == 0 and
// C % 4 == 0 (a B chunk spans one tap when C % 8 == 0, else two taps of 4).
struct ConvWgradRTProb {
  static constexpr int kKind = 4;
  ConvGeo g;
  FastDiv dHoWo, dWo;
  const float* x;
  const float* dy;
  int M, N, K;  // M = Co, N = KH*KW*C, K = B*Ho*Wo
  struct RA {
    int co, ok;
  };
  struct RB {
    int kh0, kw0, ci0, kh1, kw1, ci1, nv;  // taps of rows n..n+3 and n+4..n+7; valid rows
  };
  DEV RA rowA(int m) const { return RA{m, m < M}; }
  DEV RB rowB(int n) const {
    RB r{0, 0, 0, 0, 0, 0, max(0, min(8, N - n))};
    const int t0 = n / g.C, t1 = (n + 4) / g.C;
    r.ci0 = n - t0 * g.C;
    r.kh0 = t0 / g.KW;
    r.kw0 = t0 - r.kh0 * g.KW;
    r.ci1 = n + 4 - t1 * g.C;
    r.kh1 = t1 / g.KW;
    r.kw1 = t1 - r.kh1 * g.KW;
    return r;
  }
  DEV void a8(const RA& r, int k, float v[8]) const {
    if (!r.ok || k >= K) return zero8(v);
    load8(dy + (size_t)k * g.Co + r.co, v);
  }
  DEV void b8(const RB& r, int k, float v[8]) const {
    if (r.nv <= 0 || k >= K) return zero8(v);
    const int b = dHoWo.div(k), q = k - b * g.Ho * g.Wo;
    const int ho = dWo.div(q), wo = q - ho * g.Wo;
    const int hb = ho * g.stride - g.pad, wb = wo * g.stride - g.pad;
    const float* xb = x + (size_t)b * g.H * g.W * g.C;
    auto quad = [&](int kh, int kw, int ci, float* o) {
      const int hi = hb + kh, wi = wb + kw;
      if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W) {
        const float4 t = *(const float4*)(xb + ((size_t)hi * g.W + wi) * g.C + ci);
        o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
      } else {
        o[0] = o[1] = o[2] = o[3] = 0.f;
      }
    };
    quad(r.kh0, r.kw0, r.ci0, v);
    if (r.nv > 4) quad(r.kh1, r.kw1, r.ci1, v + 4);
    else v[4] = v[5] = v[6] = v[7] = 0.f;
    for (int e = r.nv; e < 4; ++e) v[e] = 0.f;
  }
};

// Dense: A(m, k) = a[m*lda + k] (or a[k*lda + m] when TA), B(n, k) = b[n*ldb + k]
// (or b[k*ldb + n] when TB).
template <typename TAe, typename TBe, bool TA, bool TB>
struct DenseProb {
  static constexpr int kKind = 8 + 4 * (int)(sizeof(TBe) == 2) + 2 * (int)TA + (int)TB;
  const TAe* a;
  const TBe* b;
  int lda, ldb;
  int M, N, K;
  struct RA {
    int m, ok;
  };
  typedef RA RB;
  DEV RA rowA(int m) const { return RA{m, m < M}; }
  DEV RB rowB(int n) const { return RB{n, n < N}; }
  template <typename T, bool TR>
  DEV static void get(const T* base, int ld, int row, int k, int K, float v[8]) {
    if (!TR) {
      const T* p = base + (size_t)row * ld + k;
      if (k + 8 <= K && aligned16(p)) return load8(p, v);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k + e < K) ? ldf(p + e) : 0.f;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = (k + e < K) ? ldf(base + (size_t)(k + e) * ld + row) : 0.f;
    }
  }
  DEV void a8(const RA& r, int k, float v[8]) const {
    if (!r.ok) return zero8(v);
    get<TAe, TA>(a, lda, r.m, k, K, v);
  }
  DEV void b8(const RB& r, int k, float v[8]) const {
    if (!r.ok) return zero8(v);
    get<TBe, TB>(b, ldb, r.m, k, K, v);
  }
};

// Bytes per element of a convolution's weight operand (the B rows of the
// forward product); 0 for other products (GEMM launch timer's byte count).
template <class P> struct WeightBytes { static constexpr int v = 0; };
template <typename TW> struct WeightBytes<ConvFwdProb<TW>> { static constexpr int v = (int)sizeof(TW); };

// Is the operand contiguous along rows (so lanes should walk rows)?  RT:
// chunks are 8 rows at one k (vector loads along rows, transposed LDS writes).
template <class P> struct Layout;
template <> struct Layout<ConvWgradRTProb> {
  static constexpr bool A_ROWS = false, B_ROWS = false, A_RT = true, B_RT = true;
};
template <typename TW> struct Layout<ConvFwdProb<TW>> {
  static constexpr bool A_ROWS = false, B_ROWS = false, A_RT = false, B_RT = false;
};
template <typename TW> struct Layout<ConvDgradProb<TW>> {
  static constexpr bool A_ROWS = false, B_ROWS = false, A_RT = false, B_RT = false;
};
template <> struct Layout<ConvWgradProb> {
  static constexpr bool A_ROWS = true, B_ROWS = true, A_RT = false, B_RT = false;
};
template <typename A_, typename B_, bool TA, bool TB>
struct Layout<DenseProb<A_, B_, TA, TB>> {
  static constexpr bool A_ROWS = TA, B_ROWS = TB, A_RT = false, B_RT = false;
};

// ------------------------------------------------------------- MFMA
template <typename TC>
struct Mma;
template <>
struct Mma<bf16_t> {  // v_mfma_f32_32x32x16_bf16
  static constexpr int FR = 32, NOUT = 16;
  typedef v16f Acc;
  DEV static int row(int l) { return l & 31; }
  DEV static int kof(int l) { return (l >> 5) * 8; }
  DEV static Acc zero() {
    Acc a;
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = 0.f;
    return a;
  }
  DEV static Acc mma(const bf16_t* a, const bf16_t* b, Acc c) {
    const v8bf x = *(const v8bf*)a, y = *(const v8bf*)b;
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
  }
  // accumulator element r of lane l
  DEV static int orow(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  DEV static int ocol(int l) { return l & 31; }
};
template <>
struct Mma<float> {  // 4 x v_mfma_f32_16x16x4_f32 per 16-k step
  static constexpr int FR = 16, NOUT = 4;
  typedef v4f Acc;
  DEV static int row(int l) { return l & 15; }
  DEV static int kof(int l) { return (l >> 4) * 4; }
  DEV static Acc zero() { return v4f{0.f, 0.f, 0.f, 0.f}; }
  DEV static Acc mma(const float* a, const float* b, Acc c) {
    const float4 x = *(const float4*)a, y = *(const float4*)b;
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, y.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, y.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, y.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, y.w, c, 0, 0, 0);
    return c;
  }
  DEV static int orow(int l, int r) { return 4 * (l >> 4) + r; }
  DEV static int ocol(int l) { return l & 15; }
};

// 8 floats -> LDS row segment in the operand type (hi part; lo = residual).
DEV void put8(float* d, const float v[8], float*) {
  *(float4*)d = make_float4(v[0], v[1], v[2], v[3]);
  *(float4*)(d + 4) = make_float4(v[4], v[5], v[6], v[7]);
}
// Two floats -> packed bfloat16 pair, round to nearest even (v_cvt_pk_bf16_f32).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
DEV uint32_t pk_bf16(float a, float b) {
  const bf16x2_t r = __builtin_convertvector((f32x2_t){a, b}, bf16x2_t);
  return __builtin_bit_cast(uint32_t, r);
}
DEV void put8(bf16_t* d, const float v[8], bf16_t* lo) {
  uint32_t h[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) h[i] = pk_bf16(v[2 * i], v[2 * i + 1]);
  *(uint4*)d = make_uint4(h[0], h[1], h[2], h[3]);
  if (lo) {
    uint32_t l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float a = __uint_as_float(h[i] << 16), b = __uint_as_float(h[i] & 0xffff0000u);
      l[i] = pk_bf16(v[2 * i] - a, v[2 * i + 1] - b);
    }
    *(uint4*)lo = make_uint4(l[0], l[1], l[2], l[3]);
  }
}

// Two chunks at k and k+1 -> columns k, k+1 of 8 consecutive LDS rows
// (stride ld elements; k even): one 64-bit (float pair) or 32-bit (bfloat16
// pair) store per row.  The lanes of a wavefront walk k, so each store
// instruction covers consecutive LDS words of a row: a column of 16-bit
// stores down the rows would put most lanes of a wavefront on a few banks.
DEV void put8t2(float* d, int ld, const float v0[8], const float v1[8], float*) {
#pragma unroll
  for (int e = 0; e < 8; ++e) *(float2*)(d + e * ld) = make_float2(v0[e], v1[e]);
}
DEV void put8t2(bf16_t* d, int ld, const float v0[8], const float v1[8], bf16_t* lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t h = pk_bf16(v0[e], v1[e]);
    *(uint32_t*)(d + e * ld) = h;
    if (lo) {
      const float a = __uint_as_float(h << 16), b = __uint_as_float(h & 0xffff0000u);
      *(uint32_t*)(lo + e * ld) = pk_bf16(v0[e] - a, v1[e] - b);
    }
  }
}

// ------------------------------------------------------------- kernel
template <class Prob, typename TC, int BM, int BN, int WGM, int WGN, bool SPLIT>
__global__ void __launch_bounds__(256) gemm_kernel(Prob p, Epi e, int tiles_n, int k_per_split) {
  using MM = Mma<TC>;
  constexpr int BK = 32;
  constexpr int FR = MM::FR;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / FR, FN = WTN / FR;
  static_assert(WGM * WGN == 4 && FM >= 1 && FN >= 1, "bad tile");
  constexpr int LDK = BK + 16 / (int)sizeof(TC);  // padded LDS row (elements)
  constexpr bool AR = Layout<Prob>::A_ROWS, BR = Layout<Prob>::B_ROWS;
  constexpr bool ART = Layout<Prob>::A_RT, BRT = Layout<Prob>::B_RT;
  // work units per K tile: a chunk (one row, 8 k), or for RT operands two
  // chunks (8 rows at k and k+1, stored by put8t2)
  constexpr int CA = ART ? (BM / 8) * (BK / 2) : BM * BK / 8, CB = BRT ? (BN / 8) * (BK / 2) : BN * BK / 8;
  constexpr int QA = (CA + 255) / 256, QB = (CB + 255) / 256;
  constexpr int VA = ART ? 2 : 1, VB = BRT ? 2 : 1;
  constexpr int NSPL = SPLIT ? 2 : 1;
  __shared__ __attribute__((aligned(16))) TC sA[NSPL][2][BM * LDK];
  __shared__ __attribute__((aligned(16))) TC sB[2][BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x - tm * tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = blockIdx.y * k_per_split;
  const int kend = min(p.K, kbeg + k_per_split);
  const int wm0 = (wave / WGN) * WTM, wn0 = (wave % WGN) * WTN;

  // unit c -> (row, k offset): lanes walk k for k-contiguous operands and
  // rows for row-contiguous ones
  // (RT: unit c -> first row 8*(c / (BK/2)) of an 8-row group and the k
  // pair 2*(c % (BK/2)): lanes walk the k pairs)
  auto a_row = [&](int c) { return ART ? (c / (BK / 2)) * 8 : AR ? c % BM : c / (BK / 8); };
  auto a_kc = [&](int c) { return ART ? (c % (BK / 2)) * 2 : AR ? (c / BM) * 8 : (c % (BK / 8)) * 8; };
  auto b_row = [&](int c) { return BRT ? (c / (BK / 2)) * 8 : BR ? c % BN : c / (BK / 8); };
  auto b_kc = [&](int c) { return BRT ? (c % (BK / 2)) * 2 : BR ? (c / BN) * 8 : (c % (BK / 8)) * 8; };

  typename Prob::RA ra[QA];
  typename Prob::RB rb[QB];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int c = tid + 256 * q;
    ra[q] = p.rowA(c < CA ? m0 + a_row(c) : 1 << 30);
  }
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int c = tid + 256 * q;
    rb[q] = p.rowB(c < CB ? n0 + b_row(c) : 1 << 30);
  }

  typename MM::Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = MM::zero();

  float va[QA][VA][8], vb[QB][VB][8];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int c = tid + 256 * q;
      const int k = k0 + a_kc(c);
#pragma unroll
      for (int h = 0; h < VA; ++h) {
        if (c < CA && k + h < kend) p.a8(ra[q], k + h, va[q][h]);
        else zero8(va[q][h]);
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int c = tid + 256 * q;
      const int k = k0 + b_kc(c);
#pragma unroll
      for (int h = 0; h < VB; ++h) {
        if (c < CB && k + h < kend) p.b8(rb[q], k + h, vb[q][h]);
        else zero8(vb[q][h]);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int c = tid + 256 * q;
      if (c < CA) {
        const int o = a_row(c) * LDK + a_kc(c);
        if constexpr (ART)
          put8t2(&sA[0][buf][o], LDK, va[q][0], va[q][VA - 1], SPLIT ? &sA[NSPL - 1][buf][o] : (TC*)nullptr);
        else
          put8(&sA[0][buf][o], va[q][0], SPLIT ? &sA[NSPL - 1][buf][o] : (TC*)nullptr);
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int c = tid + 256 * q;
      if (c < CB) {
        if constexpr (BRT)
          put8t2(&sB[buf][b_row(c) * LDK + b_kc(c)], LDK, vb[q][0], vb[q][VB - 1], (TC*)nullptr);
        else
          put8(&sB[buf][b_row(c) * LDK + b_kc(c)], vb[q][0], (TC*)nullptr);
      }
    }
  };

  const int ntiles = kbeg < kend ? (kend - kbeg + BK - 1) / BK : 0;
  if (ntiles > 0) {
    gload(kbeg);
    sstore(0);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
      const int cur = t & 1;
      if (t + 1 < ntiles) gload(kbeg + (t + 1) * BK);
#pragma unroll
      for (int ks = 0; ks < BK; ks += 16) {
        const int ko = ks + MM::kof(lane);
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const int ao = (wm0 + i * FR + MM::row(lane)) * LDK + ko;
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const TC* bp = &sB[cur][(wn0 + j * FR + MM::row(lane)) * LDK + ko];
            acc[i][j] = MM::mma(&sA[0][cur][ao], bp, acc[i][j]);
            if (SPLIT) acc[i][j] = MM::mma(&sA[NSPL - 1][cur][ao], bp, acc[i][j]);
          }
        }
      }
      if (t + 1 < ntiles) sstore(cur ^ 1);
      __syncthreads();
    }
  }

  if (e.gm_p > 0 && (e.partial || !e.gm_split_only)) {
    // group-major stores (plain values): the image and pixel of the fragment's
    // first row once, later rows step from it
    float* dst = e.partial ? e.partial + (size_t)blockIdx.y * p.M * p.N : e.C;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn0 + j * FR + MM::ocol(lane);
      if (n >= p.N) continue;
      const int g = n / e.gm_cg, cc = n - g * e.gm_cg, G = p.N / e.gm_cg;
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int mb = m0 + wm0 + i * FR;
        const int b0 = mb / e.gm_p, pb = mb - b0 * e.gm_p;
#pragma unroll
        for (int r = 0; r < MM::NOUT; ++r) {
          const int m = mb + MM::orow(lane, r);
          if (m < p.M) {
            int b = b0, px = pb + MM::orow(lane, r);
            if (px >= e.gm_p) {  // the fragment crosses into later images
              const int q = px / e.gm_p;
              b += q;
              px -= q * e.gm_p;
            }
            dst[(((size_t)b * G + g) * e.gm_p + px) * e.gm_cg + cc] = acc[i][j][r];
          }
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn0 + j * FR + MM::ocol(lane);
#pragma unroll
      for (int r = 0; r < MM::NOUT; ++r) {
        const int m = m0 + wm0 + i * FR + MM::orow(lane, r);
        if (m < p.M && n < p.N) {
          float v = acc[i][j][r];
          if (e.partial) {
            e.partial[((size_t)blockIdx.y * p.M + m) * p.N + n] = v;
          } else {
            v *= e.alpha;
            float* cp = e.C + crow(e, m) * e.ldc + n;
            if (e.accumulate) v += *cp;
            if (e.bias) v += e.bias[n];
            if (e.relu) v = fmaxf(v, 0.f);
            *cp = v;
          }
        }
      }
    }
}
