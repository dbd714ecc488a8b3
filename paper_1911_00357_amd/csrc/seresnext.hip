// SE-ResNeXt blocks (App. "Agent Design", visual encoder; Xie et al.'s
// aggregated transform, Hu et al.'s squeeze-excite gate), NHWC float32
// activations:
//
//   grouped 3x3 convolution  input and output channels in G equal slices,
//                            output slice g convolves input slice g with its
//                            own filters [Co][3][3][C/G].  Its FLOPs are 1/G of
//                            a dense 3x3 and its per-group products (K = 9C/G,
//                            N = Co/G, as small as 36 x 4) would leave most of
//                            a matrix-core tile empty, so it is a direct
//                            vector-ALU convolution bound by the activation
//                            traffic: one workgroup per (pixel tile, group)
//                            with the group's filters staged in LDS.
//   squeeze-excite           z = per-channel pixel mean of the branch y,
//                            s = sigmoid(W2 relu(W1 z + b1) + b2), then
//                            out = relu(s * y + shortcut); the FCs are tiny
//                            (C x C/16 per frame) and run in float32 FMAs,
//                            spread over (frame, unit tile) workgroups.
//
// Precision: with bfloat16 weights every product operand of the convolution
// is rounded to bfloat16 (activation at load, weight as stored), as the
// matrix-core path does; gradients multiply the incoming float32 gradient
// with the rounded operand.  All reductions run in a fixed order
// (deterministic).
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kThreads = 256;

// nearest bfloat16 value (ties to even) by the hardware conversion
typedef __bf16 se_bf16x2 __attribute__((ext_vector_type(2)));
typedef float se_f32x2 __attribute__((ext_vector_type(2)));
DEV float rnd_bf16(float x) {
  const se_bf16x2 r = __builtin_convertvector((se_f32x2){x, 0.f}, se_bf16x2);
  return __uint_as_float(__builtin_bit_cast(uint32_t, r) << 16);
}

// A group's filters [og][9cg] (contiguous in w) into LDS as dst[perm(co, k)],
// with every thread's loads issued before its stores.
template <typename TW, typename Perm>
DEV void stage_filters(const TW* __restrict__ w, int n, float* dst, Perm perm) {
  constexpr int kU = 8;
  for (int e0 = threadIdx.x; e0 < n; e0 += kU * 256) {
    float v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * 256;
      v[u] = ldf(w + min(e, n - 1));
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * 256;
      if (e < n) dst[perm(e)] = v[u];
    }
  }
}

template <bool BF>
DEV float opnd(float x) {
  return BF ? rnd_bf16(x) : x;
}

DEV void ld4(const float* p, float* v) {
  const float4 t = *(const float4*)p;
  v[0] = t.x;
  v[1] = t.y;
  v[2] = t.z;
  v[3] = t.w;
}

// Index sizes are checked on the host to fit in 31 bits; quotients by
// runtime sizes use precomputed multiply-shift divisors.
struct PixDiv {
  FastDiv plane, row;  // pixels per image, pixels per row (of the indexed map)
};

// ---------------------------------------------------------------- forward
// Workgroup: `pix` consecutive output pixels of one group; thread t owns
// output channel t % og of pixel rows t / og + k (256 / og).  CG > 0: the
// group's input width as a compile-time constant, so the 9 taps' channel
// loads (float4, unconditional: an out-of-range tap reads the image origin
// and is zeroed) are all issued before the products.
template <typename TW, int CG>
__global__ void __launch_bounds__(kThreads) gconv_fwd_kernel(const float* __restrict__ x, const TW* __restrict__ w,
                                                            float* __restrict__ y, ConvGeo g, int G, int pix,
                                                            PixDiv dv) {
  extern __shared__ float ws[];  // [9][cg][og]
  constexpr bool BF = sizeof(TW) == 2;
  const int cg = CG > 0 ? CG : g.C / G, og = g.Co / G, grp = blockIdx.y;
  const int kw9 = 9 * cg;
  stage_filters(w + (size_t)grp * og * kw9, og * kw9, ws, [=](int e) {
    const int co = e / kw9, k = e - co * kw9;                 // w[grp*og + co][k] -> ws[k][co]
    return k * og + co;
  });
  __syncthreads();
  const int rows = kThreads / og, co = threadIdx.x % og, r0 = threadIdx.x / og;
  if (r0 >= rows) return;
  const int plane = g.Ho * g.Wo, P = g.B * plane;
  const int p0 = blockIdx.x * pix, pend = min(P, p0 + pix);
  for (int p = p0 + r0; p < pend; p += rows) {
    const int b = dv.plane.div(p), q = p - b * plane;
    const int ho = dv.row.div(q), wo = q - ho * g.Wo;
    const float* xb = x + (size_t)b * g.H * g.W * g.C + grp * cg;
    float acc = 0.f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int hi = ho * g.stride - g.pad + tap / 3, wi = wo * g.stride - g.pad + tap % 3;
      const bool ok = (unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W;
      const float* xp = xb + (ok ? ((size_t)hi * g.W + wi) * g.C : 0);
      const float* wp = ws + tap * cg * og + co;
      if (CG > 0) {
        float v[CG > 0 ? CG : 4];
#pragma unroll
        for (int c4 = 0; c4 < CG / 4; ++c4) ld4(xp + 4 * c4, v + 4 * c4);
#pragma unroll
        for (int ci = 0; ci < CG; ++ci) acc = fmaf(ok ? opnd<BF>(v[ci]) : 0.f, wp[ci * og], acc);
      } else {
        for (int c4 = 0; c4 < cg; c4 += 4) {
          float v[4];
          ld4(xp + c4, v);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc = fmaf(ok ? opnd<BF>(v[e]) : 0.f, wp[(c4 + e) * og], acc);
        }
      }
    }
    y[(size_t)p * g.Co + grp * og + co] = acc;
  }
}

// ----------------------------------------------------------- data gradient
// dx[b][hi][wi][grp*cg + ci] = sum over taps (kh, kw) whose output pixel
// ho = (hi + pad - kh) / stride is whole and in range, and over the group's
// output channels co, of dy[b][ho][wo][grp*og + co] * w[grp*og + co][kh][kw][ci].
// Stride 1 or 2.  OG > 0: the group's output width at compile time.
template <typename TW, int OG>
__global__ void __launch_bounds__(kThreads) gconv_dgrad_kernel(const float* __restrict__ dy,
                                                              const TW* __restrict__ w, float* __restrict__ dx,
                                                              ConvGeo g, int G, int pix, PixDiv dv,
                                                              int accumulate) {
  extern __shared__ float ws[];  // [9][og][cg]
  const int cg = g.C / G, og = OG > 0 ? OG : g.Co / G, grp = blockIdx.y;
  const int kw9 = 9 * cg;
  stage_filters(w + (size_t)grp * og * kw9, og * kw9, ws, [=](int e) {
    const int co = e / kw9, k = e - co * kw9, tap = k / cg, ci = k - tap * cg;
    return (tap * og + co) * cg + ci;                         // -> ws[tap][co][ci]
  });
  __syncthreads();
  const int rows = kThreads / cg, ci = threadIdx.x % cg, r0 = threadIdx.x / cg;
  if (r0 >= rows) return;
  const int plane = g.H * g.W, P = g.B * plane;
  const int sh = g.stride == 2 ? 1 : 0;
  const int p0 = blockIdx.x * pix, pend = min(P, p0 + pix);
  for (int p = p0 + r0; p < pend; p += rows) {
    const int b = dv.plane.div(p), q = p - b * plane;
    const int hi = dv.row.div(q), wi = q - hi * g.W;
    const float* db = dy + (size_t)b * g.Ho * g.Wo * g.Co + grp * og;
    float acc = 0.f;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int th = hi + g.pad - tap / 3, tw = wi + g.pad - tap % 3;
      const int ho = th >> sh, wo = tw >> sh;
      const bool ok = th >= 0 && tw >= 0 && ((th | tw) & sh) == 0 && ho < g.Ho && wo < g.Wo;
      const float* dp = db + (ok ? ((size_t)ho * g.Wo + wo) * g.Co : 0);
      const float* wp = ws + tap * og * cg + ci;
      if (OG > 0) {
        float v[OG > 0 ? OG : 4];
#pragma unroll
        for (int c4 = 0; c4 < OG / 4; ++c4) ld4(dp + 4 * c4, v + 4 * c4);
#pragma unroll
        for (int co = 0; co < OG; ++co) acc = fmaf(ok ? v[co] : 0.f, wp[co * cg], acc);
      } else {
        for (int c4 = 0; c4 < og; c4 += 4) {
          float v[4];
          ld4(dp + c4, v);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc = fmaf(ok ? v[e] : 0.f, wp[(c4 + e) * cg], acc);
        }
      }
    }
    float* o = dx + (size_t)p * g.C + grp * cg + ci;
    *o = accumulate ? *o + acc : acc;
  }
}

// --------------------------------------------------------- weight gradient
// Partial dw of one group over one chunk of output pixels:
//   part[chunk][(grp*og + co) * 9cg + k] = sum_{p in chunk} dy[p][grp*og + co] * xcol[p][k],
// xcol[p][(kh*3 + kw)*cg + ci] the (rounded) input under tap (kh, kw).
// Pixels are staged PT at a time in LDS (the group's dy columns, and its
// im2col rows copied as float4); thread t owns outputs t, t + 256, ... (at
// most kEPT).
constexpr int kEPT = 36;   // og * 9cg <= 256 * 36 (group widths up to 32)
constexpr int kLdsFloats = 10240;

struct WgradDiv {
  PixDiv pix;          // output map
  FastDiv og, k9c4, cg4;  // og; 9cg/4 float4 per im2col row; cg/4 float4 per tap
};

template <bool BF>
__global__ void __launch_bounds__(kThreads) gconv_wgrad_kernel(const float* __restrict__ x,
                                                              const float* __restrict__ dy,
                                                              float* __restrict__ part, ConvGeo g, int G, int pix,
                                                              int PT, WgradDiv dv) {
  extern __shared__ float sm[];  // dys [PT][og], xs [PT][9cg], coordinates [PT][3]
  const int cg = g.C / G, og = g.Co / G, grp = blockIdx.y;
  const int kw9 = 9 * cg, ne = og * kw9, k9c4 = kw9 / 4, cg4 = cg / 4;
  float* xs = sm;                      // 16-byte aligned: PT * 9cg floats
  float* dys = sm + PT * kw9;
  int* pc = (int*)(dys + PT * og);
  float acc[kEPT];
#pragma unroll
  for (int j = 0; j < kEPT; ++j) acc[j] = 0.f;
  const int plane = g.Ho * g.Wo, P = g.B * plane;
  const int p0 = blockIdx.x * pix, pend = min(P, p0 + pix);
  for (int pt = p0; pt < pend; pt += PT) {
    const int np = min(PT, pend - pt);
    __syncthreads();
    for (int i = threadIdx.x; i < PT; i += kThreads) {
      int b = -1, ho = 0, wo = 0;
      if (i < np) {
        const int p = pt + i;
        b = dv.pix.plane.div(p);
        const int q = p - b * plane;
        ho = dv.pix.row.div(q);
        wo = q - ho * g.Wo;
      }
      pc[3 * i] = b;
      pc[3 * i + 1] = ho * g.stride - g.pad;
      pc[3 * i + 2] = wo * g.stride - g.pad;
    }
    for (int e = threadIdx.x; e < PT * og; e += kThreads) {
      const int i = dv.og.div(e), co = e - i * og;
      dys[e] = i < np ? dy[(size_t)(pt + i) * g.Co + grp * og + co] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < PT * k9c4; e += kThreads) {
      const int i = dv.k9c4.div(e), r = e - i * k9c4;
      const int tap = dv.cg4.div(r), c4 = r - tap * cg4;
      const int b = pc[3 * i], hi = pc[3 * i + 1] + tap / 3, wi = pc[3 * i + 2] + tap % 3;
      const bool ok = b >= 0 && (unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (ok) {
        ld4(x + (((size_t)b * g.H + hi) * g.W + wi) * g.C + grp * cg + 4 * c4, v);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = opnd<BF>(v[q]);
      }
      *(float4*)(xs + i * kw9 + tap * cg + 4 * c4) = make_float4(v[0], v[1], v[2], v[3]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kEPT; ++j) {
      const int e = threadIdx.x + j * kThreads;
      if (e < ne) {
        const int co = e / kw9, k = e - co * kw9;
        float a = acc[j];
        for (int i = 0; i < np; ++i) a = fmaf(dys[i * og + co], xs[i * kw9 + k], a);
        acc[j] = a;
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * g.Co * kw9 + (size_t)grp * ne;
#pragma unroll
  for (int j = 0; j < kEPT; ++j) {
    const int e = threadIdx.x + j * kThreads;
    if (e < ne) out[e] = acc[j];
  }
}

// dst[i] = sum over chunks z (in order) of part[z][i]
__global__ void __launch_bounds__(kThreads) chunk_sum_kernel(const float* __restrict__ part, int chunks, int n,
                                                            float* __restrict__ dst) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    float s = 0.f;
    for (int z = 0; z < chunks; ++z) s += part[(size_t)z * n + i];
    dst[i] = s;
  }
}

// ---------------------------------------------------------- squeeze-excite
// Per-channel sums over a slice of the pixels (grid F x ceil(C/64) x S;
// thread (lane, row): channel lane, pixels row, row + 4, ... of slice z):
// zpart[z][f][c] = sum_{p in slice z} y[f][p][c].  The slices' sums are
// added in order by the kernel that consumes them.
__global__ void __launch_bounds__(kThreads) se_squeeze_kernel(const float* __restrict__ y, int HW, int C, int F,
                                                             int slice, float* __restrict__ zpart) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int f = blockIdx.x, c = blockIdx.y * 64 + lane, z = blockIdx.z;
  const int pend = min(HW, (z + 1) * slice);
  float s0 = 0.f, s1 = 0.f;
  if (c < C) {
    const float* yf = y + (size_t)f * HW * C + c;
    int p = z * slice + row;
    for (; p + 4 < pend; p += 8) {
      s0 += yf[(size_t)p * C];
      s1 += yf[(size_t)(p + 4) * C];
    }
    if (p < pend) s0 += yf[(size_t)p * C];
  }
  red[row][lane] = s0 + s1;
  __syncthreads();
  if (row == 0 && c < C)
    zpart[((size_t)z * F + f) * C + c] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Hidden layer of the gate, workgroup (f, y): z = (sum of the slices) / HW
// (workgroup y == 0 stores it), then a1 = W1 z + b1 for the 16 hidden units
// 16y .. 16y + 15, four per wavefront, each a lane-strided dot product over
// the channels with its loads unrolled.
__global__ void __launch_bounds__(kThreads) se_hidden_kernel(const float* __restrict__ zpart, int S, int F,
                                                            float inv_hw, int C, int R,
                                                            const float* __restrict__ w1,
                                                            const float* __restrict__ b1, float* __restrict__ z,
                                                            float* __restrict__ a1) {
  extern __shared__ float zs[];  // [C]
  const int f = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < C; c += kThreads) {
    float t = 0.f;
    for (int k = 0; k < S; ++k) t += zpart[((size_t)k * F + f) * C + c];
    t *= inv_hw;
    zs[c] = t;
    if (blockIdx.y == 0) z[(size_t)f * C + c] = t;
  }
  __syncthreads();
  const int jb = blockIdx.y * 16 + wv * 4;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  const float* wr[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wr[q] = w1 + (size_t)min(jb + q, R - 1) * C;
  for (int c = lane; c < C; c += 64) {
    const float zv = zs[c];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = fmaf(wr[q][c], zv, acc[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float v = wave_sum(acc[q]);
    if (lane == 0 && jb + q < R) a1[(size_t)f * R + jb + q] = v + b1[jb + q];
  }
}

// Gate, workgroup (f, y): s = sigmoid(W2 relu(a1) + b2) for channels
// 64y .. 64y + 63, four wavefronts each summing a quarter of the hidden
// units, added in a fixed order.
__global__ void __launch_bounds__(kThreads) se_gate_kernel(const float* __restrict__ a1, int C, int R,
                                                          const float* __restrict__ w2,
                                                          const float* __restrict__ b2, float* __restrict__ s) {
  extern __shared__ float sm[];  // hs [R], red [4][64]
  float* hs = sm;
  float* red = sm + R;
  const int f = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < R; j += kThreads) hs[j] = fmaxf(a1[(size_t)f * R + j], 0.f);
  __syncthreads();
  const int c = blockIdx.y * 64 + lane;
  const int q = (R + 3) / 4, j0 = wv * q, j1 = min(R, j0 + q);
  float acc = 0.f;
  if (c < C) {
    const float* wr = w2 + (size_t)c * R;
#pragma unroll 8
    for (int j = j0; j < j1; ++j) acc = fmaf(wr[j], hs[j], acc);
  }
  red[wv * 64 + lane] = acc;
  __syncthreads();
  if (wv == 0 && c < C)
    s[(size_t)f * C + c] = sigm(b2[c] + ((red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane])));
}

// out = relu(s[f][c] * y + res), four channels per thread (C % 4 == 0)
__global__ void __launch_bounds__(kThreads) se_excite_kernel(const float* __restrict__ y,
                                                            const float* __restrict__ s,
                                                            const float* __restrict__ res, int n4, FastDiv dhwc4,
                                                            FastDiv dc4, int C4, float* __restrict__ out) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n4; i += gridDim.x * kThreads) {
    const int f = dhwc4.div(i), c4 = i - dc4.div(i) * C4;
    const float4 yv = ((const float4*)y)[i], rv = ((const float4*)res)[i];
    const float4 sv = ((const float4*)s)[f * C4 + c4];
    ((float4*)out)[i] = make_float4(fmaxf(fmaf(sv.x, yv.x, rv.x), 0.f), fmaxf(fmaf(sv.y, yv.y, rv.y), 0.f),
                                    fmaxf(fmaf(sv.z, yv.z, rv.z), 0.f), fmaxf(fmaf(sv.w, yv.w, rv.w), 0.f));
  }
}

// Backward, first pass (grid F x ceil(C/64) x S): dpre = dout * [out > 0]
// into dres (the shortcut's gradient) and dspart[z][f][c] = sum over slice z
// of dpre * y.
__global__ void __launch_bounds__(kThreads) se_bwd_reduce_kernel(const float* __restrict__ dout,
                                                                const float* __restrict__ out,
                                                                const float* __restrict__ y, int HW, int C, int F,
                                                                int slice, float* __restrict__ dres,
                                                                float* __restrict__ dspart) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int f = blockIdx.x, c = blockIdx.y * 64 + lane, z = blockIdx.z;
  const int pend = min(HW, (z + 1) * slice);
  float acc = 0.f;
  if (c < C) {
    const size_t base = (size_t)f * HW * C + c;
    for (int p = z * slice + row; p < pend; p += 4) {
      const size_t i = base + (size_t)p * C;
      const float o = out[i], g = dout[i], yv = y[i];
      const float d = o > 0.f ? g : 0.f;
      dres[i] = d;
      acc = fmaf(d, yv, acc);
    }
  }
  red[row][lane] = acc;
  __syncthreads();
  if (row == 0 && c < C)
    dspart[((size_t)z * F + f) * C + c] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Backward through the gate, one workgroup per frame:
//   ds = sum of the slices;  da2 = ds * s (1 - s);  da1 = (W2^T da2) * [a1 > 0];  dz = W1^T da1.
__global__ void __launch_bounds__(kThreads) se_fc_bwd_kernel(const float* __restrict__ dspart, int S, int F,
                                                            const float* __restrict__ s,
                                                            const float* __restrict__ a1, int C, int R,
                                                            const float* __restrict__ w1,
                                                            const float* __restrict__ w2, float* __restrict__ da2,
                                                            float* __restrict__ da1, float* __restrict__ dz) {
  extern __shared__ float sm[];  // d2 [C], d1 [R]
  float* d2 = sm;
  float* d1 = sm + C;
  const int f = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < C; c += kThreads) {
    float ds = 0.f;
    for (int k = 0; k < S; ++k) ds += dspart[((size_t)k * F + f) * C + c];
    const float sv = s[(size_t)f * C + c];
    const float v = ds * sv * (1.f - sv);
    d2[c] = v;
    da2[(size_t)f * C + c] = v;
  }
  __syncthreads();
  for (int j = wv; j < R; j += kThreads / 64) {
    float acc = 0.f;
    for (int c = lane; c < C; c += 64) acc = fmaf(w2[(size_t)c * R + j], d2[c], acc);
    acc = wave_sum(acc);
    if (lane == 0) {
      const float v = a1[(size_t)f * R + j] > 0.f ? acc : 0.f;
      d1[j] = v;
      da1[(size_t)f * R + j] = v;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += kThreads) {
    float acc = 0.f;
    for (int j = 0; j < R; ++j) acc = fmaf(w1[(size_t)j * C + c], d1[j], acc);
    dz[(size_t)f * C + c] = acc;
  }
}

// Gate weight gradients, one thread per element, frames summed in order:
//   dW1[j][c] = sum_f da1[f][j] z[f][c],  db1[j] = sum_f da1[f][j],
//   dW2[c][j] = sum_f da2[f][c] relu(a1[f][j]),  db2[c] = sum_f da2[f][c].
__global__ void __launch_bounds__(kThreads) se_fc_wgrad_kernel(const float* __restrict__ z,
                                                              const float* __restrict__ a1,
                                                              const float* __restrict__ da1,
                                                              const float* __restrict__ da2, int F, int C, int R,
                                                              float* __restrict__ gw1, float* __restrict__ gb1,
                                                              float* __restrict__ gw2, float* __restrict__ gb2) {
  const int n1 = R * C, n2 = n1 + R, n3 = n2 + C * R, n4 = n3 + C;
  for (int e = blockIdx.x * kThreads + threadIdx.x; e < n4; e += gridDim.x * kThreads) {
    float acc = 0.f;
    if (e < n1) {
      const int j = e / C, c = e - j * C;
      for (int f = 0; f < F; ++f) acc = fmaf(da1[(size_t)f * R + j], z[(size_t)f * C + c], acc);
      gw1[e] = acc;
    } else if (e < n2) {
      const int j = e - n1;
      for (int f = 0; f < F; ++f) acc += da1[(size_t)f * R + j];
      gb1[j] = acc;
    } else if (e < n3) {
      const int q = e - n2, c = q / R, j = q - c * R;
      for (int f = 0; f < F; ++f) acc = fmaf(da2[(size_t)f * C + c], fmaxf(a1[(size_t)f * R + j], 0.f), acc);
      gw2[q] = acc;
    } else {
      const int c = e - n3;
      for (int f = 0; f < F; ++f) acc += da2[(size_t)f * C + c];
      gb2[c] = acc;
    }
  }
}

// dy = s[f][c] * dpre + dz[f][c] / HW  (the gradient at the branch y), four channels per thread
__global__ void __launch_bounds__(kThreads) se_excite_bwd_kernel(const float* __restrict__ dpre,
                                                                const float* __restrict__ s,
                                                                const float* __restrict__ dz, int n4,
                                                                FastDiv dhwc4, FastDiv dc4, int C4, float inv_hw,
                                                                float* __restrict__ dy) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n4; i += gridDim.x * kThreads) {
    const int f = dhwc4.div(i), c4 = i - dc4.div(i) * C4;
    const float4 d = ((const float4*)dpre)[i];
    const float4 sv = ((const float4*)s)[f * C4 + c4], zv = ((const float4*)dz)[f * C4 + c4];
    ((float4*)dy)[i] = make_float4(fmaf(sv.x, d.x, zv.x * inv_hw), fmaf(sv.y, d.y, zv.y * inv_hw),
                                   fmaf(sv.z, d.z, zv.z * inv_hw), fmaf(sv.w, d.w, zv.w * inv_hw));
  }
}

unsigned grid_for(long n) { return (unsigned)std::max<long>(1, std::min<long>(cdiv(n, kThreads), 8192)); }

// Output pixels per workgroup: about 2048 workgroups in all, at most 16
// passes of the workgroup's rows.
int pix_per_block(long P, int rows, int G) {
  const long per_group = std::max<long>(1, 2048 / G);
  long pix = (P + per_group - 1) / per_group;
  pix = std::max<long>(rows, std::min<long>(pix, (long)rows * 16));
  return (int)((pix + rows - 1) / rows * rows);
}

// Pixel slices of the squeeze reductions: about 512 workgroups, slices of
// at least 16 pixels, at most kMaxSlices.
int se_slices(int F, int HW, int C) {
  const int base = F * cdiv(C, 64);
  int S = std::max(1, 512 / std::max(base, 1));
  S = std::min(S, std::max(1, HW / 16));
  return std::min(S, kSeMaxSlices);
}

template <typename TW>
void gconv_fwd_dispatch(int cg, dim3 grid, size_t sh, hipStream_t s, const float* x, const TW* w, float* y,
                        const ConvGeo& g, int G, int pix, PixDiv dv) {
  switch (cg) {
    case 4: hipLaunchKernelGGL((gconv_fwd_kernel<TW, 4>), grid, dim3(kThreads), sh, s, x, w, y, g, G, pix, dv); break;
    case 8: hipLaunchKernelGGL((gconv_fwd_kernel<TW, 8>), grid, dim3(kThreads), sh, s, x, w, y, g, G, pix, dv); break;
    case 16: hipLaunchKernelGGL((gconv_fwd_kernel<TW, 16>), grid, dim3(kThreads), sh, s, x, w, y, g, G, pix, dv); break;
    case 32: hipLaunchKernelGGL((gconv_fwd_kernel<TW, 32>), grid, dim3(kThreads), sh, s, x, w, y, g, G, pix, dv); break;
    default: hipLaunchKernelGGL((gconv_fwd_kernel<TW, 0>), grid, dim3(kThreads), sh, s, x, w, y, g, G, pix, dv);
  }
}

template <typename TW>
void gconv_dgrad_dispatch(int og, dim3 grid, size_t sh, hipStream_t s, const float* dy, const TW* w, float* dx,
                          const ConvGeo& g, int G, int pix, PixDiv dv, int acc) {
  switch (og) {
    case 4: hipLaunchKernelGGL((gconv_dgrad_kernel<TW, 4>), grid, dim3(kThreads), sh, s, dy, w, dx, g, G, pix, dv, acc); break;
    case 8: hipLaunchKernelGGL((gconv_dgrad_kernel<TW, 8>), grid, dim3(kThreads), sh, s, dy, w, dx, g, G, pix, dv, acc); break;
    case 16: hipLaunchKernelGGL((gconv_dgrad_kernel<TW, 16>), grid, dim3(kThreads), sh, s, dy, w, dx, g, G, pix, dv, acc); break;
    case 32: hipLaunchKernelGGL((gconv_dgrad_kernel<TW, 32>), grid, dim3(kThreads), sh, s, dy, w, dx, g, G, pix, dv, acc); break;
    default: hipLaunchKernelGGL((gconv_dgrad_kernel<TW, 0>), grid, dim3(kThreads), sh, s, dy, w, dx, g, G, pix, dv, acc);
  }
}

}  // namespace

bool gconv_supported(const ConvGeo& g, int G) {
  if (G <= 0 || g.C % G || g.Co % G || g.KH != 3 || g.KW != 3 || g.pad != 1) return false;
  if (g.stride != 1 && g.stride != 2) return false;
  const int cg = g.C / G, og = g.Co / G;
  // float4 channel loads; one output channel (input channel for the data
  // gradient) per thread of a row; every weight-gradient element among a
  // thread's kEPT; filters of a group within the LDS budget
  if (cg % 4 || og % 4 || cg > kThreads || og > kThreads || og * 9 * cg > kThreads * kEPT) return false;
  if ((size_t)9 * cg * og > (size_t)kLdsFloats || og + 9 * cg > kLdsFloats / 8) return false;
  // 31-bit indices (checked per call for the pixel counts)
  return true;
}

bool gconv_fits(const ConvGeo& g) {
  return (long)g.B * g.H * g.W * g.C < (1L << 31) && (long)g.B * g.Ho * g.Wo * g.Co < (1L << 31);
}

void launch_gconv_fwd(int prec, const ConvGeo& g, int G, const float* x, const void* w, float* y,
                      hipStream_t s) {
  const int cg = g.C / G, og = g.Co / G, rows = kThreads / og;
  const long P = (long)g.B * g.Ho * g.Wo;
  const int pix = pix_per_block(P, rows, G);
  const dim3 grid((unsigned)cdiv(P, pix), (unsigned)G);
  const size_t sh = (size_t)9 * cg * og * sizeof(float);
  const PixDiv dv{fast_div(g.Ho * g.Wo), fast_div(g.Wo)};
  if (prec == 1) gconv_fwd_dispatch<bf16_t>(cg, grid, sh, s, x, (const bf16_t*)w, y, g, G, pix, dv);
  else gconv_fwd_dispatch<float>(cg, grid, sh, s, x, (const float*)w, y, g, G, pix, dv);
}

void launch_gconv_dgrad(int prec, const ConvGeo& g, int G, const float* dy, const void* w, float* dx,
                        int accumulate, hipStream_t s) {
  const int cg = g.C / G, og = g.Co / G, rows = kThreads / cg;
  const long P = (long)g.B * g.H * g.W;
  const int pix = pix_per_block(P, rows, G);
  const dim3 grid((unsigned)cdiv(P, pix), (unsigned)G);
  const size_t sh = (size_t)9 * cg * og * sizeof(float);
  const PixDiv dv{fast_div(g.H * g.W), fast_div(g.W)};
  if (prec == 1) gconv_dgrad_dispatch<bf16_t>(og, grid, sh, s, dy, (const bf16_t*)w, dx, g, G, pix, dv, accumulate);
  else gconv_dgrad_dispatch<float>(og, grid, sh, s, dy, (const float*)w, dx, g, G, pix, dv, accumulate);
}

void launch_gconv_wgrad(int prec, const ConvGeo& g, int G, const float* x, const float* dy, float* dw,
                        float* part, size_t part_bytes, hipStream_t s) {
  const int cg = g.C / G, og = g.Co / G;
  const long n = (long)g.Co * 9 * cg;
  const long P = (long)g.B * g.Ho * g.Wo;
  // pixels staged per round: the LDS budget over one pixel's dy columns and im2col row
  const int PT = std::max(8, std::min(256, kLdsFloats / (og + 9 * cg)) / 8 * 8);
  const long cap = std::max<long>(1, (long)(part_bytes / ((size_t)n * sizeof(float))));
  // chunks of at least 256 pixels, about 4096 workgroups, within the partial buffer
  long chunks = std::min<long>(std::max<long>(1, 4096 / G), std::max<long>(1, P / 256));
  chunks = std::max<long>(1, std::min(chunks, cap));
  long pix = (P + chunks - 1) / chunks;
  pix = (pix + PT - 1) / PT * PT;
  chunks = (P + pix - 1) / pix;
  const size_t sh = (size_t)PT * (og + 9 * cg) * sizeof(float) + (size_t)PT * 3 * sizeof(int);
  const dim3 grid((unsigned)chunks, (unsigned)G);
  const WgradDiv dv{{fast_div(g.Ho * g.Wo), fast_div(g.Wo)}, fast_div(og), fast_div(9 * cg / 4), fast_div(cg / 4)};
  if (prec == 1)
    hipLaunchKernelGGL(gconv_wgrad_kernel<true>, grid, dim3(kThreads), sh, s, x, dy, part, g, G, (int)pix, PT, dv);
  else
    hipLaunchKernelGGL(gconv_wgrad_kernel<false>, grid, dim3(kThreads), sh, s, x, dy, part, g, G, (int)pix, PT, dv);
  hipLaunchKernelGGL(chunk_sum_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, part, (int)chunks, (int)n, dw);
}

void launch_se_forward(const float* y, const float* res, int F, int HW, int C, int R, const float* w1,
                       const float* b1, const float* w2, const float* b2, float* zpart, float* z, float* a1,
                       float* gate, float* out, hipStream_t s) {
  const int S = se_slices(F, HW, C), slice = cdiv(HW, S);
  hipLaunchKernelGGL(se_squeeze_kernel, dim3(F, cdiv(C, 64), S), dim3(kThreads), 0, s, y, HW, C, F, slice, zpart);
  hipLaunchKernelGGL(se_hidden_kernel, dim3(F, cdiv(R, 16)), dim3(kThreads), (size_t)C * sizeof(float), s, zpart,
                     S, F, 1.f / HW, C, R, w1, b1, z, a1);
  hipLaunchKernelGGL(se_gate_kernel, dim3(F, cdiv(C, 64)), dim3(kThreads), (size_t)(R + 256) * sizeof(float), s, a1,
                     C, R, w2, b2, gate);
  const int n4 = F * HW * C / 4;
  hipLaunchKernelGGL(se_excite_kernel, dim3(grid_for(n4)), dim3(kThreads), 0, s, y, gate, res, n4,
                     fast_div(HW * C / 4), fast_div(C / 4), C / 4, out);
}

void launch_se_backward(const float* dout, const float* out, const float* y, const float* z, const float* a1,
                        const float* gate, int F, int HW, int C, int R, const float* w1, const float* w2,
                        float* dres, float* dspart, float* da2, float* da1, float* dz, float* gw1, float* gb1,
                        float* gw2, float* gb2, float* dy, hipStream_t s) {
  const int S = se_slices(F, HW, C), slice = cdiv(HW, S);
  hipLaunchKernelGGL(se_bwd_reduce_kernel, dim3(F, cdiv(C, 64), S), dim3(kThreads), 0, s, dout, out, y, HW, C, F,
                     slice, dres, dspart);
  hipLaunchKernelGGL(se_fc_bwd_kernel, dim3(F), dim3(kThreads), (size_t)(C + R) * sizeof(float), s, dspart, S, F,
                     gate, a1, C, R, w1, w2, da2, da1, dz);
  const long nw = 2L * R * C + R + C;
  hipLaunchKernelGGL(se_fc_wgrad_kernel, dim3(grid_for(nw)), dim3(kThreads), 0, s, z, a1, da1, da2, F, C, R, gw1,
                     gb1, gw2, gb2);
  const int n4 = F * HW * C / 4;
  hipLaunchKernelGGL(se_excite_bwd_kernel, dim3(grid_for(n4)), dim3(kThreads), 0, s, dres, gate, dz, n4,
                     fast_div(HW * C / 4), fast_div(C / 4), C / 4, 1.f / HW, dy);
}
