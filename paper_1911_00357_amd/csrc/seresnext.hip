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
//                            (C x C/16 per frame) and run in float32 FMAs.
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

DEV float rnd_bf16(float x) { return bf2f(f2bf(x)); }

template <bool BF>
DEV float opnd(float x) {
  return BF ? rnd_bf16(x) : x;
}

// ---------------------------------------------------------------- forward
// Workgroup: `pix` consecutive output pixels of one group; thread t owns
// output channel t % og of pixel rows t / og + k * (256 / og).
template <typename TW>
__global__ void __launch_bounds__(kThreads) gconv_fwd_kernel(const float* __restrict__ x, const TW* __restrict__ w,
                                                            float* __restrict__ y, ConvGeo g, int G, int pix) {
  extern __shared__ float ws[];  // [9][cg][og]
  constexpr bool BF = sizeof(TW) == 2;
  const int cg = g.C / G, og = g.Co / G, grp = blockIdx.y;
  const int kw9 = 9 * cg;
  for (int e = threadIdx.x; e < og * kw9; e += kThreads) {
    const int co = e / kw9, k = e - co * kw9;                 // w[grp*og + co][k]
    ws[k * og + co] = ldf(w + (size_t)(grp * og + co) * kw9 + k);
  }
  __syncthreads();
  const int rows = kThreads / og, co = threadIdx.x % og, r0 = threadIdx.x / og;
  if (r0 >= rows) return;
  const long P = (long)g.B * g.Ho * g.Wo;
  const long p0 = (long)blockIdx.x * pix;
  const long pend = min(P, p0 + pix);
  for (long p = p0 + r0; p < pend; p += rows) {
    const int b = (int)(p / ((long)g.Ho * g.Wo));
    const int q = (int)(p - (long)b * g.Ho * g.Wo);
    const int ho = q / g.Wo, wo = q - ho * g.Wo;
    const float* xb = x + (size_t)b * g.H * g.W * g.C + grp * cg;
    float acc = 0.f;
    for (int kh = 0; kh < 3; ++kh) {
      const int hi = ho * g.stride - g.pad + kh;
      if ((unsigned)hi >= (unsigned)g.H) continue;
      for (int kw = 0; kw < 3; ++kw) {
        const int wi = wo * g.stride - g.pad + kw;
        if ((unsigned)wi >= (unsigned)g.W) continue;
        const float* xp = xb + ((size_t)hi * g.W + wi) * g.C;
        const float* wp = ws + (kh * 3 + kw) * cg * og + co;
        for (int ci = 0; ci < cg; ++ci) acc = fmaf(opnd<BF>(xp[ci]), wp[ci * og], acc);
      }
    }
    y[(size_t)p * g.Co + grp * og + co] = acc;
  }
}

// ----------------------------------------------------------- data gradient
// dx[b][hi][wi][grp*cg + ci] = sum over taps (kh, kw) whose output pixel
// ho = (hi + pad - kh) / stride is whole and in range, and over the group's
// output channels co, of dy[b][ho][wo][grp*og + co] * w[grp*og + co][kh][kw][ci].
template <typename TW>
__global__ void __launch_bounds__(kThreads) gconv_dgrad_kernel(const float* __restrict__ dy,
                                                              const TW* __restrict__ w, float* __restrict__ dx,
                                                              ConvGeo g, int G, int pix, int accumulate) {
  extern __shared__ float ws[];  // [9][og][cg]
  const int cg = g.C / G, og = g.Co / G, grp = blockIdx.y;
  const int kw9 = 9 * cg;
  for (int e = threadIdx.x; e < og * kw9; e += kThreads) {
    const int co = e / kw9, k = e - co * kw9, tap = k / cg, ci = k - tap * cg;
    ws[(tap * og + co) * cg + ci] = ldf(w + (size_t)(grp * og + co) * kw9 + k);
  }
  __syncthreads();
  const int rows = kThreads / cg, ci = threadIdx.x % cg, r0 = threadIdx.x / cg;
  if (r0 >= rows) return;
  const long P = (long)g.B * g.H * g.W;
  const long p0 = (long)blockIdx.x * pix;
  const long pend = min(P, p0 + pix);
  for (long p = p0 + r0; p < pend; p += rows) {
    const int b = (int)(p / ((long)g.H * g.W));
    const int q = (int)(p - (long)b * g.H * g.W);
    const int hi = q / g.W, wi = q - hi * g.W;
    const float* db = dy + (size_t)b * g.Ho * g.Wo * g.Co + grp * og;
    float acc = 0.f;
    for (int kh = 0; kh < 3; ++kh) {
      const int th = hi + g.pad - kh;
      if (th < 0 || th % g.stride) continue;
      const int ho = th / g.stride;
      if (ho >= g.Ho) continue;
      for (int kw = 0; kw < 3; ++kw) {
        const int tw = wi + g.pad - kw;
        if (tw < 0 || tw % g.stride) continue;
        const int wo = tw / g.stride;
        if (wo >= g.Wo) continue;
        const float* dp = db + ((size_t)ho * g.Wo + wo) * g.Co;
        const float* wp = ws + (kh * 3 + kw) * og * cg + ci;
        for (int co = 0; co < og; ++co) acc = fmaf(dp[co], wp[co * cg], acc);
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
// Pixels are staged kPT at a time in LDS (dy columns of the group and the
// group's im2col rows); thread t owns outputs t, t + 256, ... (at most kEPT).
constexpr int kPT = 32;
constexpr int kEPT = 36;   // og * 9cg <= 256 * 36 (group widths up to 32)

template <bool BF>
__global__ void __launch_bounds__(kThreads) gconv_wgrad_kernel(const float* __restrict__ x,
                                                              const float* __restrict__ dy,
                                                              float* __restrict__ part, ConvGeo g, int G,
                                                              int pix) {
  extern __shared__ float sm[];  // dys [kPT][og], xs [kPT][9cg]
  const int cg = g.C / G, og = g.Co / G, grp = blockIdx.y;
  const int kw9 = 9 * cg, ne = og * kw9;
  float* dys = sm;
  float* xs = sm + kPT * og;
  float acc[kEPT];
#pragma unroll
  for (int j = 0; j < kEPT; ++j) acc[j] = 0.f;
  const long P = (long)g.B * g.Ho * g.Wo;
  const long p0 = (long)blockIdx.x * pix;
  const long pend = min(P, p0 + pix);
  for (long pt = p0; pt < pend; pt += kPT) {
    const int np = (int)min((long)kPT, pend - pt);
    __syncthreads();
    for (int e = threadIdx.x; e < kPT * og; e += kThreads) {
      const int i = e / og, co = e - i * og;
      dys[e] = i < np ? dy[(size_t)(pt + i) * g.Co + grp * og + co] : 0.f;
    }
    for (int e = threadIdx.x; e < kPT * kw9; e += kThreads) {
      const int i = e / kw9, k = e - i * kw9;
      float v = 0.f;
      if (i < np) {
        const long p = pt + i;
        const int b = (int)(p / ((long)g.Ho * g.Wo));
        const int q = (int)(p - (long)b * g.Ho * g.Wo);
        const int ho = q / g.Wo, wo = q - ho * g.Wo;
        const int tap = k / cg, ci = k - tap * cg, kh = tap / 3, kw = tap - kh * 3;
        const int hi = ho * g.stride - g.pad + kh, wi = wo * g.stride - g.pad + kw;
        if ((unsigned)hi < (unsigned)g.H && (unsigned)wi < (unsigned)g.W)
          v = opnd<BF>(x[(((size_t)b * g.H + hi) * g.W + wi) * g.C + grp * cg + ci]);
      }
      xs[e] = v;
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
__global__ void __launch_bounds__(kThreads) chunk_sum_kernel(const float* __restrict__ part, int chunks, long n,
                                                            float* __restrict__ dst) {
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
    float s = 0.f;
    for (int z = 0; z < chunks; ++z) s += part[(size_t)z * n + i];
    dst[i] = s;
  }
}

// ---------------------------------------------------------- squeeze-excite
// z[f][c] = mean over the HW pixels of y[f][.][c]  (grid F x ceil(C/64);
// thread (lane, row): channel lane, pixels row, row + 4, ...).
__global__ void __launch_bounds__(kThreads) se_squeeze_kernel(const float* __restrict__ y, int HW, int C,
                                                             float* __restrict__ z) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int f = blockIdx.x, c = blockIdx.y * 64 + lane;
  float s = 0.f;
  if (c < C) {
    const float* yf = y + (size_t)f * HW * C + c;
    for (int p = row; p < HW; p += 4) s += yf[(size_t)p * C];
  }
  red[row][lane] = s;
  __syncthreads();
  if (row == 0 && c < C) z[(size_t)f * C + c] = ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) / HW;
}

// One workgroup per frame: a1 = W1 z + b1 (stored, pre-activation),
// h = relu(a1), s = sigmoid(W2 h + b2).
__global__ void __launch_bounds__(kThreads) se_fc_fwd_kernel(const float* __restrict__ z, int C, int R,
                                                            const float* __restrict__ w1,
                                                            const float* __restrict__ b1,
                                                            const float* __restrict__ w2,
                                                            const float* __restrict__ b2, float* __restrict__ a1,
                                                            float* __restrict__ s) {
  extern __shared__ float sm[];  // zs [C], hs [R]
  float* zs = sm;
  float* hs = sm + C;
  const int f = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = threadIdx.x; c < C; c += kThreads) zs[c] = z[(size_t)f * C + c];
  __syncthreads();
  for (int j = wv; j < R; j += kThreads / 64) {
    float acc = 0.f;
    for (int c = lane; c < C; c += 64) acc = fmaf(w1[(size_t)j * C + c], zs[c], acc);
    acc = wave_sum(acc) + b1[j];
    if (lane == 0) {
      a1[(size_t)f * R + j] = acc;
      hs[j] = fmaxf(acc, 0.f);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += kThreads) {
    float acc = b2[c];
    for (int j = 0; j < R; ++j) acc = fmaf(w2[(size_t)c * R + j], hs[j], acc);
    s[(size_t)f * C + c] = sigm(acc);
  }
}

// out = relu(s[f][c] * y + res)
__global__ void __launch_bounds__(kThreads) se_excite_kernel(const float* __restrict__ y,
                                                            const float* __restrict__ s,
                                                            const float* __restrict__ res, long n, int HWC, int C,
                                                            float* __restrict__ out) {
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
    const long f = i / HWC;
    const int c = (int)(i % C);
    out[i] = fmaxf(fmaf(s[f * C + c], y[i], res[i]), 0.f);
  }
}

// Backward, first pass (grid F x ceil(C/64)): dpre = dout * [out > 0] into
// dres (the shortcut's gradient) and ds[f][c] = sum over pixels of dpre * y.
__global__ void __launch_bounds__(kThreads) se_bwd_reduce_kernel(const float* __restrict__ dout,
                                                                const float* __restrict__ out,
                                                                const float* __restrict__ y, int HW, int C,
                                                                float* __restrict__ dres, float* __restrict__ ds) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int f = blockIdx.x, c = blockIdx.y * 64 + lane;
  float acc = 0.f;
  if (c < C) {
    const size_t base = (size_t)f * HW * C + c;
    for (int p = row; p < HW; p += 4) {
      const size_t i = base + (size_t)p * C;
      const float d = out[i] > 0.f ? dout[i] : 0.f;
      dres[i] = d;
      acc = fmaf(d, y[i], acc);
    }
  }
  red[row][lane] = acc;
  __syncthreads();
  if (row == 0 && c < C) ds[(size_t)f * C + c] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Backward through the gate, one workgroup per frame:
//   da2 = ds * s (1 - s);  da1 = (W2^T da2) * [a1 > 0];  dz = W1^T da1.
__global__ void __launch_bounds__(kThreads) se_fc_bwd_kernel(const float* __restrict__ ds,
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
    const float sv = s[(size_t)f * C + c];
    const float v = ds[(size_t)f * C + c] * sv * (1.f - sv);
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
  const long n1 = (long)R * C, n2 = n1 + R, n3 = n2 + (long)C * R, n4 = n3 + C;
  for (long e = (long)blockIdx.x * kThreads + threadIdx.x; e < n4; e += (long)gridDim.x * kThreads) {
    float acc = 0.f;
    if (e < n1) {
      const int j = (int)(e / C), c = (int)(e - (long)j * C);
      for (int f = 0; f < F; ++f) acc = fmaf(da1[(size_t)f * R + j], z[(size_t)f * C + c], acc);
      gw1[e] = acc;
    } else if (e < n2) {
      const int j = (int)(e - n1);
      for (int f = 0; f < F; ++f) acc += da1[(size_t)f * R + j];
      gb1[j] = acc;
    } else if (e < n3) {
      const long q = e - n2;
      const int c = (int)(q / R), j = (int)(q - (long)c * R);
      for (int f = 0; f < F; ++f) acc = fmaf(da2[(size_t)f * C + c], fmaxf(a1[(size_t)f * R + j], 0.f), acc);
      gw2[q] = acc;
    } else {
      const int c = (int)(e - n3);
      for (int f = 0; f < F; ++f) acc += da2[(size_t)f * C + c];
      gb2[c] = acc;
    }
  }
}

// dy = s[f][c] * dpre + dz[f][c] / HW  (the gradient at the branch y)
__global__ void __launch_bounds__(kThreads) se_excite_bwd_kernel(const float* __restrict__ dpre,
                                                                const float* __restrict__ s,
                                                                const float* __restrict__ dz, long n, int HWC, int C,
                                                                float inv_hw, float* __restrict__ dy) {
  for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
    const long f = i / HWC;
    const int c = (int)(i % C);
    dy[i] = fmaf(s[f * C + c], dpre[i], dz[f * C + c] * inv_hw);
  }
}

unsigned grid_for(long n) { return (unsigned)std::max<long>(1, std::min<long>(cdiv(n, kThreads), 8192)); }

// Output pixels per workgroup: enough workgroups to fill the chip, at most
// 16 passes of the workgroup's rows.
int pix_per_block(long P, int rows, int G) {
  const long per_group = std::max<long>(1, 2048 / G);   // about 2048 workgroups in all
  long pix = (P + per_group - 1) / per_group;
  pix = std::max<long>(rows, std::min<long>(pix, (long)rows * 16));
  return (int)((pix + rows - 1) / rows * rows);
}

}  // namespace

bool gconv_supported(const ConvGeo& g, int G) {
  if (G <= 0 || g.C % G || g.Co % G || g.KH != 3 || g.KW != 3) return false;
  const int cg = g.C / G, og = g.Co / G;
  // one output channel (input channel for the data gradient) per thread of a
  // row, every weight-gradient element among a thread's kEPT, LDS within 64 KB
  const size_t lds = std::max((size_t)9 * cg * og, (size_t)kPT * (og + 9 * cg)) * sizeof(float);
  return cg <= kThreads && og <= kThreads && og * 9 * cg <= kThreads * kEPT && lds <= 65536;
}

void launch_gconv_fwd(int prec, const ConvGeo& g, int G, const float* x, const void* w, float* y,
                      hipStream_t s) {
  const int og = g.Co / G, rows = kThreads / og;
  const long P = (long)g.B * g.Ho * g.Wo;
  const int pix = pix_per_block(P, rows, G);
  const dim3 grid((unsigned)cdiv(P, pix), (unsigned)G);
  const size_t sh = (size_t)9 * (g.C / G) * og * sizeof(float);
  if (prec == 1)
    hipLaunchKernelGGL(gconv_fwd_kernel<bf16_t>, grid, dim3(kThreads), sh, s, x, (const bf16_t*)w, y, g, G, pix);
  else
    hipLaunchKernelGGL(gconv_fwd_kernel<float>, grid, dim3(kThreads), sh, s, x, (const float*)w, y, g, G, pix);
}

void launch_gconv_dgrad(int prec, const ConvGeo& g, int G, const float* dy, const void* w, float* dx,
                        int accumulate, hipStream_t s) {
  const int cg = g.C / G, rows = kThreads / cg;
  const long P = (long)g.B * g.H * g.W;
  const int pix = pix_per_block(P, rows, G);
  const dim3 grid((unsigned)cdiv(P, pix), (unsigned)G);
  const size_t sh = (size_t)9 * cg * (g.Co / G) * sizeof(float);
  if (prec == 1)
    hipLaunchKernelGGL(gconv_dgrad_kernel<bf16_t>, grid, dim3(kThreads), sh, s, dy, (const bf16_t*)w, dx, g, G,
                       pix, accumulate);
  else
    hipLaunchKernelGGL(gconv_dgrad_kernel<float>, grid, dim3(kThreads), sh, s, dy, (const float*)w, dx, g, G, pix,
                       accumulate);
}

void launch_gconv_wgrad(int prec, const ConvGeo& g, int G, const float* x, const float* dy, float* dw,
                        float* part, size_t part_bytes, hipStream_t s) {
  const int cg = g.C / G, og = g.Co / G;
  const long n = (long)g.Co * 9 * cg;
  const long P = (long)g.B * g.Ho * g.Wo;
  const long cap = std::max<long>(1, (long)(part_bytes / ((size_t)n * sizeof(float))));
  // chunks of at least 256 pixels, about 4096 workgroups, within the partial buffer
  long chunks = std::min<long>(std::max<long>(1, 4096 / G), std::max<long>(1, P / 256));
  chunks = std::max<long>(1, std::min(chunks, cap));
  long pix = (P + chunks - 1) / chunks;
  pix = (pix + kPT - 1) / kPT * kPT;
  chunks = (P + pix - 1) / pix;
  const size_t sh = (size_t)kPT * (og + 9 * cg) * sizeof(float);
  const dim3 grid((unsigned)chunks, (unsigned)G);
  if (prec == 1)
    hipLaunchKernelGGL(gconv_wgrad_kernel<true>, grid, dim3(kThreads), sh, s, x, dy, part, g, G, (int)pix);
  else
    hipLaunchKernelGGL(gconv_wgrad_kernel<false>, grid, dim3(kThreads), sh, s, x, dy, part, g, G, (int)pix);
  hipLaunchKernelGGL(chunk_sum_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, part, (int)chunks, n, dw);
}

void launch_se_forward(const float* y, const float* res, int F, int HW, int C, int R, const float* w1,
                       const float* b1, const float* w2, const float* b2, float* z, float* a1, float* gate,
                       float* out, hipStream_t s) {
  hipLaunchKernelGGL(se_squeeze_kernel, dim3(F, cdiv(C, 64)), dim3(kThreads), 0, s, y, HW, C, z);
  hipLaunchKernelGGL(se_fc_fwd_kernel, dim3(F), dim3(kThreads), (size_t)(C + R) * sizeof(float), s, z, C, R, w1,
                     b1, w2, b2, a1, gate);
  const long n = (long)F * HW * C;
  hipLaunchKernelGGL(se_excite_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, y, gate, res, n, HW * C, C, out);
}

void launch_se_backward(const float* dout, const float* out, const float* y, const float* z, const float* a1,
                        const float* gate, int F, int HW, int C, int R, const float* w1, const float* w2,
                        float* dres, float* ds, float* da2, float* da1, float* dz, float* gw1, float* gb1,
                        float* gw2, float* gb2, float* dy, hipStream_t s) {
  hipLaunchKernelGGL(se_bwd_reduce_kernel, dim3(F, cdiv(C, 64)), dim3(kThreads), 0, s, dout, out, y, HW, C, dres,
                     ds);
  hipLaunchKernelGGL(se_fc_bwd_kernel, dim3(F), dim3(kThreads), (size_t)(C + R) * sizeof(float), s, ds, gate, a1,
                     C, R, w1, w2, da2, da1, dz);
  const long nw = 2L * R * C + R + C;
  hipLaunchKernelGGL(se_fc_wgrad_kernel, dim3(grid_for(nw)), dim3(kThreads), 0, s, z, a1, da1, da2, F, C, R, gw1,
                     gb1, gw2, gb2);
  const long n = (long)F * HW * C;
  hipLaunchKernelGGL(se_excite_bwd_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, dres, gate, dz, n, HW * C, C,
                     1.f / HW, dy);
}
