// GroupNorm forward/backward, max pool 3x3/2, frame preparation (2x2 average
// pool + NCHW -> NHWC), and small elementwise helpers.
//
// Activations are [B][P][C] (NHWC, P = H*W pixels).  GroupNorm statistics are
// gathered in two steps: every workgroup reduces one chunk of pixels of one
// image for all channels into per-channel shifted sums, then one wavefront
// per (image, group) merges the chunk results with the exact
// parallel-variance formula (each chunk's centred second moment plus n_i
// (mean_i - mean)^2), all in float32.
#include "common.h"
#include "kernels.h"

// ------------------------------------------------------------------ forward
// part[(b*S + s)*C + c] = {sum(y - K), sum((y - K)^2), K}, K = y at the chunk's
// first pixel.
__global__ void __launch_bounds__(256) gn_partial_kernel(const float* __restrict__ y, int P, int C,
                                                         int S, float4* __restrict__ part) {
  // lanes take channel quads (float4 loads), the rest of the block walks pixels
  __shared__ float4 s1[256], s2[256];
  const int b = blockIdx.y, s = blockIdx.x, tid = threadIdx.x;
  const int chunk = (P + S - 1) / S;
  const int p0 = s * chunk, p1 = min(P, p0 + chunk);
  const float* yb = y + (size_t)b * P * C;
  const int C4 = C >> 2;
  const int QT = C4 < 256 ? C4 : 256;  // channel quads per pass
  const int PR = 256 / QT;             // pixel lanes
  const int q0 = tid % QT, pr = tid / QT;
  for (int qb = 0; qb < C4; qb += QT) {
    const int c = 4 * (qb + q0);
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), q = a, K = a;
    if (p0 < p1 && pr < PR) {
      K = *(const float4*)(yb + (size_t)p0 * C + c);
      for (int p = p0 + pr; p < p1; p += PR) {
        const float4 v = *(const float4*)(yb + (size_t)p * C + c);
        const float4 d = make_float4(v.x - K.x, v.y - K.y, v.z - K.z, v.w - K.w);
        a.x += d.x; a.y += d.y; a.z += d.z; a.w += d.w;
        q.x += d.x * d.x; q.y += d.y * d.y; q.z += d.z * d.z; q.w += d.w * d.w;
      }
    }
    s1[tid] = a;
    s2[tid] = q;
    __syncthreads();
    if (pr == 0) {
      for (int r = 1; r < PR; ++r) {
        const float4 u = s1[r * QT + q0], w = s2[r * QT + q0];
        a.x += u.x; a.y += u.y; a.z += u.z; a.w += u.w;
        q.x += w.x; q.y += w.y; q.z += w.z; q.w += w.w;
      }
      const float n = (float)max(0, p1 - p0);
      float4* o = part + ((size_t)b * S + s) * C + c;
      o[0] = make_float4(a.x, q.x, K.x, n);
      o[1] = make_float4(a.y, q.y, K.y, n);
      o[2] = make_float4(a.z, q.z, K.z, n);
      o[3] = make_float4(a.w, q.w, K.w, n);
    }
    __syncthreads();
  }
}

// One wavefront per (b, g): mean and 1/sqrt(var + eps) of the group.
__global__ void __launch_bounds__(256) gn_finalize_kernel(const float4* __restrict__ part, int B, int S,
                                                          int C, int G, float eps,
                                                          float2* __restrict__ stats) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (wid >= B * G) return;
  const int b = wid / G, g = wid % G, Cg = C / G;
  const int nparts = S * Cg;
  float sn = 0.f, sx = 0.f;
#pragma unroll 4
  for (int i = lane; i < nparts; i += 64) {
    const int s = i / Cg, c = g * Cg + i % Cg;
    const float4 v = part[((size_t)b * S + s) * C + c];
    sn += v.w;
    sx += fmaf(v.w, v.z, v.x);  // n K + sum(y - K)
  }
  sn = wave_sum(sn);
  sx = wave_sum(sx);
  const float mean = sn > 0.f ? sx / sn : 0.f;
  float m2 = 0.f;
#pragma unroll 4
  for (int i = lane; i < nparts; i += 64) {
    const int s = i / Cg, c = g * Cg + i % Cg;
    const float4 v = part[((size_t)b * S + s) * C + c];
    if (v.w > 0.f) {
      const float n = v.w, a = v.x / n;  // chunk mean - K
      const float m2i = fmaxf(v.y - v.x * a, 0.f);
      const float d = (v.z - mean) + a;
      m2 += fmaf(n * d, d, m2i);
    }
  }
  m2 = wave_sum(m2);
  if (lane == 0) {
    const float var = sn > 0.f ? fmaxf(m2 / sn, 0.f) : 0.f;
    stats[wid] = make_float2(mean, 1.0f / sqrtf(var + eps));
  }
}

// out = [relu]( (y - mean) rstd gamma + beta [+ res] ), written NHWC or,
// with out_chw, as [B][C][P].
__global__ void __launch_bounds__(256) gn_apply_kernel(const float* __restrict__ y, int B, int P,
                                                       int C, int G, const float2* __restrict__ stats,
                                                       const float* __restrict__ gamma,
                                                       const float* __restrict__ beta,
                                                       const float* __restrict__ res, int relu,
                                                       float* __restrict__ out, int out_chw) {
  const int C4 = C >> 2, Cg = C / G;
  const int rows = B * P, n4 = rows * C4;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n4; i += gridDim.x * 256) {
    const int row = i / C4, c = 4 * (i - row * C4);
    const int b = row / P, p = row - b * P;
    const size_t e = (size_t)row * C + c;
    const float4 v = *(const float4*)(y + e);
    const float r[4] = {v.x, v.y, v.z, v.w};
    float4 rr = make_float4(0.f, 0.f, 0.f, 0.f);
    if (res) rr = *(const float4*)(res + e);
    const float ra[4] = {rr.x, rr.y, rr.z, rr.w};
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 st = stats[b * G + (c + j) / Cg];
      o[j] = (r[j] - st.x) * st.y * gamma[c + j] + beta[c + j] + ra[j];
      if (relu) o[j] = fmaxf(o[j], 0.f);
    }
    if (!out_chw) {
      *(float4*)(out + e) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) out[((size_t)b * C + c + j) * P + p] = o[j];
    }
  }
}

void launch_gn_forward(const float* y, int B, int P, int C, int G, float eps, const float* gamma,
                       const float* beta, const float* res, int relu, float* out, int out_chw,
                       float2* stats, float4* part, int S, hipStream_t s) {
  hipLaunchKernelGGL(gn_partial_kernel, dim3(S, B), dim3(256), 0, s, y, P, C, S, part);
  hipLaunchKernelGGL(gn_finalize_kernel, dim3(cdiv((long)B * G, 4)), dim3(256), 0, s, part, B, S, C,
                     G, eps, stats);
  const size_t n4 = (size_t)B * P * C / 4;
  const int nb = (int)std::min<size_t>(8192, (n4 + 255) / 256);
  hipLaunchKernelGGL(gn_apply_kernel, dim3(nb), dim3(256), 0, s, y, B, P, C, G, stats, gamma, beta,
                     res, relu, out, out_chw);
}

// ----------------------------------------------------------------- backward
// dz = dout * [out > 0] (when relu), xhat = (y - mean) rstd.
// bpart[(b*S + s)*C + c] = {sum dz, sum dz xhat}.
DEV size_t io_index(int b, int p, int c, int P, int C, int chw) {
  return chw ? ((size_t)b * C + c) * P + p : ((size_t)b * P + p) * C + c;
}

__global__ void __launch_bounds__(256) gnb_partial_kernel(const float* __restrict__ dout,
                                                          const float* __restrict__ out, int chw,
                                                          const float* __restrict__ y, int P, int C,
                                                          int G, int S, const float2* __restrict__ stats,
                                                          float2* __restrict__ bpart) {
  __shared__ float4 s1[256], s2[256];
  const int b = blockIdx.y, s = blockIdx.x, tid = threadIdx.x;
  const int chunk = (P + S - 1) / S;
  const int p0 = s * chunk, p1 = min(P, p0 + chunk);
  const int C4 = C >> 2;
  const int QT = C4 < 256 ? C4 : 256;
  const int PR = 256 / QT;
  const int q0 = tid % QT, pr = tid / QT;
  const int Cg = C / G;
  for (int qb = 0; qb < C4; qb += QT) {
    const int c = 4 * (qb + q0);
    float a[4] = {0.f, 0.f, 0.f, 0.f}, q[4] = {0.f, 0.f, 0.f, 0.f};
    if (pr < PR) {
      float2 st[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) st[j] = stats[b * G + (c + j) / Cg];
      for (int p = p0 + pr; p < p1; p += PR) {
        const size_t e = ((size_t)b * P + p) * C + c;
        float dz[4], om[4] = {1.f, 1.f, 1.f, 1.f};
        if (!chw) {
          const float4 d = *(const float4*)(dout + e);
          dz[0] = d.x; dz[1] = d.y; dz[2] = d.z; dz[3] = d.w;
          if (out) {
            const float4 m = *(const float4*)(out + e);
            om[0] = m.x; om[1] = m.y; om[2] = m.z; om[3] = m.w;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const size_t io = ((size_t)b * C + c + j) * P + p;
            dz[j] = dout[io];
            if (out) om[j] = out[io];
          }
        }
        const float4 yv = *(const float4*)(y + e);
        const float yy[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float z = om[j] > 0.f ? dz[j] : 0.f;
          a[j] += z;
          q[j] += z * (yy[j] - st[j].x) * st[j].y;
        }
      }
    }
    s1[tid] = make_float4(a[0], a[1], a[2], a[3]);
    s2[tid] = make_float4(q[0], q[1], q[2], q[3]);
    __syncthreads();
    if (pr == 0) {
      for (int r = 1; r < PR; ++r) {
        const float4 u = s1[r * QT + q0], w = s2[r * QT + q0];
        a[0] += u.x; a[1] += u.y; a[2] += u.z; a[3] += u.w;
        q[0] += w.x; q[1] += w.y; q[2] += w.z; q[3] += w.w;
      }
      float2* o = bpart + ((size_t)b * S + s) * C + c;
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] = make_float2(a[j], q[j]);
    }
    __syncthreads();
  }
}

// Two reductions of the chunk partials in one launch (one wavefront per item):
//   items [0, B G):    coef[b*G+g] = {sum_c gamma_c sum dz / n, sum_c gamma_c sum dz xhat / n}
//   items [B G, +C):   dgamma[c] = sum_{b,s} sum dz xhat, dbeta[c] = sum_{b,s} sum dz
__global__ void __launch_bounds__(256) gnb_coef_affine_kernel(const float2* __restrict__ bpart, int B, int S,
                                                              int C, int G, int P,
                                                              const float* __restrict__ gamma,
                                                              float2* __restrict__ coef, float* __restrict__ dgamma,
                                                              float* __restrict__ dbeta) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (wid < B * G) {
    const int b = wid / G, g = wid % G, Cg = C / G;
    float a = 0.f, q = 0.f;
#pragma unroll 4
    for (int i = lane; i < S * Cg; i += 64) {
      const int s = i / Cg, c = g * Cg + i % Cg;
      const float2 v = bpart[((size_t)b * S + s) * C + c];
      a = fmaf(gamma[c], v.x, a);
      q = fmaf(gamma[c], v.y, q);
    }
    a = wave_sum(a);
    q = wave_sum(q);
    if (lane == 0) {
      const float n = (float)P * (float)Cg;
      coef[wid] = make_float2(a / n, q / n);
    }
    return;
  }
  const int c = wid - B * G;
  if (c >= C) return;
  float a = 0.f, q = 0.f;
#pragma unroll 4
  for (int i = lane; i < B * S; i += 64) {
    const float2 v = bpart[(size_t)i * C + c];
    a += v.x;
    q += v.y;
  }
  a = wave_sum(a);
  q = wave_sum(q);
  if (lane == 0) {
    dgamma[c] = q;
    dbeta[c] = a;
  }
}

// dgamma / dbeta only (the one-launch backward's per-image partials, S = 1).
__global__ void __launch_bounds__(256) gnb_affine_kernel(const float2* __restrict__ bpart, int B, int S,
                                                         int C, float* __restrict__ dgamma,
                                                         float* __restrict__ dbeta) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= C) return;
  float a = 0.f, q = 0.f;
#pragma unroll 4
  for (int i = lane; i < B * S; i += 64) {
    const float2 v = bpart[(size_t)i * C + c];
    a += v.x;
    q += v.y;
  }
  a = wave_sum(a);
  q = wave_sum(q);
  if (lane == 0) {
    dgamma[c] = q;
    dbeta[c] = a;
  }
}

// dy = rstd (dz gamma - coef.x - xhat coef.y); dres (optional) = dz.  NHWC outputs.
__global__ void __launch_bounds__(256) gnb_apply_kernel(const float* __restrict__ dout,
                                                        const float* __restrict__ out, int chw,
                                                        const float* __restrict__ y, int B, int P, int C,
                                                        int G, const float2* __restrict__ stats,
                                                        const float2* __restrict__ coef,
                                                        const float* __restrict__ gamma,
                                                        float* __restrict__ dy, float* __restrict__ dres) {
  const int C4 = C >> 2, Cg = C / G;
  const int rows = B * P, n4 = rows * C4;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n4; i += gridDim.x * 256) {
    const int row = i / C4, c = 4 * (i - row * C4);
    const int b = row / P, p = row - b * P;
    const size_t e = (size_t)row * C + c;
    float dz[4], om[4] = {1.f, 1.f, 1.f, 1.f};
    if (!chw) {
      const float4 d = *(const float4*)(dout + e);
      dz[0] = d.x; dz[1] = d.y; dz[2] = d.z; dz[3] = d.w;
      if (out) {
        const float4 m = *(const float4*)(out + e);
        om[0] = m.x; om[1] = m.y; om[2] = m.z; om[3] = m.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const size_t io = ((size_t)b * C + c + j) * P + p;
        dz[j] = dout[io];
        if (out) om[j] = out[io];
      }
    }
    const float4 yv = *(const float4*)(y + e);
    const float yy[4] = {yv.x, yv.y, yv.z, yv.w};
    float o[4], zz[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int bg = b * G + (c + j) / Cg;
      const float2 st = stats[bg], cf = coef[bg];
      const float z = om[j] > 0.f ? dz[j] : 0.f;
      zz[j] = z;
      o[j] = st.y * (z * gamma[c + j] - cf.x - (yy[j] - st.x) * st.y * cf.y);
    }
    *(float4*)(dy + e) = make_float4(o[0], o[1], o[2], o[3]);
    if (dres) *(float4*)(dres + e) = make_float4(zz[0], zz[1], zz[2], zz[3]);
  }
}

void launch_gn_backward(const float* dout, const float* out, int chw, const float* y, int B, int P,
                        int C, int G, const float2* stats, const float* gamma, float* dy, float* dres,
                        float* dgamma, float* dbeta, float2* bpart, float2* coef, int S,
                        hipStream_t s) {
  hipLaunchKernelGGL(gnb_partial_kernel, dim3(S, B), dim3(256), 0, s, dout, out, chw, y, P, C, G, S,
                     stats, bpart);
  hipLaunchKernelGGL(gnb_coef_affine_kernel, dim3(cdiv((long)B * G + C, 4)), dim3(256), 0, s, bpart, B, S, C,
                     G, P, gamma, coef, dgamma, dbeta);
  const size_t n = (size_t)B * P * C / 4;
  const int nb = (int)std::min<size_t>(8192, (n + 255) / 256);
  hipLaunchKernelGGL(gnb_apply_kernel, dim3(nb), dim3(256), 0, s, dout, out, chw, y, B, P, C, G, stats,
                     coef, gamma, dy, dres);
}

// ------------------------------------------------------------------ pooling
// 3x3 window, stride 2, padding 1; arg = index 0..8 of the first maximum in
// row-major window order.
__global__ void __launch_bounds__(256) maxpool_fwd_kernel(const float* __restrict__ x, int B, int H,
                                                          int W, int C, int Ho, int Wo,
                                                          float* __restrict__ y,
                                                          uint8_t* __restrict__ arg) {
  const size_t n = (size_t)B * Ho * Wo * C;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const int c = (int)(e % C);
    size_t r = e / C;
    const int wo = (int)(r % Wo);
    r /= Wo;
    const int ho = (int)(r % Ho);
    const int b = (int)(r / Ho);
    // all nine window loads first (outside taps read a clamped in-bounds
    // element and are skipped), then the first maximum in window order
    float v[9];
    bool ok[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int hi = 2 * ho - 1 + t / 3, wi = 2 * wo - 1 + t % 3;
      ok[t] = hi >= 0 && hi < H && wi >= 0 && wi < W;
      v[t] = x[(((size_t)b * H + min(max(hi, 0), H - 1)) * W + min(max(wi, 0), W - 1)) * C + c];
    }
    float best = -INFINITY;
    int bi = 0;
#pragma unroll
    for (int t = 0; t < 9; ++t)
      if (ok[t] && v[t] > best) {
        best = v[t];
        bi = t;
      }
    y[e] = best;
    arg[e] = (uint8_t)bi;
  }
}

// dx[b,h,w,c] = sum of dy over the (at most 4) windows whose winner is (h, w).
__global__ void __launch_bounds__(256) maxpool_bwd_kernel(const float* __restrict__ dy,
                                                          const uint8_t* __restrict__ arg, int B, int H,
                                                          int W, int C, int Ho, int Wo,
                                                          float* __restrict__ dx) {
  const size_t n = (size_t)B * H * W * C;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const int c = (int)(e % C);
    size_t r = e / C;
    const int w = (int)(r % W);
    r /= W;
    const int h = (int)(r % H);
    const int b = (int)(r / H);
    float acc = 0.f;
    const int ho_lo = max(0, h / 2), ho_hi = min(Ho - 1, (h + 1) / 2);
    const int wo_lo = max(0, w / 2), wo_hi = min(Wo - 1, (w + 1) / 2);
    for (int ho = ho_lo; ho <= ho_hi; ++ho)
      for (int wo = wo_lo; wo <= wo_hi; ++wo) {
        const int kh = h - (2 * ho - 1), kw = w - (2 * wo - 1);
        if (kh < 0 || kh > 2 || kw < 0 || kw > 2) continue;
        const size_t o = (((size_t)b * Ho + ho) * Wo + wo) * C + c;
        if (arg[o] == kh * 3 + kw) acc += dy[o];
      }
    dx[e] = acc;
  }
}

void launch_maxpool_fwd(const float* x, int B, int H, int W, int C, float* y, uint8_t* arg,
                        hipStream_t s) {
  const int Ho = (H - 1) / 2 + 1, Wo = (W - 1) / 2 + 1;
  const size_t n = (size_t)B * Ho * Wo * C;
  hipLaunchKernelGGL(maxpool_fwd_kernel, dim3((int)std::min<size_t>(8192, (n + 255) / 256)), dim3(256),
                     0, s, x, B, H, W, C, Ho, Wo, y, arg);
}

void launch_maxpool_bwd(const float* dy, const uint8_t* arg, int B, int H, int W, int C, float* dx,
                        hipStream_t s) {
  const int Ho = (H - 1) / 2 + 1, Wo = (W - 1) / 2 + 1;
  const size_t n = (size_t)B * H * W * C;
  hipLaunchKernelGGL(maxpool_bwd_kernel, dim3((int)std::min<size_t>(8192, (n + 255) / 256)), dim3(256),
                     0, s, dy, arg, B, H, W, C, Ho, Wo, dx);
}

// ------------------------------------------------------------ frame prep
// x0[f][h][w][c] = mean of the 2x2 block (or the pixel) of frame src[f]
// (obs + src[f]*C*Hin*Win, NCHW, float32 or bfloat16).
template <typename T>
__global__ void __launch_bounds__(256) prep_kernel(const T* __restrict__ obs,
                                                   const int32_t* __restrict__ src, int F, int C,
                                                   int Hin, int Win, int pool, float* __restrict__ x0) {
  const int Ho = pool ? Hin / 2 : Hin, Wo = pool ? Win / 2 : Win;
  const size_t n = (size_t)F * Ho * Wo * C;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256) {
    const int c = (int)(e % C);
    size_t r = e / C;
    const int w = (int)(r % Wo);
    r /= Wo;
    const int h = (int)(r % Ho);
    const int f = (int)(r / Ho);
    const size_t fr = src ? (size_t)src[f] : (size_t)f;
    const T* p = obs + (fr * C + c) * Hin * Win;
    float v;
    if (pool) {
      const T* q = p + (size_t)(2 * h) * Win + 2 * w;
      v = 0.25f * ((ldf(q) + ldf(q + 1)) + (ldf(q + Win) + ldf(q + Win + 1)));
    } else {
      v = ldf(p + (size_t)h * Win + w);
    }
    x0[e] = v;
  }
}

void launch_prep(const void* obs, int bf16, const int32_t* src, int F, int C, int Hin, int Win,
                 int pool, float* x0, hipStream_t s) {
  const int Ho = pool ? Hin / 2 : Hin, Wo = pool ? Win / 2 : Win;
  const size_t n = (size_t)F * Ho * Wo * C;
  const int nb = (int)std::min<size_t>(8192, (n + 255) / 256);
  if (bf16)
    hipLaunchKernelGGL(prep_kernel<bf16_t>, dim3(nb), dim3(256), 0, s, (const bf16_t*)obs, src, F, C,
                       Hin, Win, pool, x0);
  else
    hipLaunchKernelGGL(prep_kernel<float>, dim3(nb), dim3(256), 0, s, (const float*)obs, src, F, C, Hin,
                       Win, pool, x0);
}

// dx = dy * [y > 0]
__global__ void __launch_bounds__(256) relu_grad_kernel(const float* __restrict__ dy,
                                                        const float* __restrict__ y, size_t n,
                                                        float* __restrict__ dx) {
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (size_t)gridDim.x * 256)
    dx[e] = y[e] > 0.f ? dy[e] : 0.f;
}

void launch_relu_grad(const float* dy, const float* y, size_t n, float* dx, hipStream_t s) {
  const int nb = (int)std::min<size_t>(8192, (n + 255) / 256);
  hipLaunchKernelGGL(relu_grad_kernel, dim3(nb), dim3(256), 0, s, dy, y, n, dx);
}

// ------------------------------------------------------ fused GroupNorm
// One workgroup per (image b, group g) holds the group's P*Cg values in
// registers (NPT per thread, element e = p*Cg + cc, so a thread keeps one
// channel when 256 % Cg == 0): exact two-pass mean / variance, then the
// apply.  The input is the convolution output, or the sum of its split-K
// partial tiles (src + z*zstride), in which case the summed output can also
// be stored (u_out) for the backward.
// Two block sums in one reduction.
template <int NT>
DEV float2 block_sum2(float v0, float v1, float2* red) {
  const float d0 = wave_sum(v0), d1 = wave_sum(v1);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = make_float2(d0, d1);
  __syncthreads();
  float2 t = make_float2(0.f, 0.f);
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    t.x += red[i].x;
    t.y += red[i].y;
  }
  return t;
}

template <int NT = 256>
DEV float block_sum(float v, float* red) {
  const float d = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = d;
  __syncthreads();
  float t = 0.f;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

template <int NPT, int NT, bool DUAL>
__global__ void __launch_bounds__(NT) gn_fused_kernel(const float* __restrict__ src, int nsplit, size_t zstride,
                                                       float* __restrict__ u_out, int P, int C, int G, float eps,
                                                       const float* __restrict__ gamma,
                                                       const float* __restrict__ beta,
                                                       const float* __restrict__ res, int relu,
                                                       float* __restrict__ out, int out_chw,
                                                       float2* __restrict__ stats, int src_gm,
                                                       float* __restrict__ pool_out, int H, int W,
                                                       const float* __restrict__ src2, int nsplit2, int src2_gm,
                                                       const float* __restrict__ gamma2,
                                                       const float* __restrict__ beta2,
                                                       float2* __restrict__ stats2) {
  __shared__ float red[NT / 64];
  __shared__ float2 red2[DUAL ? NT / 64 : 1];
  extern __shared__ float s_slab[];  // pool_out: the normalised slab [p][cc] (P Cg floats)
  const int b = blockIdx.x / G, g = blockIdx.x - b * G;
  const int Cg = C / G, n = P * Cg;
  // element j of this thread: pixel p0 + j*pstep, channel c (NT % Cg == 0)
  const int cc = threadIdx.x % Cg, p0 = threadIdx.x / Cg, pstep = NT / Cg, c = g * Cg + cc;
  const size_t base = ((size_t)b * P + p0) * C + c, jstr = (size_t)pstep * C;
  // a group-major input holds this (b, g) slab contiguously, element (p, cc) at
  // p Cg + cc: this thread's element j at threadIdx.x + j NT (coalesced)
  const size_t sbase = src_gm ? (size_t)blockIdx.x * n + threadIdx.x : base;
  const size_t sjstr = src_gm ? (size_t)NT : jstr;
  // the split-K partials, ZB splits per round with every load of a round in
  // flight together (summed in split order: deterministic)
  constexpr int ZB = NPT >= 16 ? 1 : 16 / NPT;
  // the affine parameters and the residual are loaded up front, so their
  // latency overlaps the input loads and the reductions
  const float gm = gamma[c], be = beta[c];
  float rv[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) rv[j] = (res && p0 + j * pstep < P) ? res[base + j * jstr] : 0.f;
  float x[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) x[j] = 0.f;
  for (int z0 = 0; z0 < nsplit; z0 += ZB) {
    float y[ZB][NPT];
#pragma unroll
    for (int q = 0; q < ZB; ++q)
#pragma unroll
      for (int j = 0; j < NPT; ++j)
        y[q][j] = (z0 + q < nsplit && p0 + j * pstep < P) ? src[(size_t)(z0 + q) * zstride + sbase + j * sjstr] : 0.f;
#pragma unroll
    for (int q = 0; q < ZB; ++q)
#pragma unroll
      for (int j = 0; j < NPT; ++j) x[j] += y[q][j];
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    if (u_out && p0 + j * pstep < P) u_out[base + j * jstr] = x[j];
    s += x[j];
  }
  float mean, var;
  if constexpr (DUAL) {
    // a second GroupNorm of the same shape (a projection shortcut) whose
    // output is this one's residual: its partials summed, its statistics and
    // apply taken with the same per-thread sums and reductions as a launch of
    // its own, so the residual is that launch's output bit for bit
    const size_t sbase2 = src2_gm ? (size_t)blockIdx.x * n + threadIdx.x : base;
    const size_t sjstr2 = src2_gm ? (size_t)NT : jstr;
    float x2[NPT];
#pragma unroll
    for (int j = 0; j < NPT; ++j) x2[j] = 0.f;
    for (int z0 = 0; z0 < nsplit2; z0 += ZB) {
      float y[ZB][NPT];
#pragma unroll
      for (int q = 0; q < ZB; ++q)
#pragma unroll
        for (int j = 0; j < NPT; ++j)
          y[q][j] = (z0 + q < nsplit2 && p0 + j * pstep < P) ? src2[(size_t)(z0 + q) * zstride + sbase2 + j * sjstr2]
                                                               : 0.f;
#pragma unroll
      for (int q = 0; q < ZB; ++q)
#pragma unroll
        for (int j = 0; j < NPT; ++j) x2[j] += y[q][j];
    }
    float s2 = 0.f;
#pragma unroll
    for (int j = 0; j < NPT; ++j) s2 += x2[j];
    const float2 m12 = block_sum2<NT>(s, s2, red2);
    const float mean1 = m12.x / n, mean2 = m12.y / n;
    float q1 = 0.f, q2 = 0.f;
#pragma unroll
    for (int j = 0; j < NPT; ++j)
      if (p0 + j * pstep < P) {
        q1 += (x[j] - mean1) * (x[j] - mean1);
        q2 += (x2[j] - mean2) * (x2[j] - mean2);
      }
    const float2 v12 = block_sum2<NT>(q1, q2, red2);
    const float rstd2 = 1.0f / sqrtf(v12.y / n + eps);
    if (threadIdx.x == 0) stats2[blockIdx.x] = make_float2(mean2, rstd2);
    const float ga2 = gamma2[c] * rstd2, be2 = beta2[c];
#pragma unroll
    for (int j = 0; j < NPT; ++j) rv[j] = (x2[j] - mean2) * ga2 + be2 + 0.f;
    mean = mean1;       // this GroupNorm's statistics from the same sums as a launch of its own
    var = v12.x / n;
  } else {
    mean = block_sum<NT>(s, red) / n;
    float q = 0.f;
#pragma unroll
    for (int j = 0; j < NPT; ++j)
      if (p0 + j * pstep < P) q += (x[j] - mean) * (x[j] - mean);
    var = block_sum<NT>(q, red) / n;
  }
  const float rstd = 1.0f / sqrtf(var + eps);
  if (threadIdx.x == 0) stats[blockIdx.x] = make_float2(mean, rstd);
  const float ga = gm * rstd;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int p = p0 + j * pstep;
    if (p < P) {
      const size_t idx = base + j * jstr;
      float o = (x[j] - mean) * ga + be + rv[j];
      if (relu) o = fmaxf(o, 0.f);
      if (pool_out)
        s_slab[p * Cg + cc] = o;
      else
        out[out_chw ? ((size_t)b * C + c) * P + p : idx] = o;
    }
  }
  if (pool_out) {
    // 3x3 / 2 max pool (pad 1) of this group's channels from LDS; the plain
    // output is not written.  The window maximum over the in-bounds taps is
    // the same value max_pool's first maximum takes.
    __syncthreads();
    const int Ho = (H - 1) / 2 + 1, Wo = (W - 1) / 2 + 1, no = Ho * Wo * Cg;
    for (int e = threadIdx.x; e < no; e += NT) {
      const int c2 = e % Cg, q = e / Cg, wo = q % Wo, ho = q / Wo;
      float best = -INFINITY;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int hi = 2 * ho - 1 + t / 3, wi = 2 * wo - 1 + t % 3;
        if (hi >= 0 && hi < H && wi >= 0 && wi < W) {
          const float v = s_slab[(hi * W + wi) * Cg + c2];
          if (v > best) best = v;
        }
      }
      pool_out[(((size_t)b * Ho + ho) * Wo + wo) * C + g * Cg + c2] = best;
    }
  }
}

// Backward per (b, g): dz = dout [* (out > 0)], xhat = (y - mean) rstd;
// dy = rstd (dz gamma - mean(dz gamma) - xhat mean(dz gamma xhat)), dres = dz;
// bpart[b*C + c] = {sum_p dz, sum_p dz xhat} for the dgamma / dbeta reduction.
template <int NPT, int NT>
__global__ void __launch_bounds__(NT) gnb_fused_kernel(const float* __restrict__ dout,
                                                        const float* __restrict__ outm, int chw,
                                                        const float* __restrict__ y, int P, int C, int G,
                                                        const float2* __restrict__ stats,
                                                        const float* __restrict__ gamma, float* __restrict__ dy,
                                                        float* __restrict__ dres, float2* __restrict__ bpart) {
  __shared__ float2 red2[NT / 64];
  __shared__ float2 cred[NT];
  const int b = blockIdx.x / G, g = blockIdx.x - b * G;
  const int Cg = C / G, n = P * Cg;
  const float2 st = stats[blockIdx.x];
  const int cc = threadIdx.x % Cg, p0 = threadIdx.x / Cg, pstep = NT / Cg, c = g * Cg + cc;
  const size_t base = ((size_t)b * P + p0) * C + c, jstr = (size_t)pstep * C;
  const float gm = gamma[c];
  float dz[NPT], xh[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int p = p0 + j * pstep;
    float zv = 0.f, om = 1.f, yv = st.x;
    if (p < P) {
      const size_t io = chw ? ((size_t)b * C + c) * P + p : base + j * jstr;
      zv = dout[io];
      if (outm) om = outm[io];
      yv = y[base + j * jstr];
    }
    dz[j] = om > 0.f ? zv : 0.f;
    xh[j] = (yv - st.x) * st.y;
  }
  float s1 = 0.f, s2 = 0.f, cz = 0.f, czx = 0.f;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    s1 += dz[j] * gm;
    s2 += dz[j] * gm * xh[j];
    cz += dz[j];
    czx += dz[j] * xh[j];
  }
  const float2 sm = block_sum2<NT>(s1, s2, red2);
  const float m1 = sm.x / n, m2 = sm.y / n;
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    if (p0 + j * pstep < P) {
      const size_t idx = base + j * jstr;
      dy[idx] = st.y * (dz[j] * gm - m1 - xh[j] * m2);
      if (dres) dres[idx] = dz[j];
    }
  }
  cred[threadIdx.x] = make_float2(cz, czx);
  __syncthreads();
  if (threadIdx.x < Cg) {
    float a = 0.f, q = 0.f;
    for (int t = threadIdx.x; t < NT; t += Cg) {
      a += cred[t].x;
      q += cred[t].y;
    }
    bpart[(size_t)b * C + g * Cg + threadIdx.x] = make_float2(a, q);
  }
}

// Elements per thread (1..32) of the fused kernels, 0 when unsupported; the
// block has 256 threads up to 512 elements per (image, group), else 1024.
int gn_fused_npt(int P, int Cg) {
  const int n = P * Cg;
  if (256 % Cg) return 0;
  const int nt = n <= 256 * 2 ? 256 : 1024;
  for (int k = 1; k <= 32; k *= 2)
    if (n <= nt * k) return k;
  return 0;
}

#define GN_NPT_SWITCH(NT_, NPT_, CALL) \
  if (NT_ == 256) {                    \
    switch (NPT_) {                    \
      case 1: CALL(1, 256); break;     \
      case 2: CALL(2, 256); break;     \
      case 4: CALL(4, 256); break;     \
      default: CALL(8, 256); break;    \
    }                                  \
  } else {                             \
    switch (NPT_) {                    \
      case 1: CALL(1, 1024); break;    \
      case 2: CALL(2, 1024); break;    \
      case 4: CALL(4, 1024); break;    \
      case 8: CALL(8, 1024); break;    \
      case 16: CALL(16, 1024); break;  \
      default: CALL(32, 1024); break;  \
    }                                  \
  }

bool gn_pool_fits(int P, int Cg) { return (long)P * Cg * (long)sizeof(float) <= kGnPoolLds; }

void launch_gn_fused(const float* src, int nsplit, size_t zstride, float* u_out, int B, int P, int C, int G,
                     float eps, const float* gamma, const float* beta, const float* res, int relu, float* out,
                     int out_chw, float2* stats, hipStream_t s, int src_gm, float* pool_out, int H, int W,
                     const GnSecond* second) {
  const float* src2 = second ? second->src : nullptr;
  const int nsplit2 = second ? second->nsplit : 0, src2_gm = second ? second->src_gm : 0;
  const float* gamma2 = second ? second->gamma : nullptr;
  const float* beta2 = second ? second->beta : nullptr;
  float2* stats2 = second ? second->stats : nullptr;
  const int npt = gn_fused_npt(P, C / G), nt = (long)P * (C / G) <= 256 * 2 ? 256 : 1024;
  const size_t lds = pool_out ? (size_t)P * (C / G) * sizeof(float) : 0;
#define GN_CALL_D(K, T, D)                                                                                        \
  hipLaunchKernelGGL((gn_fused_kernel<K, T, D>), dim3(B * G), dim3(T), lds, s, src, nsplit, zstride, u_out, P, C, \
                     G, eps, gamma, beta, res, relu, out, out_chw, stats, src_gm, pool_out, H, W, src2, nsplit2,      \
                     src2_gm, gamma2, beta2, stats2)
#define GN_CALL(K, T) GN_CALL_D(K, T, false)
#define GN_CALL2(K, T) GN_CALL_D(K, T, true)
  if (second) {
    GN_NPT_SWITCH(nt, npt, GN_CALL2)
  } else {
    GN_NPT_SWITCH(nt, npt, GN_CALL)
  }
#undef GN_CALL
#undef GN_CALL2
#undef GN_CALL_D
}

void launch_gnb_fused(const float* dout, const float* outm, int chw, const float* y, int B, int P, int C, int G,
                      const float2* stats, const float* gamma, float* dy, float* dres, float* dgamma,
                      float* dbeta, float2* bpart, hipStream_t s) {
  const int npt = gn_fused_npt(P, C / G), nt = (long)P * (C / G) <= 256 * 2 ? 256 : 1024;
#define GNB_CALL(K, T)                                                                                       \
  hipLaunchKernelGGL((gnb_fused_kernel<K, T>), dim3(B * G), dim3(T), 0, s, dout, outm, chw, y, P, C, G, stats, \
                     gamma, dy, dres, bpart)
  GN_NPT_SWITCH(nt, npt, GNB_CALL)
#undef GNB_CALL
  hipLaunchKernelGGL(gnb_affine_kernel, dim3(cdiv(C, 4)), dim3(256), 0, s, bpart, B, 1, C, dgamma, dbeta);
}
